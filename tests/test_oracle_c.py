"""The plain C build of the oracle's server evaluation against the numpy oracle and the stored digests.

The C code (oracle/c/he_oracle.c) follows the same steps in C for timing on host cores; it must
give the numpy oracle's words on small rings (several shapes, first / last layer patterns, FC
with several blocks) and reproduce the stored full-size digests of the x1 plain-20 stack
(tests/golden/server_digests.json, written from the numpy oracle), and the single conv workload.
"""
import json
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import bfv, cserver, packing

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import cases  # noqa: E402

T = wl.T_PLAIN


@pytest.fixture(scope="module", autouse=True)
def built():
    cserver.build()


CONV = [
    # N, L, c_i, c_o, H, stride
    (256, 2, 3, 8, 4, 1),
    (256, 2, 6, 4, 4, 1),      # K_in = 2
    (256, 2, 4, 8, 4, 2),      # stride 2, K_out = 2
    (256, 2, 5, 3, 4, 1),      # ragged
    (1024, 3, 16, 24, 6, 1),
]


@pytest.mark.parametrize("N,L,c_i,c_o,H,stride", CONV)
@pytest.mark.parametrize("first,last", [(False, False), (True, False), (False, True)])
@pytest.mark.parametrize("threads", [1, 3])
def test_c_conv_matches_numpy(N, L, c_i, c_o, H, stride, first, last, threads):
    ctx = bfv.make_ctx(N, L, T)
    g = packing.conv_geometry(N, c_i, c_o, H, H, 3, stride, 1)
    rng = np.random.default_rng(N + 31 * c_i + c_o)
    F = rng.integers(-7, 8, (c_o, c_i, 3, 3))
    rho = rng.integers(0, T, (g.K_in, c_o, N))
    fh = packing.pack_conv_filters(F, g)
    c0 = wl.uniform_per_modulus(rng, (g.K_in,), ctx.primes, N).astype(np.uint64)
    sh = None if first else rng.integers(0, T, (g.K_in, N))
    shn = None if last else rng.integers(0, T, (g.K_out, N))
    want = bfv.server_conv(ctx, g, c0, rho, fh, sh, shn)
    got = cserver.server_conv(ctx, g, c0, cserver.conv_setup(ctx, rho, fh, threads), sh, shn, threads)
    assert (got == want).all()


@pytest.mark.parametrize("N,n_i,n_o", [(256, 16, 10), (1024, 20, 5), (1024, 64, 100)])
@pytest.mark.parametrize("with_sh,with_shn", [(True, False), (True, True), (False, True)])
def test_c_fc_matches_numpy(N, n_i, n_o, with_sh, with_shn):
    ctx = bfv.make_ctx(N, 2, T)
    g = packing.fc_geometry(N, n_i, n_o)
    rng = np.random.default_rng(N + n_i + n_o)
    W = rng.integers(-7, 8, (n_o, n_i))
    w = packing.pack_fc_weights(W, g)
    d = packing.pack_fc_bias(rng.integers(-7, 8, n_o), g)
    rho = rng.integers(0, T, (g.blocks, N))
    c0 = wl.uniform_per_modulus(rng, (), ctx.primes, N).astype(np.uint64)
    sh = rng.integers(0, T, N) if with_sh else None
    shn = rng.integers(0, T, (g.blocks, g.n_o_p)) if with_shn else None
    want = bfv.server_fc(ctx, g, c0, rho, w, d, sh, shn)
    got = cserver.server_fc(ctx, g, c0, cserver.fc_setup(ctx, rho, w), d, sh, shn, threads=2)
    assert (got == want).all()


def _golden():
    with open(os.path.join(HERE, "golden", "server_digests.json")) as f:
        return json.load(f)["cases"]


def test_c_single_conv_digest():
    gold = _golden()["single_conv"]["layers"]["0"]["digest"]
    ctx = bfv.make_ctx(4096, 3, T)
    _, b = cases.client_key(ctx, wl.CONFIG_SINGLE_CONV, 0)
    shp = wl.single_conv_layer()
    inp = cases.conv_inputs(ctx, shp, wl.image(wl.CONFIG_SINGLE_CONV, 0), wl.CONFIG_SINGLE_CONV, 0, 0, 0, True,
                            False, b)
    g = inp["geom"]
    out = cserver.server_conv(ctx, g, inp["c0"], cserver.conv_setup(ctx, inp["rho"], inp["fhat"], 0), inp["sh"],
                              inp["sh_next"], threads=0)
    assert cases.digest(out) == gold


def test_c_plain20_x1_digests():
    """Every layer of the x1 stack (N = 8192, 4 limbs) on the closed-loop inputs of the stored case."""
    gold = _golden()["plain20_x1"]["layers"]
    name, cfg, width, classes, N, L, _ = cases.PLAIN20_X1
    ctx = bfv.make_ctx(N, L, T)
    _, b = cases.client_key(ctx, cfg, 0)
    layers, Ws, Bs, ins, outs = cases.plain20_layer_inputs(width, classes, cfg, 0)
    for k, shp in enumerate(layers):
        first, last = k == 0, k == len(layers) - 1
        if shp.kind == "conv":
            inp = cases.conv_inputs(ctx, shp, ins[k], cfg, 0, width, k, first, last, b)
            g = inp["geom"]
            out = cserver.server_conv(ctx, g, inp["c0"], cserver.conv_setup(ctx, inp["rho"], inp["fhat"], 0),
                                      inp["sh"], inp["sh_next"], threads=0)
        else:
            inp = cases.fc_inputs(ctx, shp, ins[k], cfg, 0, width, k, first, last, b)
            g = inp["geom"]
            out = cserver.server_fc(ctx, g, inp["c0"], cserver.fc_setup(ctx, inp["rho"], inp["w"], 0), inp["d"],
                                    inp["sh"], inp["sh_next"], threads=0)
        assert cases.digest(out) == gold[str(k)]["digest"], f"layer {k}"
