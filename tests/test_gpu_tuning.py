"""Every tuning-knob value must give the same words: an adversarial sweep of the
register radix of the forward NTT, inverse NTT and residue-class tail, and of
the MAC kernel choice, against the oracle (small rings) and the golden digest
(a full-size x1 layer); the autotuner's picks must be valid and exact too."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import bfv, packing
from gpu_helpers import dev, gpu_conv, host

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import cases  # noqa: E402

pytestmark = pytest.mark.gpu
T = wl.T_PLAIN


@pytest.fixture(scope="module")
def he():
    from paper_2409_05205_amd import he as h
    h.load_library()
    return h


def _case(N, L, c_i, c_o, H, stride, seed, B):
    octx = bfv.make_ctx(N, L, T)
    g = packing.conv_geometry(N, c_i, c_o, H, H, 3, stride, 1)
    rng = np.random.default_rng(seed)
    F = rng.integers(-7, 8, (c_o, c_i, 3, 3))
    rho = rng.integers(0, T, (g.K_in, c_o, N))
    c0 = np.stack([wl.uniform_per_modulus(rng, (g.K_in,), octx.primes, N) for _ in range(B)])
    sh = rng.integers(0, T, (B, g.K_in, N))
    shn = rng.integers(0, T, (B, g.K_out, N))
    fh = packing.pack_conv_filters(F, g)
    want = [bfv.server_conv(octx, g, c0[b].astype(np.uint64), rho, fh, sh[b], shn[b]) for b in range(B)]
    return g, F, rho, c0, sh, shn, want


@pytest.mark.parametrize("knob_name,values", [("HE_TUNE_NTT_FWD", [2, 3, 4, 5]), ("HE_TUNE_TAIL", [2, 3, 4, 5]),
                                              ("HE_TUNE_NTT_INV", [2, 3, 4, 5]), ("HE_TUNE_MAC", [0, 1, 2, 3, 4, 5, 6, 9])])
def test_knob_sweep_is_exact(he, knob_name, values):
    N, L = 1024, 2
    knob = getattr(he, knob_name)
    cases_ = [_case(N, L, 16, 16, 6, 1, 3, 5), _case(N, L, 3, 8, 4, 1, 4, 2), _case(N, L, 16, 32, 6, 2, 5, 4)]
    for flags in (0, 1):
        for v in values:
            ctx = he.Context(N, L, T)
            ctx.tune_force(knob, v)
            for g, F, rho, c0, sh, shn, want in cases_:
                layer = ctx.pack_conv(he.ConvSpec(g.c_i, g.c_o, g.H, g.W, 3, g.stride, 1), F, rho, flags)
                got = host(ctx.conv_layer(layer, dev(c0), dev(sh), dev(shn)))
                for b in range(len(want)):
                    assert (got[b] == want[b]).all(), f"{knob_name}={v} flags={flags} image {b}"


def test_knob_sweep_fullsize_digest(he):
    """Layer 1 of the x1 stack (N = 8192, 4 limbs) under every forward / tail radix."""
    with open(os.path.join(HERE, "golden", "server_digests.json")) as f:
        gold = json.load(f)["cases"]["plain20_x1"]["layers"]["1"]["digest"]
    octx = bfv.make_ctx(8192, 4, T)
    _, b = cases.client_key(octx, wl.CONFIG_PLAIN20_X1, 0)
    layers, Ws, Bs, ins, outs = cases.plain20_layer_inputs(1, 10, wl.CONFIG_PLAIN20_X1, 0)
    inp = cases.conv_inputs(octx, layers[1], ins[1], wl.CONFIG_PLAIN20_X1, 0, 1, 1, False, False, b)
    for fwd in (3, 4, 5):
        for tail in (2, 3, 4):
            ctx = he.Context(8192, 4, T)
            ctx.tune_force(he.HE_TUNE_NTT_FWD, fwd)
            ctx.tune_force(he.HE_TUNE_TAIL, tail)
            got = gpu_conv(ctx, inp["geom"], inp["F"], inp["rho"], inp["c0"], inp["sh"], inp["sh_next"], 0)
            assert cases.digest(got) == gold, f"fwd={fwd} tail={tail}"


def test_autotune_picks_are_exact(he):
    N, L = 1024, 2
    g, F, rho, c0, sh, shn, want = _case(N, L, 16, 16, 6, 1, 9, 6)
    ctx = he.Context(N, L, T)
    layer = ctx.pack_conv(he.ConvSpec(16, 16, 6, 6), F, rho)
    ctx.autotune(layer, 6)
    rows = 6 * g.K_in * L * 2
    pick = ctx.tune_get(he.HE_TUNE_NTT_FWD, 10, rows)
    assert pick in (2, 3, 4, 5)
    got = host(ctx.conv_layer(layer, dev(c0), dev(sh), dev(shn)))
    for b in range(6):
        assert (got[b] == want[b]).all()
