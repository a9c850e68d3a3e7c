"""Full-size GPU parity: every layer of the x1 plain-20 stack (N = 8192, 4 limbs)
and one layer per tiling of the x2 / x4 variants (N = 8192 / 16384), compared
bit-exactly with the oracle through the SHA-256 of c0^r stored by
tests/golden/make_golden.py (which also checked that the x1 stack decrypts to
the integer forward pass layer by layer).  Both inverse-transform forms must
give the same words.
"""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import cases  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import bfv  # noqa: E402
from gpu_helpers import dev, gpu_conv, gpu_fc, host  # noqa: E402

pytestmark = pytest.mark.gpu

_GOLD = {}


def gold():
    if not _GOLD:
        with open(os.path.join(HERE, "golden", "server_digests.json")) as f:
            _GOLD.update(json.load(f)["cases"])
    return _GOLD


@pytest.fixture(scope="module")
def he():
    from paper_2409_05205_amd import he as h
    h.load_library()
    return h


_CTX = {}


def contexts(he, N, L):
    if (N, L) not in _CTX:
        _CTX[(N, L)] = (he.Context(N, L, wl.T_PLAIN), bfv.make_ctx(N, L, wl.T_PLAIN))
    return _CTX[(N, L)]


def _stack_params():
    out = []
    for name, cfg, width, classes, N, L, idx in [cases.PLAIN20_X1] + cases.WIDE_SAMPLES:
        for k in (range(20) if idx is None else idx):
            out.append((name, cfg, width, classes, N, L, k))
    return out


_STACK = {}


def stack(width, classes, cfg):
    key = (width, classes, cfg)
    if key not in _STACK:
        _STACK[key] = cases.plain20_layer_inputs(width, classes, cfg, 0)
    return _STACK[key]


@pytest.mark.parametrize("name,cfg,width,classes,N,L,k", _stack_params())
def test_plain20_layer_digest(he, name, cfg, width, classes, N, L, k):
    ctx, octx = contexts(he, N, L)
    _, b = cases.client_key(octx, cfg, 0)
    layers, Ws, Bs, ins, outs = stack(width, classes, cfg)
    shp = layers[k]
    first, last = k == 0, k == len(layers) - 1
    want = gold()[name]["layers"][str(k)]["digest"]
    print(f"case {name} layer {k} {shp}", flush=True)
    if shp.kind == "conv":
        inp = cases.conv_inputs(octx, shp, ins[k], cfg, 0, width, k, first, last, b)
        flag_set = (0, 1) if N <= 8192 else (0,)
        for flags in flag_set:
            got = gpu_conv(ctx, inp["geom"], inp["F"], inp["rho"], inp["c0"], inp["sh"], inp["sh_next"], flags)
            assert cases.digest(got) == want, f"flags={flags}"
    else:
        inp = cases.fc_inputs(octx, shp, ins[k], cfg, 0, width, k, first, last, b)
        got = gpu_fc(ctx, inp["geom"], inp["W"], inp["bias"], inp["rho"], inp["c0"], inp["sh"], inp["sh_next"])
        assert cases.digest(got) == want


def test_single_conv_digest(he):
    ctx, octx = contexts(he, 4096, 3)
    _, b = cases.client_key(octx, wl.CONFIG_SINGLE_CONV, 0)
    shp = wl.single_conv_layer()
    x = wl.image(wl.CONFIG_SINGLE_CONV, 0)
    inp = cases.conv_inputs(octx, shp, x, wl.CONFIG_SINGLE_CONV, 0, 0, 0, True, False, b)
    for flags in (0, 1):
        got = gpu_conv(ctx, inp["geom"], inp["F"], inp["rho"], inp["c0"], inp["sh"], inp["sh_next"], flags)
        assert cases.digest(got) == gold()["single_conv"]["layers"]["0"]["digest"]


@pytest.mark.parametrize("case", cases.BATCHED_SAMPLES, ids=lambda c: c[0])
def test_batched_layer_digest(he, case):
    """A full batch of 64 images through one wide layer under every batched MAC variant (the
    LDS-staged one walking several slot ranges per workgroup at this size); the sampled
    images must match the oracle's digests."""
    name, cfg, width, classes, N, L, k, B, images = case
    ctx, octx = contexts(he, N, L)
    inp = cases.batched_layer_inputs(cfg, width, classes, k, B, N, octx.primes)
    g = inp["geom"]
    want = gold()[name]["images"]
    print(f"case {name} layer {k} B={B} s={g.s}", flush=True)
    spec = he.ConvSpec(g.c_i, g.c_o, g.H, g.W, g.f, g.stride, g.pad)
    layer = ctx.pack_conv(spec, inp["F"], inp["rho"])
    c0, sh, shn = dev(inp["c0"]), dev(inp["sh"]), dev(inp["sh_next"])
    try:
        for mac in (9, 3, 4, 5, 6, 1, 0):
            ctx.tune_force(he.HE_TUNE_MAC, mac)
            got = host(ctx.conv_layer(layer, c0, sh, shn))
            for b in images:
                assert cases.digest(got[b]) == want[str(b)], f"mac={mac} image {b}"
    finally:
        ctx.tune_force(he.HE_TUNE_MAC, -1)
