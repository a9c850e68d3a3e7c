"""ResNet-50-shaped layers (the NEXT-4 workload): the geometries its body adds to
plain-20 -- 1x1 convolutions without padding, 1x1 stride-2 projections, 3x3 stride 2
on even sizes -- against the oracle on small rings at batch one (fused kernel) and
batch five (LDS-staged MAC), and three full-size ResNet-50 layers (N = 16384, 6
limbs: a 3x3 at 28x28, a 1x1 expansion at 14x14, a 3x3 at 7x7) by the oracle's
digests."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import bfv, packing
from gpu_helpers import dev, host

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import cases  # noqa: E402

pytestmark = pytest.mark.gpu
T = wl.T_PLAIN

# (N, c_i, c_o, H, f, stride, pad)
SMALL = [
    (1024, 16, 32, 8, 1, 1, 0),      # 1x1 expansion
    (1024, 32, 8, 8, 1, 1, 0),       # 1x1 reduction
    (1024, 16, 32, 8, 1, 2, 0),      # 1x1 stride-2 projection
    (1024, 8, 8, 8, 3, 2, 1),        # 3x3 stride 2, even size
    (2048, 64, 16, 4, 1, 1, 0),      # 1x1 on a small map, s = 128
]


@pytest.fixture(scope="module")
def he():
    from paper_2409_05205_amd import he as h
    h.load_library()
    return h


@pytest.mark.parametrize("shape", SMALL, ids=lambda s: "N%d_c%d-%d_H%d_f%d_st%d_p%d" % s)
def test_resnet_geometry_matches_oracle(he, shape):
    N, c_i, c_o, H, f, stride, pad = shape
    L, B = 2, 5
    octx = bfv.make_ctx(N, L, T)
    g = packing.conv_geometry(N, c_i, c_o, H, H, f, stride, pad)
    rng = np.random.default_rng(sum(shape))
    F = rng.integers(-7, 8, (c_o, c_i, f, f))
    rho = rng.integers(0, T, (g.K_in, c_o, N))
    c0 = np.stack([wl.uniform_per_modulus(rng, (g.K_in,), octx.primes, N) for _ in range(B)])
    sh = rng.integers(0, T, (B, g.K_in, N))
    shn = rng.integers(0, T, (B, g.K_out, N))
    fh = packing.pack_conv_filters(F, g)
    want = [bfv.server_conv(octx, g, c0[b].astype(np.uint64), rho, fh, sh[b], shn[b]) for b in range(B)]
    ctx = he.Context(N, L, T)
    layer = ctx.pack_conv(he.ConvSpec(c_i, c_o, H, H, f, stride, pad), F, rho)
    for nb in (1, B):
        got = host(ctx.conv_layer(layer, dev(c0[:nb]), dev(sh[:nb]), dev(shn[:nb])))
        for b in range(nb):
            assert (got[b] == want[b]).all(), f"B={nb} image {b} s={g.s}"


@pytest.mark.parametrize("case", cases.RESNET_SAMPLES, ids=lambda c: c[0])
def test_resnet50_layer_digest(he, case):
    name, k = case
    with open(os.path.join(HERE, "golden", "server_digests.json")) as fh_:
        want = json.load(fh_)["cases"][name]["layers"][str(k)]["digest"]
    ctx = he.Context(16384, 6, T)
    octx = bfv.make_ctx(16384, 6, T)
    inp = cases.resnet_layer_inputs(k, 16384, octx.primes)
    g, shp = inp["geom"], inp["shape"]
    print(f"case {name} {shp} s={g.s}", flush=True)
    layer = ctx.pack_conv(he.ConvSpec(shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad), inp["F"],
                          inp["rho"])
    got = host(ctx.conv_layer(layer, dev(inp["c0"][None]), dev(inp["sh"][None]), dev(inp["sh_next"][None])))[0]
    assert cases.digest(got) == want
    layer.free()
