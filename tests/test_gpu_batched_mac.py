"""GPU parity of the LDS-staged batched MAC (HE_TUNE_MAC = 3, and 4 with XCD-contiguous
workgroup order; 5 and 6 the same with the stages moved by LDS DMA; 9 the matrix-core form,
which the layers with s = 2 leave for the streaming one) against the oracle:
every staging geometry its host planner produces (one or several slot groups
per block, stages that hold whole blocks or part of one, image and channel tiles
wider than the batch or the layer), ragged batches and channel counts, with and
without the input share."""
import numpy as np
import pytest

import workloads as wl
from oracle import bfv, packing
from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu
T = wl.T_PLAIN

# (N, c_i, c_o, H, stride, B)
CASES = [
    (1024, 2, 4, 14, 1, 8),      # s = 4, one group per block
    (1024, 16, 12, 14, 1, 5),    # s = 4, K_in = 4, ragged channels and batch
    (1024, 2, 2, 20, 1, 17),     # s = 2
    (1024, 4, 12, 6, 1, 3),      # s = 16, g_o = 8, ragged output group
    (1024, 16, 32, 6, 2, 6),     # s = 16, stride 2
    (2048, 8, 8, 2, 1, 2),       # s = 128, several stages per block, two groups per block
    (4096, 16, 32, 2, 2, 4),     # s = 256
    (1024, 8, 64, 2, 1, 9),      # s = 64, many channels
    (1024, 8, 24, 6, 1, 5),      # s = 64, channels a multiple of 8 but not of 64 (matrix-core tile)
    (4096, 1024, 8, 6, 1, 3),    # s = 64, K_in = 16: 2048 products per block sum (32 matrix-core chunks)
]


@pytest.fixture(scope="module")
def he():
    from paper_2409_05205_amd import he as h
    h.load_library()
    return h


@pytest.mark.parametrize("case", CASES, ids=lambda c: "N%d_c%d-%d_H%d_st%d_B%d" % c)
def test_lds_mac_matches_oracle(he, case):
    N, c_i, c_o, H, stride, B = case
    L = 2
    octx = bfv.make_ctx(N, L, T)
    g = packing.conv_geometry(N, c_i, c_o, H, H, 3, stride, 1)
    rng = np.random.default_rng(sum(case))
    F = rng.integers(-7, 8, (c_o, c_i, 3, 3))
    rho = rng.integers(0, T, (g.K_in, c_o, N))
    c0 = np.stack([wl.uniform_per_modulus(rng, (g.K_in,), octx.primes, N) for _ in range(B)])
    sh = rng.integers(0, T, (B, g.K_in, N))
    shn = rng.integers(0, T, (B, g.K_out, N))
    fh = packing.pack_conv_filters(F, g)
    ctx = he.Context(N, L, T)
    layer = ctx.pack_conv(he.ConvSpec(c_i, c_o, H, H, 3, stride, 1), F, rho)
    for use_sh in (True, False):
        want = [bfv.server_conv(octx, g, c0[b].astype(np.uint64), rho, fh, sh[b] if use_sh else None, shn[b])
                for b in range(B)]
        for mac in (3, 4, 5, 6, 9):    # register / DMA staging, round-robin / XCD-contiguous order; matrix cores
            ctx.tune_force(he.HE_TUNE_MAC, mac)
            got = host(ctx.conv_layer(layer, dev(c0), dev(sh) if use_sh else None, dev(shn)))
            for b in range(B):
                assert (got[b] == want[b]).all(), f"mac={mac} image {b} sh={use_sh} s={g.s}"
