"""GPU parity of the fused conv MAC + residue-class tail (HE_TUNE_MAC = 2)
against the oracle, next to the two-launch form (HE_TUNE_MAC = 0), on every slot
stride the fused kernel serves (s = 1 .. 256, block sums in registers, within a
4-slot chunk, or across 1 .. 64 lanes), ragged output groups, batches of one and
three images, and with the input share and the next-layer share each present or
absent (first and last layers)."""
import numpy as np
import pytest

import workloads as wl
from oracle import bfv, packing
from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu
T = wl.T_PLAIN

# (N, c_i, c_o, H, stride): s from 1 to 256, g_o < c_o with a ragged last group
SHAPES = [
    (1024, 1, 1, 30, 1),     # s = 1: M = N
    (1024, 2, 2, 20, 1),     # s = 2
    (1024, 2, 4, 14, 1),     # s = 4: one lane per block
    (1024, 8, 8, 14, 1),     # s = 4, K_in = 2
    (1024, 16, 12, 14, 1),   # s = 4, K_in = 4 (eight input rows with the share), ragged
    (1024, 4, 12, 6, 1),     # s = 16, g_o = 8, ragged second group
    (1024, 3, 16, 4, 1),     # s = 16, first-layer channel count
    (2048, 8, 8, 2, 1),      # s = 128: 32 lanes per block, M = 16
    (4096, 16, 32, 2, 2),    # s = 256: 64 lanes per block, stride 2
]


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
    return octx, g, F, rho, c0, sh, shn


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "N%d_c%d-%d_H%d_st%d" % s)
def test_fused_matches_oracle(he, shape):
    N, c_i, c_o, H, stride = shape
    L, B = 2, 3
    octx, g, F, rho, c0, sh, shn = _case(N, L, c_i, c_o, H, stride, sum(shape), B)
    fh = packing.pack_conv_filters(F, g)
    for use_sh, use_shn in ((True, True), (False, True), (True, False), (False, False)):
        want = [bfv.server_conv(octx, g, c0[b].astype(np.uint64), rho, fh, sh[b] if use_sh else None,
                                shn[b] if use_shn else None) for b in range(B)]
        for mac in (2, 0):
            ctx = he.Context(N, L, T)
            ctx.tune_force(he.HE_TUNE_MAC, mac)
            layer = ctx.pack_conv(he.ConvSpec(c_i, c_o, H, H, 3, stride, 1), F, rho)
            assert layer.info.s == g.s
            for nb in (1, B):
                got = host(ctx.conv_layer(layer, dev(c0[:nb]), dev(sh[:nb]) if use_sh else None,
                                          dev(shn[:nb]) if use_shn else None))
                for b in range(nb):
                    assert (got[b] == want[b]).all(), \
                        f"mac={mac} B={nb} image {b} sh={use_sh} shn={use_shn} s={g.s}"


def test_fused_is_the_default_at_batch_one(he):
    """B = 1 runs the fused launch (one HE_K_MAC_TAIL, no HE_K_MAC / HE_K_TAIL)."""
    N, L = 1024, 2
    octx, g, F, rho, c0, sh, shn = _case(N, L, 4, 12, 6, 1, 7, 1)
    ctx = he.Context(N, L, T)
    layer = ctx.pack_conv(he.ConvSpec(4, 12, 6, 6, 3, 1, 1), F, rho)
    ctx.profile_reset()
    ctx.profile_enable(he.HE_K_MAC | he.HE_K_TAIL | he.HE_K_MAC_TAIL)
    got = host(ctx.conv_layer(layer, dev(c0), dev(sh), dev(shn)))
    assert ctx.profile_read(he.HE_K_MAC_TAIL)[0] == 1
    assert ctx.profile_read(he.HE_K_MAC)[0] == 0 and ctx.profile_read(he.HE_K_TAIL)[0] == 0
    ctx.profile_enable(0)
    want = bfv.server_conv(octx, g, c0[0].astype(np.uint64), rho, packing.pack_conv_filters(F, g), sh[0], shn[0])
    assert (got[0] == want).all()


def test_streaming_is_the_default_for_few_rows_and_several_inputs(he):
    """B = 1 with K_in >= 2 and at most 64 output rows (K_out g_o L) takes the streaming MAC and a
    tail launch instead of the fused launch, with the same words."""
    N, L = 1024, 2
    c_i, c_o, H = 16, 12, 14            # s = 4, K_in = 4, K_out = 3, g_o = 4: 24 rows
    octx, g, F, rho, c0, sh, shn = _case(N, L, c_i, c_o, H, 1, 23, 1)
    assert g.K_in >= 2 and g.K_out * g.g_o * L <= 64
    ctx = he.Context(N, L, T)
    layer = ctx.pack_conv(he.ConvSpec(c_i, c_o, H, H, 3, 1, 1), F, rho)
    ctx.profile_reset()
    ctx.profile_enable(he.HE_K_MAC | he.HE_K_TAIL | he.HE_K_MAC_TAIL)
    got = host(ctx.conv_layer(layer, dev(c0), dev(sh), dev(shn)))
    assert ctx.profile_read(he.HE_K_MAC_TAIL)[0] == 0
    assert ctx.profile_read(he.HE_K_MAC)[0] == 1 and ctx.profile_read(he.HE_K_TAIL)[0] == 1
    ctx.profile_enable(0)
    want = bfv.server_conv(octx, g, c0[0].astype(np.uint64), rho, packing.pack_conv_filters(F, g), sh[0], shn[0])
    assert (got[0] == want).all()


# (N, L, c_i, c_o, H, B): launches of several hundred output rows (B K_out g_o L), more than
# the chip has CUs, at M = 4096, 2048 and 512, with ragged last groups.
MANY = [
    (4096, 3, 2, 127, 44, 1),    # s = 1, M = 4096: 381 rows
    (4096, 3, 2, 129, 44, 1),    # 387 rows
    (8192, 3, 1, 126, 40, 1),    # s = 4, M = 2048: 32 groups of 4, 384 rows, ragged
    (8192, 3, 1, 124, 40, 1),    # 31 groups: 372 rows
    (4096, 3, 4, 60, 20, 2),     # s = 8, M = 512: 8 groups of 8 per image, 384 rows, ragged
    (4096, 3, 4, 60, 20, 1),     # 192 rows
]


@pytest.mark.parametrize("case", MANY, ids=lambda c: "N%d_L%d_c%d-%d_H%d_B%d" % c)
def test_fused_many_rows_matches_oracle(he, case):
    N, L, c_i, c_o, H, B = case
    octx, g, F, rho, c0, sh, shn = _case(N, L, c_i, c_o, H, 1, sum(case), B)
    fh = packing.pack_conv_filters(F, g)
    rows = B * g.K_out * g.g_o * L
    ctx = he.Context(N, L, T)
    ctx.tune_force(he.HE_TUNE_MAC, 2)
    layer = ctx.pack_conv(he.ConvSpec(c_i, c_o, H, H, 3, 1, 1), F, rho)
    ctx.profile_reset()
    ctx.profile_enable(he.HE_K_MAC_TAIL)
    got = host(ctx.conv_layer(layer, dev(c0), dev(sh), dev(shn)))
    assert ctx.profile_read(he.HE_K_MAC_TAIL)[0] == 1
    ctx.profile_enable(0)
    for b in range(B):
        want = bfv.server_conv(octx, g, c0[b].astype(np.uint64), rho, fh, sh[b], shn[b])
        assert (got[b] == want).all(), f"image {b} of {B}, {rows} rows, s={g.s}"
