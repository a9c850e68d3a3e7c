"""GPU parity of he_conv_layer / he_fc_layer against the oracle, element by element.

Small rings (N = 256, 1024) span several MAC tiles, ragged channel groups,
K_in > 1, stride 2 and both inverse-transform forms; the single-conv workload
(N = 4096, 3 limbs) runs through every party and must decrypt to the integer
convolution.  Batched calls must equal one call per image.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import bfv, network, packing
from gpu_helpers import dev, gpu_conv, gpu_fc, host

pytestmark = pytest.mark.gpu

T = wl.T_PLAIN


@pytest.fixture(scope="module")
def he():
    from paper_2409_05205_amd import he as h
    h.load_library()
    return h


def _conv_case(octx, c_i, c_o, H, stride, seed, first, last, f=3, pad=1):
    N = octx.N
    g = packing.conv_geometry(N, c_i, c_o, H, H, f, stride, pad)
    rng = np.random.default_rng(seed)
    F = rng.integers(-7, 8, (c_o, c_i, f, f))
    rho = rng.integers(0, T, (g.K_in, c_o, N))
    c0 = wl.uniform_per_modulus(rng, (g.K_in,), octx.primes, N).astype(np.uint64)
    sh = None if first else rng.integers(0, T, (g.K_in, N))
    shn = None if last else rng.integers(0, T, (g.K_out, N))
    return g, F, rho, c0, sh, shn


SMALL_CONV = [
    # N, L, c_i, c_o, H, stride
    (256, 2, 3, 8, 4, 1),
    (256, 2, 6, 4, 4, 1),      # K_in = 2
    (256, 2, 4, 8, 4, 2),      # stride 2, K_out = 2
    (256, 2, 5, 3, 4, 1),      # ragged: c_o not a power of two
    (1024, 3, 16, 24, 6, 1),   # ragged last output group (g_o = 16), K_in = 1
    (1024, 2, 20, 4, 4, 1),    # K_in = 2 with a ragged input group, s = 16
    (1024, 2, 2, 2, 30, 1),    # s = 1: one class, full-length tail
    (256, 2, 2, 32, 1, 1),     # 3x3 padded input: s = 16, tail of 16 points, one thread per row
    (256, 2, 8, 16, (2, 2, 0), 1),  # 2x2 input, 2x2 filter, no padding: s = 64, 4-point tail
]


@pytest.mark.parametrize("N,L,c_i,c_o,H,stride", SMALL_CONV)
@pytest.mark.parametrize("flags", [0, 1])
@pytest.mark.parametrize("first,last", [(True, False), (False, False), (False, True)])
def test_conv_layer_matches_oracle(he, N, L, c_i, c_o, H, stride, flags, first, last):
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    f, pad = 3, 1
    if isinstance(H, tuple):
        H, f, pad = H
    g, F, rho, c0, sh, shn = _conv_case(octx, c_i, c_o, H, stride, N + c_i * 7 + c_o, first, last, f, pad)
    want = bfv.server_conv(octx, g, c0, rho, packing.pack_conv_filters(F, g), sh, shn)
    got = gpu_conv(ctx, g, F, rho, c0, sh, shn, flags)
    assert got.shape == want.shape
    assert (got == want).all()


@pytest.mark.parametrize("flags", [0, 1])
def test_single_conv_workload_decrypts(he, flags):
    """Single conv 3->16 on 3x32x32, N = 4096, 3 limbs: every party, real encryption."""
    N, L = 4096, 3
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    shp = wl.single_conv_layer()
    img = wl.image(wl.CONFIG_SINGLE_CONV, 0)
    F = wl.layer_weights(wl.CONFIG_SINGLE_CONV, 0, 0, shp)
    seen = {}

    def server(c0, rho, fhat, sh, sh_next):
        g = packing.conv_geometry(N, 3, 16, 32, 32)
        seen["want"] = bfv.server_conv(octx, g, c0, rho, fhat, sh, sh_next)
        seen["got"] = gpu_conv(ctx, g, F, rho, c0, sh, sh_next, flags)
        return seen["got"]

    for first in (True, False):
        res = network.run_conv_protocol(octx, shp, img, F, (wl.CONFIG_SINGLE_CONV, 0, 0, 0), first, False,
                                        server_fn=server)
        assert (seen["got"] == seen["want"]).all()
        assert (network.centred(res["decrypted"], T) == res["reference"]).all()


@pytest.mark.parametrize("flags", [0, 1])
def test_batched_call_equals_per_image(he, flags):
    N, L = 1024, 2
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    g, F, rho, _, _, _ = _conv_case(octx, 16, 32, 6, 1, 5, False, False)
    from paper_2409_05205_amd import he as h
    layer = ctx.pack_conv(h.ConvSpec(16, 32, 6, 6), F, rho, flags)
    rng = np.random.default_rng(11)
    B = 5
    c0 = np.stack([wl.uniform_per_modulus(rng, (g.K_in,), octx.primes, N) for _ in range(B)])
    sh = rng.integers(0, T, (B, g.K_in, N))
    shn = rng.integers(0, T, (B, g.K_out, N))
    got = host(ctx.conv_layer(layer, dev(c0), dev(sh), dev(shn)))
    fh = packing.pack_conv_filters(F, g)
    for b in range(B):
        want = bfv.server_conv(octx, g, c0[b].astype(np.uint64), rho, fh, sh[b], shn[b])
        assert (got[b] == want).all()
        alone = host(ctx.conv_layer(layer, dev(c0[b:b + 1]), dev(sh[b:b + 1]), dev(shn[b:b + 1])))
        assert (alone[0] == got[b]).all()


FC_CASES = [(256, 2, 4, 2), (256, 2, 16, 10), (256, 2, 64, 10), (1024, 3, 100, 7), (8192, 4, 64, 10),
            (16384, 6, 256, 100)]


@pytest.mark.parametrize("N,L,n_i,n_o", FC_CASES)
@pytest.mark.parametrize("first,last", [(True, False), (False, True), (False, False)])
def test_fc_layer_matches_oracle(he, N, L, n_i, n_o, first, last):
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    g = packing.fc_geometry(N, n_i, n_o)
    rng = np.random.default_rng(N + n_i + n_o)
    W = rng.integers(-7, 8, (n_o, n_i))
    B = rng.integers(-7, 8, n_o)
    rho = rng.integers(0, T, (g.blocks, N))
    c0 = wl.uniform_per_modulus(rng, (), octx.primes, N).astype(np.uint64)
    sh = None if first else rng.integers(0, T, N)
    shn = None if last else rng.integers(0, T, (g.blocks, g.n_o_p))
    want = bfv.server_fc(octx, g, c0, rho, packing.pack_fc_weights(W, g), packing.pack_fc_bias(B, g), sh, shn)
    got = gpu_fc(ctx, g, W, B, rho, c0, sh, shn)
    assert (got == want).all()


def test_fc_protocol_decrypts(he):
    N, L = 8192, 4
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    rng = np.random.default_rng(3)
    vec = rng.integers(0, 16, 64)
    W = rng.integers(-7, 8, (10, 64))
    Bb = rng.integers(-7, 8, 10)

    def server(c0, rho, w, d, sh, sh_next):
        g = packing.fc_geometry(N, 64, 10)
        return gpu_fc(ctx, g, W, Bb, rho, c0, sh, sh_next)

    res = network.run_fc_protocol(octx, wl.FCShape(64, 10), vec, W, Bb, (2, 0, 1, 19), False, True,
                                  server_fn=server)
    assert (network.centred(res["decrypted"], T) == res["reference"]).all()


def test_empty_batch_is_noop(he):
    import torch
    N, L = 256, 2
    ctx = he.Context(N, L, T)
    from paper_2409_05205_amd import he as h
    layer = ctx.pack_conv(h.ConvSpec(3, 8, 4, 4), np.ones((8, 3, 3, 3)), np.zeros((1, 8, N)))
    c0 = torch.zeros((0, 1, L, N), dtype=torch.int32, device="cuda:0")
    out = ctx.conv_layer(layer, c0)
    assert out.shape == (0, layer.K_out, L, N)


BATCHED_FULL = [(16, 16, 32, 1), (32, 32, 16, 1), (64, 64, 8, 1), (16, 32, 32, 2)]


@pytest.mark.parametrize("c_i,c_o,H,stride", BATCHED_FULL)
@pytest.mark.parametrize("flags", [0, 1])
def test_batched_fullsize_layer(he, c_i, c_o, H, stride, flags):
    """B = 6 images at N = 8192, 4 limbs (register-blocked MAC, ragged image tile):
    sampled images bit-exact vs the oracle, every image equal to its single-image call."""
    N, L = 8192, 4
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    g = packing.conv_geometry(N, c_i, c_o, H, H, 3, stride, 1)
    rng = np.random.default_rng(c_i * 100 + c_o + H + flags)
    F = rng.integers(-7, 8, (c_o, c_i, 3, 3))
    rho = rng.integers(0, T, (g.K_in, c_o, N))
    from paper_2409_05205_amd import he as h
    layer = ctx.pack_conv(h.ConvSpec(c_i, c_o, H, H, 3, stride, 1), F, rho, flags)
    B = 6
    c0 = np.stack([wl.uniform_per_modulus(rng, (g.K_in,), octx.primes, N) for _ in range(B)])
    sh = rng.integers(0, T, (B, g.K_in, N))
    shn = rng.integers(0, T, (B, g.K_out, N))
    got = host(ctx.conv_layer(layer, dev(c0), dev(sh), dev(shn)))
    fh = packing.pack_conv_filters(F, g)
    for b in (0, B - 1):
        want = bfv.server_conv(octx, g, c0[b].astype(np.uint64), rho, fh, sh[b], shn[b])
        assert (got[b] == want).all(), f"image {b}"
    for b in range(B):
        alone = host(ctx.conv_layer(layer, dev(c0[b:b + 1]), dev(sh[b:b + 1]), dev(shn[b:b + 1])))
        assert (alone[0] == got[b]).all(), f"image {b} alone"
