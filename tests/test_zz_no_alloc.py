"""he_conv_layer_noalloc (static device scratch, no allocation) against he_conv_layer.

Two calls in a row on the same GPU, the second with a smaller batch, must each give
the words of he_conv_layer on the same inputs (every quantity is an integer residue,
so the bar is equality).  A small ring is also checked against the oracle, and a
batch whose workspace exceeds the static scratch must be refused before any launch
with nothing written.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import bfv, packing
from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

T = wl.T_PLAIN


@pytest.fixture(scope="module")
def he():
    from paper_2409_05205_amd import he as h
    h.load_library()
    return h


def _inputs(primes, N, g, B, seed):
    rng = np.random.default_rng(seed)
    c0 = np.stack([wl.uniform_per_modulus(rng, (g.K_in,), primes, N) for _ in range(B)])
    sh = rng.integers(0, T, (B, g.K_in, N))
    shn = rng.integers(0, T, (B, g.K_out, N))
    return c0, sh, shn


@pytest.mark.parametrize("first", [False, True])
def test_noalloc_matches_conv_layer_twice(he, first):
    """x1 plain-20 layer 16->16 at 32x32, N = 8192, 4 limbs: B = 3, then B = 1."""
    import torch
    N, L = 8192, 4
    ctx = he.Context(N, L, T)
    g = packing.conv_geometry(N, 16, 16, 32, 32, 3, 1, 1)
    rng = np.random.default_rng(11)
    F = rng.integers(-7, 8, (16, 16, 3, 3))
    rho = rng.integers(0, T, (g.K_in, 16, N))
    layer = ctx.pack_conv(he.ConvSpec(16, 16, 32, 32), F, rho)
    for B, seed in ((3, 21), (1, 22)):
        c0, sh, shn = _inputs(ctx.primes, N, g, B, seed)
        tc0, tshn = dev(c0), dev(shn)
        tsh = None if first else dev(sh)
        want = host(ctx.conv_layer(layer, tc0, tsh, tshn))
        out = torch.full((B, g.K_out, L, N), -1, dtype=torch.int32, device="cuda:0")
        got = host(ctx.conv_layer_noalloc(layer, tc0, out, tsh, tshn))
        print(f"noalloc B={B} first={first}: {got.shape}", flush=True)
        assert got.shape == want.shape
        assert (got == want).all()


def test_noalloc_small_ring_matches_oracle(he):
    """N = 1024, 2 limbs, K_in = 2 with a ragged input group, B = 2 then B = 1, against the oracle."""
    import torch
    N, L = 1024, 2
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    g = packing.conv_geometry(N, 20, 4, 4, 4, 3, 1, 1)
    rng = np.random.default_rng(5)
    F = rng.integers(-7, 8, (4, 20, 3, 3))
    rho = rng.integers(0, T, (g.K_in, 4, N))
    layer = ctx.pack_conv(he.ConvSpec(20, 4, 4, 4), F, rho)
    fhat = packing.pack_conv_filters(F, g)
    for B, seed in ((2, 31), (1, 32)):
        c0, sh, shn = _inputs(octx.primes, N, g, B, seed)
        out = torch.zeros((B, g.K_out, L, N), dtype=torch.int32, device="cuda:0")
        got = host(ctx.conv_layer_noalloc(layer, dev(c0), out, dev(sh), dev(shn)))
        for b in range(B):
            want = bfv.server_conv(octx, g, c0[b].astype(np.uint64), rho, fhat, sh[b], shn[b])
            assert (got[b] == want).all()


def test_noalloc_refuses_batch_beyond_scratch(he):
    import torch
    N, L = 8192, 4
    ctx = he.Context(N, L, T)
    g = packing.conv_geometry(N, 16, 16, 32, 32, 3, 1, 1)
    rng = np.random.default_rng(3)
    layer = ctx.pack_conv(he.ConvSpec(16, 16, 32, 32), rng.integers(-7, 8, (16, 16, 3, 3)),
                          rng.integers(0, T, (g.K_in, 16, N)))
    B = 1
    while layer.workspace_bytes(B) <= he.NOALLOC_SCRATCH_BYTES:
        B *= 2
    c0 = torch.zeros((B, g.K_in, L, N), dtype=torch.int32, device="cuda:0")
    out = torch.full((B, g.K_out, L, N), 7, dtype=torch.int32, device="cuda:0")
    with pytest.raises(he.HEError) as ei:
        ctx.conv_layer_noalloc(layer, c0, out)
    assert ei.value.code == he.HE_ENOMEM
    torch.cuda.synchronize()
    assert bool((out == 7).all())
