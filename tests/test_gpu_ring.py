"""GPU parity of the ring primitives: NTT -> INTT identity, products vs the oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle import bfv, ring
from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

T = wl.T_PLAIN


@pytest.fixture(scope="module")
def he():
    from paper_2409_05205_amd import he as h
    h.load_library()
    return h


@pytest.mark.parametrize("N,L", [(256, 2), (4096, 3), (8192, 4), (16384, 6)])
def test_ntt_roundtrip_on_device(he, N, L):
    ctx = he.Context(N, L, T)
    x = wl.uniform_per_modulus(np.random.default_rng(N), (3,), ctx.primes, N)
    X = ctx.ntt_forward(dev(x))
    back = ctx.ntt_inverse(X)
    assert (host(back) == x.astype(np.uint64)).all()
    # the transform is not the identity and lands in [0, q)
    Xh = host(X)
    assert not (Xh == x.astype(np.uint64)).all()
    for l, q in enumerate(ctx.primes):
        assert Xh[:, l, :].max() < q


@pytest.mark.parametrize("N,L", [(4096, 3), (8192, 4), (16384, 6)])
def test_forward_split_rows_match_whole_rows(he, N, L):
    """A launch of at most 128 (64) limb rows shares each row between 2 (4) workgroups; the words
    must be those of the one-workgroup-per-row transform of a larger launch, and round-trip."""
    ctx = he.Context(N, L, T)
    R = 256 // L + 1                                # > 128 limb rows: whole rows
    x = wl.uniform_per_modulus(np.random.default_rng(N + 7), (R,), ctx.primes, N)
    whole = host(ctx.ntt_forward(dev(x)))
    # 2-way, 4-way, one poly, and both sides of the 64- and 128-row boundaries
    for r in sorted({100 // L, 40 // L, 1, 64 // L, 64 // L + 1, 128 // L, 128 // L + 1}):
        part = ctx.ntt_forward(dev(x[:r]))
        assert (host(part) == whole[:r]).all(), f"{r} polys of {L} limbs"
        assert (host(ctx.ntt_inverse(part)) == x[:r].astype(np.uint64)).all()


@pytest.mark.parametrize("N,L", [(256, 2), (1024, 2)])
def test_poly_mul_matches_schoolbook(he, N, L):
    ctx = he.Context(N, L, T)
    rng = np.random.default_rng(N + 1)
    a = wl.uniform_per_modulus(rng, (2,), ctx.primes, N)
    b = wl.uniform_per_modulus(rng, (2,), ctx.primes, N)
    c = host(ctx.poly_mul(dev(a), dev(b)))
    for r in range(2):
        for l, q in enumerate(ctx.primes):
            assert (c[r, l] == ring.negacyclic_schoolbook(a[r, l], b[r, l], q)).all()


@pytest.mark.parametrize("N,L", [(4096, 3), (8192, 4), (16384, 6)])
def test_poly_mul_matches_oracle_ntt_product(he, N, L):
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    rng = np.random.default_rng(N + 2)
    a = wl.uniform_per_modulus(rng, (1,), ctx.primes, N)
    b = wl.uniform_per_modulus(rng, (1,), ctx.primes, N)
    c = host(ctx.poly_mul(dev(a), dev(b)))
    for l, q in enumerate(ctx.primes):
        assert (c[0, l] == ring.negacyclic_ntt(a[0, l], b[0, l], q, octx.psis[l])).all()


def test_monomial_product_on_device(he):
    """X^a * X^b = +-X^((a+b) mod N): a closed form, independent of the oracle."""
    N, L = 4096, 3
    ctx = he.Context(N, L, T)
    pairs = [(0, 0), (1, N - 1), (N - 1, N - 1), (1234, 3000), (2048, 2048)]
    A = np.zeros((len(pairs), L, N), dtype=np.int64)
    B = np.zeros_like(A)
    for r, (x, y) in enumerate(pairs):
        A[r, :, x] = 1
        B[r, :, y] = 1
    C = host(ctx.poly_mul(dev(A), dev(B)))
    for r, (x, y) in enumerate(pairs):
        for l, q in enumerate(ctx.primes):
            expect = np.zeros(N, dtype=np.uint64)
            e = x + y
            expect[e % N] = 1 if e < N else q - 1
            assert (C[r, l] == expect).all()


def test_context_parameters_match_oracle(he):
    for N, L in [(4096, 3), (8192, 4), (16384, 6)]:
        ctx = he.Context(N, L, T)
        octx = bfv.make_ctx(N, L, T)
        assert ctx.primes == octx.primes
        assert ctx.delta_l == octx.delta_l


@pytest.mark.parametrize("N,L", [(4096, 3), (8192, 4), (16384, 6)])
def test_forward_in_place_matches_out_of_place(he, N, L):
    """In place (destination = source) the launcher keeps one workgroup per row, which reads its
    row whole before it stores; the words must equal the out-of-place transform at 1, 8, 64 and
    128 limb rows (the launch sizes whose out-of-place form shares rows between workgroups)."""
    import torch
    ctx = he.Context(N, L, T)
    for limb_rows in (1, 8, 64, 128):
        polys = max(1, limb_rows // L)
        x = wl.uniform_per_modulus(np.random.default_rng(N + limb_rows), (polys,), ctx.primes, N)
        ref = host(ctx.ntt_forward(dev(x)))
        t = dev(x)
        ctx.ntt_forward(t, out=t)
        torch.cuda.synchronize()
        assert (host(t) == ref).all(), f"{polys} polys of {L} limbs in place"


def test_layer_geometry_matches_oracle_packing(he):
    """he_layer_geometry (the library's tiling rule) against the oracle's own implementation of
    the rule, on every plain-20 width and the ResNet-50 body shapes."""
    from oracle import packing
    shapes = []
    for width in (1, 2, 4):
        shapes += [(8192 if width < 4 else 16384, s) for s in wl.plain20(width, 10 if width < 4 else 100)]
    shapes += [(16384, s) for s in set(wl.resnet50_body())]
    ctxs = {}
    for N, shp in shapes:
        ctx = ctxs.setdefault(N, he.Context(N, 1, T))
        if shp.kind == "conv":
            g = packing.conv_geometry(N, shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
            i = ctx.geometry(he.ConvSpec(shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad))
            assert (i.s, i.g_i, i.g_o, i.K_in, i.K_out) == (g.s, g.g_i, g.g_o, g.K_in, g.K_out), shp
            assert i.resident_bytes == shp.c_o * 1 * 2 * g.K_in * N * 4
        else:
            g = packing.fc_geometry(N, shp.n_i, shp.n_o)
            i = ctx.geometry(he.FCSpec(shp.n_i, shp.n_o))
            assert (i.n_o_p, i.n_i_p, i.blocks) == (g.n_o_p, g.n_i_p, g.blocks), shp


def test_layer_call_without_reserved_workspace_fails_cleanly(he):
    """A layer call never allocates: with nothing reserved for its stream it returns HE_ENOMEM
    before any launch, and succeeds once the workspace is reserved."""
    import ctypes
    import torch
    N, L = 1024, 2
    ctx = he.Context(N, L, T)
    rng = np.random.default_rng(3)
    spec = he.ConvSpec(3, 8, 6, 6)
    K_in = ctx.geometry(spec).K_in
    layer = ctx.pack_conv(spec, rng.integers(-7, 8, (8, 3, 3, 3)), rng.integers(0, T, (K_in, 8, N)))
    c0 = dev(wl.uniform_per_modulus(rng, (1, layer.K_in), ctx.primes, N))
    out = torch.zeros((1, layer.K_out, L, N), dtype=torch.int32, device="cuda:0")
    s = torch.cuda.Stream()
    lib = he.load_library()
    rc = lib.he_conv_layer(ctx.handle, layer.handle, 1, c0.data_ptr(), None, None, out.data_ptr(),
                           ctypes.c_void_p(s.cuda_stream))
    assert rc == he.HE_ENOMEM
    assert b"he_workspace_reserve" in lib.he_last_error()
    torch.cuda.synchronize()
    assert int(out.abs().sum()) == 0                      # nothing was launched
    ctx.reserve(layer.workspace_bytes(1), s)
    ctx.conv_layer(layer, c0, out=out, stream=s)
    ref = ctx.conv_layer(layer, c0)
    torch.cuda.synchronize()
    assert (host(out) == host(ref)).all()
