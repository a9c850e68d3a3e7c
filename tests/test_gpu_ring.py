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
