"""Pins for the oracle's negacyclic arithmetic.

The schoolbook product is pinned to hand-worked small products, the monomial
closed form X^a X^b = +-X^((a+b) mod N) and an integer linear convolution
folded by X^N = -1.  The NTT is pinned to the schoolbook product, to direct
evaluation at the odd powers of psi, and to its inverse.
"""
import numpy as np
import pytest

from oracle import params, ring

SMALL = [(8, 17), (16, 97), (32, 193), (64, 257)]
BIG_Q = [1073692673, 1072496641]


def test_schoolbook_hand_examples():
    q = 97
    # (1 + X)^2 = 1 + 2X + X^2 in Z[X]/(X^4 + 1)
    assert ring.negacyclic_schoolbook([1, 1, 0, 0], [1, 1, 0, 0], q).tolist() == [1, 2, 1, 0]
    # X^3 * X = X^4 = -1
    assert ring.negacyclic_schoolbook([0, 0, 0, 1], [0, 1, 0, 0], q).tolist() == [q - 1, 0, 0, 0]
    # (1 + 2X + 3X^2 + 4X^3) X = -4 + X + 2X^2 + 3X^3
    assert ring.negacyclic_schoolbook([1, 2, 3, 4], [0, 1, 0, 0], q).tolist() == [q - 4, 1, 2, 3]


@pytest.mark.parametrize("N", [4, 8, 16])
def test_schoolbook_monomials(N):
    q = 257
    for a in range(N):
        for b in range(N):
            xa = np.zeros(N, dtype=np.int64); xa[a] = 1
            xb = np.zeros(N, dtype=np.int64); xb[b] = 1
            expect = np.zeros(N, dtype=np.int64)
            e = a + b
            expect[e % N] = 1 if e < N else q - 1
            assert (ring.negacyclic_schoolbook(xa, xb, q) == expect).all()


@pytest.mark.parametrize("N,q", SMALL + [(64, BIG_Q[0])])
def test_schoolbook_vs_folded_linear_convolution(N, q):
    rng = np.random.default_rng(N)
    a = rng.integers(-20, 20, N)
    b = rng.integers(-20, 20, N)
    lin = np.convolve(a, b)                     # exact integer product, degree <= 2N-2
    folded = lin[:N].copy()
    folded[: N - 1] -= lin[N:]                  # X^(N+k) = -X^k
    assert (ring.negacyclic_schoolbook(a, b, q) == folded % q).all()


@pytest.mark.parametrize("N,q", SMALL + [(32, BIG_Q[0]), (64, BIG_Q[1])])
def test_ntt_product_equals_schoolbook(N, q):
    psi = params.primitive_2n_root(q, N)
    rng = np.random.default_rng(q % 1000 + N)
    for _ in range(3):
        a = rng.integers(0, q, N)
        b = rng.integers(0, q, N)
        assert (ring.negacyclic_ntt(a, b, q, psi) == ring.negacyclic_schoolbook(a, b, q)).all()


@pytest.mark.parametrize("N,q", [(16, 97), (64, BIG_Q[0])])
def test_ntt_is_evaluation_at_odd_powers(N, q):
    psi = params.primitive_2n_root(q, N)
    a = np.random.default_rng(7).integers(0, q, N)
    A = ring.ntt(a, q, psi)
    for k in range(N):
        assert int(A[k]) == ring.evaluate(a, pow(psi, 2 * k + 1, q), q)


@pytest.mark.parametrize("N,q", [(4096, BIG_Q[0]), (16384, BIG_Q[1])])
def test_intt_inverts_ntt(N, q):
    psi = params.primitive_2n_root(q, N)
    a = np.random.default_rng(3).integers(0, q, (2, N)).astype(np.uint64)
    assert (ring.intt(ring.ntt(a, q, psi), q, psi) == a).all()
    assert (ring.ntt(ring.intt(a, q, psi), q, psi) == a).all()
