"""Pins for the oracle's parameters: primes, roots, Delta, CRT (closed forms)."""
import numpy as np
import pytest

from oracle import params

T = 786433


def _trial_division_prime(n: int) -> bool:
    """Independent primality check (trial division), for pinning Miller-Rabin."""
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    r = int(n ** 0.5) + 1
    cand = np.arange(3, r + 1, 2, dtype=np.int64)
    return not np.any(n % cand == 0)


def test_plaintext_modulus():
    assert _trial_division_prime(T)
    assert T - 1 == 3 * 2 ** 18


@pytest.mark.parametrize("n", [2, 3, 4, 17, 97, 561, 7681, 12289, 65537, 1 << 31, (1 << 31) - 1,
                               1073692673, 1073692671, 3215031751])
def test_miller_rabin_matches_trial_division(n):
    assert params.is_prime(n) == _trial_division_prime(n)


@pytest.mark.parametrize("N,L", [(4096, 3), (8192, 4), (16384, 6)])
def test_prime_rule(N, L):
    ps = params.ntt_primes(N, L)
    assert len(ps) == L and ps == sorted(ps, reverse=True)
    for q in ps:
        assert q < 2 ** 30 and q % (2 * N) == 1 and _trial_division_prime(q)
    # no larger admissible prime was skipped
    chosen = set(ps)
    q = ((1 << 30) - 1) // (2 * N) * (2 * N) + 1
    while q >= ps[-1]:
        if q < (1 << 30) and q not in chosen:
            assert not _trial_division_prime(q)
        q -= 2 * N


@pytest.mark.parametrize("N,q", [(8, 17), (16, 97), (4096, 1073692673), (16384, 1072496641)])
def test_primitive_root(N, q):
    psi = params.primitive_2n_root(q, N)
    assert pow(psi, N, q) == q - 1
    assert pow(psi, 2 * N, q) == 1


def test_delta_and_crt_roundtrip():
    ps = params.ntt_primes(8192, 4)
    Q = params.modulus_product(ps)
    D = params.delta(ps, T)
    assert 0 <= Q - T * D < T
    rng = np.random.default_rng(0)
    for _ in range(50):
        x = int(rng.integers(0, 2 ** 62)) * int(rng.integers(0, 2 ** 58)) % Q
        assert params.crt([x % q for q in ps], ps) == x
    assert params.crt([0] * 4, ps) == 0
    assert params.crt([q - 1 for q in ps], ps) == Q - 1
