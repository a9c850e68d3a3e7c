"""Ring parameters: NTT-friendly primes, roots of unity, Delta and CRT.

Oracle (test infrastructure).  The paper works over R_Q = Z_Q[X]/(X^N + 1) with
Q a product of word-size primes handled through the CRT (Sec. I, Sec. II-A).
The prime rule (the L largest primes below 2^30 with q = 1 mod 2N) and the
exact BFV scale Delta = floor(Q / t) are this repository's readings of the
paper's unspecified parameters.
"""
from __future__ import annotations

from functools import reduce
from typing import List, Sequence


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin, exact for n < 3.3e24 with these bases."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)
    for p in small:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(N: int, L: int, bits: int = 30) -> List[int]:
    """The L largest primes q < 2^bits with q = 1 (mod 2N), in descending order."""
    step = 2 * N
    q = ((1 << bits) - 1) // step * step + 1
    if q >= (1 << bits):
        q -= step
    out = []
    while len(out) < L:
        if q < 2:
            raise ValueError("not enough primes")
        if is_prime(q):
            out.append(q)
        q -= step
    return out


def primitive_2n_root(q: int, N: int) -> int:
    """A primitive 2N-th root of unity psi mod q (psi^N = -1).

    Since 2N is a power of two, any x with x^N = -1 has order exactly 2N.
    Candidates are g^((q-1)/2N) for g = 2, 3, ...
    """
    if (q - 1) % (2 * N):
        raise ValueError("q != 1 mod 2N")
    e = (q - 1) // (2 * N)
    for g in range(2, q):
        psi = pow(g, e, q)
        if pow(psi, N, q) == q - 1:
            return psi
    raise ValueError("no root")


def modulus_product(primes: Sequence[int]) -> int:
    return reduce(lambda x, y: x * y, primes, 1)


def delta(primes: Sequence[int], t: int) -> int:
    """BFV plaintext scale Delta = floor(Q / t)."""
    return modulus_product(primes) // t


def crt(residues: Sequence[int], primes: Sequence[int]) -> int:
    """The unique x in [0, Q) with x = residues[l] (mod primes[l])."""
    Q = modulus_product(primes)
    x = 0
    for r, q in zip(residues, primes):
        Mi = Q // q
        x += int(r) * Mi * pow(Mi, -1, q)
    return x % Q
