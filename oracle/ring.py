"""Negacyclic polynomial arithmetic in Z_q[X]/(X^N + 1).

Oracle (test infrastructure).  The ring of Sec. II-A: coefficients mod q,
every product reduced by X^N + 1.  Two product routines:

* ``negacyclic_schoolbook`` is the definition written out:
  c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j  (mod q).
* ``ntt`` / ``intt`` form a textbook transform used as a primitive (the paper
  multiplies through NTTs and coefficient-wise products, Sec. IV-A-1).  It is
  the twisted cyclic form: pre-multiply coefficient i by psi^i, run a radix-2
  cyclic DFT with omega = psi^2 over natural order, so that output k equals the
  evaluation a(psi^(2k+1)).  It is pinned against the schoolbook definition and
  against direct evaluation, never trusted on its own.

All arithmetic is on numpy uint64 with residues < 2^30, so every product of two
residues (< 2^60) is exact.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

U64 = np.uint64


def reduce_signed(a, q: int) -> np.ndarray:
    """Map signed integers to residues in [0, q)."""
    return (np.asarray(a, dtype=np.int64) % np.int64(q)).astype(U64)


def negacyclic_schoolbook(a, b, q: int) -> np.ndarray:
    """Product a*b mod (X^N + 1, q) by the definition (O(N^2)).

    Accumulates a_i * (X^i b): multiplying by X^i shifts b up by i places and
    negates the coefficients that wrap past X^N (since X^N = -1).
    """
    a = reduce_signed(a, q)
    b = reduce_signed(b, q)
    N = a.shape[0]
    qq = U64(q)
    acc = np.zeros(N, dtype=U64)
    for i in range(N):
        ai = a[i]
        if ai == 0:
            continue
        shifted = np.empty(N, dtype=U64)
        shifted[i:] = b[: N - i]
        shifted[:i] = (qq - b[N - i:]) % qq
        acc = (acc + ai * shifted % qq) % qq
    return acc


@lru_cache(maxsize=None)
def _tables(N: int, q: int, psi: int):
    """Powers used by the twisted cyclic transform (cached per (N, q, psi))."""
    assert pow(psi, N, q) == q - 1, "psi must be a primitive 2N-th root"
    omega = psi * psi % q
    twist = np.array([pow(psi, i, q) for i in range(N)], dtype=U64)
    untwist = np.array([pow(psi, -i, q) for i in range(N)], dtype=U64)
    rev = np.zeros(N, dtype=np.int64)
    bits = N.bit_length() - 1
    for i in range(N):
        rev[i] = int(format(i, f"0{bits}b")[::-1], 2) if bits else 0
    stages_f, stages_i = [], []
    length = 2
    while length <= N:
        half = length // 2
        wl = pow(omega, N // length, q)
        wli = pow(wl, -1, q)
        stages_f.append(np.array([pow(wl, j, q) for j in range(half)], dtype=U64))
        stages_i.append(np.array([pow(wli, j, q) for j in range(half)], dtype=U64))
        length *= 2
    return twist, untwist, rev, stages_f, stages_i, pow(N, -1, q)


def _cyclic_dft(x: np.ndarray, q: int, rev: np.ndarray, stages) -> np.ndarray:
    """Iterative radix-2 decimation-in-time cyclic DFT over Z_q (natural order out)."""
    N = x.shape[-1]
    qq = U64(q)
    y = x[..., rev].copy()
    length = 2
    for tw in stages:
        half = length // 2
        shp = y.shape[:-1] + (N // length, 2, half)
        z = y.reshape(shp)
        u = z[..., 0, :]
        v = z[..., 1, :] * tw % qq
        top = (u + v) % qq
        bot = (u + qq - v) % qq
        y = np.stack([top, bot], axis=-2).reshape(y.shape)
        length *= 2
    return y


def ntt(a, q: int, psi: int) -> np.ndarray:
    """Forward negacyclic NTT along the last axis: out[..., k] = a(psi^(2k+1)) mod q."""
    a = np.asarray(a, dtype=U64) % U64(q)
    N = a.shape[-1]
    twist, _, rev, sf, _, _ = _tables(N, q, psi)
    return _cyclic_dft(a * twist % U64(q), q, rev, sf)


def intt(A, q: int, psi: int) -> np.ndarray:
    """Inverse of ``ntt`` along the last axis."""
    A = np.asarray(A, dtype=U64) % U64(q)
    N = A.shape[-1]
    _, untwist, rev, _, si, ninv = _tables(N, q, psi)
    y = _cyclic_dft(A, q, rev, si)
    return y * U64(ninv) % U64(q) * untwist % U64(q)


def negacyclic_ntt(a, b, q: int, psi: int) -> np.ndarray:
    """Product a*b mod (X^N + 1, q) through the NTT (primitive, pinned to the schoolbook)."""
    a = reduce_signed(a, q)
    b = reduce_signed(b, q)
    return intt(ntt(a, q, psi) * ntt(b, q, psi) % U64(q), q, psi)


def evaluate(a, x: int, q: int) -> int:
    """a(x) mod q by Horner's rule (used to pin the NTT's evaluation definition)."""
    acc = 0
    for c in reversed([int(v) for v in np.asarray(a).tolist()]):
        acc = (acc * x + c) % q
    return acc
