"""Coefficient packing of Conv and FC layers (Sec. II-C, Sec. III-A, Sec. III-B).

Oracle (test infrastructure).

Conv.  The paper packs all c_i input channels of one image into i(X)
(Eq. i_batch: channel m's pixel (k, l) at exponent s(k h_i + l) + m, up to a
fixed offset) and all filters of output channel n into
f^(n)(X) = X^(n c_i / c_o) * sum_m f^(m,n),<s>(X) X^(-m) (Eq. k_batch_new), so
that output channel n's results land on the residue class n c_i/c_o mod s.
The paper assumes N = c_i w^2, c_o | c_i and valid padding.  The plain-20
shapes break all three, so this module uses the generalised tiling below (the
paper's case is recovered exactly: s = c_i, g_o = c_o, o_n = n c_i / c_o):

  H_p = H + 2 pad, W_p = W + 2 pad             (zero padding is packed in)
  s   = 2^floor(log2(N / (H_p W_p)))           slot stride, needs s >= 1
  g_i = min(c_i, s)                             input channels per input poly
  g_o = largest power of two <= min(c_o, s)     output channels per output poly
  K_in = ceil(c_i / g_i), K_out = ceil(c_o / g_o)
  o_n = (n mod g_o) * (s / g_o)                 residue class of channel n

  input poly j :  coefficient s (y W_p + x) + m'  =  I_pad^(j g_i + m')[y][x]
  filter (j,n) :  sum_{m' < g_i, ky, kx} F^(j g_i + m', n)[ky][kx]
                      * X^(o_n - s (ky W_p + kx) - m')     with X^-e = -X^(N-e)

Exponents are the paper's (ConvFHE's) with the input shifted up by s f W_p and
the filter shifted down by the same amount, so the product is identical.
Output channel n, position (oy, ox) of a stride-sigma layer is coefficient
s (sigma oy W_p + sigma ox) + o_n of output poly floor(n / g_o).  Exact (no
aliasing) whenever s H_p W_p <= N and g_i <= s.

FC.  Eq. i(x) formula / w(x) formula with n_o' = n_o rounded up to a power of
two (zero-padded rows) and n_i' = N / n_o' (zero-padded columns); when
n_i n_o' > N the matrix is split into blocks of n_o' = 2^floor(log2(N / n_i))
rows (the paper's floor(N / n_i) rows per polynomial, Sec. IV-A-3).  By
Theorem 1 coefficient k < n_o' of i(X) w_b(X) + d_b(X) is output b n_o' + k.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _pow2_floor(x: int) -> int:
    return 1 << (int(x).bit_length() - 1)


def _pow2_ceil(x: int) -> int:
    return 1 << (int(x) - 1).bit_length() if x > 1 else 1


@dataclass(frozen=True)
class ConvGeom:
    N: int
    c_i: int
    c_o: int
    H: int
    W: int
    f: int
    stride: int
    pad: int
    H_p: int
    W_p: int
    s: int
    g_i: int
    g_o: int
    K_in: int
    K_out: int
    H_o: int
    W_o: int

    def class_of(self, n: int) -> int:
        """Residue class o_n holding output channel n."""
        return (n % self.g_o) * (self.s // self.g_o)


def conv_geometry(N: int, c_i: int, c_o: int, H: int, W: int, f: int = 3,
                  stride: int = 1, pad: int = 1) -> ConvGeom:
    H_p, W_p = H + 2 * pad, W + 2 * pad
    if H_p * W_p > N:
        raise ValueError("padded image does not fit in one polynomial")
    s = _pow2_floor(N // (H_p * W_p))
    g_i = min(c_i, s)
    g_o = _pow2_floor(min(c_o, s))
    K_in = -(-c_i // g_i)
    K_out = -(-c_o // g_o)
    # output size, valid windows over the padded image (Sec. II-B)
    H_o = (H_p - f) // stride + 1
    W_o = (W_p - f) // stride + 1
    return ConvGeom(N, c_i, c_o, H, W, f, stride, pad, H_p, W_p, s, g_i, g_o,
                    K_in, K_out, H_o, W_o)


def pack_conv_input(img: np.ndarray, g: ConvGeom) -> np.ndarray:
    """Input image [c_i][H][W] -> K_in integer polynomials [K_in][N] (Eq. i_batch)."""
    img = np.asarray(img, dtype=np.int64)
    out = np.zeros((g.K_in, g.N), dtype=np.int64)
    for m in range(g.c_i):
        j, mp = divmod(m, g.g_i)
        for y in range(g.H):
            for x in range(g.W):
                yp, xp = y + g.pad, x + g.pad
                out[j, g.s * (yp * g.W_p + xp) + mp] = img[m, y, x]
    return out


def pack_conv_filters(F: np.ndarray, g: ConvGeom) -> np.ndarray:
    """Filters [c_o][c_i][f][f] -> f-hat [K_in][c_o][N] signed integers (Eq. k_batch_new)."""
    F = np.asarray(F, dtype=np.int64)
    N = g.N
    out = np.zeros((g.K_in, g.c_o, N), dtype=np.int64)
    for n in range(g.c_o):
        o_n = g.class_of(n)
        for m in range(g.c_i):
            j, mp = divmod(m, g.g_i)
            for ky in range(g.f):
                for kx in range(g.f):
                    e = o_n - g.s * (ky * g.W_p + kx) - mp
                    w = int(F[n, m, ky, kx])
                    if e >= 0:
                        out[j, n, e] += w
                    else:                      # X^e = -X^(N+e) for -N < e < 0
                        out[j, n, N + e] -= w
    return out


def conv_output_coeff(g: ConvGeom, n: int, oy: int, ox: int):
    """(output poly index, coefficient index) of output channel n at (oy, ox)."""
    k = g.s * (g.stride * oy * g.W_p + g.stride * ox) + g.class_of(n)
    return n // g.g_o, k


def decode_conv_output(r: np.ndarray, g: ConvGeom) -> np.ndarray:
    """Plaintext output polys [K_out][N] -> [c_o][H_o][W_o]."""
    out = np.zeros((g.c_o, g.H_o, g.W_o), dtype=np.int64)
    for n in range(g.c_o):
        for oy in range(g.H_o):
            for ox in range(g.W_o):
                p, k = conv_output_coeff(g, n, oy, ox)
                out[n, oy, ox] = r[p, k]
    return out


@dataclass(frozen=True)
class FCGeom:
    N: int
    n_i: int
    n_o: int
    n_o_p: int      # rows per block (power of two), the paper's n_o in Eq. w(x)
    n_i_p: int      # padded input length N / n_o_p
    blocks: int


def fc_geometry(N: int, n_i: int, n_o: int) -> FCGeom:
    n_o_p = _pow2_ceil(n_o)
    if n_i * n_o_p > N:
        n_o_p = _pow2_floor(N // n_i)
    if n_o_p < 1 or n_i > N:
        raise ValueError("FC input does not fit in one polynomial")
    n_i_p = N // n_o_p
    blocks = -(-n_o // n_o_p)
    return FCGeom(N, n_i, n_o, n_o_p, n_i_p, blocks)


def pack_fc_input(I: np.ndarray, g: FCGeom) -> np.ndarray:
    """Eq. i(x) formula: i(X) = sum_l I_l X^(l n_o')."""
    out = np.zeros(g.N, dtype=np.int64)
    for l in range(g.n_i):
        out[l * g.n_o_p] = int(I[l])
    return out


def _padded_matrix(W: np.ndarray, g: FCGeom) -> np.ndarray:
    Wp = np.zeros((g.blocks * g.n_o_p, g.n_i_p), dtype=np.int64)
    Wp[: g.n_o, : g.n_i] = np.asarray(W, dtype=np.int64)
    return Wp


def pack_fc_weights(W: np.ndarray, g: FCGeom) -> np.ndarray:
    """Eq. w(x) formula per block b (rows b n_o' ... b n_o' + n_o' - 1):

    w_b(X) = sum_k W_{k,0} X^k - sum_k sum_{l=1}^{n_i'-1} W_{k, n_i'-l} X^(l n_o' + k).
    """
    Wp = _padded_matrix(W, g)
    out = np.zeros((g.blocks, g.N), dtype=np.int64)
    for b in range(g.blocks):
        rows = Wp[b * g.n_o_p:(b + 1) * g.n_o_p]
        for k in range(g.n_o_p):
            out[b, k] = rows[k, 0]
            for l in range(1, g.n_i_p):
                out[b, l * g.n_o_p + k] = -rows[k, g.n_i_p - l]
    return out


def pack_fc_bias(B, g: FCGeom) -> np.ndarray:
    """d_b(X) = sum_k B_{b n_o' + k} X^k, as [blocks][n_o'] (zero-padded)."""
    out = np.zeros((g.blocks, g.n_o_p), dtype=np.int64)
    if B is None:
        return out
    flat = np.zeros(g.blocks * g.n_o_p, dtype=np.int64)
    flat[: g.n_o] = np.asarray(B, dtype=np.int64)
    return flat.reshape(g.blocks, g.n_o_p)


def decode_fc_output(r: np.ndarray, g: FCGeom) -> np.ndarray:
    """[blocks][n_o'] plaintext -> the n_o outputs."""
    return np.asarray(r, dtype=np.int64).reshape(-1)[: g.n_o].copy()
