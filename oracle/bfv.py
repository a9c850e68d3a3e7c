"""Exact (BFV-style) reading of the paper's server-client layer procedure.

Oracle (test infrastructure).  Follows Alg. 1 (Conv) and Alg. 2 (FC) of
Sec. III in the paper's order, in the exact-integer reading used by this
repository:

* Scheme.  The paper uses CKKS (Sec. II-A).  Here the plaintext ring is Z_t,
  Delta = floor(Q / t), and the per-share rescale by Delta^-1 (Alg. 1 lines
  after the products, Alg. 2 server and client lines) is replaced by one
  scale-and-round after the two shares are added (reading R1).
* Encryption of -i (Alg. 1 client encryption, Eq. encryption): the client sends
  c0 = -(v b + Delta i + e0) mod Q, the negation of the fresh encryption of i,
  keeping v.  This is the sign choice under which v rho b cancels between the
  server line c0 rho - sh f and the client line v p1 + i p2 (reading R2).
* Scale placement (reading R3): the server subtracts Delta sh f-hat; the
  client mask is p2 = Delta (f-hat + rho) + e2 and the client multiplies it by
  its unscaled plaintext i in [0, t).
* rho, sh, sh' are uniform in [0, t) (reading R4); in Alg. 2 the server line
  reads c0 rho (reading R5).
* Extraction (Alg. 1, the loop over j and n): output poly g receives, for each
  channel n of its group, the coefficients in residue class o_n mod s of
  c0^(n); the other coefficients are zero before Delta sh' is added to every
  coefficient (reading R10).
* Decryption rounds half up: r = floor((t x + floor(Q/2)) / Q) mod t with x the
  CRT lift of c0^r + c1^r (reading R11).

Polynomials are numpy int64/uint64 arrays; a limb axis of length L holds the
residues mod each prime.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import params, ring
from .packing import ConvGeom, FCGeom

U64 = np.uint64


@dataclass
class Ctx:
    N: int
    t: int
    primes: List[int]
    psis: List[int]
    Q: int
    Delta: int
    delta_l: List[int]

    @property
    def L(self) -> int:
        return len(self.primes)


def make_ctx(N: int, L: int, t: int, primes: Optional[Sequence[int]] = None) -> Ctx:
    primes = list(primes) if primes is not None else params.ntt_primes(N, L)
    psis = [params.primitive_2n_root(q, N) for q in primes]
    Q = params.modulus_product(primes)
    D = Q // t
    return Ctx(N, t, primes, psis, Q, D, [D % q for q in primes])


# ------------------------------------------------------------------ helpers
def _limbs(ctx: Ctx, a) -> np.ndarray:
    """Signed integer polynomial(s) [..., N] -> residues [..., L, N]."""
    a = np.asarray(a, dtype=np.int64)
    return np.stack([ring.reduce_signed(a, q) for q in ctx.primes], axis=-2)


def _sum_of_products(ctx: Ctx, l: int, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """sum_j xs[j] * ys[j, ...] in Z_q[X]/(X^N+1) for limb l.

    xs: [J][N] residues, ys: [J][M][N] residues -> [M][N].  Uses the NTT as a
    multiplication primitive: transform, coefficient-wise multiply-add,
    one inverse transform per output.
    """
    q, psi = ctx.primes[l], ctx.psis[l]
    qq = U64(q)
    X = ring.ntt(xs, q, psi)                      # [J][N]
    Y = ring.ntt(ys, q, psi)                      # [J][M][N]
    acc = np.zeros(Y.shape[1:], dtype=U64)
    for j in range(X.shape[0]):
        acc = (acc + Y[j] * X[j][None, :] % qq) % qq
    return ring.intt(acc, q, psi)


# ------------------------------------------------------------------ client keys
def keygen(ctx: Ctx, s, a, e) -> np.ndarray:
    """Public key part b = -a s + e mod Q (Sec. II-A).  a: [L][N] residues; s, e signed.

    Returns b as [L][N] residues (pk = (b, a)).
    """
    b = np.zeros((ctx.L, ctx.N), dtype=U64)
    for l, q in enumerate(ctx.primes):
        qq = U64(q)
        as_ = ring.negacyclic_ntt(a[l], s, q, ctx.psis[l])
        b[l] = (ring.reduce_signed(e, q) + qq - as_) % qq
    return b


def encrypt_c0(ctx: Ctx, i_poly, v, e0, b) -> np.ndarray:
    """c0 of the encryption of -i (Alg. 1 / Alg. 2 client encryption; reading R2).

    c0 = -(v b + Delta i + e0) mod Q, for i with coefficients in [0, t).
    Returns [L][N] residues.
    """
    out = np.zeros((ctx.L, ctx.N), dtype=U64)
    i_poly = np.asarray(i_poly, dtype=np.int64)
    for l, q in enumerate(ctx.primes):
        qq = U64(q)
        vb = ring.negacyclic_ntt(v, b[l], q, ctx.psis[l])
        di = ring.reduce_signed(i_poly, q) * U64(ctx.delta_l[l]) % qq
        tot = (vb + di + ring.reduce_signed(e0, q)) % qq
        out[l] = (qq - tot) % qq
    return out


# ------------------------------------------------------------------ server side
def server_conv(ctx: Ctx, g: ConvGeom, c0, rho, fhat, sh=None, sh_next=None) -> np.ndarray:
    """Server evaluation of one Conv layer (Alg. 1, server evaluation).

    c0    [K_in][L][N] residues (coefficient domain)
    rho   [K_in][c_o][N] integers in [0, t)        (server masks)
    fhat  [K_in][c_o][N] signed packed filters     (Eq. k_batch_new, generalised)
    sh    [K_in][N] in [0, t) or None (first layer: no share to remove)
    sh_next [K_out][N] in [0, t) or None (last layer: no fresh share)
    returns c0^r as [K_out][L][N] residues.

    Steps: c0^(n) = sum_j c0_j rho_j^(n) - Delta sh_j fhat_j^(n); extract the
    residue class o_n of each c0^(n) into output poly floor(n / g_o); add
    Delta sh'.
    """
    N, L = ctx.N, ctx.L
    out = np.zeros((g.K_out, L, N), dtype=U64)
    k = np.arange(N)
    for l, q in enumerate(ctx.primes):
        qq = U64(q)
        A = _sum_of_products(ctx, l, np.asarray(c0)[:, l, :], ring.reduce_signed(rho, q))
        if sh is not None:
            P = _sum_of_products(ctx, l, ring.reduce_signed(sh, q), ring.reduce_signed(fhat, q))
            A = (A + qq - P * U64(ctx.delta_l[l]) % qq) % qq
        for n in range(g.c_o):
            sel = (k % g.s) == g.class_of(n)
            out[n // g.g_o, l, sel] = A[n, sel]
        if sh_next is not None:
            add = ring.reduce_signed(sh_next, q) * U64(ctx.delta_l[l]) % qq
            out[:, l, :] = (out[:, l, :] + add) % qq
    return out


def server_fc(ctx: Ctx, g: FCGeom, c0, rho, w, d=None, sh=None, sh_next=None) -> np.ndarray:
    """Server evaluation of one FC layer (Alg. 2, server evaluation).

    c0 [L][N]; rho [blocks][N] in [0, t); w [blocks][N] signed (Eq. w(x) formula);
    d [blocks][n_o'] signed bias; sh [N] in [0, t) or None; sh_next [blocks][n_o']
    or None.  Returns [blocks][L][n_o']: the first n_o' coefficients of
    c0 rho_b - Delta sh w_b, plus Delta ((d_b + sh'_b) mod t).
    """
    L, no = ctx.L, g.n_o_p
    out = np.zeros((g.blocks, L, no), dtype=U64)
    c0 = np.asarray(c0)
    dd = np.zeros((g.blocks, no), dtype=np.int64) if d is None else np.asarray(d, dtype=np.int64)
    msg = dd + (0 if sh_next is None else np.asarray(sh_next, dtype=np.int64))
    msg = msg % ctx.t
    for l, q in enumerate(ctx.primes):
        qq = U64(q)
        A = _sum_of_products(ctx, l, c0[l][None, :], ring.reduce_signed(rho, q)[None])
        if sh is not None:
            P = _sum_of_products(ctx, l, ring.reduce_signed(sh, q)[None, :], ring.reduce_signed(w, q)[None])
            A = (A + qq - P * U64(ctx.delta_l[l]) % qq) % qq
        out[:, l, :] = (A[:, :no] + msg.astype(U64) * U64(ctx.delta_l[l]) % qq) % qq
    return out


# ------------------------------------------------------------------ client side
def client_masks(ctx: Ctx, rho, fhat, b, e1, e2):
    """Server-initialisation masks sent to the client (Alg. 1 / Alg. 2 initialisation).

    p1 = rho b + e1, p2 = Delta (fhat + rho) + e2 (reading R3).
    rho, fhat, e1, e2: [..., N] integers; b: [L][N].  Returns p1, p2 as [..., L, N].
    """
    rho = np.asarray(rho, dtype=np.int64)
    lead = rho.shape[:-1]
    p1 = np.zeros(lead + (ctx.L, ctx.N), dtype=U64)
    p2 = np.zeros_like(p1)
    flat_r = rho.reshape(-1, ctx.N)
    flat_f = np.asarray(fhat, dtype=np.int64).reshape(-1, ctx.N)
    flat_e1 = np.asarray(e1, dtype=np.int64).reshape(-1, ctx.N)
    flat_e2 = np.asarray(e2, dtype=np.int64).reshape(-1, ctx.N)
    p1v = p1.reshape(-1, ctx.L, ctx.N)
    p2v = p2.reshape(-1, ctx.L, ctx.N)
    for l, q in enumerate(ctx.primes):
        qq, psi = U64(q), ctx.psis[l]
        Bh = ring.ntt(b[l], q, psi)
        Rh = ring.ntt(ring.reduce_signed(flat_r, q), q, psi)
        p1v[:, l, :] = (ring.intt(Rh * Bh[None, :] % qq, q, psi) + ring.reduce_signed(flat_e1, q)) % qq
        fr = ring.reduce_signed(flat_f + flat_r, q) * U64(ctx.delta_l[l]) % qq
        p2v[:, l, :] = (fr + ring.reduce_signed(flat_e2, q)) % qq
    return p1, p2


def client_conv(ctx: Ctx, g: ConvGeom, v, i_polys, p1, p2) -> np.ndarray:
    """Client evaluation of one Conv layer (Alg. 1, client evaluation).

    c1^(n) = sum_j v_j p1_j^(n) + i_j p2_j^(n); the same residue-class
    extraction as the server, no share.  v, i_polys: [K_in][N]; p1, p2:
    [K_in][c_o][L][N].  Returns c1^r as [K_out][L][N].
    """
    N = ctx.N
    out = np.zeros((g.K_out, ctx.L, N), dtype=U64)
    k = np.arange(N)
    for l, q in enumerate(ctx.primes):
        qq = U64(q)
        A = _sum_of_products(ctx, l, ring.reduce_signed(v, q), np.asarray(p1)[:, :, l, :])
        B = _sum_of_products(ctx, l, ring.reduce_signed(i_polys, q), np.asarray(p2)[:, :, l, :])
        C = (A + B) % qq
        for n in range(g.c_o):
            sel = (k % g.s) == g.class_of(n)
            out[n // g.g_o, l, sel] = C[n, sel]
    return out


def client_fc(ctx: Ctx, g: FCGeom, v, i_poly, p1, p2) -> np.ndarray:
    """Client evaluation of one FC layer (Alg. 2): first n_o' coefficients of v p1_b + i p2_b.

    v, i_poly: [N]; p1, p2: [blocks][L][N].  Returns [blocks][L][n_o'].
    """
    out = np.zeros((g.blocks, ctx.L, g.n_o_p), dtype=U64)
    for l, q in enumerate(ctx.primes):
        qq = U64(q)
        A = _sum_of_products(ctx, l, ring.reduce_signed(v, q)[None, :], np.asarray(p1)[None, :, l, :])
        B = _sum_of_products(ctx, l, ring.reduce_signed(i_poly, q)[None, :], np.asarray(p2)[None, :, l, :])
        out[:, l, :] = ((A + B) % qq)[:, : g.n_o_p]
    return out


# ------------------------------------------------------------------ decryption
def add_shares(ctx: Ctx, c0r, c1r) -> np.ndarray:
    """r = c0^r + c1^r limb-wise (Alg. 1 / Alg. 2, last client line)."""
    out = np.zeros(np.shape(c0r), dtype=U64)
    for l, q in enumerate(ctx.primes):
        out[..., l, :] = (np.asarray(c0r)[..., l, :] + np.asarray(c1r)[..., l, :]) % U64(q)
    return out


def crt_lift(ctx: Ctx, x) -> np.ndarray:
    """[..., L, M] residues -> object array [..., M] of integers in [0, Q)."""
    x = np.asarray(x)
    lead = x.shape[:-2]
    M = x.shape[-1]
    flat = x.reshape(-1, ctx.L, M)
    out = np.empty((flat.shape[0], M), dtype=object)
    Q = ctx.Q
    coefs = []
    for q in ctx.primes:
        Mi = Q // q
        coefs.append(Mi * pow(Mi, -1, q))
    for r in range(flat.shape[0]):
        acc = np.zeros(M, dtype=object)
        for l in range(ctx.L):
            acc = acc + flat[r, l].astype(object) * coefs[l]
        out[r] = acc % Q
    return out.reshape(lead + (M,))


def decrypt(ctx: Ctx, x) -> np.ndarray:
    """Scale and round the share sum: floor((t x + floor(Q/2)) / Q) mod t, per coefficient."""
    X = crt_lift(ctx, x)
    half = ctx.Q // 2
    fn = np.frompyfunc(lambda z: ((ctx.t * z + half) // ctx.Q) % ctx.t, 1, 1)
    return fn(X).astype(np.int64)


def noise_magnitude(ctx: Ctx, x, m) -> int:
    """max |x - Delta m| over coefficients, centred mod Q, for x ~ Delta m + noise."""
    X = crt_lift(ctx, x)
    M = np.asarray(m, dtype=np.int64).astype(object) % ctx.t
    E = (X - M * ctx.Delta) % ctx.Q
    E = np.where(E > ctx.Q // 2, E - ctx.Q, E)
    return int(max(abs(int(e)) for e in E.reshape(-1)))
