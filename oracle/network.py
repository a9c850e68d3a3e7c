"""Integer layer references and the client-side harness between layers.

Oracle (test infrastructure).

* ``conv2d`` is Eq. siso_conv_formula / Eq. batch_conv_formula written out: a
  cross-correlation summed over input channels, valid windows of the zero-padded
  input, stride sigma (output size floor((w_i - f_w + 1) / s_w), Sec. II-B).
* ``fc`` is R = W I + B (Sec. II-B).
* ``relu_requant`` / ``gap`` simulate what the client obtains between layers
  (the paper runs ReLU through an OT protocol, Sec. III-C, out of scope here):
  centred lift of the decrypted value mod t, ReLU, then the smallest right
  shift that brings the maximum into [0, 15].  The paper does not define this
  requantisation: parity unpinned, and the same harness feeds both sides.
* ``run_layer_protocol`` drives one layer through every party's steps (client
  encryption, server evaluation, client evaluation, decryption) with keyed
  random inputs; ``server_fn`` lets a test substitute another server.
"""
from __future__ import annotations

from typing import Callable, Optional

import numpy as np

import workloads as wl

from . import bfv, packing


def conv2d(img, F, stride: int = 1, pad: int = 1) -> np.ndarray:
    img = np.asarray(img, dtype=np.int64)
    F = np.asarray(F, dtype=np.int64)
    c_o, c_i, f, _ = F.shape
    x = np.pad(img, ((0, 0), (pad, pad), (pad, pad)))
    Hp, Wp = x.shape[1:]
    Ho = (Hp - f) // stride + 1
    Wo = (Wp - f) // stride + 1
    out = np.zeros((c_o, Ho, Wo), dtype=np.int64)
    for ky in range(f):
        for kx in range(f):
            win = x[:, ky: ky + stride * (Ho - 1) + 1: stride, kx: kx + stride * (Wo - 1) + 1: stride]
            out += np.einsum("nm,myx->nyx", F[:, :, ky, kx], win)
    return out


def fc(I, W, B=None) -> np.ndarray:
    r = np.asarray(W, dtype=np.int64) @ np.asarray(I, dtype=np.int64)
    return r if B is None else r + np.asarray(B, dtype=np.int64)


def centred(x, t: int) -> np.ndarray:
    """Lift residues mod t to (-t/2, t/2]."""
    x = np.asarray(x, dtype=np.int64) % t
    return np.where(x > t // 2, x - t, x)


def relu_requant(z) -> np.ndarray:
    """ReLU then the smallest right shift k >= 0 with max >> k <= 15 (whole tensor)."""
    r = np.maximum(np.asarray(z, dtype=np.int64), 0)
    k = 0
    mx = int(r.max()) if r.size else 0
    while (mx >> k) > 15:
        k += 1
    return r >> k


def gap(x) -> np.ndarray:
    """Global average pool, floor of the mean over the spatial axes."""
    x = np.asarray(x, dtype=np.int64)
    return x.reshape(x.shape[0], -1).sum(axis=1) // (x.shape[1] * x.shape[2])


def plaintext_forward(img, layers, Ws, Bs):
    """Integer forward pass of a conv/FC stack with the harness between layers.

    Returns the list of raw (pre-ReLU) integer outputs of every layer and the
    list of inputs each layer saw.
    """
    outs, ins = [], []
    x = np.asarray(img, dtype=np.int64)
    for idx, (shp, W, B) in enumerate(zip(layers, Ws, Bs)):
        if shp.kind == "conv":
            ins.append(x)
            y = conv2d(x, W, shp.stride, shp.pad)
            outs.append(y)
            a = relu_requant(y)
            nxt = layers[idx + 1] if idx + 1 < len(layers) else None
            x = gap(a) if (nxt is not None and nxt.kind == "fc") else a
        else:
            ins.append(x)
            y = fc(x, W, B)
            outs.append(y)
            x = relu_requant(y)
    return outs, ins


# ------------------------------------------------------------------ protocol
def run_conv_protocol(ctx: bfv.Ctx, shape, img, F, seed_key, first: bool, last: bool,
                      server_fn: Optional[Callable] = None):
    """One Conv layer through Alg. 1 with keyed randomness.

    seed_key = (config, client, variant, layer).  Returns a dict with the
    decrypted output tensor [c_o][H_o][W_o] (share removed), the exact integer
    result, the server output c0^r and the inputs the server saw.
    """
    cfg, cl, var, lay = seed_key
    N, t = ctx.N, ctx.t
    g = packing.conv_geometry(N, shape.c_i, shape.c_o, shape.H, shape.W, shape.f, shape.stride, shape.pad)
    x_poly = packing.pack_conv_input(img, g)                     # true input, packed
    fhat = packing.pack_conv_filters(F, g)
    rho = wl.uniform_below(wl.rng(cfg, 0, var, lay, "rho"), (g.K_in, g.c_o, N), t)
    sh = None if first else wl.uniform_below(wl.rng(cfg, cl, var, lay, "sh"), (g.K_in, N), t)
    sh_next = None if last else wl.uniform_below(wl.rng(cfg, cl, var, lay, "shnext"), (g.K_out, N), t)
    # client keys
    s = wl.ternary(wl.rng(cfg, cl, 0, 0, "s"), N)
    a = wl.uniform_per_modulus(wl.rng(cfg, cl, 0, 0, "a"), (), ctx.primes, N)
    e = wl.gaussian(wl.rng(cfg, cl, 0, 0, "e"), N)
    b = bfv.keygen(ctx, s, a, e)
    # client plaintext i_j = (x_j + sh_j) mod t, encrypt -i_j
    i_polys = x_poly % t if sh is None else (x_poly + sh) % t
    c0 = np.zeros((g.K_in, ctx.L, N), dtype=np.uint64)
    vs = np.zeros((g.K_in, N), dtype=np.int64)
    for j in range(g.K_in):
        v = wl.encryption_v(wl.rng(cfg, cl, var, lay, "v", j), N)
        e0 = wl.gaussian(wl.rng(cfg, cl, var, lay, "e0", j), N)
        c0[j] = bfv.encrypt_c0(ctx, i_polys[j], v, e0, b)
        vs[j] = v
    # server
    srv = server_fn or (lambda *args: bfv.server_conv(ctx, g, *args))
    c0r = srv(c0, rho, fhat, sh, sh_next)
    # client masks (server initialisation), client evaluation, decryption
    e1 = wl.gaussian(wl.rng(cfg, 0, var, lay, "e1"), (g.K_in, g.c_o, N))
    e2 = wl.gaussian(wl.rng(cfg, 0, var, lay, "e2"), (g.K_in, g.c_o, N))
    p1, p2 = bfv.client_masks(ctx, rho, fhat, b, e1, e2)
    c1r = bfv.client_conv(ctx, g, vs, i_polys, p1, p2)
    tot = bfv.add_shares(ctx, c0r, c1r)
    r = bfv.decrypt(ctx, tot)                                  # [K_out][N]
    if sh_next is not None:
        r = (r - sh_next) % t
    dec = packing.decode_conv_output(r, g)
    ref = conv2d(img, F, shape.stride, shape.pad)
    return dict(geom=g, decrypted=dec, reference=ref, c0r=c0r, c0=c0, rho=rho, fhat=fhat,
                sh=sh, sh_next=sh_next, total=tot, r=r)


def run_fc_protocol(ctx: bfv.Ctx, shape, vec, W, B, seed_key, first: bool, last: bool,
                    server_fn: Optional[Callable] = None):
    """One FC layer through Alg. 2 with keyed randomness (see run_conv_protocol)."""
    cfg, cl, var, lay = seed_key
    N, t = ctx.N, ctx.t
    g = packing.fc_geometry(N, shape.n_i, shape.n_o)
    x_poly = packing.pack_fc_input(vec, g)
    w = packing.pack_fc_weights(W, g)
    d = packing.pack_fc_bias(B, g)
    rho = wl.uniform_below(wl.rng(cfg, 0, var, lay, "rho"), (g.blocks, N), t)
    sh = None if first else wl.uniform_below(wl.rng(cfg, cl, var, lay, "sh"), (N,), t)
    sh_next = None if last else wl.uniform_below(wl.rng(cfg, cl, var, lay, "shnext"), (g.blocks, g.n_o_p), t)
    s = wl.ternary(wl.rng(cfg, cl, 0, 0, "s"), N)
    a = wl.uniform_per_modulus(wl.rng(cfg, cl, 0, 0, "a"), (), ctx.primes, N)
    e = wl.gaussian(wl.rng(cfg, cl, 0, 0, "e"), N)
    b = bfv.keygen(ctx, s, a, e)
    i_poly = x_poly % t if sh is None else (x_poly + sh) % t
    v = wl.encryption_v(wl.rng(cfg, cl, var, lay, "v", 0), N)
    e0 = wl.gaussian(wl.rng(cfg, cl, var, lay, "e0", 0), N)
    c0 = bfv.encrypt_c0(ctx, i_poly, v, e0, b)
    srv = server_fn or (lambda *args: bfv.server_fc(ctx, g, *args))
    c0r = srv(c0, rho, w, d, sh, sh_next)
    e1 = wl.gaussian(wl.rng(cfg, 0, var, lay, "e1"), (g.blocks, N))
    e2 = wl.gaussian(wl.rng(cfg, 0, var, lay, "e2"), (g.blocks, N))
    p1, p2 = bfv.client_masks(ctx, rho, w, b, e1, e2)
    c1r = bfv.client_fc(ctx, g, v, i_poly, p1, p2)
    tot = bfv.add_shares(ctx, c0r, c1r)
    r = bfv.decrypt(ctx, tot)                                  # [blocks][n_o']
    if sh_next is not None:
        r = (r - sh_next) % t
    dec = packing.decode_fc_output(r, g)
    ref = fc(vec, W, B)
    return dict(geom=g, decrypted=dec, reference=ref, c0r=c0r, c0=c0, rho=rho, w=w, d=d,
                sh=sh, sh_next=sh_next, total=tot, r=r)
