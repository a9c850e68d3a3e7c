"""Seeded full-size parity cases shared by the golden-digest script and the GPU tests.

Each case rebuilds the server's inputs for one layer from the keyed workload
generators and the oracle's client (key generation and c0 encryption of the
layer's true input plus the server share).  Layer inputs follow the plain-20
harness: the true input of layer k+1 is the ReLU / requantised integer output
of layer k (the value the client decrypts, checked by the golden script), so
the sequence is the closed loop without re-running the client per layer.
"""
from __future__ import annotations

import hashlib
from typing import Dict

import numpy as np

import workloads as wl
from oracle import bfv, network, packing


def digest(arr) -> str:
    a = np.ascontiguousarray(np.asarray(arr).astype("<u4"))
    return hashlib.sha256(a.tobytes()).hexdigest()


def client_key(ctx: bfv.Ctx, cfg: int, client: int):
    s = wl.ternary(wl.rng(cfg, client, 0, 0, "s"), ctx.N)
    a = wl.uniform_per_modulus(wl.rng(cfg, client, 0, 0, "a"), (), ctx.primes, ctx.N)
    e = wl.gaussian(wl.rng(cfg, client, 0, 0, "e"), ctx.N)
    return s, bfv.keygen(ctx, s, a, e)


def conv_inputs(ctx: bfv.Ctx, shape, x, cfg, client, variant, layer, first, last, b) -> Dict:
    """Server inputs of one conv layer whose true (plaintext) input is x [c_i][H][W]."""
    N, t = ctx.N, ctx.t
    g = packing.conv_geometry(N, shape.c_i, shape.c_o, shape.H, shape.W, shape.f, shape.stride, shape.pad)
    F = wl.layer_weights(cfg, variant, layer, shape)
    rho = wl.uniform_below(wl.rng(cfg, 0, variant, layer, "rho"), (g.K_in, g.c_o, N), t)
    sh = None if first else wl.uniform_below(wl.rng(cfg, client, variant, layer, "sh"), (g.K_in, N), t)
    shn = None if last else wl.uniform_below(wl.rng(cfg, client, variant, layer, "shnext"), (g.K_out, N), t)
    xp = packing.pack_conv_input(x, g)
    ip = xp % t if sh is None else (xp + sh) % t
    c0 = np.zeros((g.K_in, ctx.L, N), dtype=np.uint64)
    vs = np.zeros((g.K_in, N), dtype=np.int64)
    for j in range(g.K_in):
        v = wl.encryption_v(wl.rng(cfg, client, variant, layer, "v", j), N)
        e0 = wl.gaussian(wl.rng(cfg, client, variant, layer, "e0", j), N)
        c0[j] = bfv.encrypt_c0(ctx, ip[j], v, e0, b)
        vs[j] = v
    return dict(geom=g, F=F, rho=rho, fhat=packing.pack_conv_filters(F, g), sh=sh, sh_next=shn, c0=c0,
                v=vs, i_polys=ip)


def fc_inputs(ctx: bfv.Ctx, shape, x, cfg, client, variant, layer, first, last, b) -> Dict:
    N, t = ctx.N, ctx.t
    g = packing.fc_geometry(N, shape.n_i, shape.n_o)
    W = wl.layer_weights(cfg, variant, layer, shape)
    B = wl.layer_bias(cfg, variant, layer, shape)
    rho = wl.uniform_below(wl.rng(cfg, 0, variant, layer, "rho"), (g.blocks, N), t)
    sh = None if first else wl.uniform_below(wl.rng(cfg, client, variant, layer, "sh"), (N,), t)
    shn = None if last else wl.uniform_below(wl.rng(cfg, client, variant, layer, "shnext"), (g.blocks, g.n_o_p), t)
    xp = packing.pack_fc_input(x, g)
    ip = xp % t if sh is None else (xp + sh) % t
    v = wl.encryption_v(wl.rng(cfg, client, variant, layer, "v", 0), N)
    e0 = wl.gaussian(wl.rng(cfg, client, variant, layer, "e0", 0), N)
    c0 = bfv.encrypt_c0(ctx, ip, v, e0, b)
    return dict(geom=g, W=W, bias=B, rho=rho, w=packing.pack_fc_weights(W, g), d=packing.pack_fc_bias(B, g),
                sh=sh, sh_next=shn, c0=c0, v=v, i_poly=ip)


def plain20_layer_inputs(width: int, classes: int, cfg: int, client: int):
    """(layers, weights, biases, true inputs, integer outputs) of the plain-20 stack on one image."""
    layers = wl.plain20(width, classes)
    Ws = [wl.layer_weights(cfg, width, k, s) for k, s in enumerate(layers)]
    Bs = [wl.layer_bias(cfg, width, k, s) for k, s in enumerate(layers)]
    img = wl.image(cfg, client, width)
    outs, ins = network.plaintext_forward(img, layers, Ws, Bs)
    return layers, Ws, Bs, ins, outs


# Full-size cases: (name, config, width, classes, N, L, layer indices or None for all)
PLAIN20_X1 = ("plain20_x1", wl.CONFIG_PLAIN20_X1, 1, 10, 8192, 4, None)
# one layer per distinct tiling of the wider variants (stage entry, stride-2, stage body, FC)
WIDE_SAMPLES = [
    ("plain20_x2", wl.CONFIG_BATCHED, 2, 10, 8192, 4, [0, 1, 7, 8, 13, 14, 19]),
    ("plain20_x2_c100", wl.CONFIG_BATCHED, 2, 100, 8192, 4, [19]),
    ("plain20_x4", wl.CONFIG_STRESS, 4, 100, 16384, 6, [0, 7, 13, 14, 19]),
]

# Batched full-size layers: (name, config, width, classes, N, L, layer, batch, sampled images).
# The GPU runs the whole batch; the oracle digests of the sampled images are stored.
BATCHED_SAMPLES = [
    ("batched_x1_l7", wl.CONFIG_BATCHED, 1, 10, 8192, 4, 7, 64, [5, 60]),
    ("batched_x2_l1", wl.CONFIG_BATCHED, 2, 10, 8192, 4, 1, 64, [3, 62]),
    ("batched_x4_l1", wl.CONFIG_BATCHED, 4, 100, 16384, 6, 1, 64, [0, 45]),
]


def batched_layer_inputs(cfg, width, classes, k, B, N, primes):
    """Server inputs of conv layer k of a plain-20 width variant for a batch of B images, drawn as
    the batched benchmark draws them: c0 uniform per limb, shares uniform in [0, t)."""
    shp = wl.plain20(width, classes)[k]
    g = packing.conv_geometry(N, shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
    L = len(primes)
    F = wl.layer_weights(cfg, width, k, shp)
    rho = wl.mask_polys(cfg, width, k, g.K_in * shp.c_o, N).reshape(g.K_in, shp.c_o, N)
    c0 = wl.ciphertext_polys(cfg, 0, width, k, B * g.K_in, primes, N).reshape(B, g.K_in, L, N)
    sh = wl.share_polys(cfg, 0, width, k, B * g.K_in, N).reshape(B, g.K_in, N)
    shn = wl.share_polys(cfg, 0, width, k, B * g.K_out, N, "shnext").reshape(B, g.K_out, N)
    return {"shape": shp, "geom": g, "F": F, "rho": rho, "c0": c0, "sh": sh, "sh_next": shn}

# ResNet-50-shaped layers at N = 16384, L = 6 (one image): (name, layer index in
# workloads.resnet50_body()); the stride-2 1x1 projection of stage 2 packed on the subsampled
# 28x28 map (256 -> 512), a 3x3 at 28x28 (s = 16), a 1x1 expansion at 14x14 (s = 64) and a 3x3
# at 7x7 (s = 128).
RESNET_SAMPLES = [("resnet50_l13", 13), ("resnet50_l15", 15), ("resnet50_l29", 29), ("resnet50_l47", 47)]


def resnet_layer_inputs(k, N, primes):
    """Server inputs of ResNet-50 body layer k for one image: c0 uniform per limb, shares
    uniform in [0, t)."""
    cfg = wl.CONFIG_RESNET50
    shp = wl.resnet50_body()[k]
    g = packing.conv_geometry(N, shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
    F = wl.layer_weights(cfg, 0, k, shp)
    rho = wl.mask_polys(cfg, 0, k, g.K_in * shp.c_o, N).reshape(g.K_in, shp.c_o, N)
    c0 = wl.ciphertext_polys(cfg, 0, 0, k, g.K_in, primes, N)
    sh = wl.share_polys(cfg, 0, 0, k, g.K_in, N)
    shn = wl.share_polys(cfg, 0, 0, k, g.K_out, N, "shnext")
    return {"shape": shp, "geom": g, "F": F, "rho": rho, "c0": c0, "sh": sh, "sh_next": shn}
