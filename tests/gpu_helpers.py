"""Helpers for the GPU tests: device transfer and GPU-backed server callbacks."""
from __future__ import annotations

import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.int32))).to("cuda:0")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.int64).astype(np.uint64)


def gpu_conv(ctx, geom, F, rho, c0, sh, sh_next, flags=0):
    """One image through he_pack_filters + he_conv_layer; returns c0^r [K_out][L][N]."""
    from paper_2409_05205_amd import he
    spec = he.ConvSpec(geom.c_i, geom.c_o, geom.H, geom.W, geom.f, geom.stride, geom.pad)
    layer = ctx.pack_conv(spec, F, rho, flags)
    out = ctx.conv_layer(layer, dev(np.asarray(c0)[None]), None if sh is None else dev(np.asarray(sh)[None]),
                         None if sh_next is None else dev(np.asarray(sh_next)[None]))
    return host(out)[0]


def gpu_fc(ctx, geom, W, bias, rho, c0, sh, sh_next):
    from paper_2409_05205_amd import he
    layer = ctx.pack_fc(he.FCSpec(geom.n_i, geom.n_o), W, rho, bias)
    out = ctx.fc_layer(layer, dev(np.asarray(c0)[None]), None if sh is None else dev(np.asarray(sh)[None]),
                       None if sh_next is None else dev(np.asarray(sh_next)[None]))
    return host(out)[0]
