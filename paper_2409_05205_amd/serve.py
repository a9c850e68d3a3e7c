"""Served form: many clients streaming single-layer requests to one GPU.

Builds the packed plain-20 variants (the server's resident NTT-domain operands),
per-client resident ciphertext buffers for every layer, a Poisson arrival trace
in which each request names a uniformly random client and layer type, and
replays it through the native continuous-batching server (he_server_*).  The
same trace replayed with one stream and batch 1 is the plain first-come
first-served one-request-per-launch server it is compared against.

Per-client inputs are synthetic: c0 shares uniform per limb (what RLWE
ciphertexts look like to the server), shares uniform in [0, t), drawn on the
device from a seeded generator per (variant, layer).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

import workloads as wl

from . import he


@dataclass
class Variant:
    """One packed plain-20 width variant on its own ring."""
    width: int
    classes: int
    ctx: "he.Context"
    shapes: List[object]
    layers: List["he.Layer"] = field(default_factory=list)


def pack_variant(width: int, classes: int, ctx: "he.Context", cfg: int = wl.CONFIG_SERVED) -> Variant:
    v = Variant(width, classes, ctx, wl.plain20(width, classes))
    N = ctx.N
    for k, shp in enumerate(v.shapes):
        W = wl.layer_weights(cfg, width, k, shp)
        if shp.kind == "conv":
            spec = he.ConvSpec(shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
            K_in = ctx.geometry(spec).K_in
            rho = wl.mask_polys(cfg, width, k, K_in * shp.c_o, N).reshape(K_in, shp.c_o, N)
            v.layers.append(ctx.pack_conv(spec, W, rho))
        else:
            spec = he.FCSpec(shp.n_i, shp.n_o)
            rho = wl.mask_polys(cfg, width, k, ctx.geometry(spec).blocks, N)
            v.layers.append(ctx.pack_fc(spec, W, rho, wl.layer_bias(cfg, width, k, shp)))
    return v


def _uniform_limbs(shape_lead, primes, N, gen, device):
    import torch
    L = len(primes)
    out = torch.empty(tuple(shape_lead) + (L, N), dtype=torch.int32, device=device)
    for l, q in enumerate(primes):
        out[..., l, :] = torch.randint(0, int(q), tuple(shape_lead) + (N,), generator=gen, device=device,
                                       dtype=torch.int32)
    return out


@dataclass
class LayerBuffers:
    c0: object
    sh: Optional[object]
    shn: Optional[object]
    out: object


def client_buffers(v: Variant, clients: int, seed: int, device="cuda:0") -> List[LayerBuffers]:
    """Resident per-client inputs and outputs of every layer of a variant: tensors [clients][...]."""
    import torch
    bufs = []
    ctx = v.ctx
    N, L, t = ctx.N, ctx.L, ctx.t
    for k, (shp, ly) in enumerate(zip(v.shapes, v.layers)):
        g = torch.Generator(device=device)
        g.manual_seed(seed * 1000003 + v.width * 101 + k)
        first, last = k == 0, k == len(v.shapes) - 1
        i = ly.info
        if shp.kind == "conv":
            c0 = _uniform_limbs((clients, i.K_in), ctx.primes, N, g, device)
            sh = None if first else torch.randint(0, t, (clients, i.K_in, N), generator=g, device=device,
                                                 dtype=torch.int32)
            shn = None if last else torch.randint(0, t, (clients, i.K_out, N), generator=g, device=device,
                                                 dtype=torch.int32)
            out = torch.empty((clients, i.K_out, L, N), dtype=torch.int32, device=device)
        else:
            c0 = _uniform_limbs((clients,), ctx.primes, N, g, device)
            sh = torch.randint(0, t, (clients, N), generator=g, device=device, dtype=torch.int32)
            shn = None if last else torch.randint(0, t, (clients, i.blocks, i.n_o_p), generator=g, device=device,
                                                 dtype=torch.int32)
            out = torch.empty((clients, i.blocks, L, i.n_o_p), dtype=torch.int32, device=device)
        bufs.append(LayerBuffers(c0, sh, shn, out))
    return bufs


def poisson_trace(rate: float, n: int, layer_types: int, clients: int, seed: int):
    """Arrival times (s), layer-type index and client index of n requests."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([wl.MASTER_SEED, wl.CONFIG_SERVED, seed])))
    gaps = rng.exponential(1.0 / rate, n)
    arrival = np.cumsum(gaps) - gaps[0]
    return arrival, rng.integers(0, layer_types, n), rng.integers(0, clients, n)


def run_trace(variants: List[Variant], buffers: List[List[LayerBuffers]], arrival, ltype, client,
              streams: int, max_batch: int, budget: int, timeout_s: float = 0.0):
    """Replay a trace through he_server; returns the server's per-request results and the type table."""
    srv = he.Server(streams, max_batch, budget, timeout_s)
    table = []      # layer-type index -> (variant index, layer index, server layer id)
    for vi, v in enumerate(variants):
        for k, ly in enumerate(v.layers):
            table.append((vi, k, srv.add_layer(v.ctx, ly)))
    for a, lt, cl in zip(arrival, ltype, client):
        vi, k, lid = table[int(lt)]
        b = buffers[vi][k]
        srv.add_request(lid, float(a), b.c0[cl], None if b.sh is None else b.sh[cl],
                        None if b.shn is None else b.shn[cl], b.out[cl])
    rc = srv.run()
    res = srv.results()
    srv.free()
    res["rc"] = rc
    return res


def latency_stats(res, warmup: int):
    """Latency percentiles and throughput over the requests after `warmup` that succeeded; a failed
    request (e.g. rejected for memory at dispatch) completes at once and would flatter both."""
    ok = res["status"][warmup:] == 0
    lat = (res["complete"] - res["arrival"])[warmup:][ok]
    a = res["arrival"][warmup:]
    c = res["complete"][warmup:][ok]
    span = c.max() - a.min() if len(c) else float("nan")
    return {
        "requests": int(len(ok)),
        "failed": int((~ok).sum()),
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
        "mean_ms": float(lat.mean() * 1e3) if len(lat) else None,
        "layers_per_s": float(len(lat) / span) if len(lat) else 0.0,
        "mean_batch": float(res["batch"][warmup:].mean()),
    }


def run_clients(variant: Variant, buffers: List[LayerBuffers], clients: int, streams: int, max_batch: int,
                budget: int, start_gap: float = 0.0, timeout_s: float = 0.0):
    """Every client streams the whole stack: layer k of a client is issued when its layer k-1
    returns (he_server request dependencies).  Clients start start_gap seconds apart.
    Returns per-request results plus the request table [client][layer] -> index."""
    srv = he.Server(streams, max_batch, budget, timeout_s)
    lids = [srv.add_layer(variant.ctx, ly) for ly in variant.layers]
    n_layers = len(variant.layers)
    index = np.zeros((clients, n_layers), dtype=np.int64)
    idx = 0
    # independent first layers in arrival order, then the dependent chain of each client
    for cl in range(clients):
        b = buffers[0]
        srv.add_request_after(lids[0], cl * start_gap, -1, b.c0[cl], None if b.sh is None else b.sh[cl],
                              None if b.shn is None else b.shn[cl], b.out[cl])
        index[cl, 0] = idx
        idx += 1
    for k in range(1, n_layers):
        b = buffers[k]
        for cl in range(clients):
            srv.add_request_after(lids[k], 0.0, int(index[cl, k - 1]), b.c0[cl],
                                  None if b.sh is None else b.sh[cl], None if b.shn is None else b.shn[cl],
                                  b.out[cl])
            index[cl, k] = idx
            idx += 1
    rc = srv.run()
    res = srv.results()
    srv.free()
    res["rc"] = rc
    res["index"] = index
    return res


def client_stats(res):
    """Per-inference latency (first layer issued to last layer returned) and throughput."""
    index = res["index"]
    ok_req = res["status"] == 0
    # an inference counts only when every one of its layers succeeded (a failure fails its dependants)
    ok_inf = ok_req[index].all(axis=1)
    start = res["arrival"][index[ok_inf, 0]]
    end = res["complete"][index[ok_inf, -1]]
    inf = end - start
    lat = (res["complete"] - res["arrival"])[ok_req]
    span = res["complete"][ok_req].max() - res["arrival"].min() if ok_req.any() else float("nan")
    return {
        "clients": int(index.shape[0]),
        "requests": int(index.size),
        "failed": int((~ok_req).sum()),
        "inference_p50_ms": float(np.percentile(inf, 50) * 1e3) if len(inf) else None,
        "inference_p99_ms": float(np.percentile(inf, 99) * 1e3) if len(inf) else None,
        "layer_p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
        "layer_p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
        "layers_per_s": float(ok_req.sum() / span) if ok_req.any() else 0.0,
        "mean_batch": float(res["batch"].mean()),
    }
