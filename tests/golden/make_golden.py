"""Write tests/golden/server_digests.json from the CPU oracle only.

For every full-size case in cases.py this script runs the oracle's server
evaluation (Alg. 1 / Alg. 2, exact reading) on the seeded inputs and stores the
SHA-256 of c0^r as little-endian u32 words (for the batched layers, of the
sampled images of the batch).  For the x1 plain-20 stack and the
single-conv workload it also runs the oracle client (masks p1/p2, client
evaluation, decryption) and asserts that every decrypted output minus the fresh
share equals the integer layer output mod t, i.e. that the closed loop of the
harness holds.  Nothing here touches the GPU library.

Usage: python tests/golden/make_golden.py [--only NAME ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import cases  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import bfv, network, packing  # noqa: E402


def check_conv_decrypt(ctx, cfg, variant, k, inp, out, ref, b):
    g = inp["geom"]
    e1 = wl.gaussian(wl.rng(cfg, 0, variant, k, "e1"), (g.K_in, g.c_o, ctx.N))
    e2 = wl.gaussian(wl.rng(cfg, 0, variant, k, "e2"), (g.K_in, g.c_o, ctx.N))
    p1, p2 = bfv.client_masks(ctx, inp["rho"], inp["fhat"], b, e1, e2)
    c1r = bfv.client_conv(ctx, g, inp["v"], inp["i_polys"], p1, p2)
    r = bfv.decrypt(ctx, bfv.add_shares(ctx, out, c1r))
    if inp["sh_next"] is not None:
        r = (r - inp["sh_next"]) % ctx.t
    dec = network.centred(packing.decode_conv_output(r, g), ctx.t)
    assert (dec == ref).all(), f"conv layer {k}: decryption does not match the integer conv"


def check_fc_decrypt(ctx, cfg, variant, k, inp, out, ref, b):
    g = inp["geom"]
    e1 = wl.gaussian(wl.rng(cfg, 0, variant, k, "e1"), (g.blocks, ctx.N))
    e2 = wl.gaussian(wl.rng(cfg, 0, variant, k, "e2"), (g.blocks, ctx.N))
    p1, p2 = bfv.client_masks(ctx, inp["rho"], inp["w"], b, e1, e2)
    c1r = bfv.client_fc(ctx, g, inp["v"], inp["i_poly"], p1, p2)
    r = bfv.decrypt(ctx, bfv.add_shares(ctx, out, c1r))
    if inp["sh_next"] is not None:
        r = (r - inp["sh_next"]) % ctx.t
    dec = network.centred(packing.decode_fc_output(r, g), ctx.t)
    assert (dec == ref).all(), f"fc layer {k}: decryption does not match the integer FC"


def run_stack(name, cfg, width, classes, N, L, idx, decrypt):
    ctx = bfv.make_ctx(N, L, wl.T_PLAIN)
    _, b = cases.client_key(ctx, cfg, 0)
    layers, Ws, Bs, ins, outs = cases.plain20_layer_inputs(width, classes, cfg, 0)
    idx = list(range(len(layers))) if idx is None else idx
    res = {"config": cfg, "width": width, "classes": classes, "N": N, "L": L, "layers": {}}
    for k in idx:
        shp = layers[k]
        first, last = k == 0, k == len(layers) - 1
        t0 = time.time()
        if shp.kind == "conv":
            inp = cases.conv_inputs(ctx, shp, ins[k], cfg, 0, width, k, first, last, b)
            out = bfv.server_conv(ctx, inp["geom"], inp["c0"], inp["rho"], inp["fhat"], inp["sh"], inp["sh_next"])
            if decrypt:
                check_conv_decrypt(ctx, cfg, width, k, inp, out, outs[k], b)
        else:
            inp = cases.fc_inputs(ctx, shp, ins[k], cfg, 0, width, k, first, last, b)
            out = bfv.server_fc(ctx, inp["geom"], inp["c0"], inp["rho"], inp["w"], inp["d"], inp["sh"],
                                inp["sh_next"])
            if decrypt:
                check_fc_decrypt(ctx, cfg, width, k, inp, out, outs[k], b)
        res["layers"][str(k)] = {"kind": shp.kind, "digest": cases.digest(out), "shape": list(out.shape)}
        print(f"{name} layer {k} {shp} {time.time() - t0:.1f}s", flush=True)
    return res


def case_single_conv():
    # single conv workload: conv 3->16 on 3x32x32, N=4096, L=3, first layer with a fresh share
    ctx = bfv.make_ctx(4096, 3, wl.T_PLAIN)
    _, b = cases.client_key(ctx, wl.CONFIG_SINGLE_CONV, 0)
    shp = wl.single_conv_layer()
    x = wl.image(wl.CONFIG_SINGLE_CONV, 0)
    inp = cases.conv_inputs(ctx, shp, x, wl.CONFIG_SINGLE_CONV, 0, 0, 0, True, False, b)
    o = bfv.server_conv(ctx, inp["geom"], inp["c0"], inp["rho"], inp["fhat"], inp["sh"], inp["sh_next"])
    F = wl.layer_weights(wl.CONFIG_SINGLE_CONV, 0, 0, shp)
    check_conv_decrypt(ctx, wl.CONFIG_SINGLE_CONV, 0, 0, inp, o, network.conv2d(x, F), b)
    return {"config": 1, "N": 4096, "L": 3,
            "layers": {"0": {"kind": "conv", "digest": cases.digest(o), "shape": list(o.shape)}}}


def case_batched(name, cfg, width, classes, N, L, k, B, images):
    ctx = bfv.make_ctx(N, L, wl.T_PLAIN)
    inp = cases.batched_layer_inputs(cfg, width, classes, k, B, N, ctx.primes)
    g = inp["geom"]
    fh = packing.pack_conv_filters(inp["F"], g)
    res = {"config": cfg, "width": width, "classes": classes, "N": N, "L": L, "layer": k, "batch": B,
           "images": {}}
    for b in images:
        t0 = time.time()
        o = bfv.server_conv(ctx, g, inp["c0"][b].astype(np.uint64), inp["rho"], fh, inp["sh"][b],
                            inp["sh_next"][b])
        res["images"][str(b)] = cases.digest(o)
        print(f"{name} image {b} {time.time() - t0:.1f}s", flush=True)
    return res


def case_resnet(name, k):
    ctx = bfv.make_ctx(16384, 6, wl.T_PLAIN)
    t0 = time.time()
    inp = cases.resnet_layer_inputs(k, 16384, ctx.primes)
    g = inp["geom"]
    o = bfv.server_conv(ctx, g, inp["c0"].astype(np.uint64), inp["rho"], packing.pack_conv_filters(inp["F"], g),
                        inp["sh"], inp["sh_next"])
    print(f"{name} {inp['shape']} {time.time() - t0:.1f}s", flush=True)
    return {"config": wl.CONFIG_RESNET50, "N": 16384, "L": 6, "layer": k,
            "layers": {str(k): {"kind": "conv", "digest": cases.digest(o), "shape": list(o.shape)}}}


def all_cases():
    """name -> function computing the case's record."""
    out = {"single_conv": case_single_conv}
    name, cfg, width, classes, N, L, idx = cases.PLAIN20_X1
    out[name] = lambda a=(name, cfg, width, classes, N, L, idx): run_stack(*a, decrypt=True)
    for name, cfg, width, classes, N, L, idx in cases.WIDE_SAMPLES:
        out[name] = lambda a=(name, cfg, width, classes, N, L, idx): run_stack(*a, decrypt=False)
    for c in cases.BATCHED_SAMPLES:
        out[c[0]] = lambda c=c: case_batched(*c)
    for name, k in cases.RESNET_SAMPLES:
        out[name] = lambda a=(name, k): case_resnet(*a)
    return out


def main(argv):
    """Every case, or with --only NAME [NAME ...] just those, merged into the stored file."""
    path = os.path.join(HERE, "server_digests.json")
    table = all_cases()
    if argv[:1] == ["--only"]:
        names = argv[1:]
        unknown = [n for n in names if n not in table]
        if unknown:
            raise SystemExit(f"unknown cases: {unknown}")
        with open(path) as f:
            out = json.load(f)
    else:
        names = list(table)
        out = {"note": "SHA-256 of the oracle's c0^r (little-endian u32) per layer; written by make_golden.py",
               "cases": {}}
    for n in names:
        out["cases"][n] = table[n]()
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote server_digests.json")


if __name__ == "__main__":
    main(sys.argv[1:])
