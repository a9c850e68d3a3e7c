#!/usr/bin/env python
"""Benchmark of the rotation-free HE Conv/FC server path on one MI355X.

Workload (the `value` line): the full plain-20 x1 linear stack (19 convs + FC
64->10), ring degree N = 8192 with 4 limbs of 30-bit primes, t = 786433, one
image per layer call.  A step is one image through all 20 server layers (the
whole hot path: forward NTTs, coefficient-wise MAC, residue-class inverse
transform and extraction).  Inputs are synthetic and resident in HBM before
timing: c0 shares uniform per limb (indistinguishable from real encryptions),
shares uniform in [0, t), uint4-activation-shaped layers, weights in [-7, 7].

Forms reported beside the value:
  plain_host  one he_*_layer call per layer from Python, synchronising after each
  plain       one image, the 20 layer calls issued back to back by the native runtime
  graph       the same 20 calls captured once into a HIP graph, one replay per image
  batched     64 images through the x1, x2 (N = 8192, 4 limbs) and x4 (N = 16384,
              6 limbs) stacks, heads of 10 and 100 classes, graph replay per variant

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batched] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

HBM_PEAK_GBS = 8000.0
CUS, CLOCK_GHZ = 256, 2.4
# Integer-ALU roofs (whole chip, G operations per second): he_probe_rate (csrc/kernels_probe.hip)
# on an MI355X, the figures of profiles/alu_rates_MI355X.md; a run replaces them with its own
# measurement unless --no-rates.  A Shoup butterfly is 9 vector instructions (1 mul_hi, 2 mul_lo,
# 6 add / sub / min); the MAC's inner product is one v_mad_u64_u32 per product.
BFLY_PEAK_G = 4084.5
GSBFLY_PEAK_G = 4368.0
MAD64_PEAK_G = 32825.4
# the matrix cores' published dense int8 rate (T operations per second, 2 per multiply-add)
INT8_PEAK_T = 5000.0


def alu_rates(he):
    """Measured integer-ALU rates of the chip (he_probe_rate), as G ops/s and per CU-clock."""
    out = {}
    for name, kind in [("butterfly_ct", he.HE_PROBE_BFLY), ("butterfly_gs", he.HE_PROBE_GSBFLY),
                       ("mad_u64_u32", he.HE_PROBE_MAD64), ("add_u32", he.HE_PROBE_ADD),
                       ("mul_lo_u32", he.HE_PROBE_MULLO), ("mul_hi_u32", he.HE_PROBE_MULHI)]:
        ops, ms = he.probe_rate(kind, 8192)
        out[name] = {"G_per_s": round(ops / 1e9, 1), "per_CU_clock": round(ops / (CUS * CLOCK_GHZ * 1e9), 3),
                     "ms": round(ms, 3)}
    return out
# HBM traffic per launch from the FETCH_SIZE / WRITE_SIZE counter runs (calibrated on a 256 MiB
# copy: FETCH_SIZE x 2, WRITE_SIZE x 1), valid while the kernel source is the one that was measured.
PMC_TRAFFIC = {
    # the launch that carries each layer's MAC, per layer of the stack with every layer pinned to each
    # form in turn: k_mac_tail (F, fused MAC and inverse), k_mac_class / k_mac_full (S, split), and
    # the whole layer in one launch, k_fused_layer (O) or k_fused_rows (R; the FC head runs O).  Each
    # form is valid while the sources of its kernels are the ones that were measured
    # (profiles/pmc_traffic_plain20_x1_N8192_L4_per_layer.md).
    "layers": {
        "forms": {
            "F": {"sources": ['paper_2409_05205_amd/csrc/kernels_ntt.hip', 'paper_2409_05205_amd/csrc/ntt_device.h', 'paper_2409_05205_amd/csrc/he_device.h', 'paper_2409_05205_amd/csrc/he_kernels.h'],
                  "sha256": "8d1ea5ef077d446825896ff12ca053fd17508c6d584bab342ab22c7bc30a3008"},
            "S": {"sources": ['paper_2409_05205_amd/csrc/kernels_mac.hip', 'paper_2409_05205_amd/csrc/mac_device.h', 'paper_2409_05205_amd/csrc/he_device.h', 'paper_2409_05205_amd/csrc/he_kernels.h'],
                  "sha256": "a7faeb2207bf7d8972ef6a84f4dce52fd05e94139fd72f17b001672f5dfcbb0c"},
            "O": {"sources": ['paper_2409_05205_amd/csrc/kernels_fused.hip', 'paper_2409_05205_amd/csrc/mac_device.h', 'paper_2409_05205_amd/csrc/ntt_device.h', 'paper_2409_05205_amd/csrc/he_device.h', 'paper_2409_05205_amd/csrc/he_kernels.h'],
                  "sha256": "645ce1a77c03a9d6853cd08c333e990aea30effd7100a5746eaf85749a3bdfb6"},
            "R": {"sources": ['paper_2409_05205_amd/csrc/kernels_fused.hip', 'paper_2409_05205_amd/csrc/mac_device.h', 'paper_2409_05205_amd/csrc/ntt_device.h', 'paper_2409_05205_amd/csrc/he_device.h', 'paper_2409_05205_amd/csrc/he_kernels.h'],
                  "sha256": "645ce1a77c03a9d6853cd08c333e990aea30effd7100a5746eaf85749a3bdfb6"},
        },
        "per_layer": [
            {"F": 4734832, "S": 2794366, "O": 8171361, "R": 5412329},
            {"F": 21246894, "S": 18389014, "O": 27299716, "R": 24147928},
            {"F": 21246693, "S": 18389014, "O": 27304469, "R": 24146264},
            {"F": 21246657, "S": 18389014, "O": 27301124, "R": 24146173},
            {"F": 21246492, "S": 18389014, "O": 27299021, "R": 24146191},
            {"F": 21246565, "S": 18389069, "O": 27301763, "R": 24146721},
            {"F": 21246492, "S": 18389014, "O": 27302513, "R": 24146228},
            {"F": 40117782, "S": 35688643, "O": 48298221, "R": 43046101},
            {"F": 19031735, "S": 17602847, "O": 22431035, "R": 20820773},
            {"F": 19031204, "S": 17602646, "O": 22431638, "R": 20820627},
            {"F": 19031332, "S": 17602792, "O": 22431967, "R": 20820773},
            {"F": 19031460, "S": 17602646, "O": 22430632, "R": 20820773},
            {"F": 19031479, "S": 17602646, "O": 22430523, "R": 20820810},
            {"F": 36854486, "S": 34641026, "O": 41334202, "R": 38794379},
            {"F": 17956058, "S": 17209462, "O": 19849457, "R": 19257527},
            {"F": 17956003, "S": 17209462, "O": 19850371, "R": 19257454},
            {"F": 17956039, "S": 17209462, "O": 19852748, "R": 19262811},
            {"F": 17956167, "S": 17209608, "O": 19849859, "R": 19261823},
            {"F": 17956039, "S": 17209315, "O": 19852620, "R": 19257472},
            {"F": None, "S": 704442, "O": 2251866, "R": 2253143},
        ]},
    "ntt_fwd": {"sources": ['paper_2409_05205_amd/csrc/kernels_ntt.hip', 'paper_2409_05205_amd/csrc/ntt_device.h', 'paper_2409_05205_amd/csrc/he_device.h'],
                "sha256": "c280e448cab85526766aa78838073e79e0eb9474054d251a16fa52e20c135e11",
                "bytes_per_launch": 2834205},
}


def pmc_traffic(kind, plan=None, only=None):
    """Counter-measured HBM bytes per launch, or None once a measured source has changed.  For a
    per-layer table, `plan` gives the form of each layer (O / R one launch, F fused, S split: the
    launch that carries the MAC) and the result is the mean over the layers `only` selects (all
    by default); None if a selected layer ran in a form the table has no entry for."""
    import hashlib

    def fresh(r):
        h = hashlib.sha256()
        for src in r["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        return h.hexdigest() == r["sha256"]

    rec = PMC_TRAFFIC.get(kind)
    if rec is None:
        return None
    if "per_layer" not in rec:
        return rec["bytes_per_launch"] if fresh(rec) else None
    table = rec["per_layer"]
    if plan is None or len(plan) != len(table):
        return None
    sel = [k for k in range(len(table)) if only is None or only[k]]
    if not sel or any(table[k].get(plan[k]) is None for k in sel):
        return None
    if not all(fresh(rec["forms"][c]) for c in {plan[k] for k in sel}):
        return None
    return round(sum(table[k][plan[k]] for k in sel) / len(sel))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ stack setup
class Stack:
    """Packed layers and resident per-image inputs of one plain-20 variant."""

    def __init__(self, he, ctx, cfg, width, classes_list, B_list, N, L):
        import torch
        self.ctx = ctx
        self.layers_shape = wl.plain20(width, classes_list[0])
        self.layers = []
        self.steps = []          # (layer, B, c0, sh, sh_next)
        self.rows = []           # output channels (conv) or row blocks (fc) per step
        dev = torch.device("cuda:0")
        t = ctx.t
        for k, shp in enumerate(self.layers_shape):
            first, last = k == 0, k == len(self.layers_shape) - 1
            if shp.kind == "conv":
                spec = he.ConvSpec(shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
                til = ctx.geometry(spec)
                W = wl.layer_weights(cfg, width, k, shp)
                rho = wl.mask_polys(cfg, width, k, til.K_in * shp.c_o, N).reshape(til.K_in, shp.c_o, N)
                ly = ctx.pack_conv(spec, W, rho)
                self.layers.append(ly)
                B = sum(B_list)
                c0 = torch.from_numpy(wl.ciphertext_polys(cfg, 0, width, k, B * til.K_in, ctx.primes, N)
                                      .reshape(B, til.K_in, L, N).astype(np.int32)).to(dev)
                sh = None if first else torch.from_numpy(
                    wl.share_polys(cfg, 0, width, k, B * til.K_in, N).reshape(B, til.K_in, N)
                    .astype(np.int32)).to(dev)
                shn = None if last else torch.from_numpy(
                    wl.share_polys(cfg, 0, width, k, B * til.K_out, N, "shnext").reshape(B, til.K_out, N)
                    .astype(np.int32)).to(dev)
                self.steps.append((ly, B, c0, sh, shn))
                self.rows.append(shp.c_o)
            else:
                for h, (classes, B) in enumerate(zip(classes_list, B_list)):
                    fshp = wl.FCShape(shp.n_i, classes)
                    W = wl.layer_weights(cfg, width * 10 + h, k, fshp)
                    bias = wl.layer_bias(cfg, width * 10 + h, k, fshp)
                    fspec = he.FCSpec(shp.n_i, classes)
                    blocks = ctx.geometry(fspec).blocks
                    rho = wl.mask_polys(cfg, width * 10 + h, k, blocks, N)
                    ly = ctx.pack_fc(fspec, W, rho, bias)
                    self.layers.append(ly)
                    c0 = torch.from_numpy(wl.ciphertext_polys(cfg, 0, width * 10 + h, k, B, ctx.primes, N)
                                          .astype(np.int32)).to(dev)
                    sh = torch.from_numpy(wl.share_polys(cfg, 0, width * 10 + h, k, B, N).astype(np.int32)).to(dev)
                    self.steps.append((ly, B, c0, sh, None))
                    self.rows.append(blocks)
        self.seq = he.Sequence(ctx)
        for ly, B, c0, sh, shn in self.steps:
            self.seq.add(ly, c0, sh, shn)

    def autotune(self):
        """Time every kernel variant on each layer's launch shapes; keep the fastest."""
        for ly, B, c0, sh, shn in self.steps:
            self.ctx.autotune(ly, B)

    def image_layers(self):
        """Image-layer evaluations per pass (conv layers count B images, FC heads their B)."""
        return sum(B for _, B, _, _, _ in self.steps)

    def mac_plan(self, he):
        """Which launch carries each layer's MAC: 'one' / 'rows' (the whole layer in one launch:
        work items of sub-blocks, chunks and tails / one MAC + inverse item per output row), 'fused'
        (MAC + residue-class tail in one launch, after a forward-transform launch), 'split' (MAC
        launch, then tail / inverse launch) or 'mfma' (the same with the MAC on the matrix cores),
        read from the kernel kinds one call of the layer records."""
        plan = []
        kinds = he.HE_K_MAC | he.HE_K_MAC_TAIL | he.HE_K_LAYER | he.HE_K_LAYER_ROWS | he.HE_K_MAC_MFMA
        for ly, B, c0, sh, shn in self.steps:
            self.ctx.profile_reset()
            self.ctx.profile_enable(kinds)
            if ly.kind == he.HE_LAYER_CONV:
                self.ctx.conv_layer(ly, c0, sh, shn)
            else:
                self.ctx.fc_layer(ly, c0, sh, shn)
            one = self.ctx.profile_read(he.HE_K_LAYER)[0] > 0
            rows = self.ctx.profile_read(he.HE_K_LAYER_ROWS)[0] > 0
            fused = self.ctx.profile_read(he.HE_K_MAC_TAIL)[0] > 0
            mfma = self.ctx.profile_read(he.HE_K_MAC_MFMA)[0] > 0
            self.ctx.profile_enable(0)
            plan.append("one" if one else ("rows" if rows else ("fused" if fused else ("mfma" if mfma else "split"))))
        self.ctx.profile_reset()
        return plan

    def mac_kernel_bytes(self, plan, only=None):
        """Algorithmic bytes of the launches that carry the MAC in one pass: resident operand
        rows once, NTT-domain inputs once per image, and what the launch writes (block sums or
        products for a split MAC; output polynomials, after reading sh', for a fused one)."""
        tot = 0
        L, N = self.ctx.L, self.ctx.N
        for k, ((ly, B, c0, sh, shn), c_o, form) in enumerate(zip(self.steps, self.rows, plan)):
            if only is not None and not only[k]:
                continue
            i = ly.info
            J = i.K_in * (2 if sh is not None else 1)
            tot += J * c_o * L * N * 4 + B * J * L * N * 4
            if form == "fused":
                tot += B * i.K_out * L * N * 4 + (B * i.K_out * N * 4 if shn is not None else 0)
            else:
                out_per = N // i.s if ly.kind == 0 and i.flags == 0 else N
                tot += B * c_o * L * out_per * 4
        return tot

    def layer_bytes(self, only=None):
        """Algorithmic HBM bytes of one pass of whole layer calls: c0, sh and sh' read, the resident
        operand rows read once, the output polynomials (FC: their n_o' kept coefficients) written."""
        L, N = self.ctx.L, self.ctx.N
        tot = 0
        for k, ((ly, B, c0, sh, shn), rows) in enumerate(zip(self.steps, self.rows)):
            if only is not None and not only[k]:
                continue
            i = ly.info
            J = i.K_in * (2 if sh is not None else 1)
            tot += J * rows * L * N * 4 + B * i.K_in * L * N * 4
            if sh is not None:
                tot += B * i.K_in * N * 4
            if ly.kind == 0:
                tot += B * i.K_out * L * N * 4 + (B * i.K_out * N * 4 if shn is not None else 0)
            else:
                tot += B * rows * L * i.n_o_p * 4 + (B * rows * i.n_o_p * 4 if shn is not None else 0)
        return tot

    def fwd_bytes(self, only=None):
        """Algorithmic HBM bytes of one pass's forward transforms: each c0 row read and written per
        limb; each sh row read once and written for every limb."""
        L, N = self.ctx.L, self.ctx.N
        tot = 0
        for k, (ly, B, c0, sh, shn) in enumerate(self.steps):
            if only is not None and not only[k]:
                continue
            rows = B * ly.info.K_in
            tot += rows * L * N * 8
            if sh is not None:
                tot += rows * N * 4 + rows * L * N * 4
        return tot

    def inverse_bytes(self, only=None):
        """Algorithmic HBM bytes of one pass's inverse launches: the MAC output read (block sums
        of every channel, or full rows for FC and full-form conv), sh' read once per output
        polynomial, the output polynomials (FC: their n_o' kept coefficients) written."""
        L, N = self.ctx.L, self.ctx.N
        tot = 0
        for k, ((ly, B, c0, sh, shn), rows) in enumerate(zip(self.steps, self.rows)):
            if only is not None and not only[k]:
                continue
            i = ly.info
            if ly.kind == 0:
                per = N // i.s if i.flags == 0 else N
                tot += B * rows * L * per * 4 + B * i.K_out * L * N * 4
                tot += B * i.K_out * N * 4 if shn is not None else 0
            else:
                tot += B * rows * L * N * 4 + B * rows * L * i.n_o_p * 4
                tot += B * rows * i.n_o_p * 4 if shn is not None else 0
        return tot

    def butterflies_fwd(self, only=None):
        """Forward-NTT butterflies of one pass (c0 rows, plus sh rows where present)."""
        L, N = self.ctx.L, self.ctx.N
        per_row = (N // 2) * (N.bit_length() - 1)
        tot = 0
        for k, (ly, B, c0, sh, shn) in enumerate(self.steps):
            if only is not None and not only[k]:
                continue
            tot += B * ly.info.K_in * L * (2 if sh is not None else 1) * per_row
        return tot

    def tail_butterflies(self, only=None):
        """Inverse-transform butterflies of one pass: the (N/s)-point residue-class inverse of
        every real output channel (conv), the N-point inverse of every row block (FC)."""
        L, N = self.ctx.L, self.ctx.N
        tot = 0
        for k, ((ly, B, c0, sh, shn), rows) in enumerate(zip(self.steps, self.rows)):
            if only is not None and not only[k]:
                continue
            M = N // ly.info.s if ly.kind == 0 and ly.info.flags == 0 else N
            tot += B * rows * L * (M // 2) * (M.bit_length() - 1)
        return tot

    def modmuls(self, only=None):
        """Coefficient-wise modular multiplications of the MAC in one pass."""
        tot = 0
        L, N = self.ctx.L, self.ctx.N
        for k, ((ly, B, c0, sh, shn), c_o) in enumerate(zip(self.steps, self.rows)):
            if only is not None and not only[k]:
                continue
            J = ly.info.K_in * (2 if sh is not None else 1)
            tot += B * J * c_o * L * N
        return tot


def time_loop(fn, steps, warmup, sync):
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return time.perf_counter() - t0


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[k]


def batched_rooflines(he, ctx, st, stream, sync, passes=2, plan=None):
    """Per-kind kernel time of eager passes over a batched stack (HIP events on the launch
    stream), against the integer roofs: forward and inverse butterflies against the measured
    butterfly rate, MAC products against the 64-bit multiply-add rate.  Each kind also gets its
    algorithmic HBM bytes per pass over its time as a fraction of HBM (`hbm_frac`).  Layers the
    tuner put in a one-launch form (`plan`) are reported apart, against HBM."""
    import torch
    kinds = [("ntt_fwd", he.HE_K_NTT_FWD), ("mac", he.HE_K_MAC), ("tail", he.HE_K_TAIL), ("intt", he.HE_K_INTT),
             ("mac_tail", he.HE_K_MAC_TAIL), ("layer", he.HE_K_LAYER), ("layer_rows", he.HE_K_LAYER_ROWS),
             ("mac_mfma", he.HE_K_MAC_MFMA)]
    ctx.profile_reset()
    ctx.profile_enable(sum(k for _, k in kinds))
    with torch.cuda.stream(stream):
        for _ in range(passes):
            st.seq.run(stream)
    sync()
    ms = {}
    for name, kind in kinds:
        n, t = ctx.profile_read(kind)
        ms[name] = t / passes
    ctx.profile_enable(0)
    ctx.profile_reset()
    out = {}
    one = [p in ("one", "rows") for p in plan] if plan is not None else [False] * len(st.steps)
    multi = [not o for o in one]
    on_mfma = [p == "mfma" for p in plan] if plan is not None else [False] * len(st.steps)
    valu_mac = [m and not f for m, f in zip(multi, on_mfma)]

    def hbm(nbytes, t_ms):
        gbs = nbytes / (t_ms / 1e3) / 1e9
        return {"hbm_bytes_per_batch": int(nbytes), "hbm_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}

    if ms["ntt_fwd"]:
        fwd_rate = st.butterflies_fwd(multi) / (ms["ntt_fwd"] / 1e3) / 1e9
        out["ntt_fwd"] = {"ms_per_batch": round(ms["ntt_fwd"], 3), "bound": "alu", "achieved": round(fwd_rate, 1),
                          "peak": BFLY_PEAK_G, "unit": "Gbutterfly/s", "frac": round(fwd_rate / BFLY_PEAK_G, 4),
                          **hbm(st.fwd_bytes(multi), ms["ntt_fwd"])}
    mac_ms = ms["mac"] + ms["mac_tail"]
    if mac_ms:
        mac_rate = st.modmuls(valu_mac) / (mac_ms / 1e3) / 1e9
        out["mac"] = {"ms_per_batch": round(mac_ms, 3), "bound": "alu", "achieved": round(mac_rate, 1),
                      "peak": MAD64_PEAK_G, "unit": "Gmodmul/s", "frac": round(mac_rate / MAD64_PEAK_G, 4),
                      "layers": sum(valu_mac)}
        if plan is not None:
            out["mac"].update(hbm(st.mac_kernel_bytes(plan, only=valu_mac), mac_ms))
    if ms["mac_mfma"]:
        # each modular product is 16 products of 8-bit digits (2 int8 ops each) on the matrix cores
        mm = st.modmuls(on_mfma)
        tops = 32 * mm / (ms["mac_mfma"] / 1e3) / 1e12
        out["mac_mfma"] = {"ms_per_batch": round(ms["mac_mfma"], 3), "bound": "mfma", "achieved": round(tops, 1),
                           "peak": INT8_PEAK_T, "unit": "TOP/s (int8)", "frac": round(tops / INT8_PEAK_T, 4),
                           "Gmodmul_per_s": round(mm / (ms["mac_mfma"] / 1e3) / 1e9, 1), "layers": sum(on_mfma),
                           **hbm(st.mac_kernel_bytes(plan, only=on_mfma), ms["mac_mfma"])}
    inv_ms = ms["tail"] + ms["intt"]
    if inv_ms:
        inv_rate = st.tail_butterflies(multi) / (inv_ms / 1e3) / 1e9
        out["inverse"] = {"ms_per_batch": round(inv_ms, 3), "bound": "alu", "achieved": round(inv_rate, 1),
                          "peak": GSBFLY_PEAK_G, "unit": "Gbutterfly/s", "frac": round(inv_rate / GSBFLY_PEAK_G, 4),
                          **hbm(st.inverse_bytes(multi), inv_ms)}
    lay_ms = ms["layer"] + ms["layer_rows"]
    if lay_ms:
        out["one_launch_layers"] = {"ms_per_batch": round(lay_ms, 3), "layers": sum(one),
                                    **hbm(st.layer_bytes(one), lay_ms)}
    return out


def grouped_form(he, ctx, args, widths, stream, sync):
    """The batched stacks of every width resident at once and evaluated by grouped launches
    (he_group_*): one launch per layer index (the k-th call of every width together), and one
    launch for every call of every width.  Each pass is the same work as one pass of each width's
    captured sequence.  Roofline: the algorithmic HBM bytes of a pass (resident operands once per
    layer, inputs and outputs once) over the grouped launch's own time (HIP events)."""
    import torch
    stacks, ctxs = [], {}
    for width in widths:
        N, L = (8192, 4) if width < 4 else (16384, 6)
        if (N, L) not in ctxs:
            ctxs[(N, L)] = ctx if N == 8192 else he.Context(N, L, wl.T_PLAIN)
        log(f"setup: grouped x{width} N={N} L={L}")
        stacks.append(Stack(he, ctxs[(N, L)], wl.CONFIG_BATCHED, width, [10, 100], [32, 32], N, L))
    sync()
    per_layer = []
    for k in range(max(len(st.steps) for st in stacks)):
        g = he.Group()
        for st in stacks:
            if k < len(st.steps):
                ly, B, c0, sh, shn = st.steps[k]
                g.add(ly, c0, sh, shn)
        per_layer.append(g.build())
    whole = he.Group()
    for st in stacks:
        for ly, B, c0, sh, shn in st.steps:
            whole.add(ly, c0, sh, shn)
    whole.build()
    if not args.no_tune:
        for g in per_layer:
            g.tune(stream)
        whole.tune(stream)
    il = sum(st.image_layers() for st in stacks)
    nbytes = sum(st.layer_bytes() for st in stacks)
    steps = args.batched_steps
    out = {"widths": widths, "image_layers_per_pass": il, "algorithmic_bytes_per_pass": int(nbytes)}
    with torch.cuda.stream(stream):
        T = time_loop(lambda: [g.run(stream) for g in per_layer], steps, 1, sync)
    for g in per_layer:
        g.check(stream)
    out["per_layer_index"] = {"launches_per_pass": len(per_layer), "layers_per_s": round(il * steps / T, 1),
                              "ms_per_pass": round(T / steps * 1e3, 3)}
    with torch.cuda.stream(stream):
        T = time_loop(lambda: whole.run(stream), steps, 1, sync)
    whole.check(stream)
    items, tiled, ws = whole.items()
    c0ctx = stacks[0].ctx
    c0ctx.profile_reset()
    c0ctx.profile_enable(he.HE_K_GROUP)
    with torch.cuda.stream(stream):
        time_loop(lambda: whole.run(stream), 3, 0, sync)
    n, ms = c0ctx.profile_read(he.HE_K_GROUP)
    c0ctx.profile_enable(0)
    c0ctx.profile_reset()
    kern_s = ms / 1e3 / max(1, n)
    gbs = nbytes / kern_s / 1e9
    out["one_launch"] = {"launches_per_pass": 1, "calls": len(whole), "layers_per_s": round(il * steps / T, 1),
                         "xcd_chunk": 1 << whole.chunk_log,
                         "ms_per_pass": round(T / steps * 1e3, 3), "items_ntt_mac_inverse": list(items),
                         "image_tiled_calls": tiled, "workspace_bytes": ws,
                         "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                                      "avg_launch_ms": round(kern_s * 1e3, 3), "kernel": "k_fused_group"}}
    for g in per_layer:
        g.free()
    whole.free()
    del stacks
    torch.cuda.empty_cache()
    # single images: every layer of every width once (one image per call, one FC head each), as
    # captured per-context sequences of layer calls against one grouped launch
    singles = [Stack(he, ctxs[(8192, 4) if w < 4 else (16384, 6)], wl.CONFIG_BATCHED, w, [10], [1],
                     8192 if w < 4 else 16384, 4 if w < 4 else 6) for w in widths]
    seqs = {}
    for st in singles:
        for ly, B, c0, sh, shn in st.steps:
            key = id(st.ctx)
            if key not in seqs:
                seqs[key] = he.Sequence(st.ctx)
            seqs[key].add(ly, c0, sh, shn)
    sync()
    with torch.cuda.stream(stream):
        for q in seqs.values():
            q.capture(stream)
        T_seq = time_loop(lambda: [q.replay(stream) for q in seqs.values()], steps * 4, 2, sync)
    g1 = he.Group()
    for st in singles:
        for ly, B, c0, sh, shn in st.steps:
            g1.add(ly, c0, sh, shn)
    g1.build()
    if not args.no_tune:
        g1.tune(stream)
    with torch.cuda.stream(stream):
        T_grp = time_loop(lambda: g1.run(stream), steps * 4, 2, sync)
    g1.check(stream)
    il1 = sum(st.image_layers() for st in singles)
    out["single_images"] = {"calls": len(g1), "sequences_layers_per_s": round(il1 * steps * 4 / T_seq, 1),
                            "sequences_ms_per_pass": round(T_seq / (steps * 4) * 1e3, 3),
                            "group_layers_per_s": round(il1 * steps * 4 / T_grp, 1),
                            "group_ms_per_pass": round(T_grp / (steps * 4) * 1e3, 3),
                            "group_items_ntt_mac_inverse": list(g1.items()[0])}
    g1.free()
    del seqs, singles
    torch.cuda.empty_cache()
    log(f"grouped: {json.dumps(out)}")
    return out


def paper_protocol_form(he, ctx, st, stream, steps, warmup, sync):
    """Seconds for `steps` images of the stack under the paper's protocol (see the caller): the
    server's share transforms run as one chain on a second stream, each layer waiting only for
    the transform of its own share."""
    import torch
    side = torch.cuda.Stream()
    n = len(st.steps)
    xs, outs = [], [None] * n
    for ly, B, c0, sh, shn in st.steps:
        x = ctx.input_buffer(ly, B)
        ctx.inputs_ntt(ly, x, c0=c0)              # the client's NTT(c0), before timing
        xs.append(x)
    ready = [torch.cuda.Event() if st.steps[k][3] is not None else None for k in range(n)]

    def body():
        main = torch.cuda.current_stream()
        side.wait_stream(main)
        with torch.cuda.stream(side):
            for k, (ly, B, c0, sh, shn) in enumerate(st.steps):
                if sh is not None:
                    ctx.inputs_ntt(ly, xs[k], sh=sh)
                    ready[k].record(side)
        for k, (ly, B, c0, sh, shn) in enumerate(st.steps):
            if ready[k] is not None:
                main.wait_event(ready[k])
            outs[k] = ctx.layer_from_ntt(ly, xs[k], sh is not None, shn, out=outs[k])
        main.wait_stream(side)
    # an eager pass allocates every workspace and output before the capture
    with torch.cuda.stream(stream):
        body()
    sync()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        body()
    sync()
    with torch.cuda.stream(stream):
        return time_loop(g.replay, steps, warmup, sync)


def single_conv_form(he, args, stream, sync):
    """The single conv workload (conv 3->16 on 3x32x32, pad 1, N = 4096, 3 limbs, a network's first
    layer: no input share, a fresh output share): layer calls back to back (throughput), per-call
    latency with a synchronisation after each call (p50 / p99), and the kernel time per launch kind
    against HBM (algorithmic bytes of the launches that carry the layer)."""
    import torch
    N, L = 4096, 3
    ctx = he.Context(N, L, wl.T_PLAIN)
    shp = wl.single_conv_layer()
    spec = he.ConvSpec(shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
    til = ctx.geometry(spec)
    cfg = wl.CONFIG_SINGLE_CONV
    W = wl.layer_weights(cfg, 0, 0, shp)
    rho = wl.mask_polys(cfg, 0, 0, til.K_in * shp.c_o, N).reshape(til.K_in, shp.c_o, N)
    ly = ctx.pack_conv(spec, W, rho)
    dev = torch.device("cuda:0")
    c0 = torch.from_numpy(wl.ciphertext_polys(cfg, 0, 0, 0, til.K_in, ctx.primes, N)
                          .reshape(1, til.K_in, L, N).astype(np.int32)).to(dev)
    shn = torch.from_numpy(wl.share_polys(cfg, 0, 0, 0, til.K_out, N, "shnext").reshape(1, til.K_out, N)
                           .astype(np.int32)).to(dev)
    if not args.no_tune:
        ctx.autotune(ly, 1)
    seq = he.Sequence(ctx)
    seq.add(ly, c0, None, shn)
    reps = max(200, args.steps)
    with torch.cuda.stream(stream):
        T = time_loop(lambda: seq.run(stream), reps, 20, sync)
    lat = []
    for _ in range(reps):
        t0 = time.perf_counter()
        ctx.conv_layer(ly, c0, None, shn, stream=stream)
        stream.synchronize()
        lat.append(time.perf_counter() - t0)
    kinds = [("ntt_fwd", he.HE_K_NTT_FWD), ("mac", he.HE_K_MAC), ("tail", he.HE_K_TAIL), ("intt", he.HE_K_INTT),
             ("mac_tail", he.HE_K_MAC_TAIL), ("layer", he.HE_K_LAYER), ("layer_rows", he.HE_K_LAYER_ROWS)]
    ctx.profile_reset()
    ctx.profile_enable(sum(k for _, k in kinds))
    with torch.cuda.stream(stream):
        time_loop(lambda: seq.run(stream), 100, 0, sync)
    kern = {}
    for name, kind in kinds:
        n, ms = ctx.profile_read(kind)
        if n:
            kern[name] = {"launches_per_call": n // 100, "avg_us": round(ms * 1e3 / n, 3)}
    ctx.profile_enable(0)
    ctx.profile_reset()
    # algorithmic bytes of the call: c0 read, resident operand rows (c0 rows only: no input share)
    # read once, sh' read, output polynomials written
    nbytes = (til.K_in * L * N + til.K_in * shp.c_o * L * N + til.K_out * N + til.K_out * L * N) * 4
    call_us = sum(v["avg_us"] * v["launches_per_call"] for v in kern.values())
    ach = nbytes / (call_us * 1e-6) / 1e9
    out = {"workload": "conv 3->16 on 3x32x32, pad 1, N=4096, 3 limbs, first layer (no input share)",
           "layers_per_s": round(reps / T, 1), "ms_per_layer": round(T / reps * 1e3, 4),
           "latency_p50_ms": round(percentile(lat, 50) * 1e3, 4),
           "latency_p99_ms": round(percentile(lat, 99) * 1e3, 4), "kernels": kern,
           "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_call": nbytes,
                        "kernel_us_per_call": round(call_us, 3)}}
    log(f"single_conv: {json.dumps(out)}")
    ly.free()
    return out


def resnet50_form(he, args, stream, sync):
    """ResNet-50-shaped layers (the body after the stem: 52 convs + FC 2048 -> 1000) at
    N = 16384, 6 limbs.  Each distinct shape is packed, tuned and timed on its own (resident
    operands of one shape at a time) at batch 1 and batch 16; per-image totals weight each
    shape by how often the body uses it."""
    import collections
    import torch
    ctx = he.Context(16384, 6, wl.T_PLAIN)
    N, L, t = 16384, 6, wl.T_PLAIN
    body = wl.resnet50_body()
    count = collections.Counter(body)
    first = {}
    for k, shp in enumerate(body):
        first.setdefault(shp, k)
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(wl.MASTER_SEED + wl.CONFIG_RESNET50)
    reps = args.resnet50_reps
    rows, tot1, tot16, resident = [], 0.0, 0.0, 0
    for shp, k in sorted(first.items(), key=lambda kv: kv[1]):
        W = wl.layer_weights(wl.CONFIG_RESNET50, 0, k, shp)
        if shp.kind == "conv":
            spec = he.ConvSpec(shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
            K_in = ctx.geometry(spec).K_in
            rho = wl.mask_polys(wl.CONFIG_RESNET50, 0, k, K_in * shp.c_o, N).reshape(K_in, shp.c_o, N)
            ly = ctx.pack_conv(spec, W, rho)
        else:
            fspec = he.FCSpec(shp.n_i, shp.n_o)
            rho = wl.mask_polys(wl.CONFIG_RESNET50, 0, k, ctx.geometry(fspec).blocks, N)
            ly = ctx.pack_fc(fspec, W, rho, wl.layer_bias(wl.CONFIG_RESNET50, 0, k, shp))
        del rho
        i = ly.info
        resident += i.resident_bytes * count[shp]
        res = {}
        for B in (1, 16):
            if shp.kind == "conv":
                c0 = torch.randint(0, 1 << 29, (B, i.K_in, L, N), generator=gen, device=dev, dtype=torch.int32)
                sh = torch.randint(0, t, (B, i.K_in, N), generator=gen, device=dev, dtype=torch.int32)
                shn = torch.randint(0, t, (B, i.K_out, N), generator=gen, device=dev, dtype=torch.int32)
            else:
                c0 = torch.randint(0, 1 << 29, (B, L, N), generator=gen, device=dev, dtype=torch.int32)
                sh = torch.randint(0, t, (B, N), generator=gen, device=dev, dtype=torch.int32)
                shn = None
            if not args.no_tune:
                ctx.autotune(ly, B)
            seq = he.Sequence(ctx)
            for _ in range(reps):
                seq.add(ly, c0, sh, shn)
            with torch.cuda.stream(stream):
                T = time_loop(lambda: seq.run(stream), 3, 1, sync)
            res[B] = T / 3 / reps
            del seq, c0, sh, shn
            torch.cuda.empty_cache()
        tot1 += res[1] * count[shp]
        tot16 += res[16] * count[shp]
        rows.append({"layer": k, "shape": f"{shp.c_i}->{shp.c_o} {shp.H}x{shp.W} f{shp.f} s{shp.stride}"
                     if shp.kind == "conv" else f"fc {shp.n_i}->{shp.n_o}",
                     "count": count[shp], "slot_stride": int(getattr(i, "s", 0)),
                     "resident_GB": round(i.resident_bytes / 1e9, 3),
                     "ms_b1": round(res[1] * 1e3, 4), "ms_per_image_b16": round(res[16] / 16 * 1e3, 4)})
        log(f"resnet50 {rows[-1]}")
        ly.free()
        torch.cuda.empty_cache()
    n = len(body)
    return {"layers": n, "distinct_shapes": len(first), "N": N, "limbs": L,
            "resident_GB_whole_body": round(resident / 1e9, 1),
            "b1": {"ms_per_image": round(tot1 * 1e3, 3), "layers_per_s": round(n / tot1, 1)},
            "b16": {"ms_per_image": round(tot16 / 16 * 1e3, 3), "layers_per_s": round(16 * n / tot16, 1)},
            "per_shape": rows,
            "note": "synthetic inputs; the 224x224 stem is not included (needs N >= 65536 in this packing)"}


# ------------------------------------------------------------------ CPU baseline
def _host_description():
    """nproc and the CPU model of this host (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(reps_one=1, reps_all=3):
    """The oracle's plain C build (textbook NTT, u64 % reduction, -O2, OpenMP over (limb, channel)
    units) over every layer of the x1 stack for one image, on one core and on all host cores.  The
    set-up transforms of the masks and filters (kept by the server, Sec. IV-A-1) are not timed."""
    from oracle import bfv, cserver, packing
    N, L = 8192, 4
    ctx = bfv.make_ctx(N, L, wl.T_PLAIN)
    layers = wl.plain20(1, 10)
    cfg = wl.CONFIG_PLAIN20_X1
    calls = []
    for k, shp in enumerate(layers):
        if shp.kind == "conv":
            g = packing.conv_geometry(N, shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
            F = wl.layer_weights(cfg, 1, k, shp)
            rho = wl.mask_polys(cfg, 1, k, g.K_in * shp.c_o, N).reshape(g.K_in, shp.c_o, N)
            ops = cserver.conv_setup(ctx, rho, packing.pack_conv_filters(F, g), 0)
            c0 = wl.ciphertext_polys(cfg, 0, 1, k, g.K_in, ctx.primes, N).astype(np.uint64)
            sh = None if k == 0 else wl.share_polys(cfg, 0, 1, k, g.K_in, N)
            shn = wl.share_polys(cfg, 0, 1, k, g.K_out, N, "shnext")
            calls.append(lambda th, g=g, c0=c0, ops=ops, sh=sh, shn=shn:
                         cserver.server_conv(ctx, g, c0, ops, sh, shn, th))
        else:
            g = packing.fc_geometry(N, shp.n_i, shp.n_o)
            w = packing.pack_fc_weights(wl.layer_weights(cfg, 1, k, shp), g)
            d = packing.pack_fc_bias(wl.layer_bias(cfg, 1, k, shp), g)
            ops = cserver.fc_setup(ctx, wl.mask_polys(cfg, 1, k, g.blocks, N), w, 0)
            c0 = wl.ciphertext_polys(cfg, 0, 1, k, 1, ctx.primes, N)[0].astype(np.uint64)
            sh = wl.share_polys(cfg, 0, 1, k, 1, N)[0]
            calls.append(lambda th, g=g, c0=c0, ops=ops, d=d, sh=sh: cserver.server_fc(ctx, g, c0, ops, d, sh, None, th))

    def stack_s(threads, reps):
        t0 = time.perf_counter()
        for _ in range(reps):
            for fn in calls:
                fn(threads)
        return (time.perf_counter() - t0) / reps

    nproc, model = _host_description()
    # the host cores this process may use (OMP_NUM_THREADS, where set, caps them)
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (nproc or 1)
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        avail = min(avail, int(os.environ["OMP_NUM_THREADS"]))
    t_one = stack_s(1, reps_one)
    threads = cserver.threads_used(avail)
    t_all = stack_s(threads, reps_all)
    n = len(layers)
    return {"value": round(n / t_all, 2), "unit": "layers/s", "cores": threads, "kind": "oracle",
            "sample": f"plain C build of the oracle's server evaluation (oracle/c/he_oracle.c: textbook NTT, u64 "
                      f"% reduction, gcc -O2, OpenMP over (limb, channel) units): the whole {n}-layer x1 stack "
                      f"(N=8192, 4 limbs), one image, {reps_all} passes on {threads} threads; set-up transforms of "
                      f"the masks and filters untimed",
            "single_core": {"value": round(n / t_one, 2), "unit": "layers/s", "cores": 1,
                            "s_per_image": round(t_one, 3), "passes": reps_one},
            "s_per_image": round(t_all, 3), "nproc": nproc, "cpu_model": model}


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-group", action="store_true", help="skip the grouped launches of the batched form")
    ap.add_argument("--batched-widths", default="1,2,4", help="plain-20 widths of the batched form")
    ap.add_argument("--no-resnet50", action="store_true",
                    help="skip the ResNet-50-shaped layers (each distinct shape packed and timed in turn)")
    ap.add_argument("--resnet50-reps", type=int, default=10)
    ap.add_argument("--batched-tail", type=int, default=None,
                    help="pin the residue-class tail form of the batched form (HE_TUNE_TAIL value)")
    ap.add_argument("--batched-mac", type=int, default=None,
                    help="pin the MAC variant of the batched form (HE_TUNE_MAC value) instead of tuning it")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=20000)
    ap.add_argument("--served-warmup", type=int, default=1000)
    ap.add_argument("--served-rate", type=float, default=2000.0)
    ap.add_argument("--served-sweep", default="2000,8000,16000,32000,64000",
                    help="offered rates (req/s) of the load sweep, served against plain FCFS at each ('' skips)")
    ap.add_argument("--sweep-requests", type=int, default=4000)
    ap.add_argument("--no-single", action="store_true", help="skip the single conv workload (N=4096, 3 limbs)")
    ap.add_argument("--no-stress", action="store_true")
    ap.add_argument("--stress-clients", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-rates", action="store_true",
                    help="keep the stored integer-ALU roofs instead of measuring them (he_probe_rate)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="also run one 256 MiB device-to-device copy (known bytes) for counter calibration")
    ap.add_argument("--pmc-mac-form", choices=["F", "S", "O", "R"], default=None,
                    help="counter runs: pin every layer of the plain stack to the fused (F) or split (S) MAC "
                         "form or a one-launch form (O work items, R rows; the FC head takes O), run only the "
                         "plain loop and print the plan (the per-layer traffic table)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path shards across GPUs by "
              f"independent requests, which this benchmark does not exercise", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_05205_amd import he
    he.load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    sync = torch.cuda.synchronize
    rates = None
    if not args.no_rates:
        global BFLY_PEAK_G, GSBFLY_PEAK_G, MAD64_PEAK_G
        rates = alu_rates(he)
        BFLY_PEAK_G = rates["butterfly_ct"]["G_per_s"]
        GSBFLY_PEAK_G = rates["butterfly_gs"]["G_per_s"]
        MAD64_PEAK_G = rates["mad_u64_u32"]["G_per_s"]
        log(f"alu rates: {json.dumps(rates)}")

    # ---------------- plain x1 stack, one image per call
    log("setup: x1 stack N=8192 L=4")
    ctx = he.Context(8192, 4, wl.T_PLAIN)
    st = Stack(he, ctx, wl.CONFIG_PLAIN20_X1, 1, [10], [1], 8192, 4)
    n_layers = len(st.steps)
    if args.pmc_mac_form is not None:
        ctx.tune_force(he.HE_TUNE_MAC, {"F": 2, "S": 0, "O": 7, "R": 8}[args.pmc_mac_form])
    elif not args.no_tune:
        st.autotune()
    sync()

    if args.pmc_calibration:
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda:0")     # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        sync()
        del src, dst

    # plain: native runtime, one image, 20 calls back to back
    with torch.cuda.stream(stream):
        T_plain = time_loop(lambda: st.seq.run(stream), args.steps, args.warmup, sync)
    log(f"plain: {T_plain / args.steps * 1e3:.3f} ms/step")
    if args.pmc_mac_form is not None:
        # layer order of the MAC launches above is the stack order, one per layer per call
        plan = "".join({"one": "O", "rows": "R", "fused": "F", "split": "S", "mfma": "M"}[p] for p in st.mac_plan(he))
        print(json.dumps({"pmc_mac_form": args.pmc_mac_form, "plan": plan,
                          "calls": args.warmup + args.steps + 1}), flush=True)
        return

    # kernel timing of the same calls (HIP events on the launch stream)
    plan = st.mac_plan(he)
    ctx.profile_reset()
    ctx.profile_enable(he.HE_K_MAC | he.HE_K_NTT_FWD | he.HE_K_TAIL | he.HE_K_INTT | he.HE_K_MAC_TAIL | he.HE_K_LAYER |
                       he.HE_K_LAYER_ROWS)
    with torch.cuda.stream(stream):
        T_prof = time_loop(lambda: st.seq.run(stream), args.steps, 0, sync)
    kern = {}
    for name, kind in [("ntt_fwd", he.HE_K_NTT_FWD), ("mac", he.HE_K_MAC), ("tail", he.HE_K_TAIL),
                       ("intt", he.HE_K_INTT), ("mac_tail", he.HE_K_MAC_TAIL), ("layer", he.HE_K_LAYER),
                       ("layer_rows", he.HE_K_LAYER_ROWS)]:
        n, ms = ctx.profile_read(kind)
        kern[name] = {"launches": n, "total_ms": ms, "avg_us": (ms * 1e3 / n) if n else None}
    ctx.profile_enable(0)
    ctx.profile_reset()
    log("kernels:", json.dumps(kern))

    # graph: capture once, replay per image
    seq_g = he.Sequence(ctx)
    for ly, B, c0, sh, shn in st.steps:
        seq_g.add(ly, c0, sh, shn)
    with torch.cuda.stream(stream):
        seq_g.capture(stream)
        T_graph = time_loop(lambda: seq_g.replay(stream), args.steps, args.warmup, sync)
    log(f"graph: {T_graph / args.steps * 1e3:.3f} ms/step")

    # paper_protocol: the same stack and calls under the paper's protocol (Sec. IV-A-1). The client
    # sends NTT(c0) (its transform is client work, done before timing); the server draws its shares
    # and transforms them on a second stream, ahead of the layers that read them, and each layer is
    # then one launch on the main stream. Captured once into a graph, one replay per image.
    T_proto = paper_protocol_form(he, ctx, st, stream, args.steps, args.warmup, sync)
    log(f"paper_protocol: {T_proto / args.steps * 1e3:.3f} ms/step")

    # plain_host: per-layer Python calls with a sync after each layer, per-layer latency
    lat = []

    def host_step():
        for ly, B, c0, sh, shn in st.steps:
            t0 = time.perf_counter()
            if ly.kind == he.HE_LAYER_CONV:
                ctx.conv_layer(ly, c0, sh, shn, stream=stream)
            else:
                ctx.fc_layer(ly, c0, sh, shn, stream=stream)
            stream.synchronize()
            lat.append(time.perf_counter() - t0)
    host_steps = max(5, args.steps // 4)
    T_host = time_loop(host_step, host_steps, 2, sync)
    lat = lat[2 * n_layers:]
    log(f"plain_host: {T_host / host_steps * 1e3:.3f} ms/step")

    # the launches that carry the MAC: fused MAC + tail (conv layers at batch one) and the
    # split MAC (FC head, and any layer the tuner gave the two-launch form)
    rooflines = {}
    per_step = {}
    plan_letters = "".join({"one": "O", "rows": "R", "fused": "F", "split": "S", "mfma": "M"}[p] for p in plan)
    one_sel = [p in ("one", "rows") for p in plan]
    n_one = sum(one_sel)
    lay_n = kern["layer"]["launches"] + kern["layer_rows"]["launches"]
    if lay_n:
        # whole layers in one launch (forward transforms, MAC, inverse, extraction)
        one_bytes = st.layer_bytes(only=one_sel)
        lay_ms = kern["layer"]["total_ms"] + kern["layer_rows"]["total_ms"]
        lay_avg_s = lay_ms / 1e3 / lay_n
        ach = one_bytes / n_one / lay_avg_s / 1e9
        rooflines["layer"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(ach / HBM_PEAK_GBS, 4),
                              "traffic": pmc_traffic("layers", plan_letters, one_sel),
                              "algorithmic_bytes_per_launch": one_bytes // n_one,
                              "kernel": f"k_fused_layer / k_fused_rows (forward NTT, MAC, residue-class / prefix "
                                        f"inverse and extraction in one launch, {n_one} layers)",
                              "launches_per_step": n_one, "avg_launch_us": round(lay_avg_s * 1e6, 3)}
        per_step["layer"] = lay_ms
    mac_n = kern["mac"]["launches"] + kern["mac_tail"]["launches"]
    if mac_n:
        multi = [not o for o in one_sel]
        n_multi = sum(multi)
        mac_bytes = st.mac_kernel_bytes(plan, only=multi)
        mac_ms = kern["mac"]["total_ms"] + kern["mac_tail"]["total_ms"]
        mac_avg_s = mac_ms / 1e3 / mac_n
        achieved = mac_bytes / n_multi / mac_avg_s / 1e9
        n_fused = plan.count("fused")
        rooflines["mac"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(achieved / HBM_PEAK_GBS, 4),
                            "traffic": pmc_traffic("layers", plan_letters, multi), "mac_forms": plan_letters,
                            "algorithmic_bytes_per_launch": mac_bytes // n_multi,
                            "kernel": f"k_mac_tail (fused MAC + residue-class inverse, {n_fused} layers) / "
                                      f"k_mac_class, k_mac_full (split MAC, {n_multi - n_fused} layers)",
                            "launches_per_step": n_multi, "avg_launch_us": round(mac_avg_s * 1e6, 3)}
        per_step["mac"] = mac_ms
    if kern["ntt_fwd"]["launches"]:
        multi = [not o for o in one_sel]
        fwd_avg_s = kern["ntt_fwd"]["total_ms"] / 1e3 / kern["ntt_fwd"]["launches"]
        fwd_bfly = st.butterflies_fwd(only=multi) / sum(multi)        # one forward launch per layer
        fwd_g = fwd_bfly / fwd_avg_s / 1e9
        rooflines["ntt_fwd"] = {"bound": "alu", "achieved": round(fwd_g, 1), "peak": BFLY_PEAK_G,
                                "unit": "Gbutterfly/s", "frac": round(fwd_g / BFLY_PEAK_G, 4),
                                "traffic": pmc_traffic("ntt_fwd"), "butterflies_per_launch": int(fwd_bfly),
                                "kernel": "k_ntt_fwd (forward negacyclic NTT)", "launches_per_step": sum(multi),
                                "avg_launch_us": round(fwd_avg_s * 1e6, 3)}
        per_step["ntt_fwd"] = kern["ntt_fwd"]["total_ms"]
    if kern["tail"]["launches"] + kern["intt"]["launches"]:
        per_step["tail"] = kern["tail"]["total_ms"] + kern["intt"]["total_ms"]
    dominant = max(per_step, key=per_step.get)
    roofline = rooflines.get(dominant) or rooflines.get("mac") or rooflines["layer"]
    layers_per_s = n_layers * args.steps / T_plain
    graph_lps = n_layers * args.steps / T_graph
    result = {
        "metric": "HE Conv+FC layers/sec and p50/p99 latency, batched/served vs plain, 1 MI355X",
        "value": round(layers_per_s, 1),
        "unit": "layers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(T_plain / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "plain-20 x1 linear stack (19 conv + FC 64->10), one image per layer call",
                   "N": 8192, "limbs": 4, "t": wl.T_PLAIN, "layers": n_layers, "images_per_step": 1,
                   "form": "plain: native runtime issues the 20 layer calls back to back on one stream"},
        "limb_poly_macs_per_s": round(st.modmuls() / 8192 * args.steps / T_plain, 1),
        "roofline": roofline,
        "rooflines": rooflines,
        "alu_rates": rates,
        "layer_forms": plan_letters,
        "dominant_kernel": dominant,
        "kernels": kern,
        "forms": {
            "plain": {"layers_per_s": round(layers_per_s, 1), "ms_per_image": round(T_plain / args.steps * 1e3, 4)},
            "graph": {"layers_per_s": round(graph_lps, 1), "ms_per_image": round(T_graph / args.steps * 1e3, 4)},
            "paper_protocol": {"layers_per_s": round(n_layers * args.steps / T_proto, 1),
                               "ms_per_image": round(T_proto / args.steps * 1e3, 4),
                               "note": "c0 arrives as NTT(c0) (client's transform, untimed); the server's "
                                       "NTT(sh) of every layer runs as a chain on a second stream, each "
                                       "layer waiting for its own"},
            "plain_host": {"layers_per_s": round(n_layers * host_steps / T_host, 1),
                           "ms_per_image": round(T_host / host_steps * 1e3, 4),
                           "layer_latency_p50_ms": round(percentile(lat, 50) * 1e3, 4),
                           "layer_latency_p99_ms": round(percentile(lat, 99) * 1e3, 4)},
        },
    }
    del seq_g

    # ---------------- single conv workload: conv 3->16 on 3x32x32, N = 4096, 3 limbs, one image
    if not args.no_single:
        result["forms"]["single_conv"] = single_conv_form(he, args, stream, sync)

    # ---------------- batched: 64 images x widths 1, 2, 4
    if not args.no_batched:
        bres = {}
        tot_layers = 0
        tot_time = 0.0
        widths = [int(w) for w in args.batched_widths.split(",")]
        for width, N, L in [(w, 8192 if w < 4 else 16384, 4 if w < 4 else 6) for w in widths]:
            log(f"setup: batched x{width} N={N} L={L}")
            bctx = ctx if N == 8192 else he.Context(N, L, wl.T_PLAIN)
            bst = Stack(he, bctx, wl.CONFIG_BATCHED, width, [10, 100], [32, 32], N, L)
            if args.batched_mac is not None:
                bctx.tune_force(he.HE_TUNE_MAC, args.batched_mac)
            if args.batched_tail is not None:
                bctx.tune_force(he.HE_TUNE_TAIL, args.batched_tail)
            if not args.no_tune:
                bst.autotune()
            sync()
            bseq = he.Sequence(bctx)
            for ly, B, c0, sh, shn in bst.steps:
                bseq.add(ly, c0, sh, shn)
            with torch.cuda.stream(stream):
                bseq.capture(stream)
                T = time_loop(lambda: bseq.replay(stream), args.batched_steps, 1, sync)
            il = bst.image_layers()
            bres[f"x{width}"] = {"layers_per_s": round(il * args.batched_steps / T, 1),
                                 "ms_per_batch": round(T / args.batched_steps * 1e3, 3),
                                 "image_layers_per_batch": il,
                                 "limb_poly_macs_per_s": round(bst.modmuls() / N * args.batched_steps / T, 1),
                                 "kernel_rooflines": batched_rooflines(he, bctx, bst, stream, sync,
                                                                       plan=bst.mac_plan(he))}
            log(f"batched x{width}: {json.dumps(bres[f'x{width}'])}")
            tot_layers += il * args.batched_steps
            tot_time += T
            if args.batched_mac is not None:
                bctx.tune_force(he.HE_TUNE_MAC, -1)
            if args.batched_tail is not None:
                bctx.tune_force(he.HE_TUNE_TAIL, 0)
            del bseq, bst
            torch.cuda.empty_cache()
        bres["all_widths_layers_per_s"] = round(tot_layers / tot_time, 1)
        if not args.no_group:
            bres["grouped"] = grouped_form(he, ctx, args, widths, stream, sync)
        result["forms"]["batched"] = bres

    # ---------------- served: Poisson stream of single-layer requests, 128 clients
    if not args.no_served:
        from paper_2409_05205_amd import serve
        log("setup: served variants x1/x2 (N=8192, 10 classes), x4 (N=16384, 100 classes), 128 clients")
        ctx16 = he.Context(16384, 6, wl.T_PLAIN)
        variants = [serve.pack_variant(1, 10, ctx), serve.pack_variant(2, 10, ctx), serve.pack_variant(4, 100, ctx16)]
        clients = 128
        buffers = [serve.client_buffers(v, clients, seed=v.width) for v in variants]
        sync()
        n_types = sum(len(v.layers) for v in variants)
        n = args.served_requests + args.served_warmup
        arrival, ltype, client = serve.poisson_trace(args.served_rate, n, n_types, clients, seed=1)
        sres = {"offered_req_per_s": args.served_rate, "clients": clients, "layer_types": n_types,
                "requests": args.served_requests, "warmup_requests": args.served_warmup}
        budget = 8 << 30
        # batches of up to 16 requests: saturated 75K layers/s against 62K with batches of up to 8,
        # and at 64K req/s p99 8.0 against 10.7 ms (32 measured no better)
        SERVED_MB = 16
        for name, streams, mb in [("served", 4, SERVED_MB), ("plain_fcfs", 1, 1)]:
            res = serve.run_trace(variants, buffers, arrival, ltype, client, streams, mb, budget, timeout_s=300)
            st = serve.latency_stats(res, args.served_warmup)
            st.update({"streams": streams, "max_batch": mb, "rc": res["rc"],
                       "valid": res["rc"] == 0 and st["failed"] == 0})
            sres[name] = st
            log(f"{name}: {json.dumps(st)}")
        # capacity: the whole trace arrives at once
        sat_n = min(3000, n)
        z = np.zeros(sat_n)
        for name, streams, mb in [("served_saturated", 4, SERVED_MB), ("plain_saturated", 1, 1)]:
            res = serve.run_trace(variants, buffers, z, ltype[:sat_n], client[:sat_n], streams, mb, budget,
                                  timeout_s=300)
            span = res["complete"].max()
            sres[name] = {"requests": sat_n, "layers_per_s": sat_n / span, "mean_batch": float(res["batch"].mean()),
                          "rc": res["rc"]}
            log(f"{name}: {json.dumps(sres[name])}")
        # offered-load sweep: served against plain FCFS on the same trace at each rate
        sweep = []
        for rate in [float(r) for r in args.served_sweep.split(",") if r.strip()]:
            m = args.sweep_requests
            w = m // 10
            arr, lt, cl = serve.poisson_trace(rate, m + w, n_types, clients, seed=2)
            row = {"offered_req_per_s": rate, "requests": m, "warmup_requests": w}
            for name, streams, mb in [("served", 4, SERVED_MB), ("plain_fcfs", 1, 1)]:
                res = serve.run_trace(variants, buffers, arr, lt, cl, streams, mb, budget, timeout_s=300)
                st = serve.latency_stats(res, w)
                st["rc"] = res["rc"]
                st["valid"] = res["rc"] == 0 and st["failed"] == 0
                row[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
            log(f"sweep {json.dumps(row)}")
            sweep.append(row)
        sres["sweep"] = sweep
        result["forms"]["served"] = sres
        del variants, buffers
        torch.cuda.empty_cache()

    # ---------------- stress: x4 / 100 classes, clients streaming whole inferences
    if not args.no_stress:
        from paper_2409_05205_amd import serve
        C = args.stress_clients
        log(f"setup: stress x4 (N=16384, 6 limbs, 100 classes), {C} clients")
        ctx16s = he.Context(16384, 6, wl.T_PLAIN)
        v4 = serve.pack_variant(4, 100, ctx16s, cfg=wl.CONFIG_STRESS)
        bufs = serve.client_buffers(v4, C, seed=5)
        sync()
        stres = {}
        # batches of up to 64 requests: 69K layers/s against 57K with batches of up to 16, and lower
        # inference latency (four streams; 2 x 64 and 8 x 32 were measured below both)
        for name, streams, mb in [("served", 4, 64), ("plain_fcfs", 1, 1)]:
            res = serve.run_clients(v4, bufs, C, streams, mb, 24 << 30, timeout_s=300)
            st = serve.client_stats(res)
            st.update({"streams": streams, "max_batch": mb, "rc": res["rc"]})
            stres[name] = st
            log(f"stress {name}: {json.dumps(st)}")
        result["forms"]["stress"] = stres
        del v4, bufs
        torch.cuda.empty_cache()

    if not args.no_resnet50:
        log("setup: ResNet-50-shaped layers, N=16384, 6 limbs")
        result["forms"]["resnet50"] = resnet50_form(he, args, stream, sync)

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
