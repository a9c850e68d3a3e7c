"""Stress workload: plain-20 x4 with a 100-class head, N = 16384, 6 limbs,
256 clients each streaming the whole 19-conv + FC inference through the
continuous-batching server (a client's layer k+1 is issued when its layer k
returns).  Every client encrypts its true layer inputs on the device; every
decrypted output of every layer of every client must equal the integer forward
pass mod t.

The client's share c1^r of each output is formed, for this check, with the
masks' noise terms e1 = e2 = 0: then sum_j v_j p1_j + i_j p2_j equals the
server products applied to the inputs (v_j b + Delta i_j, t - i_j), so one more
server-kernel call per layer gives it for all clients at once (the last layer
uses an FC layer packed without bias).  The extra r_t f-hat term this adds is
far below Delta.  The integer reference runs on the device in float64 (exact
for these magnitudes) and is checked against the oracle's forward pass for two
clients.  For the first 8 clients, the first, a middle and the last layer are
also compared word for word with the oracle: the oracle's own encryption of the
same plaintext (numpy), and its server evaluation of those ciphertexts (the C
build, which the CPU suite pins to the numpy oracle and the stored digests).
"""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import bfv, cserver, network, packing
from gpu_helpers import host

pytestmark = pytest.mark.gpu

T = wl.T_PLAIN
CLIENTS = int(os.environ.get("HE_STRESS_CLIENTS", "256"))
CFG = wl.CONFIG_STRESS
WIDTH = 4
ORACLE_CLIENTS = 8
ORACLE_LAYERS = (0, 9, 19)      # first conv, a stage-two conv (128 -> 128 at 16 x 16), the FC head


def _forward_gpu(imgs, shapes, Ws, Bs):
    """Integer plain-20 forward pass with the harness between layers, batched over clients."""
    import torch
    import torch.nn.functional as Fn
    x = torch.as_tensor(imgs, dtype=torch.int64, device="cuda:0")
    ins, outs = [], []
    for k, (shp, W, B) in enumerate(zip(shapes, Ws, Bs)):
        ins.append(x)
        if shp.kind == "conv":
            y = Fn.conv2d(x.double(), torch.as_tensor(W, dtype=torch.float64, device="cuda:0"), stride=shp.stride,
                          padding=shp.pad)
            y = torch.round(y).long()
        else:
            y = torch.round(x.double() @ torch.as_tensor(W, dtype=torch.float64, device="cuda:0").T).long()
            y = y + torch.as_tensor(B, dtype=torch.int64, device="cuda:0")
        outs.append(y)
        r = torch.clamp(y, min=0)
        mx = r.reshape(r.shape[0], -1).amax(dim=1)
        bits = torch.zeros_like(mx)
        for b in range(40):
            bits = torch.where(mx >> b > 0, torch.full_like(mx, b + 1), bits)
        shift = torch.clamp(bits - 4, min=0)
        a = r >> shift.view(-1, *([1] * (r.dim() - 1)))
        nxt = shapes[k + 1] if k + 1 < len(shapes) else None
        x = a.reshape(a.shape[0], a.shape[1], -1).sum(dim=2) // (a.shape[2] * a.shape[3]) \
            if (nxt is not None and nxt.kind == "fc") else a
    return ins, outs


def _conv_pack_index(g):
    """(j, coefficient) of every (channel, y, x) of the input image (the packing of the tiling rule)."""
    m, y, x = np.meshgrid(np.arange(g.c_i), np.arange(g.H), np.arange(g.W), indexing="ij")
    j = m // g.g_i
    coef = g.s * ((y + g.pad) * g.W_p + (x + g.pad)) + m % g.g_i
    return m.ravel(), y.ravel(), x.ravel(), j.ravel(), coef.ravel()


def _conv_out_index(g):
    n, oy, ox = np.meshgrid(np.arange(g.c_o), np.arange(g.H_o), np.arange(g.W_o), indexing="ij")
    p = n // g.g_o
    k = g.s * (g.stride * oy * g.W_p + g.stride * ox) + (n % g.g_o) * (g.s // g.g_o)
    return p.ravel(), k.ravel()


def _draws(seed, shape, kind):
    import torch
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(seed)
    if kind == "share":
        return torch.randint(0, T, shape, generator=gen, device="cuda:0", dtype=torch.int64)
    if kind == "gauss":
        e = torch.round(torch.normal(0.0, wl.SIGMA, shape, generator=gen, device="cuda:0"))
        return torch.clamp(e, -np.floor(wl.ERR_BOUND), np.floor(wl.ERR_BOUND)).to(torch.int32)
    u = torch.randint(0, 4, shape, generator=gen, device="cuda:0")
    return torch.where(u < 2, 0, torch.where(u == 2, 1, -1)).to(torch.int32)


def test_stress_x4_clients_decrypt_exact():
    import torch
    from paper_2409_05205_amd import he, serve
    N, L = 16384, 6
    C = CLIENTS
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    v = serve.pack_variant(WIDTH, 100, ctx, cfg=CFG)
    shapes = v.shapes
    Ws = [wl.layer_weights(CFG, WIDTH, k, s) for k, s in enumerate(shapes)]
    Bs = [wl.layer_bias(CFG, WIDTH, k, s) for k, s in enumerate(shapes)]
    fg = packing.fc_geometry(N, shapes[-1].n_i, shapes[-1].n_o)
    fc_nobias = ctx.pack_fc(he.FCSpec(shapes[-1].n_i, shapes[-1].n_o), Ws[-1],
                            wl.mask_polys(CFG, WIDTH, 19, fg.blocks, N), None)
    imgs = np.stack([wl.image(CFG, c, WIDTH) for c in range(C)])
    print(f"stress: {C} clients, x4 stack N={N} L={L}", flush=True)
    ins, outs = _forward_gpu(imgs, shapes, Ws, Bs)
    for c in sorted({0, C - 1}):
        o_outs, o_ins = network.plaintext_forward(imgs[c], shapes, Ws, Bs)
        for k in range(len(shapes)):
            assert (o_outs[k] == outs[k][c].cpu().numpy()).all(), f"reference layer {k} client {c}"

    # keys per client: b = -a s + e on the device
    keys = []
    for c in range(C):
        s = wl.ternary(wl.rng(CFG, c, 0, 0, "s"), N)
        a = wl.uniform_per_modulus(wl.rng(CFG, c, 0, 0, "a"), (), ctx.primes, N)
        e = wl.gaussian(wl.rng(CFG, c, 0, 0, "e"), N)
        b = ctx.encrypt_c0(torch.as_tensor(s[None], dtype=torch.int32, device="cuda:0"),
                           torch.as_tensor(a, dtype=torch.int32, device="cuda:0"),
                           torch.zeros((1, N), dtype=torch.int32, device="cuda:0"),
                           torch.as_tensor(-e[None], dtype=torch.int32, device="cuda:0"))[0]
        keys.append((s, a, e, b))
    qs = torch.as_tensor(ctx.primes, dtype=torch.int64, device="cuda:0").view(1, L, 1)

    # encrypted, resident per-client inputs of every layer
    bufs, side = [], []
    for k, (shp, ly) in enumerate(zip(shapes, v.layers)):
        first, last = k == 0, k == len(shapes) - 1
        info = ly.info
        if shp.kind == "conv":
            g = packing.conv_geometry(N, shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
            mi, yi, xi, ji, ci = _conv_pack_index(g)
            packed = torch.zeros((C, g.K_in, N), dtype=torch.int64, device="cuda:0")
            dv = lambda a: torch.as_tensor(a, dtype=torch.int64, device="cuda:0")  # noqa: E731
            packed[:, dv(ji), dv(ci)] = ins[k][:, dv(mi), dv(yi), dv(xi)]
            K_in, outshape = g.K_in, (C, g.K_out, L, N)
            shn = None if last else _draws(CFG * 1000 + k * 7 + 1, (C, g.K_out, N), "share")
        else:
            packed = torch.zeros((C, 1, N), dtype=torch.int64, device="cuda:0")
            packed[:, 0, torch.arange(fg.n_i, device="cuda:0") * fg.n_o_p] = ins[k]
            K_in, outshape = 1, (C, fg.blocks, L, fg.n_o_p)
            shn = None
        sh = None if first else _draws(CFG * 1000 + k * 7 + 2, (C, K_in, N), "share")
        i_poly = packed % T if sh is None else (packed + sh) % T
        vv = _draws(CFG * 1000 + k * 7 + 3, (C, K_in, N), "v")
        e0 = _draws(CFG * 1000 + k * 7 + 4, (C, K_in, N), "gauss")
        c0 = torch.empty((C, K_in, L, N), dtype=torch.int32, device="cuda:0")
        x1 = torch.empty_like(c0)
        zeros = torch.zeros((K_in, N), dtype=torch.int32, device="cuda:0")
        i32 = i_poly.to(torch.int32)
        for c in range(C):
            ctx.encrypt_c0(vv[c], keys[c][3], i32[c], e0[c], out=c0[c])
            ctx.encrypt_c0(vv[c], keys[c][3], i32[c], zeros, out=x1[c])      # -(v b + Delta i)
        c0p = ((qs - x1.long()) % qs).to(torch.int32)                         # v b + Delta i = -c0 - e0
        shp_ = ((T - i_poly) % T).to(torch.int32)
        if shp.kind == "conv":
            bufs.append(serve.LayerBuffers(c0, None if sh is None else sh.to(torch.int32).contiguous(),
                                           None if shn is None else shn.to(torch.int32).contiguous(),
                                           torch.empty(outshape, dtype=torch.int32, device="cuda:0")))
        else:
            bufs.append(serve.LayerBuffers(c0[:, 0].contiguous(), sh[:, 0].to(torch.int32).contiguous(), None,
                                           torch.empty(outshape, dtype=torch.int32, device="cuda:0")))
        side.append(dict(c0p=c0p, shp=shp_, sh=sh, shn=shn))
        if k in ORACLE_LAYERS:
            # the first clients: the oracle's own encryption, word for word
            side[-1]["oc0"] = []
            for c in range(min(C, ORACLE_CLIENTS)):
                s0, a0, e_0, b0 = keys[c]
                ob = bfv.keygen(octx, s0, a0, e_0)
                assert (host(b0[None])[0] == ob).all(), f"key of client {c}"
                oc0 = np.stack([bfv.encrypt_c0(octx, i_poly[c, j].cpu().numpy(), vv[c, j].cpu().numpy(),
                                               e0[c, j].cpu().numpy(), ob) for j in range(K_in)])
                assert (host(c0[c:c + 1])[0] == oc0).all(), f"encryption layer {k} client {c}"
                side[-1]["oc0"].append(oc0)
        print(f"encrypted layer {k}", flush=True)

    # the bench's stress configuration: batches of up to 64 requests, which take the matrix-core MAC
    res = serve.run_clients(v, bufs, C, streams=4, max_batch=64, budget=24 << 30, timeout_s=600)
    assert res["rc"] == 0 and (res["status"] == 0).all()
    st = serve.client_stats(res)
    print("stress stats:", st, flush=True)

    # decrypt every output of every client and compare with the integer forward pass
    for k, (shp, ly) in enumerate(zip(shapes, v.layers)):
        c0p, shp_, shn = side[k]["c0p"], side[k]["shp"], side[k]["shn"]
        out = bufs[k].out
        if shp.kind == "conv":
            g = packing.conv_geometry(N, shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
            c1 = ctx.conv_layer(ly, c0p, shp_, None)
            msg = ctx.decrypt(out.reshape(C * g.K_out, L, N), c1.reshape(C * g.K_out, L, N)).long()
            msg = msg.reshape(C, g.K_out, N)
            if shn is not None:
                msg = (msg - shn) % T
            p, kk = _conv_out_index(g)
            dec = msg[:, torch.as_tensor(p, device="cuda:0"), torch.as_tensor(kk, device="cuda:0")]
            dec = torch.where(dec > T // 2, dec - T, dec).reshape(C, g.c_o, g.H_o, g.W_o)
            assert torch.equal(dec, outs[k]), f"layer {k}: decrypted output differs from the integer conv"
            if k in ORACLE_LAYERS:
                rho = wl.mask_polys(CFG, WIDTH, k, g.K_in * g.c_o, N).reshape(g.K_in, g.c_o, N)
                ops = cserver.conv_setup(octx, rho, packing.pack_conv_filters(Ws[k], g), 0)
                for c, oc0 in enumerate(side[k]["oc0"]):
                    sh_c = None if side[k]["sh"] is None else side[k]["sh"][c].cpu().numpy()
                    shn_c = None if shn is None else shn[c].cpu().numpy()
                    want = cserver.server_conv(octx, g, oc0, ops, sh_c, shn_c, 0)
                    assert (host(out[c:c + 1])[0] == want).all(), f"server words of client {c}, layer {k}"
        else:
            c1 = ctx.fc_layer(fc_nobias, c0p[:, 0].contiguous(), shp_[:, 0].contiguous(), None)
            msg = ctx.decrypt(out.reshape(C * fg.blocks, L, fg.n_o_p), c1.reshape(C * fg.blocks, L, fg.n_o_p)).long()
            msg = msg.reshape(C, fg.blocks * fg.n_o_p)[:, :fg.n_o]
            dec = torch.where(msg > T // 2, msg - T, msg)
            assert torch.equal(dec, outs[k]), "FC: decrypted output differs from the integer FC"
            ops = cserver.fc_setup(octx, wl.mask_polys(CFG, WIDTH, 19, fg.blocks, N),
                                   packing.pack_fc_weights(Ws[-1], fg), 0)
            for c, oc0 in enumerate(side[k]["oc0"]):
                want = cserver.server_fc(octx, fg, oc0[0], ops, packing.pack_fc_bias(Bs[-1], fg),
                                         side[k]["sh"][c, 0].cpu().numpy(), None, 0)
                assert (host(out[c:c + 1])[0] == want).all(), f"server words of client {c}, FC"
        print(f"checked layer {k}", flush=True)
