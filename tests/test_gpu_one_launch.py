"""GPU parity of the one-launch layer form (forward NTT, MAC and inverse in one launch).

At N = 4096 the oracle checks, word for word, conv shapes that cover every slot stride the form
takes (s = 2 .. 256), several input polys, ragged channel groups, stride 2 and the first / last
layer patterns, and FC heads with n_o' below, at and above the 16 coefficients an item forms
(two blocks).  At the plain-20 shapes (N = 8192 and 16384) the form must give the words of the
multi-launch forms, which the oracle checks elsewhere.  Batches, the NTT-domain entry points,
the counters' reset between launches (graph replays) and the wait flag are checked too.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import bfv, packing
from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

T = wl.T_PLAIN


@pytest.fixture(scope="module")
def he():
    from paper_2409_05205_amd import he as h
    h.load_library()
    return h


@pytest.fixture(scope="module")
def ctx4096(he):
    return he.Context(4096, 3, T)


def _launches(ctx, he, fn):
    ctx.profile_reset()
    ctx.profile_enable(he.HE_K_LAYER | he.HE_K_LAYER_ROWS | he.HE_K_MAC | he.HE_K_MAC_TAIL | he.HE_K_NTT_FWD)
    out = fn()
    host(out)
    # both one-launch forms (work items: HE_K_LAYER, rows: HE_K_LAYER_ROWS)
    n_layer = ctx.profile_read(he.HE_K_LAYER)[0] + ctx.profile_read(he.HE_K_LAYER_ROWS)[0]
    n_other = sum(ctx.profile_read(k)[0] for k in (he.HE_K_MAC, he.HE_K_MAC_TAIL, he.HE_K_NTT_FWD))
    ctx.profile_enable(0)
    ctx.profile_reset()
    return out, n_layer, n_other


CONV = [
    # c_i, c_o, H, stride, f, pad        slot stride s at N = 4096
    (3, 16, 32, 1, 3, 1),    # s = 2, K_in = 2 (the single-conv workload's shape)
    (16, 16, 8, 1, 3, 1),    # s = 32
    (16, 32, 16, 2, 3, 1),   # s = 8, K_in = 2, K_out = 4, stride 2
    (5, 3, 4, 1, 3, 1),      # s = 64, ragged: g_o = 2, second group holds one channel
    (64, 64, 8, 1, 3, 1),    # s = 32, K_in = 2, K_out = 2
    (4, 8, 3, 1, 3, 1),      # s = 128
    (8, 16, 2, 1, 3, 1),     # s = 256, 16-point tail
    (20, 24, 6, 1, 3, 1),    # s = 64, K_in = 1, ragged last output group
]


@pytest.mark.parametrize("c_i,c_o,H,stride,f,pad", CONV)
@pytest.mark.parametrize("first,last", [(False, False), (True, False), (False, True)])
@pytest.mark.parametrize("form", [7, 8])
def test_one_launch_conv_matches_oracle(he, ctx4096, c_i, c_o, H, stride, f, pad, first, last, form):
    """form 7: work items of NTT sub-blocks, MAC chunks and tails; 8: whole-row transforms and one
    MAC + inverse item per output row."""
    ctx = ctx4096
    ctx.tune_force(he.HE_TUNE_MAC, form)
    N, L = ctx.N, ctx.L
    octx = bfv.make_ctx(N, L, T)
    g = packing.conv_geometry(N, c_i, c_o, H, H, f, stride, pad)
    rng = np.random.default_rng(1000 + 7 * c_i + c_o + H)
    F = rng.integers(-7, 8, (c_o, c_i, f, f))
    rho = rng.integers(0, T, (g.K_in, c_o, N))
    c0 = wl.uniform_per_modulus(rng, (g.K_in,), octx.primes, N).astype(np.uint64)
    sh = None if first else rng.integers(0, T, (g.K_in, N))
    shn = None if last else rng.integers(0, T, (g.K_out, N))
    layer = ctx.pack_conv(he.ConvSpec(c_i, c_o, H, H, f, stride, pad), F, rho)
    want = bfv.server_conv(octx, g, c0, rho, packing.pack_conv_filters(F, g), sh, shn)
    out, n_layer, n_other = _launches(ctx, he, lambda: ctx.conv_layer(
        layer, dev(c0[None]), None if sh is None else dev(sh[None]), None if shn is None else dev(shn[None])))
    ctx.tune_force(he.HE_TUNE_MAC, -1)
    print(f"conv {c_i}->{c_o} H={H} s={g.s} form {form}: one-launch={n_layer} other={n_other}", flush=True)
    assert n_layer == 1 and n_other == 0
    assert (host(out)[0] == want).all()
    ctx.sync_check()


FC = [
    # n_i, n_o              n_o', blocks at N = 4096
    (64, 10),     # 16, 1
    (64, 100),    # 64, 2: coefficient groups of 16 and two blocks
    (20, 5),      # 8, 1: fewer coefficients than an item forms
    (256, 33),    # 16, 3 blocks
]


@pytest.mark.parametrize("n_i,n_o", FC)
@pytest.mark.parametrize("with_sh,with_shn", [(True, False), (True, True), (False, True)])
def test_one_launch_fc_matches_oracle(he, ctx4096, n_i, n_o, with_sh, with_shn):
    ctx = ctx4096
    N, L = ctx.N, ctx.L
    octx = bfv.make_ctx(N, L, T)
    g = packing.fc_geometry(N, n_i, n_o)
    rng = np.random.default_rng(2000 + n_i + n_o)
    W = rng.integers(-7, 8, (n_o, n_i))
    bias = rng.integers(-7, 8, n_o)
    rho = rng.integers(0, T, (g.blocks, N))
    c0 = wl.uniform_per_modulus(rng, (), octx.primes, N).astype(np.uint64)
    sh = rng.integers(0, T, N) if with_sh else None
    shn = rng.integers(0, T, (g.blocks, g.n_o_p)) if with_shn else None
    layer = ctx.pack_fc(he.FCSpec(n_i, n_o), W, rho, bias)
    want = bfv.server_fc(octx, g, c0, rho, packing.pack_fc_weights(W, g), packing.pack_fc_bias(bias, g), sh, shn)
    out, n_layer, n_other = _launches(ctx, he, lambda: ctx.fc_layer(
        layer, dev(c0[None]), None if sh is None else dev(sh[None]), None if shn is None else dev(shn[None])))
    assert n_layer == 1 and n_other == 0          # an FC layer at B = 1 takes one launch by default
    assert (host(out)[0] == want).all()
    ctx.sync_check()


def _plain20_layer(he, ctx, shp, k, B, seed):
    N, L = ctx.N, ctx.L
    rng = np.random.default_rng(seed)
    if shp.kind == "conv":
        spec = he.ConvSpec(shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
        i = ctx.geometry(spec)
        layer = ctx.pack_conv(spec, rng.integers(-7, 8, (shp.c_o, shp.c_i, shp.f, shp.f)),
                              rng.integers(0, T, (i.K_in, shp.c_o, N)))
        c0 = np.stack([wl.uniform_per_modulus(rng, (i.K_in,), ctx.primes, N) for _ in range(B)])
        sh = None if k == 0 else rng.integers(0, T, (B, i.K_in, N))
        shn = rng.integers(0, T, (B, i.K_out, N))
    else:
        fspec = he.FCSpec(shp.n_i, shp.n_o)
        i = ctx.geometry(fspec)
        layer = ctx.pack_fc(fspec, rng.integers(-7, 8, (shp.n_o, shp.n_i)), rng.integers(0, T, (i.blocks, N)),
                            rng.integers(-7, 8, shp.n_o))
        c0 = np.stack([wl.uniform_per_modulus(rng, (), ctx.primes, N) for _ in range(B)])
        sh = rng.integers(0, T, (B, N))
        shn = None
    return layer, dev(c0), None if sh is None else dev(sh), None if shn is None else dev(shn)


def _call(ctx, layer, he, c0, sh, shn):
    return host(ctx.conv_layer(layer, c0, sh, shn) if layer.kind == he.HE_LAYER_CONV else
                ctx.fc_layer(layer, c0, sh, shn))


@pytest.mark.parametrize("width", [1, 4])
def test_one_launch_matches_multi_launch_plain20(he, width):
    """Every distinct layer shape of the x1 (N = 8192, 4 limbs) and x4 (N = 16384, 6 limbs) stacks:
    one launch against the multi-launch forms (streaming and fused MAC), word for word."""
    N, L = (8192, 4) if width == 1 else (16384, 6)
    ctx = he.Context(N, L, T)
    seen = set()
    for k, shp in enumerate(wl.plain20(width, 10 if width == 1 else 100)):
        key = (shp, k == 0)
        if key in seen:
            continue
        seen.add(key)
        layer, c0, sh, shn = _plain20_layer(he, ctx, shp, k, 1, 300 + k)
        ctx.tune_force(he.HE_TUNE_MAC, 7)
        got = _call(ctx, layer, he, c0, sh, shn)
        for form in ([0, 2, 8] if shp.kind == "conv" else [0]):
            ctx.tune_force(he.HE_TUNE_MAC, form)
            want = _call(ctx, layer, he, c0, sh, shn)
            print(f"x{width} layer {k} {shp}: one-launch vs form {form}", flush=True)
            assert (got == want).all()
        ctx.tune_force(he.HE_TUNE_MAC, -1)
        layer.free()
    ctx.sync_check()


@pytest.mark.parametrize("B", [2, 5])
@pytest.mark.parametrize("form", [7, 8])
def test_one_launch_batches(he, B, form):
    """Forced at B > 1 (each image its own items) the words equal one call per image."""
    ctx = he.Context(8192, 4, T)
    for k in (1, 7, 13, 19):
        shp = wl.plain20(1, 10)[k]
        layer, c0, sh, shn = _plain20_layer(he, ctx, shp, k, B, 400 + k)
        ctx.tune_force(he.HE_TUNE_MAC, form)
        got = _call(ctx, layer, he, c0, sh, shn)
        ctx.tune_force(he.HE_TUNE_MAC, -1)
        for b in range(B):
            one = _call(ctx, layer, he, c0[b:b + 1], None if sh is None else sh[b:b + 1],
                        None if shn is None else shn[b:b + 1])
            assert (got[b:b + 1] == one).all()
        layer.free()
    ctx.sync_check()


def test_one_launch_from_ntt_inputs(he):
    """he_conv_layer_ntt / he_fc_layer_ntt in one launch (no forward items) give he_conv_layer's words."""
    ctx = he.Context(8192, 4, T)
    for k in (0, 3, 9, 19):
        shp = wl.plain20(1, 10)[k]
        layer, c0, sh, shn = _plain20_layer(he, ctx, shp, k, 1, 500 + k)
        want = _call(ctx, layer, he, c0, sh, shn)
        x = ctx.input_buffer(layer, 1)
        ctx.inputs_ntt(layer, x, c0=c0, sh=sh)
        ctx.profile_reset()
        ctx.profile_enable(he.HE_K_LAYER)
        ctx.tune_force(he.HE_TUNE_MAC, 7)
        got = host(ctx.layer_from_ntt(layer, x, sh is not None, shn))
        ctx.tune_force(he.HE_TUNE_MAC, -1)
        assert ctx.profile_read(he.HE_K_LAYER)[0] == 1
        ctx.profile_enable(0)
        assert (got == want).all()
        layer.free()
    ctx.sync_check()


def test_one_launch_graph_replays(he):
    """A captured sequence of one-launch layers replays with the counters back at zero each time:
    every replay, with eager calls between them, gives the eager words."""
    import torch
    ctx = he.Context(8192, 4, T)
    ctx.tune_force(he.HE_TUNE_MAC, 7)
    steps = []
    for k in (0, 1, 7, 13, 19):
        shp = wl.plain20(1, 10)[k]
        steps.append(_plain20_layer(he, ctx, shp, k, 1, 600 + k))
    want = [_call(ctx, ly, he, c0, sh, shn) for ly, c0, sh, shn in steps]
    seq = he.Sequence(ctx)
    outs = [seq.add(ly, c0, sh, shn) for ly, c0, sh, shn in steps]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        seq.capture(stream)
        for rep in range(4):
            for o in outs:
                o.fill_(0)
            seq.replay(stream)
            stream.synchronize()
            for o, w in zip(outs, want):
                assert (host(o) == w).all(), f"replay {rep}"
            # eager work between replays
            _call(ctx, steps[1][0], he, *steps[1][1:])
