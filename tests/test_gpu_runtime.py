"""GPU tests of the layer-sequence runtime: eager run and hipGraph replay must give
the words of one-call-per-layer execution, on every replay, with other eager
device work (output clobbering, allocations) between the replays."""
import numpy as np
import pytest

import workloads as wl
from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

T = wl.T_PLAIN


def _build(he, ctx, N, L, rng):
    steps = []
    shapes = [(4, 16, 6, 1), (16, 16, 6, 1), (16, 32, 6, 2)]
    for k, (ci, co, H, st) in enumerate(shapes):
        spec = he.ConvSpec(ci, co, H, H, 3, st, 1)
        til = ctx.geometry(spec)
        ly = ctx.pack_conv(spec, rng.integers(-7, 8, (co, ci, 3, 3)), rng.integers(0, T, (til.K_in, co, N)),
                           flags=k % 2)
        B = 3
        c0 = dev(np.stack([wl.uniform_per_modulus(rng, (til.K_in,), ctx.primes, N) for _ in range(B)]))
        sh = None if k == 0 else dev(rng.integers(0, T, (B, til.K_in, N)))
        shn = dev(rng.integers(0, T, (B, til.K_out, N)))
        steps.append((ly, c0, sh, shn))
    fly = ctx.pack_fc(he.FCSpec(32, 10), rng.integers(-7, 8, (10, 32)), rng.integers(0, T, (1, N)),
                      rng.integers(-7, 8, 10))
    c0 = dev(np.stack([wl.uniform_per_modulus(rng, (), ctx.primes, N) for _ in range(2)]))
    steps.append((fly, c0, dev(rng.integers(0, T, (2, N))), None))
    return steps


def test_sequence_and_graph_match_per_layer_calls():
    import torch
    from paper_2409_05205_amd import he
    N, L = 1024, 2
    ctx = he.Context(N, L, T)
    rng = np.random.default_rng(9)
    steps = _build(he, ctx, N, L, rng)
    want = []
    for ly, c0, sh, shn in steps:
        if ly.kind == he.HE_LAYER_CONV:
            want.append(host(ctx.conv_layer(ly, c0, sh, shn)))
        else:
            want.append(host(ctx.fc_layer(ly, c0, sh, shn)))
    stream = torch.cuda.Stream()
    seq = he.Sequence(ctx)
    outs = [seq.add(ly, c0, sh, shn) for ly, c0, sh, shn in steps]
    assert len(seq) == len(steps)
    with torch.cuda.stream(stream):
        seq.run(stream)
    stream.synchronize()
    for o, w in zip(outs, want):
        assert (host(o) == w).all()
    gseq = he.Sequence(ctx)
    gouts = [gseq.add(ly, c0, sh, shn) for ly, c0, sh, shn in steps]
    with torch.cuda.stream(stream):
        gseq.capture(stream)
    for rep in range(4):
        for o in gouts:
            o.fill_(-1)                      # eager work between replays
        scratch = torch.randint(0, 100, (1 << 20,), device="cuda:0")
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            gseq.replay(stream)
        stream.synchronize()
        for o, w in zip(gouts, want):
            assert (host(o) == w).all(), f"replay {rep}"
        del scratch


def test_kernel_timing_counts_launches():
    from paper_2409_05205_amd import he
    N, L = 1024, 2
    ctx = he.Context(N, L, T)
    rng = np.random.default_rng(2)
    steps = _build(he, ctx, N, L, rng)
    ctx.profile_reset()
    ctx.profile_enable(he.HE_K_MAC | he.HE_K_NTT_FWD | he.HE_K_TAIL | he.HE_K_INTT)
    for ly, c0, sh, shn in steps:
        if ly.kind == he.HE_LAYER_CONV:
            ctx.conv_layer(ly, c0, sh, shn)
        else:
            ctx.fc_layer(ly, c0, sh, shn)
    n_mac, ms = ctx.profile_read(he.HE_K_MAC)
    assert n_mac == 4 and ms > 0
    n_fwd, _ = ctx.profile_read(he.HE_K_NTT_FWD)
    assert n_fwd == 4                   # one launch per layer: c0, and sh when present, together
    n_tail, _ = ctx.profile_read(he.HE_K_TAIL)
    n_intt, _ = ctx.profile_read(he.HE_K_INTT)
    assert n_tail + n_intt == 4
    ctx.profile_enable(0)
    ctx.profile_reset()
    assert ctx.profile_read(he.HE_K_MAC)[0] == 0
