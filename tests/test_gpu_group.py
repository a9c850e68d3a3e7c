"""GPU parity of the grouped launch (he_group_*): independent layer calls of any contexts, shapes
and batch sizes evaluated by one kernel launch.

Small rings: one group mixes conv and FC calls of two contexts (N = 4096 with 3 limbs, N = 8192
with 2 limbs), batches of 1 to 6 images, ragged channel groups and image tiles, every first /
last-layer pattern; each image's words must equal the oracle's server evaluation (Alg. 1 /
Alg. 2), under each MAC item form (automatic, one image per item, image tiles).  Full size: one
launch holding the batch-64 layers of the x1, x2 and x4 variants (N = 8192 / 16384) must give the
oracle's stored digests of the sampled images, and plain-20 layers of both ring degrees must give
the words of the one-call path.  Repeated launches check that the counters return to zero, under
several ways of dealing the items to the XCDs and after the group's autotuner ran.
"""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import cases  # noqa: E402
import workloads as wl  # noqa: E402
from oracle import bfv, packing  # noqa: E402
from gpu_helpers import dev, host  # noqa: E402

pytestmark = pytest.mark.gpu

T = wl.T_PLAIN


@pytest.fixture(scope="module")
def he():
    from paper_2409_05205_amd import he as h
    h.load_library()
    return h


# ctx key, kind, shape, B, first, last
SMALL = [
    ("a", "conv", (3, 16, 32, 1, 3, 1), 1, True, False),     # s = 2, K_in = 2
    ("a", "conv", (16, 32, 16, 2, 3, 1), 6, False, False),   # s = 8, stride 2, K_out = 4: image tiles
    ("a", "conv", (5, 3, 4, 1, 3, 1), 5, False, True),       # s = 64, ragged channel group
    ("a", "fc", (64, 100), 2, False, False),                 # n_o' = 64, two blocks
    ("b", "conv", (16, 16, 16, 1, 3, 1), 4, False, False),   # N = 8192: s = 16
    ("b", "conv", (20, 24, 6, 1, 3, 1), 3, True, False),     # s = 128 at N = 8192, ragged last group
    ("b", "fc", (64, 10), 1, False, True),
]


def _small_case(he, ctxs, octxs, i, key, kind, shape, B, first, last):
    ctx, octx = ctxs[key], octxs[key]
    N = ctx.N
    rng = np.random.default_rng(7000 + 13 * i)
    if kind == "conv":
        c_i, c_o, H, stride, f, pad = shape
        g = packing.conv_geometry(N, c_i, c_o, H, H, f, stride, pad)
        F = rng.integers(-7, 8, (c_o, c_i, f, f))
        rho = rng.integers(0, T, (g.K_in, c_o, N))
        c0 = np.stack([wl.uniform_per_modulus(rng, (g.K_in,), octx.primes, N) for _ in range(B)])
        sh = None if first else rng.integers(0, T, (B, g.K_in, N))
        shn = None if last else rng.integers(0, T, (B, g.K_out, N))
        layer = ctx.pack_conv(he.ConvSpec(c_i, c_o, H, H, f, stride, pad), F, rho)
        fh = packing.pack_conv_filters(F, g)
        want = [bfv.server_conv(octx, g, c0[b].astype(np.uint64), rho, fh, None if sh is None else sh[b],
                                None if shn is None else shn[b]) for b in range(B)]
    else:
        n_i, n_o = shape
        g = packing.fc_geometry(N, n_i, n_o)
        W = rng.integers(-7, 8, (n_o, n_i))
        bias = rng.integers(-7, 8, n_o)
        rho = rng.integers(0, T, (g.blocks, N))
        c0 = np.stack([wl.uniform_per_modulus(rng, (), octx.primes, N) for _ in range(B)])
        sh = None if first else rng.integers(0, T, (B, N))
        shn = None if last else rng.integers(0, T, (B, g.blocks, g.n_o_p))
        layer = ctx.pack_fc(he.FCSpec(n_i, n_o), W, rho, bias)
        w, d = packing.pack_fc_weights(W, g), packing.pack_fc_bias(bias, g)
        want = [bfv.server_fc(octx, g, c0[b].astype(np.uint64), rho, w, d, None if sh is None else sh[b],
                              None if shn is None else shn[b]) for b in range(B)]
    args = (layer, dev(c0), None if sh is None else dev(sh), None if shn is None else dev(shn))
    return args, want


@pytest.mark.parametrize("flags", [0, 1, 2], ids=["auto", "per_image", "tiled"])
def test_group_small_rings_match_oracle(he, flags):
    ctxs = {"a": he.Context(4096, 3, T), "b": he.Context(8192, 2, T)}
    octxs = {k: bfv.make_ctx(c.N, c.L, T) for k, c in ctxs.items()}
    grp = he.Group()
    outs, wants = [], []
    for i, case in enumerate(SMALL):
        args, want = _small_case(he, ctxs, octxs, i, *case)
        outs.append(grp.add(*args))
        wants.append(want)
    grp.build(flags)
    items, tiled, ws = grp.items()
    print(f"flags {flags}: items {items} tiled calls {tiled} workspace {ws}", flush=True)
    if flags == 1:
        assert tiled == 0
    if flags == 2:
        assert tiled == sum(1 for c in SMALL if c[1] == "conv")
    # three launches in a row, with the items dealt to the XCDs in chunks of 64, 1 and 1024
    for rep, chunk_log in enumerate((6, 0, 10)):
        for o in outs:
            o.fill_(-1)
        grp.set_chunk(chunk_log)
        grp.run()
        grp.check()
        for i, (o, want) in enumerate(zip(outs, wants)):
            got = host(o)
            for b, w in enumerate(want):
                assert (got[b] == w).all(), f"launch {rep} call {i} {SMALL[i]} image {b}"
    grp.free()


def _gold():
    with open(os.path.join(HERE, "golden", "server_digests.json")) as f:
        return json.load(f)["cases"]


def test_group_batched_widths_one_launch(he):
    """The batch-64 sample layers of the x1, x2 and x4 variants in ONE launch (two ring degrees,
    image-tiled MAC items): the sampled images give the oracle's digests, twice in a row."""
    gold = _gold()
    ctxs = {}
    grp = he.Group()
    outs = []
    for name, cfg, width, classes, N, L, k, B, images in cases.BATCHED_SAMPLES:
        if (N, L) not in ctxs:
            ctxs[(N, L)] = he.Context(N, L, T)
        ctx = ctxs[(N, L)]
        inp = cases.batched_layer_inputs(cfg, width, classes, k, B, N, ctx.primes)
        g = inp["geom"]
        layer = ctx.pack_conv(he.ConvSpec(g.c_i, g.c_o, g.H, g.W, g.f, g.stride, g.pad), inp["F"], inp["rho"])
        out = grp.add(layer, dev(inp["c0"]), dev(inp["sh"]), dev(inp["sh_next"]))
        outs.append((name, images, out))
    grp.build()
    items, tiled, ws = grp.items()
    chunk_log = grp.tune()
    print(f"items {items} tiled calls {tiled} workspace {ws / 2**20:.0f} MiB, tuned chunk 2^{chunk_log}", flush=True)
    assert tiled == len(cases.BATCHED_SAMPLES) and 2 <= chunk_log <= 8
    for _, _, out in outs:
        out.fill_(-1)
    for rep in range(2):
        grp.run()
        grp.check()
        for name, images, out in outs:
            got = host(out)
            for b in images:
                assert cases.digest(got[b]) == gold[name]["images"][str(b)], f"launch {rep} {name} image {b}"
    grp.free()


def _plain20_call(he, ctx, shp, k, B, seed):
    N = ctx.N
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


@pytest.mark.parametrize("flags", [0, 2], ids=["auto", "tiled"])
def test_group_plain20_matches_layer_calls(he, flags):
    """Every distinct layer shape of the x1 (N = 8192, 4 limbs, B = 3) and x4 (N = 16384, 6 limbs,
    B = 2) stacks in one group: the words of one layer call each (the oracle checks those)."""
    grp = he.Group()
    calls = []
    for width, N, L, B in ((1, 8192, 4, 3), (4, 16384, 6, 2)):
        ctx = he.Context(N, L, T)
        seen = set()
        for k, shp in enumerate(wl.plain20(width, 10 if width == 1 else 100)):
            key = (shp, k == 0)
            if key in seen:
                continue
            seen.add(key)
            layer, c0, sh, shn = _plain20_call(he, ctx, shp, k, B, 900 + 31 * width + k)
            calls.append((width, k, ctx, layer, c0, sh, shn, grp.add(layer, c0, sh, shn)))
    grp.build(flags)
    print(f"{len(calls)} calls, items {grp.items()}", flush=True)
    grp.run()
    grp.check()
    for width, k, ctx, layer, c0, sh, shn, out in calls:
        want = host(ctx.conv_layer(layer, c0, sh, shn) if layer.kind == he.HE_LAYER_CONV else
                    ctx.fc_layer(layer, c0, sh, shn))
        print(f"x{width} layer {k}", flush=True)
        assert (host(out) == want).all()
    grp.free()


def test_group_rejects_full_intt_layers(he):
    """A conv layer packed for the full-length inverse is outside the grouped launch: refused at
    creation with HE_EUNSUPPORTED, before anything runs."""
    ctx = he.Context(4096, 2, T)
    rng = np.random.default_rng(5)
    spec = he.ConvSpec(3, 8, 8, 8, 3, 1, 1)
    i = ctx.geometry(spec)
    layer = ctx.pack_conv(spec, rng.integers(-7, 8, (8, 3, 3, 3)), rng.integers(0, T, (i.K_in, 8, 4096)),
                          flags=he.HE_PACK_FULL_INTT)
    c0 = dev(np.stack([wl.uniform_per_modulus(rng, (i.K_in,), ctx.primes, 4096)]))
    grp = he.Group()
    grp.add(layer, c0)
    with pytest.raises(he.HEError) as e:
        grp.build()
    assert e.value.code == he.HE_EUNSUPPORTED


def test_group_rejects_invalid_calls(he):
    """Invalid calls are refused at creation with HE_EINVAL before anything runs: a layer of
    another context, a batch of zero, a missing output, an unknown MAC flag."""
    ctx_a, ctx_b = he.Context(4096, 2, T), he.Context(4096, 2, T)
    rng = np.random.default_rng(9)
    spec = he.ConvSpec(3, 8, 8, 8, 3, 1, 1)
    i = ctx_a.geometry(spec)
    layer = ctx_a.pack_conv(spec, rng.integers(-7, 8, (8, 3, 3, 3)), rng.integers(0, T, (i.K_in, 8, 4096)))
    c0 = dev(np.stack([wl.uniform_per_modulus(rng, (i.K_in,), ctx_a.primes, 4096)]))
    out = dev(np.zeros((1, i.K_out, 2, 4096), dtype=np.int64))
    lib = he.load_library()
    import ctypes

    def create(calls, flags=0):
        arr = (he.LayerCall * len(calls))(*calls)
        h = ctypes.c_void_p()
        rc = lib.he_group_create(arr, len(calls), flags, ctypes.byref(h))
        if rc == he.HE_OK:
            lib.he_group_free(h)
        return rc

    good = he.LayerCall(ctx_a.handle, layer.handle, 1, c0.data_ptr(), None, None, out.data_ptr())
    assert create([good]) == he.HE_OK
    assert create([he.LayerCall(ctx_b.handle, layer.handle, 1, c0.data_ptr(), None, None, out.data_ptr())]) == \
        he.HE_EINVAL
    assert create([he.LayerCall(ctx_a.handle, layer.handle, 0, c0.data_ptr(), None, None, out.data_ptr())]) == \
        he.HE_EINVAL
    assert create([he.LayerCall(ctx_a.handle, layer.handle, 1, c0.data_ptr(), None, None, None)]) == he.HE_EINVAL
    assert create([good], flags=7) == he.HE_EINVAL
    assert lib.he_group_create(None, 0, 0, ctypes.byref(ctypes.c_void_p())) == he.HE_EINVAL


def test_group_graph_replays(he):
    """A grouped launch captured into a HIP graph: every replay, with eager work between the
    replays, gives the words of the eager launch (the counters return to zero inside the launch,
    so the graph needs no memset node)."""
    import torch
    ctxs = {"a": he.Context(4096, 3, T), "b": he.Context(8192, 2, T)}
    octxs = {k: bfv.make_ctx(c.N, c.L, T) for k, c in ctxs.items()}
    grp = he.Group()
    outs, wants = [], []
    for i, case in enumerate(SMALL):
        args, want = _small_case(he, ctxs, octxs, i, *case)
        outs.append(grp.add(*args))
        wants.append(want)
    grp.build()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        grp.run(stream)            # eager launch first (nothing is allocated during capture either way)
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        grp.run(stream)
    stream.synchronize()
    other_args, other_want = _small_case(he, ctxs, octxs, 99, "a", "conv", (16, 16, 16, 1, 3, 1), 2, False, False)
    for rep in range(4):
        for o in outs:
            o.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        # eager work between the replays
        other = host(ctxs["a"].conv_layer(*other_args))
        for b, w in enumerate(other_want):
            assert (other[b] == w).all()
        for i, (o, want) in enumerate(zip(outs, wants)):
            got = host(o)
            for b, w in enumerate(want):
                assert (got[b] == w).all(), f"replay {rep} call {i} image {b}"
    grp.check(stream)
    grp.free()
