"""GPU tests of the continuous-batching server (he_server_*).

Every request's output words must equal a lone layer call on the same inputs,
whether it ran alone, batched with others of its layer, or overlapped with
other layers on other streams; a budget that only fits one request at a time
still completes every request; a budget too small for a layer fails exactly
the requests of that layer with HE_ENOMEM.
"""
import numpy as np
import pytest

import workloads as wl
from gpu_helpers import host

pytestmark = pytest.mark.gpu

T = wl.T_PLAIN


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2409_05205_amd import he, serve
    N, L = 1024, 2
    ctx = he.Context(N, L, T)
    rng = np.random.default_rng(4)
    shapes = [wl.ConvShape(3, 16, 6, 6), wl.ConvShape(16, 16, 6, 6), wl.ConvShape(16, 32, 6, 6, stride=2),
              wl.FCShape(32, 10)]
    v = serve.Variant(1, 10, ctx, shapes)
    for shp in shapes:
        if shp.kind == "conv":
            spec = he.ConvSpec(shp.c_i, shp.c_o, shp.H, shp.W, 3, shp.stride, 1)
            til = ctx.geometry(spec)
            v.layers.append(ctx.pack_conv(spec, rng.integers(-7, 8, (shp.c_o, shp.c_i, 3, 3)),
                                          rng.integers(0, T, (til.K_in, shp.c_o, N))))
        else:
            v.layers.append(ctx.pack_fc(he.FCSpec(32, 10), rng.integers(-7, 8, (10, 32)),
                                        rng.integers(0, T, (1, N)), rng.integers(-7, 8, 10)))
    clients = 6
    bufs = serve.client_buffers(v, clients, seed=7)
    # references: lone calls, one per (client, layer)
    ref = []
    for ly, b in zip(v.layers, bufs):
        per = []
        for cl in range(clients):
            sl = slice(cl, cl + 1)
            if ly.kind == he.HE_LAYER_CONV:
                o = ctx.conv_layer(ly, b.c0[sl], None if b.sh is None else b.sh[sl], None if b.shn is None else b.shn[sl])
            else:
                o = ctx.fc_layer(ly, b.c0[sl], None if b.sh is None else b.sh[sl], None if b.shn is None else b.shn[sl])
            per.append(host(o)[0])
        ref.append(per)
    torch.cuda.synchronize()
    return dict(he=he, serve=serve, ctx=ctx, v=v, bufs=bufs, ref=ref, clients=clients)


def _trace_once(setup, arrival):
    """Each (client, layer) pair at most once, in a shuffled order."""
    pairs = [(k, cl) for k in range(len(setup["v"].layers)) for cl in range(setup["clients"])]
    rng = np.random.default_rng(len(arrival))
    rng.shuffle(pairs)
    pairs = pairs[: len(arrival)]
    return np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs])


def _check(setup, res, ltype, client, expect_ok=None):
    bufs, ref = setup["bufs"], setup["ref"]
    for i, (k, cl) in enumerate(zip(ltype, client)):
        if expect_ok is not None and not expect_ok(k):
            continue
        assert res["status"][i] == 0
        got = host(bufs[k].out[cl])
        assert (got == ref[k][cl]).all(), f"request {i} layer {k} client {cl}"
        assert res["complete"][i] >= res["dispatch"][i] >= res["arrival"][i] - 1e-6


def _clear(setup):
    for b in setup["bufs"]:
        b.out.fill_(-1)


@pytest.mark.parametrize("streams,max_batch", [(1, 1), (3, 8), (4, 2)])
def test_burst_batches_and_matches_lone_calls(setup, streams, max_batch):
    _clear(setup)
    n = 24
    arrival = np.zeros(n)
    ltype, client = _trace_once(setup, arrival)
    res = setup["serve"].run_trace([setup["v"]], [setup["bufs"]], arrival, ltype, client, streams, max_batch,
                                   1 << 30, timeout_s=60)
    assert res["rc"] == 0
    if max_batch > 1:
        assert res["batch"].max() > 1          # the burst was batched
    else:
        assert res["batch"].max() == 1
    _check(setup, res, ltype, client)


def test_poisson_trace_matches_lone_calls(setup):
    _clear(setup)
    n = 24
    arrival = np.cumsum(np.random.default_rng(1).exponential(2e-4, n))
    ltype, client = _trace_once(setup, arrival)
    res = setup["serve"].run_trace([setup["v"]], [setup["bufs"]], arrival, ltype, client, 4, 4, 1 << 30,
                                   timeout_s=60)
    assert res["rc"] == 0
    _check(setup, res, ltype, client)


def test_budget_for_one_request_serialises(setup):
    _clear(setup)
    v = setup["v"]
    need = max(ly.workspace_bytes(1) for ly in v.layers) + 4096
    n = 12
    arrival = np.zeros(n)
    ltype, client = _trace_once(setup, arrival)
    res = setup["serve"].run_trace([v], [setup["bufs"]], arrival, ltype, client, 4, 8, need, timeout_s=60)
    assert res["rc"] == 0
    _check(setup, res, ltype, client)


def test_budget_too_small_fails_that_layer_only(setup):
    _clear(setup)
    v = setup["v"]
    sizes = [ly.workspace_bytes(1) for ly in v.layers]
    big = int(np.argmax(sizes))
    budget = sorted(sizes)[-2] + 4096          # fits every layer but the largest
    assert budget < sizes[big]
    n = 16
    arrival = np.zeros(n)
    ltype, client = _trace_once(setup, arrival)
    res = setup["serve"].run_trace([v], [setup["bufs"]], arrival, ltype, client, 2, 1, budget, timeout_s=60)
    he = setup["he"]
    for i, k in enumerate(ltype):
        if k == big:
            assert res["status"][i] == he.HE_ENOMEM
    assert (ltype == big).any() and (ltype != big).any()
    _check(setup, res, ltype, client, expect_ok=lambda k: k != big)
