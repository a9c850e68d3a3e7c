"""Pins for oracle.counts: the communication formulas of Table II against all 16 printed cells,
and the per-layer operation counts of the generalised packing against Table I / Table III in the
paper's own setting.  The benchmark's algorithmic operation counts are checked against the same
per-layer counts on the plain-20 x1 stack (no GPU: counts read only geometry)."""
import json
import os

import pytest

import workloads as wl
from oracle import counts, packing

HERE = os.path.dirname(os.path.abspath(__file__))


def _decimals(v: float) -> int:
    s = repr(v)
    return len(s.split(".")[1]) if "." in s else 0


def test_table2_formulas_reproduce_every_printed_cell():
    fix = json.load(open(os.path.join(HERE, "golden", "table2_comm_mb.json")))
    checked = 0
    for row in fix["rows"]:
        for design in ("gazelle", "cheetah", "convfhe", "proposed"):
            mb = counts.table2_comm_bytes(design, row["w"], row["c_i"], row["c_o"]) / 1e6
            printed = row[design]
            assert round(mb, _decimals(printed)) == pytest.approx(printed), (design, row)
            checked += 1
    assert checked == 16


def test_table2_detects_a_wrong_formula():
    """Planted mistake: the output polynomials priced at the input width (log Q' taken as log Q)
    must miss the printed cell."""
    row = json.load(open(os.path.join(HERE, "golden", "table2_comm_mb.json")))["rows"][3]
    mb = counts.table2_comm_bytes("proposed", row["w"], row["c_i"], row["c_o"], log_qp=104) / 1e6
    assert round(mb, 2) != row["proposed"]


# The paper's setting of Table I: N = c_i w^2, c_o divides c_i, valid (no) padding.
PAPER_CONV = [(256, 16, 4, co) for co in (1, 2, 4, 8, 16)] + [(1024, 64, 4, 16), (4096, 16, 16, 4),
                                                              (8192, 128, 8, 32)]


@pytest.mark.parametrize("N,c_i,w,c_o", PAPER_CONV)
def test_conv_counts_reduce_to_table1(N, c_i, w, c_o):
    g = packing.conv_geometry(N, c_i, c_o, w, w, 3, 1, 0)
    assert g.K_in == 1 and g.s == c_i and g.g_o == c_o
    server, _ = counts.table1_conv(c_o)
    # the paper's protocol: c0 arrives as NTT(c0), the server transforms its share only
    assert counts.conv_layer_counts(g, first_layer=False, c0_in_ntt_form=True) == server
    # reading R9 (c0 in coefficient form at the boundary): one more forward transform
    r9 = counts.conv_layer_counts(g, first_layer=False, c0_in_ntt_form=False)
    assert (r9.ntt, r9.intt, r9.cwm) == (server.ntt + 1, server.intt, server.cwm)
    assert counts.table1_conv_memory(c_o)[0] == 2 * c_o + 1


@pytest.mark.parametrize("N,n_i,n_o", [(8192, 64, 10), (8192, 512, 100), (16384, 256, 100), (8, 4, 2),
                                       (4096, 1024, 64)])
def test_fc_counts_reduce_to_table3(N, n_i, n_o):
    g = packing.fc_geometry(N, n_i, n_o)
    server, _ = counts.table3_fc(N, n_i, n_o)
    assert counts.fc_layer_counts(g, first_layer=False, c0_in_ntt_form=True) == server
    assert counts.table3_fc_memory(N, n_i, n_o)[0] == 2 * N * g.blocks


def test_bench_operation_counts_match_layer_counts():
    """bench.py's MAC products and forward butterflies for the x1 stack at one image equal the
    per-layer counts (coefficient-form c0, as the benchmark runs it) times N, L and (N/2) log2 N."""
    import bench

    class _Info:
        def __init__(self, **k):
            self.__dict__.update(k)

    class _Layer:
        def __init__(self, kind, info):
            self.kind, self.info = kind, info

    class _Ctx:
        N, L = 8192, 4

    N, L = 8192, 4
    st = bench.Stack.__new__(bench.Stack)
    st.ctx = _Ctx()
    st.steps, st.rows = [], []
    share = object()
    cwm = ntt = 0
    layers = wl.plain20(1, 10)
    for k, shp in enumerate(layers):
        first, last = k == 0, k == len(layers) - 1
        if shp.kind == "conv":
            g = packing.conv_geometry(N, shp.c_i, shp.c_o, shp.H, shp.W, shp.f, shp.stride, shp.pad)
            info = _Info(K_in=g.K_in, K_out=g.K_out, s=g.s, flags=0, n_o_p=0)
            st.steps.append((_Layer(0, info), 1, None, None if first else share, None if last else share))
            st.rows.append(shp.c_o)
            c = counts.conv_layer_counts(g, first, c0_in_ntt_form=False)
        else:
            g = packing.fc_geometry(N, shp.n_i, shp.n_o)
            info = _Info(K_in=1, K_out=0, s=0, flags=0, n_o_p=g.n_o_p)
            st.steps.append((_Layer(1, info), 1, None, share, None))
            st.rows.append(g.blocks)
            c = counts.fc_layer_counts(g, False, c0_in_ntt_form=False)
        cwm += c.cwm
        ntt += c.ntt
    assert st.modmuls() == cwm * N * L
    assert st.butterflies_fwd() == ntt * L * (N // 2) * 13
