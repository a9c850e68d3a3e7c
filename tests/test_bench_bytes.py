"""The algorithmic byte and operation counts bench.py divides by measured times, checked against
hand counts of one residue-class conv layer and one FC layer (no GPU: the counts read only
layer geometry)."""
import bench


class _Info:
    def __init__(self, **k):
        self.__dict__.update(k)


class _Layer:
    def __init__(self, kind, info):
        self.kind = kind
        self.info = info


class _Ctx:
    L = 4
    N = 8192


def _stack():
    st = bench.Stack.__new__(bench.Stack)
    st.ctx = _Ctx()
    share = object()   # any non-None tensor stands for a present share
    # conv 16 -> 16 at 32 x 32 (s = 4, K_in = K_out = 4), 64 images, with sh and sh'; FC block of
    # n_o' = 16 rows, 32 inputs, with sh and without sh'
    st.steps = [(_Layer(0, _Info(K_in=4, K_out=4, s=4, flags=0, n_o_p=0)), 64, None, share, share),
                (_Layer(1, _Info(K_in=1, K_out=0, s=0, flags=0, n_o_p=16)), 32, None, share, None)]
    st.rows = [16, 1]
    return st


def test_forward_bytes():
    L, N = 4, 8192
    conv = 64 * 4 * L * N * 8 + 64 * 4 * N * 4 + 64 * 4 * L * N * 4    # c0 rows r+w; sh read once, written per limb
    fc = 32 * L * N * 8 + 32 * N * 4 + 32 * L * N * 4
    assert _stack().fwd_bytes() == conv + fc


def test_inverse_bytes():
    L, N, M = 4, 8192, 8192 // 4
    conv = 64 * 16 * L * M * 4 + 64 * 4 * L * N * 4 + 64 * 4 * N * 4     # block sums, out, sh'
    fc = 32 * 1 * L * N * 4 + 32 * 1 * L * 16 * 4                        # MAC rows in, n_o' out
    assert _stack().inverse_bytes() == conv + fc


def test_mac_bytes_and_counts():
    L, N, M = 4, 8192, 8192 // 4
    st = _stack()
    conv = 8 * 16 * L * N * 4 + 64 * 8 * L * N * 4 + 64 * 16 * L * M * 4   # operands, inputs, block sums
    fc = 2 * 1 * L * N * 4 + 32 * 2 * L * N * 4 + 32 * 1 * L * N * 4
    assert st.mac_kernel_bytes(["split", "split"]) == conv + fc
    # the matrix-core MAC reads and writes what the split one does (block sums, not outputs)
    assert st.mac_kernel_bytes(["mfma", "split"]) == conv + fc
    assert st.mac_kernel_bytes(["mfma", "split"], only=[True, False]) == conv
    assert st.modmuls() == 64 * 8 * 16 * L * N + 32 * 2 * 1 * L * N
    assert st.butterflies_fwd() == (64 * 4 * L * 2 + 32 * L * 2) * (N // 2) * 13
    assert st.tail_butterflies() == 64 * 16 * L * (M // 2) * 11 + 32 * 1 * L * (N // 2) * 13


def _sha(files):
    import hashlib
    import os
    h = hashlib.sha256()
    for src in files:
        with open(os.path.join(bench.ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _current(kind):
    """The counter record with the hash of every form set to the sources as they are now."""
    rec = dict(bench.PMC_TRAFFIC[kind])
    if "forms" in rec:
        rec["forms"] = {c: dict(f, sha256=_sha(f["sources"])) for c, f in rec["forms"].items()}
    else:
        rec["sha256"] = _sha(rec["sources"])
    return rec


def test_counter_traffic_follows_the_per_layer_forms(monkeypatch):
    monkeypatch.setitem(bench.PMC_TRAFFIC, "layers", _current("layers"))
    table = bench.PMC_TRAFFIC["layers"]["per_layer"]
    n = len(table)
    split = "S" * n
    assert bench.pmc_traffic("layers", split) == round(sum(r["S"] for r in table) / n)
    mixed = "F" + "S" * (n - 2) + "S"
    want = (table[0]["F"] + sum(r["S"] for r in table[1:])) / n
    assert bench.pmc_traffic("layers", mixed) == round(want)
    # a selection: the one-launch layers of a plan apart from the multi-launch ones
    plan = "O" + "S" * (n - 2) + "O"
    one = [c == "O" for c in plan]
    assert bench.pmc_traffic("layers", plan, one) == round((table[0]["O"] + table[-1]["O"]) / 2)
    assert bench.pmc_traffic("layers", plan, [not o for o in one]) == round(
        sum(r["S"] for r in table[1:-1]) / (n - 2))
    # the FC head has no fused form, a plan of the wrong length matches nothing
    assert table[-1]["F"] is None
    assert bench.pmc_traffic("layers", "F" * n) is None
    assert bench.pmc_traffic("layers", split[:-1]) is None
    assert bench.pmc_traffic("layers") is None
    # a kernel source changed since the counters were taken: only that form's entries go
    rec = _current("layers")
    rec["forms"]["F"] = dict(rec["forms"]["F"], sha256="0" * 64)
    monkeypatch.setitem(bench.PMC_TRAFFIC, "layers", rec)
    assert bench.pmc_traffic("layers", split) is not None
    assert bench.pmc_traffic("layers", mixed) is None
    monkeypatch.setitem(bench.PMC_TRAFFIC, "ntt_fwd", dict(bench.PMC_TRAFFIC["ntt_fwd"], sha256="0" * 64))
    assert bench.pmc_traffic("ntt_fwd") is None
    monkeypatch.setitem(bench.PMC_TRAFFIC, "ntt_fwd", _current("ntt_fwd"))
    assert bench.pmc_traffic("ntt_fwd") == bench.PMC_TRAFFIC["ntt_fwd"]["bytes_per_launch"]

