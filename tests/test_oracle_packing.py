"""Pins for the conv / FC packing and the integer layer references.

* conv2d is checked against an explicit loop over Eq. batch_conv_formula and a
  closed form (all-ones input and filters count the in-bounds taps).
* The generalised conv packing is checked by brute force in Z[X]/(X^N+1): the
  coefficient s (sigma oy W_p + sigma ox) + o_n of sum_j i_j f_j^(n) must be
  the integer convolution (Eq. batch_conv_formula, cross-correlation).
* In the paper's own setting (N = c_i w^2, c_o | c_i, valid padding) the packed
  polynomials are checked against Eq. i_batch and Eq. k_batch_new typed in
  with ConvFHE's exponents, up to the fixed monomial shift between the two
  exponent conventions.
* FC packing is checked by brute force of Theorem 1, including the Fig. 5
  shape n_i = 4, n_o = 2 with N = n_i n_o.
* The ResNet-50 stride-2 1x1 projections packed on the subsampled map: the
  subsampled conv equals the strided one (brute force), and the HE layer on the
  subsampled map decrypts to the strided conv of the full map.
"""
import itertools

import numpy as np
import pytest

import workloads as wl
from oracle import bfv, network, packing


def int_negacyclic(a, b):
    """Exact product in Z[X]/(X^N + 1) (integer linear convolution folded)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    N = a.shape[0]
    lin = np.convolve(a, b)
    out = lin[:N].copy()
    out[: N - 1] -= lin[N:]
    return out


def monomial_shift(a, e):
    """a(X) * X^e in Z[X]/(X^N + 1) for any integer e."""
    a = np.asarray(a, dtype=np.int64)
    N = a.shape[0]
    out = np.zeros(N, dtype=np.int64)
    for i, c in enumerate(a):
        if c == 0:
            continue
        k = i + e
        sign = 1
        q, r = divmod(k, N)        # X^(qN + r) = (-1)^q X^r
        if q % 2:
            sign = -1
        out[r] += sign * c
    return out


def loop_conv(img, F, stride, pad):
    c_o, c_i, f, _ = F.shape
    H, W = img.shape[1:]
    Ho = (H + 2 * pad - f) // stride + 1
    Wo = (W + 2 * pad - f) // stride + 1
    out = np.zeros((c_o, Ho, Wo), dtype=np.int64)
    for n, y, x in itertools.product(range(c_o), range(Ho), range(Wo)):
        acc = 0
        for m, ky, kx in itertools.product(range(c_i), range(f), range(f)):
            yy, xx = stride * y + ky - pad, stride * x + kx - pad
            if 0 <= yy < H and 0 <= xx < W:
                acc += int(F[n, m, ky, kx]) * int(img[m, yy, xx])
        out[n, y, x] = acc
    return out


@pytest.mark.parametrize("c_i,c_o,H,f,stride,pad", [(3, 4, 5, 3, 1, 1), (2, 3, 6, 3, 2, 1), (4, 2, 7, 5, 1, 2),
                                                    (1, 1, 4, 3, 1, 0)])
def test_conv2d_matches_loops(c_i, c_o, H, f, stride, pad):
    rng = np.random.default_rng(c_i * 10 + H)
    img = rng.integers(0, 16, (c_i, H, H))
    F = rng.integers(-7, 8, (c_o, c_i, f, f))
    assert (network.conv2d(img, F, stride, pad) == loop_conv(img, F, stride, pad)).all()


def test_conv2d_closed_form_ones():
    img = np.ones((2, 4, 4), dtype=np.int64)
    F = np.ones((1, 2, 3, 3), dtype=np.int64)
    out = network.conv2d(img, F, 1, 1)[0]
    # taps inside the image: corner 4, edge 6, interior 9, times 2 channels
    expect = 2 * np.array([[4, 6, 6, 4], [6, 9, 9, 6], [6, 9, 9, 6], [4, 6, 6, 4]])
    assert (out == expect).all()


CONV_CASES = [
    # N, c_i, c_o, H, f, stride, pad
    (256, 3, 8, 4, 3, 1, 1),     # c_o > c_i, one input poly
    (256, 6, 4, 4, 3, 1, 1),     # K_in = 2
    (256, 4, 8, 4, 3, 2, 1),     # stride 2, K_out = 2
    (256, 2, 2, 6, 3, 1, 1),
    (512, 5, 3, 5, 3, 1, 1),     # ragged channel tail (c_i not a multiple of g_i)
    (1024, 16, 16, 6, 3, 2, 1),  # K_in = 2 at stride 2
    (256, 4, 4, 6, 5, 1, 0),     # valid padding, f = 5
]


@pytest.mark.parametrize("N,c_i,c_o,H,f,stride,pad", CONV_CASES)
def test_conv_packing_brute_force(N, c_i, c_o, H, f, stride, pad):
    g = packing.conv_geometry(N, c_i, c_o, H, H, f, stride, pad)
    assert g.s * g.H_p * g.W_p <= N and g.g_i <= g.s
    rng = np.random.default_rng(N + c_i + c_o)
    img = rng.integers(0, 16, (c_i, H, H))
    F = rng.integers(-7, 8, (c_o, c_i, f, f))
    ip = packing.pack_conv_input(img, g)
    fh = packing.pack_conv_filters(F, g)
    ref = loop_conv(img, F, stride, pad)
    for n in range(c_o):
        prod = sum(int_negacyclic(ip[j], fh[j, n]) for j in range(g.K_in))
        for oy in range(g.H_o):
            for ox in range(g.W_o):
                p, k = packing.conv_output_coeff(g, n, oy, ox)
                assert p == n // g.g_o
                assert k % g.s == g.class_of(n)
                assert prod[k] == ref[n, oy, ox]


@pytest.mark.parametrize("c_i,c_o,w", [(4, 2, 4), (4, 4, 4), (8, 2, 4), (16, 4, 4)])
def test_conv_packing_reduces_to_paper_equations(c_i, c_o, w):
    """Paper's setting: N = c_i w^2, c_o | c_i, valid padding, f_w = f_h = 2.

    Eq. i_batch with ConvFHE's i^(m): exponent s((k - f_w) h_i + l) + m.
    Eq. k_batch_new with ConvFHE's f^(m,n): exponent
        s(h_i f_w - (k h_i + l)) + n c_i / c_o - m.
    The oracle's exponents are these shifted by +s f_w h_i (input) and
    -s f_w h_i (filter).
    """
    f = 2
    N = c_i * w * w
    g = packing.conv_geometry(N, c_i, c_o, w, w, f, 1, 0)
    assert (g.s, g.g_i, g.g_o, g.K_in, g.K_out) == (c_i, c_i, c_o, 1, 1)
    rng = np.random.default_rng(c_i * c_o)
    img = rng.integers(0, 16, (c_i, w, w))
    F = rng.integers(-7, 8, (c_o, c_i, f, f))
    s, hi = c_i, w
    paper_i = np.zeros(N, dtype=np.int64)
    for m in range(c_i):
        for k in range(w):
            for l in range(w):
                paper_i += monomial_shift(np.eye(1, N, 0, dtype=np.int64)[0] * img[m, k, l],
                                          s * ((k - f) * hi + l) + m)
    ours_i = packing.pack_conv_input(img, g)[0]
    assert (monomial_shift(ours_i, -s * f * hi) == paper_i).all()
    fh = packing.pack_conv_filters(F, g)[0]
    for n in range(c_o):
        paper_f = np.zeros(N, dtype=np.int64)
        for m in range(c_i):
            for k in range(f):
                for l in range(f):
                    e = s * (hi * f - (k * hi + l)) + n * c_i // c_o - m
                    paper_f += monomial_shift(np.eye(1, N, 0, dtype=np.int64)[0] * F[n, m, k, l], e)
        assert (monomial_shift(fh[n], s * f * hi) == paper_f).all()
        # valid entries at slots k c_i + n c_i / c_o (Sec. III-A)
        prod = int_negacyclic(paper_i, paper_f)
        ref = loop_conv(img, F, 1, 0)[n]
        for k in range(w - f + 1):
            for l in range(w - f + 1):
                assert prod[s * (k * hi + l) + n * c_i // c_o] == ref[k, l]


FC_CASES = [(8, 4, 2), (256, 4, 2), (256, 16, 10), (256, 20, 5), (256, 64, 10), (512, 100, 7), (8192, 64, 10)]


@pytest.mark.parametrize("N,n_i,n_o", FC_CASES)
def test_theorem1_brute_force(N, n_i, n_o):
    g = packing.fc_geometry(N, n_i, n_o)
    assert g.n_o_p * g.n_i_p == N and g.n_i <= g.n_i_p and g.blocks * g.n_o_p >= n_o
    rng = np.random.default_rng(N + n_i)
    I = rng.integers(0, 16, n_i)
    W = rng.integers(-7, 8, (n_o, n_i))
    B = rng.integers(-7, 8, n_o)
    ip = packing.pack_fc_input(I, g)
    w = packing.pack_fc_weights(W, g)
    d = packing.pack_fc_bias(B, g)
    got = []
    for b in range(g.blocks):
        prod = int_negacyclic(ip, w[b])
        got.append(prod[: g.n_o_p] + d[b])
    got = np.concatenate(got)[:n_o]
    assert (got == W @ I + B).all()


def test_fig5_shape_is_papers_exact_setting():
    g = packing.fc_geometry(8, 4, 2)
    assert (g.n_o_p, g.n_i_p, g.blocks) == (2, 4, 1)


def test_workload_geometries():
    """Tiling of the plain-20 shapes (rule values, regression for the GPU side)."""
    g = packing.conv_geometry(4096, 3, 16, 32, 32)
    assert (g.s, g.g_i, g.g_o, g.K_in, g.K_out) == (2, 2, 2, 2, 8)
    exp8 = {(3, 16, 32, 1): (4, 3, 4, 1, 4), (16, 16, 32, 1): (4, 4, 4, 4, 4), (16, 32, 32, 2): (4, 4, 4, 4, 8),
            (32, 32, 16, 1): (16, 16, 16, 2, 2), (32, 64, 16, 2): (16, 16, 16, 2, 4), (64, 64, 8, 1): (64, 64, 64, 1, 1)}
    for (ci, co, H, st), v in exp8.items():
        g = packing.conv_geometry(8192, ci, co, H, H, 3, st, 1)
        assert (g.s, g.g_i, g.g_o, g.K_in, g.K_out) == v
    g = packing.conv_geometry(16384, 256, 256, 8, 8)
    assert (g.s, g.g_i, g.g_o, g.K_in, g.K_out) == (128, 128, 128, 2, 2)
    f = packing.fc_geometry(8192, 64, 10)
    assert (f.n_o_p, f.n_i_p, f.blocks) == (16, 512, 1)
    f = packing.fc_geometry(16384, 256, 100)
    assert (f.n_o_p, f.n_i_p, f.blocks) == (64, 256, 2)


# ------------------------------------------------------------------ ResNet-50 stride-2 projections
def _loop_conv1x1(img, F, stride):
    """Brute force: out[n][y][x] = sum_m F[n][m] img[m][stride y][stride x], no padding."""
    c_o, c_i = F.shape[:2]
    _, H, W = img.shape
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    out = np.zeros((c_o, Ho, Wo), dtype=np.int64)
    for n in range(c_o):
        for y in range(Ho):
            for x in range(Wo):
                out[n, y, x] = sum(int(F[n, m, 0, 0]) * int(img[m, stride * y, stride * x]) for m in range(c_i))
    return out


def test_resnet50_projections_are_subsampled_1x1():
    """The stride-2 projections of the body are 1x1 stride-1 convs at the output size, fed by the
    block input of the stage's first block; the strided form is still available."""
    sub = wl.resnet50_body()
    full = wl.resnet50_body(subsample_projections=False)
    assert len(sub) == len(full) == 53
    for k, (a, b) in enumerate(zip(sub, full)):
        if k in wl.RESNET50_SUBSAMPLED_PROJECTIONS:
            assert b.f == 1 and b.stride == 2 and b.pad == 0
            assert (a.c_i, a.c_o, a.f, a.stride, a.pad) == (b.c_i, b.c_o, 1, 1, 0)
            assert a.H == b.H // 2 and a.W == b.W // 2
            # the output size of the strided conv is the subsampled map's
            assert a.H == sub[k - 1].H               # the block's 1x1 expansion at the output size
        else:
            assert a == b
    assert [k for k, s in enumerate(full) if s.kind == "conv" and s.f == 1 and s.stride == 2] == \
        list(wl.RESNET50_SUBSAMPLED_PROJECTIONS)


@pytest.mark.parametrize("c_i,c_o,H", [(3, 4, 8), (5, 2, 6), (4, 3, 7)])
def test_subsampled_projection_equals_strided_conv(c_i, c_o, H):
    """A 1x1 stride-2 conv equals the 1x1 conv of the even-pixel map (brute force; odd sizes too)."""
    rng = np.random.default_rng(c_i * 100 + c_o * 10 + H)
    img = rng.integers(0, 16, (c_i, H, H))
    F = rng.integers(-7, 8, (c_o, c_i, 1, 1))
    want = _loop_conv1x1(img, F, 2)
    assert (network.conv2d(img, F, stride=2, pad=0) == want).all()
    assert (network.conv2d(wl.projection_input(img), F, stride=1, pad=0) == want).all()


def test_subsampled_projection_protocol_decrypts_to_strided_conv():
    """The HE layer packed on the subsampled map decrypts (Alg. 1, oracle client and server) to
    the integer stride-2 1x1 conv of the full map."""
    ctx = bfv.make_ctx(256, 2, wl.T_PLAIN)
    rng = np.random.default_rng(77)
    c_i, c_o, H = 4, 6, 8
    img = rng.integers(0, 16, (c_i, H, H))
    F = rng.integers(-7, 8, (c_o, c_i, 1, 1))
    shp = wl.ConvShape(c_i, c_o, H // 2, H // 2, f=1, stride=1, pad=0)
    res = network.run_conv_protocol(ctx, shp, wl.projection_input(img), F, (99, 6, 0, c_i), False, False)
    assert (network.centred(res["decrypted"], wl.T_PLAIN) == _loop_conv1x1(img, F, 2)).all()
