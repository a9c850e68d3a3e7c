"""Pins for the oracle's protocol (Alg. 1 / Alg. 2 in the exact reading).

The decrypted layer output minus the fresh share must equal the integer
convolution / FC result mod t (Eq. c0+c1: the shares add up to
Delta (i f-hat) + small noise + Delta sh').  The noise must stay below the
analytic worst case, far under Delta / 2.  Planted mistakes (the literal sign
of the printed encryption line, a dropped share term) must break decryption,
which shows the checks can fail.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import bfv, network, packing

T = wl.T_PLAIN


@pytest.fixture(scope="module")
def ctx256():
    return bfv.make_ctx(256, 2, T)


CONV = [((3, 8, 4, 4), 1), ((6, 4, 4, 4), 1), ((4, 8, 4, 4), 2), ((2, 2, 6, 6), 1), ((5, 3, 4, 4), 1)]


@pytest.mark.parametrize("shape,stride", CONV)
@pytest.mark.parametrize("first,last", [(True, False), (False, False), (False, True), (True, True)])
def test_conv_protocol_decrypts_to_integer_conv(ctx256, shape, stride, first, last):
    c_i, c_o, H, W = shape
    shp = wl.ConvShape(c_i, c_o, H, W, stride=stride)
    rng = np.random.default_rng(c_i + 7 * c_o + stride)
    img = rng.integers(0, 16, (c_i, H, W))
    F = rng.integers(-7, 8, (c_o, c_i, 3, 3))
    res = network.run_conv_protocol(ctx256, shp, img, F, (99, 1, 0, c_i), first, last)
    assert (network.centred(res["decrypted"], T) == res["reference"]).all()


@pytest.mark.parametrize("n_i,n_o", [(4, 2), (16, 10), (20, 5), (64, 10)])
@pytest.mark.parametrize("first,last", [(True, False), (False, True)])
def test_fc_protocol_decrypts_to_integer_fc(ctx256, n_i, n_o, first, last):
    rng = np.random.default_rng(n_i * n_o)
    vec = rng.integers(0, 16, n_i)
    W = rng.integers(-7, 8, (n_o, n_i))
    B = rng.integers(-7, 8, n_o)
    res = network.run_fc_protocol(ctx256, wl.FCShape(n_i, n_o), vec, W, B, (99, 2, 0, n_i), first, last)
    assert (network.centred(res["decrypted"], T) == res["reference"]).all()


def test_single_conv_workload_end_to_end():
    """The single-conv workload (N=4096, 3 limbs, 3x32x32 -> 16) through every party."""
    ctx = bfv.make_ctx(4096, 3, T)
    shp = wl.single_conv_layer()
    img = wl.image(1, 0)
    F = wl.layer_weights(1, 0, 0, shp)
    res = network.run_conv_protocol(ctx, shp, img, F, (1, 0, 0, 0), True, False)
    assert (network.centred(res["decrypted"], T) == res["reference"]).all()
    # noise: decrypted share sum minus Delta * message, against the analytic bound
    g = res["geom"]
    m = (res["r"] + res["sh_next"]) % T
    noise = bfv.noise_magnitude(ctx, res["total"], m)
    # worst case per input poly: |e0 rho| + |v e1| + |i e2| <= N(6s)t + N(6s) + N t (6s), plus
    # the t-wrap term r_t |k f| (<= t * 63 c_i), summed over K_in polys
    e = int(np.floor(6 * wl.SIGMA))
    bound = g.K_in * (ctx.N * e * T + ctx.N * e + ctx.N * T * e) + T * 63 * g.c_i + T
    assert noise <= bound
    assert bound < ctx.Delta // 2


def test_literal_encryption_sign_fails(ctx256, monkeypatch):
    """Planted mistake: c0 = v b - Delta i + e0 (the literal reading) must not decrypt."""
    def wrong(ctx, i_poly, v, e0, b):
        out = np.zeros((ctx.L, ctx.N), dtype=np.uint64)
        from oracle import ring
        for l, q in enumerate(ctx.primes):
            qq = np.uint64(q)
            vb = ring.negacyclic_ntt(v, b[l], q, ctx.psis[l])
            di = ring.reduce_signed(i_poly, q) * np.uint64(ctx.delta_l[l]) % qq
            out[l] = (vb + qq - di + ring.reduce_signed(e0, q)) % qq
        return out
    monkeypatch.setattr(bfv, "encrypt_c0", wrong)
    shp = wl.ConvShape(3, 8, 4, 4)
    rng = np.random.default_rng(5)
    img = rng.integers(0, 16, (3, 4, 4))
    F = rng.integers(-7, 8, (8, 3, 3, 3))
    res = network.run_conv_protocol(ctx256, shp, img, F, (99, 3, 0, 0), False, False)
    assert (network.centred(res["decrypted"], T) != res["reference"]).mean() > 0.9


def test_dropped_share_term_fails(ctx256):
    """Planted mistake: a server that forgets the - Delta sh f-hat term must not decrypt."""
    shp = wl.ConvShape(3, 8, 4, 4)
    rng = np.random.default_rng(6)
    img = rng.integers(0, 16, (3, 4, 4))
    F = rng.integers(-7, 8, (8, 3, 3, 3))
    g = packing.conv_geometry(256, 3, 8, 4, 4)

    def server(c0, rho, fhat, sh, sh_next):
        return bfv.server_conv(ctx256, g, c0, rho, fhat, None, sh_next)
    res = network.run_conv_protocol(ctx256, shp, img, F, (99, 4, 0, 0), False, False, server_fn=server)
    assert (network.centred(res["decrypted"], T) != res["reference"]).mean() > 0.9


def test_server_is_deterministic(ctx256):
    shp = wl.ConvShape(3, 8, 4, 4)
    img = np.ones((3, 4, 4), dtype=np.int64)
    F = np.ones((8, 3, 3, 3), dtype=np.int64)
    a = network.run_conv_protocol(ctx256, shp, img, F, (99, 5, 0, 0), False, False)["c0r"]
    b = network.run_conv_protocol(ctx256, shp, img, F, (99, 5, 0, 0), False, False)["c0r"]
    assert (a == b).all()


def test_harness_requant():
    z = np.array([-5, 0, 3, 40, 17])
    assert network.relu_requant(z).tolist() == [0, 0, 0, 10, 4]   # shift 2: 40 >> 2 = 10
    assert network.relu_requant(np.array([-1, 15])).tolist() == [0, 15]
    x = np.arange(2 * 8 * 8).reshape(2, 8, 8)
    assert network.gap(x).tolist() == [31, 95]


# ------------------------------------------------------------------ the RLWE identity (Sec. II-A)
def _schoolbook_limbs(ctx, a_limbs, b_signed):
    """a * b per limb by the schoolbook definition (independent of the oracle's NTT)."""
    from oracle import ring
    return np.stack([ring.negacyclic_schoolbook(a_limbs[l], b_signed, q) for l, q in enumerate(ctx.primes)])


def _rlwe_case(ctx, seed):
    rng = np.random.default_rng(seed)
    N = ctx.N
    s = wl.ternary(rng, N)
    a = wl.uniform_per_modulus(rng, (), ctx.primes, N).astype(np.uint64)
    e = wl.gaussian(rng, N)
    v = wl.encryption_v(rng, N)
    e0 = wl.gaussian(rng, N)
    e1 = wl.gaussian(rng, N)
    i = rng.integers(0, T, N)
    return s, a, e, v, e0, e1, i


def _decrypt_with_key(ctx, c0, a, s, v, e1):
    """The second ciphertext element of the same encryption, c1 = -(v a + e1) (the negation of
    the fresh c1 = v a + e1 of Eq. encryption), then c0 + c1 s and the scale-and-round."""
    from oracle import ring
    va = _schoolbook_limbs(ctx, a, v)
    c1 = np.stack([(np.uint64(q) - (va[l] + ring.reduce_signed(e1, q)) % np.uint64(q)) % np.uint64(q)
                   for l, q in enumerate(ctx.primes)])
    c1s = _schoolbook_limbs(ctx, c1, s)
    x = np.stack([(c0[l] + c1s[l]) % np.uint64(q) for l, q in enumerate(ctx.primes)])
    return bfv.decrypt(ctx, x[None])[0]


@pytest.mark.parametrize("seed", [0, 1])
def test_keygen_encrypt_decrypt_rlwe_identity(seed):
    """Pins keygen (b = -a s + e), encrypt_c0 and decrypt together through the identity of
    Eq. encryption / Eq. decryption: with c1 = -(v a + e1), c0 + c1 s = -(Delta i + v e + e0 + e1 s),
    which decrypts to -i mod t.  Products by the schoolbook definition, not the oracle's NTT."""
    ctx = bfv.make_ctx(64, 2, T)
    s, a, e, v, e0, e1, i = _rlwe_case(ctx, seed)
    b = bfv.keygen(ctx, s, a, e)
    # b + a s = e per limb (the definition of the public key)
    as_ = _schoolbook_limbs(ctx, a, s)
    from oracle import ring
    for l, q in enumerate(ctx.primes):
        assert ((b[l] + as_[l]) % np.uint64(q) == ring.reduce_signed(e, q)).all()
    c0 = bfv.encrypt_c0(ctx, i, v, e0, b)
    assert (_decrypt_with_key(ctx, c0, a, s, v, e1) == (-i) % T).all()


def test_keygen_sign_flip_fails():
    """Planted mistake: b = a s + e (sign of a s flipped) must break the identity, since then
    c0 + c1 s carries -2 v a s, which is not small."""
    from oracle import ring
    ctx = bfv.make_ctx(64, 2, T)
    s, a, e, v, e0, e1, i = _rlwe_case(ctx, 5)
    as_ = _schoolbook_limbs(ctx, a, s)
    b_wrong = np.stack([(as_[l] + ring.reduce_signed(e, q)) % np.uint64(q) for l, q in enumerate(ctx.primes)])
    c0 = bfv.encrypt_c0(ctx, i, v, e0, b_wrong)
    assert (_decrypt_with_key(ctx, c0, a, s, v, e1) != (-i) % T).mean() > 0.9


# ------------------------------------------------------------------ server evaluation by the schoolbook
def _schoolbook_sum_of_products(ctx, l, xs, ys):
    """sum_j xs[j] * ys[j, m] in Z_q[X]/(X^N+1) by the schoolbook definition."""
    from oracle import ring
    q = ctx.primes[l]
    xs = np.asarray(xs)
    ys = np.asarray(ys)
    out = np.zeros(ys.shape[1:], dtype=np.uint64)
    for j in range(xs.shape[0]):
        for m in range(ys.shape[1]):
            out[m] = (out[m] + ring.negacyclic_schoolbook(xs[j], ys[j, m], q)) % np.uint64(q)
    return out


@pytest.mark.parametrize("shape", [(2, 3, 2, 2, 1), (3, 2, 2, 2, 2), (4, 4, 3, 2, 1)])
def test_server_conv_equal_with_schoolbook_products(shape, monkeypatch):
    """server_conv multiplies through the oracle's NTT; with every product taken by the schoolbook
    definition instead (tiny N), the words of c0^r must be identical."""
    c_i, c_o, H, W, stride = shape
    N = 64
    ctx = bfv.make_ctx(N, 2, T)
    g = packing.conv_geometry(N, c_i, c_o, H, W, 3, stride, 1)
    rng = np.random.default_rng(c_i * 10 + c_o)
    F = rng.integers(-7, 8, (c_o, c_i, 3, 3))
    fh = packing.pack_conv_filters(F, g)
    rho = rng.integers(0, T, (g.K_in, c_o, N))
    c0 = wl.uniform_per_modulus(rng, (g.K_in,), ctx.primes, N).astype(np.uint64)
    sh = rng.integers(0, T, (g.K_in, N))
    shn = rng.integers(0, T, (g.K_out, N))
    ref = bfv.server_conv(ctx, g, c0, rho, fh, sh, shn)
    monkeypatch.setattr(bfv, "_sum_of_products", _schoolbook_sum_of_products)
    school = bfv.server_conv(ctx, g, c0, rho, fh, sh, shn)
    assert (school == ref).all()


@pytest.mark.parametrize("n_i,n_o,N", [(4, 2, 8), (6, 5, 64), (16, 10, 64)])
def test_server_fc_equal_with_schoolbook_products(n_i, n_o, N, monkeypatch):
    """As above for server_fc, including the Fig. 5 shape (n_i = 4, n_o = 2, N = 8)."""
    ctx = bfv.make_ctx(N, 2, T)
    g = packing.fc_geometry(N, n_i, n_o)
    rng = np.random.default_rng(n_i * n_o + N)
    w = packing.pack_fc_weights(rng.integers(-7, 8, (n_o, n_i)), g)
    d = packing.pack_fc_bias(rng.integers(-7, 8, n_o), g)
    rho = rng.integers(0, T, (g.blocks, N))
    c0 = wl.uniform_per_modulus(rng, (), ctx.primes, N).astype(np.uint64)
    sh = rng.integers(0, T, N)
    shn = rng.integers(0, T, (g.blocks, g.n_o_p))
    ref = bfv.server_fc(ctx, g, c0, rho, w, d, sh, shn)
    monkeypatch.setattr(bfv, "_sum_of_products", _schoolbook_sum_of_products)
    school = bfv.server_fc(ctx, g, c0, rho, w, d, sh, shn)
    assert (school == ref).all()
