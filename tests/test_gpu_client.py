"""GPU client role: c0 encryption, key generation, decryption, the client's
masks p1, p2 built on the device from the server layer, and the client's c1^r
layer, each bit-exact against the oracle's client, and a layer that goes
through every party on the device and decrypts to the integer convolution."""
import numpy as np
import pytest

import workloads as wl
from oracle import bfv, network, packing
from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu
T = wl.T_PLAIN


@pytest.fixture(scope="module")
def he():
    from paper_2409_05205_amd import he as h
    h.load_library()
    return h


def _keys(octx, seed):
    rng = np.random.default_rng(seed)
    s = wl.ternary(rng, octx.N)
    a = wl.uniform_per_modulus(rng, (), octx.primes, octx.N)
    e = wl.gaussian(rng, octx.N)
    return s, a, e, bfv.keygen(octx, s, a, e)


@pytest.mark.parametrize("N,L", [(1024, 2), (4096, 3), (16384, 6)])
def test_keygen_and_encrypt_match_oracle(he, N, L):
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    s, a, e, b = _keys(octx, N)
    kb = host(ctx.encrypt_c0(dev(s[None]), dev(a), dev(np.zeros((1, N))), dev(-e[None])))[0]
    assert (kb == b).all()
    rng = np.random.default_rng(N + 1)
    rows = 3
    v = wl.encryption_v(rng, (rows, N))
    i = rng.integers(0, T, (rows, N))
    e0 = wl.gaussian(rng, (rows, N))
    got = host(ctx.encrypt_c0(dev(v), dev(b), dev(i), dev(e0)))
    for r in range(rows):
        assert (got[r] == bfv.encrypt_c0(octx, i[r], v[r], e0[r], b)).all()


@pytest.mark.parametrize("N,L", [(1024, 2), (8192, 4), (16384, 6)])
def test_decrypt_matches_oracle(he, N, L):
    """Fresh encryptions of random messages: -(c0) + c1 with c1 = v a + e1 is the
    standard pair; decrypt(c0 + c1 s) must give -msg mod t, as the oracle does."""
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    s, a, e, b = _keys(octx, N + 7)
    rng = np.random.default_rng(N + 8)
    rows = 2
    msg = rng.integers(0, T, (rows, N))
    v = wl.encryption_v(rng, (rows, N))
    e0 = wl.gaussian(rng, (rows, N))
    c0 = np.stack([bfv.encrypt_c0(octx, msg[r], v[r], e0[r], b) for r in range(rows)])
    # client share of -msg: c1 s with c1 = -(v a + e1); x = c0 + c1 s = -(Delta msg) + noise
    e1 = wl.gaussian(rng, (rows, N))
    x1 = np.stack([bfv.encrypt_c0(octx, np.zeros(N, dtype=np.int64), v[r], e1[r], a) for r in range(rows)])
    from oracle import ring
    x1s = np.zeros_like(x1)
    for r in range(rows):
        for l, q in enumerate(octx.primes):
            x1s[r, l] = ring.negacyclic_ntt(x1[r, l], s, q, octx.psis[l])
    want = bfv.decrypt(octx, bfv.add_shares(octx, c0, x1s))
    assert (want == (-msg) % T).all()
    got = host(ctx.decrypt(dev(c0), dev(x1s)))
    assert (got == want).all()


@pytest.mark.parametrize("flags", [0, 1])
def test_client_layer_matches_oracle_client(he, flags):
    """c1^r = extraction of sum_j v_j p1_j + i_j p2_j (Alg. 1 client evaluation)."""
    N, L = 1024, 2
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    shp = wl.ConvShape(20, 24, 6, 6)
    g = packing.conv_geometry(N, 20, 24, 6, 6)
    rng = np.random.default_rng(13)
    F = rng.integers(-7, 8, (24, 20, 3, 3))
    fh = packing.pack_conv_filters(F, g)
    rho = rng.integers(0, T, (g.K_in, 24, N))
    _, _, _, b = _keys(octx, 5)
    e1 = wl.gaussian(rng, (g.K_in, 24, N))
    e2 = wl.gaussian(rng, (g.K_in, 24, N))
    p1, p2 = bfv.client_masks(octx, rho, fh, b, e1, e2)
    v = wl.encryption_v(rng, (g.K_in, N))
    i = rng.integers(0, T, (g.K_in, N))
    want = bfv.client_conv(octx, g, v, i, p1, p2)
    layer = ctx.pack_operands(he.ConvSpec(20, 24, 6, 6), p1, p2, flags)
    vres = np.stack([np.stack([v[j] % q for q in octx.primes]) for j in range(g.K_in)])
    got = host(ctx.conv_layer(layer, dev(vres[None]), dev(i[None])))[0]
    assert (got == want).all()


def test_client_fc_layer_matches_oracle_client(he):
    N, L = 1024, 2
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    g = packing.fc_geometry(N, 100, 7)
    rng = np.random.default_rng(17)
    W = rng.integers(-7, 8, (7, 100))
    w = packing.pack_fc_weights(W, g)
    rho = rng.integers(0, T, (g.blocks, N))
    _, _, _, b = _keys(octx, 6)
    p1, p2 = bfv.client_masks(octx, rho, w, b, wl.gaussian(rng, (g.blocks, N)), wl.gaussian(rng, (g.blocks, N)))
    v = wl.encryption_v(rng, N)
    i = rng.integers(0, T, N)
    want = bfv.client_fc(octx, g, v, i, p1, p2)
    layer = ctx.pack_operands(he.FCSpec(100, 7), p1, p2)
    vres = np.stack([v % q for q in octx.primes])
    got = host(ctx.fc_layer(layer, dev(vres[None]), dev(i[None])))[0]
    assert (got == want).all()


def test_every_party_on_device_decrypts(he):
    """Single-conv workload: keys, encryption, server, client and decryption all on the GPU."""
    N, L = 4096, 3
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    shp = wl.single_conv_layer()
    g = packing.conv_geometry(N, 3, 16, 32, 32)
    img = wl.image(wl.CONFIG_SINGLE_CONV, 1)
    F = wl.layer_weights(wl.CONFIG_SINGLE_CONV, 0, 0, shp)
    fh = packing.pack_conv_filters(F, g)
    rng = np.random.default_rng(21)
    rho = rng.integers(0, T, (g.K_in, 16, N))
    s, a, e, _ = _keys(octx, 22)
    b = ctx.encrypt_c0(dev(s[None]), dev(a), dev(np.zeros((1, N))), dev(-e[None]))[0]
    sh = rng.integers(0, T, (g.K_in, N))
    shn = rng.integers(0, T, (g.K_out, N))
    i = (packing.pack_conv_input(img, g) + sh) % T
    v = wl.encryption_v(rng, (g.K_in, N))
    e0 = wl.gaussian(rng, (g.K_in, N))
    c0 = ctx.encrypt_c0(dev(v), b, dev(i), dev(e0))
    server = ctx.pack_conv(he.ConvSpec(3, 16, 32, 32), F, rho)
    c0r = ctx.conv_layer(server, c0[None], dev(sh[None]), dev(shn[None]))[0]
    client = ctx.client_masks(server, b, dev(wl.gaussian(rng, (g.K_in, 16, N))), dev(wl.gaussian(rng, (g.K_in, 16, N))))
    vres = np.stack([np.stack([v[j] % q for q in octx.primes]) for j in range(g.K_in)])
    c1r = ctx.conv_layer(client, dev(vres[None]), dev(i[None]))[0]
    r = host(ctx.decrypt(c0r, c1r)).astype(np.int64)
    dec = network.centred(packing.decode_conv_output((r - shn) % T, g), T)
    assert (dec == network.conv2d(img, F)).all()


@pytest.mark.parametrize("flags", [0, 1])
def test_client_masks_on_device_match_oracle(he, flags):
    """Masks p1 = rho b + e1, p2 = Delta (fhat + rho) + e2 formed on the device from the server
    layer's resident operands: the client layer they give equals the oracle client's c1^r."""
    N, L = 1024, 2
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    g = packing.conv_geometry(N, 20, 24, 6, 6)
    rng = np.random.default_rng(31 + flags)
    F = rng.integers(-7, 8, (24, 20, 3, 3))
    fh = packing.pack_conv_filters(F, g)
    rho = rng.integers(0, T, (g.K_in, 24, N))
    _, _, _, b = _keys(octx, 7)
    e1 = wl.gaussian(rng, (g.K_in, 24, N))
    e2 = wl.gaussian(rng, (g.K_in, 24, N))
    p1, p2 = bfv.client_masks(octx, rho, fh, b, e1, e2)
    v = wl.encryption_v(rng, (g.K_in, N))
    i = rng.integers(0, T, (g.K_in, N))
    want = bfv.client_conv(octx, g, v, i, p1, p2)
    server = ctx.pack_conv(he.ConvSpec(20, 24, 6, 6), F, rho, flags)
    client = ctx.client_masks(server, dev(b), dev(e1), dev(e2))
    vres = np.stack([np.stack([v[j] % q for q in octx.primes]) for j in range(g.K_in)])
    got = host(ctx.conv_layer(client, dev(vres[None]), dev(i[None])))[0]
    assert (got == want).all()
    # the server layer is unchanged
    sh = rng.integers(0, T, (g.K_in, N))
    c0 = wl.uniform_per_modulus(rng, (g.K_in,), octx.primes, N)
    got_s = host(ctx.conv_layer(server, dev(c0[None]), dev(sh[None])))[0]
    assert (got_s == bfv.server_conv(octx, g, c0.astype(np.uint64), rho, fh, sh, None)).all()


def test_client_fc_masks_on_device_match_oracle(he):
    N, L = 1024, 2
    ctx = he.Context(N, L, T)
    octx = bfv.make_ctx(N, L, T)
    g = packing.fc_geometry(N, 100, 7)
    rng = np.random.default_rng(37)
    W = rng.integers(-7, 8, (7, 100))
    w = packing.pack_fc_weights(W, g)
    rho = rng.integers(0, T, (g.blocks, N))
    _, _, _, b = _keys(octx, 8)
    e1 = wl.gaussian(rng, (g.blocks, N))
    e2 = wl.gaussian(rng, (g.blocks, N))
    p1, p2 = bfv.client_masks(octx, rho, w, b, e1, e2)
    v = wl.encryption_v(rng, N)
    i = rng.integers(0, T, N)
    want = bfv.client_fc(octx, g, v, i, p1, p2)
    server = ctx.pack_fc(he.FCSpec(100, 7), W, rho, rng.integers(-7, 8, 7))
    client = ctx.client_masks(server, dev(b), dev(e1), dev(e2))
    vres = np.stack([v % q for q in octx.primes])
    got = host(ctx.fc_layer(client, dev(vres[None]), dev(i[None])))[0]
    assert (got == want).all()
