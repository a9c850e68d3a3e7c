"""GPU parity of the layer split at its NTT-domain inputs (the paper's protocol: the client
sends NTT(c0), the server transforms its own share): he_layer_inputs_ntt followed by
he_conv_layer_ntt / he_fc_layer_ntt gives the oracle's words, whether c0 and sh are transformed
in one call or in two, for conv (both inverse forms, B = 1 and 3) and FC, with and without the
input share and the next-layer share."""
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


@pytest.mark.parametrize("shape", [(1024, 4, 12, 6, 1), (1024, 16, 12, 14, 1), (2048, 8, 8, 2, 1)],
                         ids=lambda s: "N%d_c%d-%d_H%d_st%d" % s)
@pytest.mark.parametrize("flags", [0, 1])
def test_conv_from_ntt_inputs_matches_oracle(he, shape, flags):
    N, c_i, c_o, H, stride = shape
    L, B = 2, 3
    octx = bfv.make_ctx(N, L, T)
    g = packing.conv_geometry(N, c_i, c_o, H, H, 3, stride, 1)
    rng = np.random.default_rng(sum(shape) + flags)
    F = rng.integers(-7, 8, (c_o, c_i, 3, 3))
    rho = rng.integers(0, T, (g.K_in, c_o, N))
    c0 = np.stack([wl.uniform_per_modulus(rng, (g.K_in,), octx.primes, N) for _ in range(B)])
    sh = rng.integers(0, T, (B, g.K_in, N))
    shn = rng.integers(0, T, (B, g.K_out, N))
    fh = packing.pack_conv_filters(F, g)
    ctx = he.Context(N, L, T)
    layer = ctx.pack_conv(he.ConvSpec(c_i, c_o, H, H, 3, stride, 1), F, rho, flags)
    for use_sh, use_shn in ((True, True), (False, True), (True, False)):
        want = [bfv.server_conv(octx, g, c0[b].astype(np.uint64), rho, fh, sh[b] if use_sh else None,
                                shn[b] if use_shn else None) for b in range(B)]
        for nb in (1, B):
            x = ctx.input_buffer(layer, nb)
            # client: NTT(c0); server: NTT(sh), a separate call
            ctx.inputs_ntt(layer, x, c0=dev(c0[:nb]))
            if use_sh:
                ctx.inputs_ntt(layer, x, sh=dev(sh[:nb]))
            got = host(ctx.layer_from_ntt(layer, x, use_sh, dev(shn[:nb]) if use_shn else None))
            for b in range(nb):
                assert (got[b] == want[b]).all(), f"B={nb} image {b} sh={use_sh} shn={use_shn}"
        # both transforms in one call
        x = ctx.input_buffer(layer, B)
        ctx.inputs_ntt(layer, x, c0=dev(c0), sh=dev(sh) if use_sh else None)
        got = host(ctx.layer_from_ntt(layer, x, use_sh, dev(shn) if use_shn else None))
        for b in range(B):
            assert (got[b] == want[b]).all()


def test_fc_from_ntt_inputs_matches_oracle(he):
    N, L, B = 1024, 2, 2
    octx = bfv.make_ctx(N, L, T)
    g = packing.fc_geometry(N, 64, 10)
    rng = np.random.default_rng(5)
    W = rng.integers(-7, 8, (10, 64))
    bias = rng.integers(-7, 8, 10)
    rho = rng.integers(0, T, (g.blocks, N))
    w = packing.pack_fc_weights(W, g)
    c0 = np.stack([wl.uniform_per_modulus(rng, (), octx.primes, N) for _ in range(B)])
    sh = rng.integers(0, T, (B, N))
    shn = rng.integers(0, T, (B, g.blocks, g.n_o_p))
    ctx = he.Context(N, L, T)
    layer = ctx.pack_fc(he.FCSpec(64, 10), W, rho, bias)
    for use_shn in (True, False):
        x = ctx.input_buffer(layer, B)
        ctx.inputs_ntt(layer, x, c0=dev(c0))
        ctx.inputs_ntt(layer, x, sh=dev(sh))
        got = host(ctx.layer_from_ntt(layer, x, True, dev(shn) if use_shn else None))
        for b in range(B):
            want = bfv.server_fc(octx, g, c0[b].astype(np.uint64), rho, w, packing.pack_fc_bias(bias, g), sh[b],
                                 shn[b] if use_shn else None)
            assert (got[b] == want).all()
