"""Seeded synthetic workloads for the rotation-free HE Conv/FC server path.

This module holds only workload shapes and keyed random draws. It contains none
of the method's arithmetic (no ring products, no packing, no scheme algebra), so
both the CPU oracle and the GPU path may take their inputs from it.

Every tensor is drawn from its own keyed stream
``SeedSequence([MASTER_SEED, config, client, variant, layer, kind, j])`` so a
tensor's value never depends on the order in which other tensors are drawn: a
request produces the same inputs whether it runs alone or inside a mix.

Distributions follow the paper's setting (Sec. II-A: ternary secret, Gaussian
errors DG(sigma^2), v in {0 w.p. 1/2, +-1 w.p. 1/4}) with the exact-integer
parameter set used throughout this repository: plaintext modulus t = 786433,
sigma = 3.2, uint4 activations in [0, 15] and integer weights in [-7, 7].
Images stand in for CIFAR (3x32x32); layer shapes are those of the plain-20
classifier and its width variants (Sec. IV-B, Table IV).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

MASTER_SEED = 2409052050
T_PLAIN = 786433          # plaintext modulus t (prime, t - 1 = 3 * 2^18)
SIGMA = 3.2               # Gaussian error width
ERR_BOUND = 6.0 * SIGMA   # errors are rounded normals clipped to |e| <= 6 sigma

KINDS = {
    "img": 0, "W": 1, "bias": 2, "rho": 3, "s": 4, "a": 5, "e": 6, "v": 7,
    "e0": 8, "e1": 9, "e2": 10, "sh": 11, "shnext": 12, "arrival": 13,
    "c0": 14, "pick": 15,
}


def rng(config: int, client: int, variant: int, layer: int, kind: str, j: int = 0) -> np.random.Generator:
    """Independent generator keyed by (config, client, variant, layer, kind, j)."""
    ss = np.random.SeedSequence([MASTER_SEED, int(config), int(client), int(variant),
                                 int(layer), KINDS[kind], int(j)])
    return np.random.Generator(np.random.PCG64(ss))


# ---------------------------------------------------------------- draws
def uint4(g: np.random.Generator, shape) -> np.ndarray:
    """Activations uniform in [0, 15]."""
    return g.integers(0, 16, size=shape, dtype=np.int64)


def weights(g: np.random.Generator, shape, lo: int = -7, hi: int = 7) -> np.ndarray:
    """Integer weights uniform in [lo, hi]."""
    return g.integers(lo, hi + 1, size=shape, dtype=np.int64)


def uniform_below(g: np.random.Generator, shape, bound: int) -> np.ndarray:
    """Uniform integers in [0, bound)."""
    return g.integers(0, int(bound), size=shape, dtype=np.int64)


def uniform_per_modulus(g: np.random.Generator, lead_shape, moduli: Sequence[int], n: int) -> np.ndarray:
    """Array of shape lead_shape + (len(moduli), n); slice l uniform in [0, moduli[l])."""
    lead_shape = tuple(lead_shape)
    out = np.empty(lead_shape + (len(moduli), n), dtype=np.int64)
    for l, q in enumerate(moduli):
        out[..., l, :] = g.integers(0, int(q), size=lead_shape + (n,), dtype=np.int64)
    return out


def ternary(g: np.random.Generator, shape) -> np.ndarray:
    """Uniform over {-1, 0, 1}."""
    return g.integers(-1, 2, size=shape, dtype=np.int64)


def gaussian(g: np.random.Generator, shape, sigma: float = SIGMA, bound: float = ERR_BOUND) -> np.ndarray:
    """Rounded normal of width sigma, clipped to |e| <= bound."""
    e = np.rint(g.normal(0.0, sigma, size=shape))
    return np.clip(e, -np.floor(bound), np.floor(bound)).astype(np.int64)


def encryption_v(g: np.random.Generator, shape) -> np.ndarray:
    """v coefficients: 0 w.p. 1/2, +1 w.p. 1/4, -1 w.p. 1/4."""
    u = g.integers(0, 4, size=shape, dtype=np.int64)
    return np.where(u < 2, 0, np.where(u == 2, 1, -1)).astype(np.int64)


# ---------------------------------------------------------------- shapes
@dataclass(frozen=True)
class ConvShape:
    c_i: int
    c_o: int
    H: int
    W: int
    f: int = 3
    stride: int = 1
    pad: int = 1
    kind: str = "conv"


@dataclass(frozen=True)
class FCShape:
    n_i: int
    n_o: int
    kind: str = "fc"


def plain20(width: int = 1, classes: int = 10) -> List[object]:
    """The plain-20 linear stack at width multiplier 1, 2 or 4.

    conv 3->c at 32x32; six 3x3 convs at c channels on 32x32 (the last six of
    stage 1); six at 2c on 16x16, the first taking c->2c with stride 2; six at
    4c on 8x8, the first taking 2c->4c with stride 2; global average pool; FC
    4c -> classes.  19 convs + 1 FC = 20 linear layers.
    """
    c = 16 * width
    L: List[object] = [ConvShape(3, c, 32, 32)]
    L += [ConvShape(c, c, 32, 32) for _ in range(6)]
    L += [ConvShape(c, 2 * c, 32, 32, stride=2)]
    L += [ConvShape(2 * c, 2 * c, 16, 16) for _ in range(5)]
    L += [ConvShape(2 * c, 4 * c, 16, 16, stride=2)]
    L += [ConvShape(4 * c, 4 * c, 8, 8) for _ in range(5)]
    L += [FCShape(4 * c, classes)]
    return L


def resnet50_body(classes: int = 1000, subsample_projections: bool = True) -> List[object]:
    """The ResNet-50 linear layers after its stem, for a 224x224 input: bottleneck blocks
    (1x1 reduce, 3x3, 1x1 expand, and a 1x1 projection on the first block of a stage) at
    56x56 (3 blocks, 64/256 channels), 28x28 (4 blocks, 128/512), 14x14 (6 blocks, 256/1024)
    and 7x7 (3 blocks, 512/2048), the stride of a stage's first block on its 3x3 and its
    projection; then global average pooling and FC 2048 -> classes.  52 convs + 1 FC.

    A 1x1 convolution of stride 2 reads only the pixels at even coordinates, so with
    subsample_projections the stride-2 projections (layers 13, 26 and 45) are the same 1x1
    convolution at stride 1 on the map subsampled to the output size (projection_input): each
    party subsamples its share of the block input before packing, and the layer packs a map a
    quarter of the size, with a quarter of the resident operands and output polynomials.

    The stem (7x7 stride-2 conv on 224x224, then max pooling) is not included: one
    zero-padded 230x230 channel needs N >= 65536 coefficients in this packing.
    """
    layers: List[object] = []
    c_in = 64
    for H_out, mid, out, blocks, stride in ((56, 64, 256, 3, 1), (28, 128, 512, 4, 2), (14, 256, 1024, 6, 2),
                                           (7, 512, 2048, 3, 2)):
        for b in range(blocks):
            st = stride if b == 0 else 1
            H_in = H_out * st
            layers.append(ConvShape(c_in, mid, H_in, H_in, f=1, stride=1, pad=0))
            layers.append(ConvShape(mid, mid, H_in, H_in, f=3, stride=st, pad=1))
            layers.append(ConvShape(mid, out, H_out, H_out, f=1, stride=1, pad=0))
            if b == 0:
                if st > 1 and subsample_projections:
                    layers.append(ConvShape(c_in, out, H_out, H_out, f=1, stride=1, pad=0))
                else:
                    layers.append(ConvShape(c_in, out, H_in, H_in, f=1, stride=st, pad=0))
            c_in = out
    layers.append(FCShape(2048, classes))
    return layers


RESNET50_SUBSAMPLED_PROJECTIONS = (13, 26, 45)   # stride-2 1x1 projections packed on the subsampled map


def projection_input(x, stride: int = 2):
    """The input of a subsampled stride-s 1x1 projection: the pixels of x [c][H][W] at
    coordinates that are multiples of s."""
    return x[:, ::stride, ::stride]


@dataclass(frozen=True)
class HEParams:
    N: int
    L: int
    t: int = T_PLAIN


# The five workloads (ring degree, limbs, network).
CONFIG_SINGLE_CONV = 1      # one conv 3->16 on 3x32x32, N=4096, 3 limbs
CONFIG_PLAIN20_X1 = 2       # full x1 stack, N=8192, 4 limbs, one image per launch
CONFIG_BATCHED = 3          # 64 images x widths 1, 2, 4
CONFIG_SERVED = 4           # Poisson stream of single-layer requests, 128 clients
CONFIG_STRESS = 5           # x4 / 100 classes, N=16384, 6 limbs, 256 clients
CONFIG_RESNET50 = 6         # ResNet-50-shaped layers (after the stem), N=16384, 6 limbs

PARAMS_BY_WIDTH = {1: HEParams(8192, 4), 2: HEParams(8192, 4), 4: HEParams(16384, 6)}
PARAMS_SINGLE = HEParams(4096, 3)


def single_conv_layer() -> ConvShape:
    return ConvShape(3, 16, 32, 32)


# ---------------------------------------------------------------- layer inputs
def layer_weights(config: int, variant: int, layer: int, shape) -> np.ndarray:
    """Conv filters [c_o][c_i][f][f] or FC matrix [n_o][n_i], integers in [-7, 7]."""
    g = rng(config, 0, variant, layer, "W")
    if shape.kind == "conv":
        return weights(g, (shape.c_o, shape.c_i, shape.f, shape.f))
    return weights(g, (shape.n_o, shape.n_i))


def layer_bias(config: int, variant: int, layer: int, shape) -> Optional[np.ndarray]:
    if shape.kind != "fc":
        return None
    return weights(rng(config, 0, variant, layer, "bias"), (shape.n_o,))


def image(config: int, client: int, variant: int = 0) -> np.ndarray:
    """A 3x32x32 uint4 image."""
    return uint4(rng(config, client, variant, 0, "img"), (3, 32, 32))


def layer_activation(config: int, client: int, variant: int, layer: int, shape) -> np.ndarray:
    """A uint4 activation of the layer's input shape (open-loop workloads)."""
    g = rng(config, client, variant, layer, "img")
    if shape.kind == "conv":
        return uint4(g, (shape.c_i, shape.H, shape.W))
    return uint4(g, (shape.n_i,))


def mask_polys(config: int, variant: int, layer: int, count: int, n: int, t: int = T_PLAIN) -> np.ndarray:
    """Server masks rho: `count` polynomials uniform in [0, t)."""
    return uniform_below(rng(config, 0, variant, layer, "rho"), (count, n), t)


def share_polys(config: int, client: int, variant: int, layer: int, count: int, n: int,
                kind: str = "sh", t: int = T_PLAIN) -> np.ndarray:
    """Server shares sh / sh' : `count` polynomials uniform in [0, t)."""
    return uniform_below(rng(config, client, variant, layer, kind), (count, n), t)


def ciphertext_polys(config: int, client: int, variant: int, layer: int, count: int,
                     moduli: Sequence[int], n: int) -> np.ndarray:
    """Stand-in c0 shares: [count][L][n], uniform per limb.

    RLWE ciphertexts are computationally indistinguishable from uniform, so the
    server's work on these is the work it does on real encryptions.  Tests that
    need real encryptions build them with the oracle client instead.
    """
    return uniform_per_modulus(rng(config, client, variant, layer, "c0"), (count,), moduli, n)
