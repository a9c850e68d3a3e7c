"""Operation counts (Table I, Table III) and communication bytes (Table II).

Oracle (test infrastructure).  Three kinds of function:

* ``table1_conv`` / ``table3_fc`` give the proposed design's server and client
  counts exactly as the paper's complexity tables state them for one layer:
  Table I (Conv, N = c_i w^2, one input polynomial) and Table III (FC, with
  floor(N / n_i) weight rows per polynomial).
* ``conv_layer_counts`` / ``fc_layer_counts`` count the same quantities for this
  repository's generalised packing (several input polynomials K_in, output
  groups of g_o channels, padding) and for either form in which c0 reaches the
  server: in NTT form as the paper's protocol sends it (the client derives
  NTT(c0) during encryption, Sec. IV-A-1), or in coefficient form (one more
  forward transform per input polynomial, reading R9).  In the paper's own
  setting (K_in = 1, c0 in NTT form) they reduce to the table entries.
* ``table2_comm_bytes`` is the communication per Conv + ReLU round of Table II
  for each design column, from its printed formula.

Counts are per RNS limb and per polynomial: one "NTT" is one length-N forward
transform of one polynomial, one "CWM" one coefficient-wise product of two
length-N polynomials (N modular multiplications).
"""
from __future__ import annotations

from dataclasses import dataclass
from math import ceil

from .packing import ConvGeom, FCGeom


@dataclass(frozen=True)
class Counts:
    ntt: int        # forward transforms
    intt: int       # inverse transforms
    cwm: int        # coefficient-wise products of two length-N polynomials
    rotations: int


def table1_conv(c_o: int):
    """Table I, proposed design: (server, client) for one Conv layer with c_o output channels."""
    server = Counts(ntt=1, intt=c_o, cwm=2 * c_o, rotations=0)
    client = Counts(ntt=3, intt=c_o, cwm=2 * c_o, rotations=0)
    return server, client


def table1_conv_memory(c_o: int):
    """Table I, proposed design: memory in length-N polynomials, (server, client)."""
    return 2 * c_o + 1, 2 * c_o + 1


def _fc_polys(N: int, n_i: int, n_o: int) -> int:
    """ceil(n_o / floor(N / n_i)): weight polynomials of an FC layer (Sec. III-B)."""
    return ceil(n_o / (N // n_i))


def table3_fc(N: int, n_i: int, n_o: int):
    """Table III, proposed design: (server, client) counts for one FC layer.  The CWM entries
    are printed as multiplications of coefficients (2 N per polynomial pair); here they are given
    in polynomial CWMs (that entry divided by N)."""
    P = _fc_polys(N, n_i, n_o)
    server = Counts(ntt=1, intt=P, cwm=2 * P, rotations=0)
    client = Counts(ntt=3, intt=P, cwm=2 * P, rotations=0)
    return server, client


def table3_fc_memory(N: int, n_i: int, n_o: int):
    """Table III, proposed design: memory in coefficients, (server, client)."""
    P = _fc_polys(N, n_i, n_o)
    return 2 * N * P, 2 * N * P + n_o


def conv_layer_counts(g: ConvGeom, first_layer: bool, c0_in_ntt_form: bool) -> Counts:
    """Server counts per limb for one conv layer of this repository's packing.

    Forward transforms: NTT(sh_j) for each input polynomial (none on a network's first layer,
    which has no share), plus NTT(c0_j) when c0 arrives in coefficient form.  Inverse transforms:
    one per output channel (each c0^(n) is recovered before its residue class is extracted).
    CWMs: c0_j rho_j^(n) and sh_j fhat_j^(n) for every (j, n) (the second only with a share).
    """
    K = g.K_in
    ntt = (0 if first_layer else K) + (0 if c0_in_ntt_form else K)
    cwm = (1 if first_layer else 2) * K * g.c_o
    return Counts(ntt=ntt, intt=g.c_o, cwm=cwm, rotations=0)


def fc_layer_counts(g: FCGeom, first_layer: bool, c0_in_ntt_form: bool) -> Counts:
    """Server counts per limb for one FC layer (one input polynomial, `blocks` weight polynomials)."""
    ntt = (0 if first_layer else 1) + (0 if c0_in_ntt_form else 1)
    return Counts(ntt=ntt, intt=g.blocks, cwm=(1 if first_layer else 2) * g.blocks, rotations=0)


def table2_comm_bytes(design: str, w: int, c_i: int, c_o: int, N: int = 8192, log_q: int = 104,
                      log_qp: int = 55) -> float:
    """Table II: bytes sent per Conv + ReLU round, client to server plus server to client, from the
    table's formulas (which give bits).  design: gazelle, cheetah, convfhe or proposed."""
    if design == "gazelle":
        bits = 2 * N * (ceil(2 * w * w * c_i / N) * log_q + ceil(2 * w * w * c_o / N) * log_qp)
    elif design == "cheetah":
        bits = 2 * N * (ceil(w * w * c_i / N) * log_q + c_o * log_qp)
    elif design == "convfhe":
        bits = 2 * N * (ceil(w * w * c_i / N) * log_q + ceil(w * w * c_o / N) * log_qp)
    elif design == "proposed":
        bits = N * ceil(w * w * c_i / N) * log_q + ceil(w * w * c_o * c_o / c_i) * log_qp
    else:
        raise ValueError(design)
    return bits / 8
