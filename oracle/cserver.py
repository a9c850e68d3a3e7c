"""ctypes binding of the plain C build of the oracle's server evaluation (oracle/c/he_oracle.c).

Oracle (test infrastructure): used by the test suite and by the benchmark's CPU-baseline leg,
never by the product path.  The C code takes the same inputs as bfv.server_conv / server_fc
(plus the set-up transforms of the masks and packed filters, Sec. IV-A-1) and must give the same
words; tests/test_oracle_c.py checks that against the numpy oracle and the stored digests.

build() compiles the library with gcc (-O2, OpenMP); server_conv / server_fc run one layer.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

from . import bfv
from .packing import ConvGeom, FCGeom

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "he_oracle.c")
LIB = os.path.join(HERE, "c", "liboracle.so")

_lib = None


def build() -> str:
    """Compile oracle/c/he_oracle.c into oracle/c/liboracle.so (gcc -O2 -fopenmp)."""
    tmp = f"{LIB}.{os.getpid()}.tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built (oracle.cserver.build())")
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        U32, I = ctypes.c_uint32, ctypes.c_int
        lib.oracle_ntt_rows.argtypes = [U32, U32, P, P, U32, P, P, I]
        lib.oracle_server_conv.argtypes = [U32, U32, P, P, P, U32, U32, U32, U32, U32, P, P, P, P, P, P, P, I]
        lib.oracle_server_fc.argtypes = [U32, U32, P, P, P, ctypes.c_uint64, U32, U32, P, P, P, P, P, P, P, I]
        lib.oracle_threads.argtypes = [I]
        _lib = lib
    return _lib


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def _i64(a) -> Optional[np.ndarray]:
    return None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _p(a) -> Optional[int]:
    return None if a is None else a.ctypes.data


def _ctx_arrays(ctx: bfv.Ctx):
    return _u64(ctx.primes), _u64(ctx.psis), _u64(ctx.delta_l)


def threads_used(threads: int) -> int:
    return int(load().oracle_threads(threads))


def ntt_rows(ctx: bfv.Ctx, rows, threads: int = 1) -> np.ndarray:
    """Set-up transforms: signed rows [..., N] -> evaluations [..., L, N] for every limb."""
    rows = _i64(rows)
    lead = rows.shape[:-1]
    flat = rows.reshape(-1, ctx.N)
    out = np.empty((flat.shape[0], ctx.L, ctx.N), dtype=np.uint64)
    pr, ps, _ = _ctx_arrays(ctx)
    rc = load().oracle_ntt_rows(ctx.N, ctx.L, _p(pr), _p(ps), flat.shape[0], _p(flat), _p(out), threads)
    if rc != 0:
        raise RuntimeError("oracle_ntt_rows failed")
    return out.reshape(lead + (ctx.L, ctx.N))


def conv_setup(ctx: bfv.Ctx, rho, fhat, threads: int = 1):
    """NTTs of rho [K_in][c_o][N] and fhat [K_in][c_o][N] (kept by the server, Sec. IV-A-1)."""
    return ntt_rows(ctx, rho, threads), ntt_rows(ctx, fhat, threads)


def server_conv(ctx: bfv.Ctx, g: ConvGeom, c0, ops, sh=None, sh_next=None, threads: int = 1) -> np.ndarray:
    """bfv.server_conv in C; ops = conv_setup(ctx, rho, fhat).  Returns [K_out][L][N]."""
    rho_h, f_h = ops
    c0 = _u64(c0)
    sh, shn = _i64(sh), _i64(sh_next)
    cls = np.ascontiguousarray(np.array([g.class_of(n) for n in range(g.c_o)], dtype=np.uint32))
    out = np.empty((g.K_out, ctx.L, ctx.N), dtype=np.uint64)
    pr, ps, dl = _ctx_arrays(ctx)
    rc = load().oracle_server_conv(ctx.N, ctx.L, _p(pr), _p(ps), _p(dl), g.K_in, g.c_o, g.g_o, g.K_out, g.s,
                                   _p(cls), _p(c0), _p(rho_h), _p(f_h), _p(sh), _p(shn), _p(out), threads)
    if rc != 0:
        raise RuntimeError("oracle_server_conv failed")
    return out


def fc_setup(ctx: bfv.Ctx, rho, w, threads: int = 1):
    """NTTs of rho [blocks][N] and the packed weights w [blocks][N]."""
    return ntt_rows(ctx, rho, threads), ntt_rows(ctx, w, threads)


def server_fc(ctx: bfv.Ctx, g: FCGeom, c0, ops, d=None, sh=None, sh_next=None, threads: int = 1) -> np.ndarray:
    """bfv.server_fc in C; ops = fc_setup(ctx, rho, w).  Returns [blocks][L][n_o']."""
    rho_h, w_h = ops
    c0 = _u64(c0)
    dd = _i64(np.zeros((g.blocks, g.n_o_p), dtype=np.int64) if d is None else d)
    sh, shn = _i64(sh), _i64(sh_next)
    out = np.empty((g.blocks, ctx.L, g.n_o_p), dtype=np.uint64)
    pr, ps, dl = _ctx_arrays(ctx)
    rc = load().oracle_server_fc(ctx.N, ctx.L, _p(pr), _p(ps), _p(dl), ctx.t, g.blocks, g.n_o_p, _p(c0),
                                 _p(rho_h), _p(w_h), _p(sh), _p(dd), _p(shn), _p(out), threads)
    if rc != 0:
        raise RuntimeError("oracle_server_fc failed")
    return out
