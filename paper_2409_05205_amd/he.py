"""ctypes binding of libhe.so (argument marshalling only).

Every computation runs in the HIP library; this module checks shapes, dtypes
and devices, passes raw pointers and the caller's HIP stream, and turns error
codes into exceptions.  Device buffers are torch tensors of dtype int32 holding
the u32 residue words (all residues are below 2^30).  There is no CPU
fallback: if the library is missing, importing the entry points fails.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhe.so")

HE_OK, HE_EINVAL, HE_EUNSUPPORTED, HE_ENOMEM, HE_EDEVICE = 0, -1, -2, -3, -4
HE_LAYER_CONV, HE_LAYER_FC = 0, 1
HE_PACK_CLASS_INTT, HE_PACK_FULL_INTT = 0, 1

EXPORTED = [
    "he_setup", "he_ctx_params", "he_pack_filters", "he_layer_info_get", "he_layer_workspace_bytes",
    "he_conv_layer", "he_conv_layer_ws", "he_fc_layer", "he_fc_layer_ws", "he_ntt_forward",
    "he_ntt_inverse", "he_poly_mul", "he_free_layer", "he_free", "he_strerror", "he_last_error",
    "he_profile_enable", "he_profile_read", "he_profile_reset",
    "he_seq_create", "he_seq_add", "he_seq_run", "he_seq_capture", "he_seq_replay", "he_seq_length",
    "he_seq_free",
    "he_server_create", "he_server_add_layer", "he_server_add_request", "he_server_run", "he_server_requests",
    "he_server_results", "he_server_free",
    "he_tune_force", "he_autotune_layer", "he_tune_get",
    "he_layer_inputs_ntt", "he_conv_layer_ntt", "he_fc_layer_ntt",
    "he_pack_operands", "he_client_masks", "he_encrypt_c0", "he_decrypt", "he_server_add_request_after",
    "he_layer_geometry", "he_ctx_workspace_bytes", "he_workspace_reserve", "he_conv_layer_noalloc",
    "he_sync_check", "he_probe_rate",
    "he_group_create", "he_group_run", "he_group_check", "he_group_items", "he_group_free", "he_group_tune",
    "he_group_set_chunk",
]
HE_PROBE_BFLY, HE_PROBE_GSBFLY, HE_PROBE_MAD64, HE_PROBE_ADD, HE_PROBE_MULLO, HE_PROBE_MULHI = 1, 2, 3, 4, 5, 6
NOALLOC_SCRATCH_BYTES = 32 << 20   # HE_NOALLOC_SCRATCH_BYTES in include/he.h
HE_TUNE_NTT_FWD, HE_TUNE_NTT_INV, HE_TUNE_TAIL, HE_TUNE_MAC = 1, 2, 3, 4
HE_K_NTT_FWD, HE_K_MAC, HE_K_TAIL, HE_K_INTT, HE_K_MAC_TAIL, HE_K_LAYER, HE_K_LAYER_ROWS = 1, 2, 4, 8, 16, 32, 64
HE_K_GROUP = 128
HE_K_MAC_MFMA = 256
HE_GROUP_MAC_AUTO, HE_GROUP_MAC_PER_IMAGE, HE_GROUP_MAC_TILED = 0, 1, 2


class HEError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        super().__init__(f"{what}: {code} ({detail})" if detail else f"{what}: {code}")


class LayerDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("c_i", ctypes.c_uint32), ("c_o", ctypes.c_uint32),
                ("H", ctypes.c_uint32), ("W", ctypes.c_uint32), ("f", ctypes.c_uint32),
                ("stride", ctypes.c_uint32), ("pad", ctypes.c_uint32), ("n_i", ctypes.c_uint32),
                ("n_o", ctypes.c_uint32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("timeout_s", ctypes.c_double)]


class LayerCall(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("layer", ctypes.c_void_p), ("B", ctypes.c_uint32),
                ("d_c0", ctypes.c_void_p), ("d_sh", ctypes.c_void_p), ("d_sh_next", ctypes.c_void_p),
                ("d_out", ctypes.c_void_p)]


class LayerInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("N", ctypes.c_uint32), ("L", ctypes.c_uint32),
                ("s", ctypes.c_uint32), ("g_i", ctypes.c_uint32), ("g_o", ctypes.c_uint32),
                ("K_in", ctypes.c_uint32), ("K_out", ctypes.c_uint32), ("H_p", ctypes.c_uint32),
                ("W_p", ctypes.c_uint32), ("H_o", ctypes.c_uint32), ("W_o", ctypes.c_uint32),
                ("n_o_p", ctypes.c_uint32), ("n_i_p", ctypes.c_uint32), ("blocks", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("resident_bytes", ctypes.c_uint64)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    # torch brings its own HIP runtime (soname libamdhip64.so.7); loading it first makes
    # libhe.so bind to that same runtime, so one process never holds two HIP runtimes.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, U32, VP, SZ = ctypes.POINTER, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t
    lib.he_setup.argtypes = [U32, U32, P(U32), U32, P(VP)]
    lib.he_ctx_params.argtypes = [VP, P(U32), P(U32), P(U32), P(U32), P(U32)]
    lib.he_pack_filters.argtypes = [VP, P(LayerDesc), VP, VP, VP, U32, P(VP)]
    lib.he_layer_info_get.argtypes = [VP, P(LayerInfo)]
    lib.he_layer_workspace_bytes.argtypes = [VP, U32]
    lib.he_layer_workspace_bytes.restype = SZ
    lib.he_layer_geometry.argtypes = [VP, P(LayerDesc), U32, P(LayerInfo)]
    lib.he_ctx_workspace_bytes.argtypes = [VP, U32]
    lib.he_ctx_workspace_bytes.restype = SZ
    lib.he_workspace_reserve.argtypes = [VP, VP, SZ]
    for name in ("he_conv_layer", "he_fc_layer"):
        getattr(lib, name).argtypes = [VP, VP, U32, VP, VP, VP, VP, VP]
    lib.he_conv_layer_noalloc.argtypes = [VP, VP, U32, VP, VP, VP, VP, VP]
    lib.he_sync_check.argtypes = [VP, VP]
    lib.he_probe_rate.argtypes = [U32, U32, P(ctypes.c_double), P(ctypes.c_double)]
    for name in ("he_conv_layer_ws", "he_fc_layer_ws"):
        getattr(lib, name).argtypes = [VP, VP, U32, VP, VP, VP, VP, VP, SZ, VP]
    lib.he_layer_inputs_ntt.argtypes = [VP, VP, U32, VP, VP, VP, VP]
    for name in ("he_conv_layer_ntt", "he_fc_layer_ntt"):
        getattr(lib, name).argtypes = [VP, VP, U32, VP, ctypes.c_int, VP, VP, VP]
    lib.he_ntt_forward.argtypes = [VP, U32, VP, VP, VP]
    lib.he_ntt_inverse.argtypes = [VP, U32, VP, VP, VP]
    lib.he_poly_mul.argtypes = [VP, U32, VP, VP, VP, VP]
    lib.he_profile_enable.argtypes = [VP, U32]
    lib.he_profile_read.argtypes = [VP, U32, P(ctypes.c_uint64), P(ctypes.c_double)]
    lib.he_profile_reset.argtypes = [VP]
    lib.he_seq_create.argtypes = [VP, P(VP)]
    lib.he_seq_add.argtypes = [VP, VP, U32, VP, VP, VP, VP]
    lib.he_seq_run.argtypes = [VP, VP]
    lib.he_seq_capture.argtypes = [VP, VP]
    lib.he_seq_replay.argtypes = [VP, VP]
    lib.he_seq_length.argtypes = [VP]
    lib.he_seq_length.restype = U32
    lib.he_seq_free.argtypes = [VP]
    lib.he_server_create.argtypes = [P(ServerConfig), P(VP)]
    lib.he_server_add_layer.argtypes = [VP, VP, VP, P(U32)]
    lib.he_server_add_request.argtypes = [VP, U32, ctypes.c_double, VP, VP, VP, VP]
    lib.he_server_add_request_after.argtypes = [VP, U32, ctypes.c_double, ctypes.c_int64, VP, VP, VP, VP]
    lib.he_server_run.argtypes = [VP]
    lib.he_server_requests.argtypes = [VP]
    lib.he_server_requests.restype = U32
    D = P(ctypes.c_double)
    lib.he_server_results.argtypes = [VP, D, D, D, P(U32), P(ctypes.c_int32)]
    lib.he_server_free.argtypes = [VP]
    lib.he_pack_operands.argtypes = [VP, P(LayerDesc), VP, VP, U32, P(VP)]
    lib.he_client_masks.argtypes = [VP, VP, VP, VP, VP, P(VP)]
    lib.he_encrypt_c0.argtypes = [VP, U32, VP, VP, VP, VP, VP, VP]
    lib.he_decrypt.argtypes = [VP, U32, U32, VP, VP, VP, VP]
    lib.he_tune_force.argtypes = [VP, U32, ctypes.c_int32]
    lib.he_autotune_layer.argtypes = [VP, VP, U32, VP]
    lib.he_tune_get.argtypes = [VP, U32, U32, U32, P(ctypes.c_int32)]
    lib.he_group_create.argtypes = [P(LayerCall), U32, U32, P(VP)]
    lib.he_group_run.argtypes = [VP, VP]
    lib.he_group_check.argtypes = [VP, VP]
    lib.he_group_items.argtypes = [VP, P(U32), P(U32), P(SZ)]
    lib.he_group_free.argtypes = [VP]
    lib.he_group_tune.argtypes = [VP, VP, P(U32)]
    lib.he_group_set_chunk.argtypes = [VP, U32]
    lib.he_free_layer.argtypes = [VP]
    lib.he_free.argtypes = [VP]
    lib.he_strerror.argtypes = [ctypes.c_int]
    lib.he_strerror.restype = ctypes.c_char_p
    lib.he_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("he_layer_workspace_bytes", "he_strerror", "he_last_error", "he_free", "he_free_layer",
                        "he_seq_length", "he_seq_free", "he_server_requests", "he_server_free", "he_group_free",
                        "he_ctx_workspace_bytes"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != HE_OK:
        lib = load_library()
        raise HEError(rc, what, f"{lib.he_strerror(rc).decode()}; {lib.he_last_error().decode()}")


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _check_dev(t, shape, name: str, allow_none: bool = False):
    import torch
    if t is None:
        if allow_none:
            return
        raise ValueError(f"{name} is required")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype not in (torch.int32, torch.uint32):
        raise ValueError(f"{name} must hold 32-bit words (int32/uint32), got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


@dataclass
class ConvSpec:
    c_i: int
    c_o: int
    H: int
    W: int
    f: int = 3
    stride: int = 1
    pad: int = 1


@dataclass
class FCSpec:
    n_i: int
    n_o: int


def _desc(spec) -> LayerDesc:
    if isinstance(spec, FCSpec):
        return LayerDesc(HE_LAYER_FC, 0, 0, 0, 0, 0, 0, 0, spec.n_i, spec.n_o)
    return LayerDesc(HE_LAYER_CONV, spec.c_i, spec.c_o, spec.H, spec.W, spec.f, spec.stride, spec.pad, 0, 0)


class Layer:
    """A packed layer: NTT-domain operands resident on the device."""

    def __init__(self, ctx: "Context", handle: int, kind: int, rows: int):
        self.ctx = ctx
        self.handle = ctypes.c_void_p(handle)
        self.kind = kind
        self.rows = rows          # output channels (conv) or row blocks (fc)
        info = LayerInfo()
        _check(load_library().he_layer_info_get(self.handle, ctypes.byref(info)), "he_layer_info_get")
        self.info = info

    def __getattr__(self, k):
        info = self.__dict__.get("info")
        if info is not None and k in dict(LayerInfo._fields_):
            return getattr(info, k)
        raise AttributeError(k)

    def workspace_bytes(self, B: int) -> int:
        return int(load_library().he_layer_workspace_bytes(self.handle, B))

    def free(self):
        if self.handle:
            load_library().he_free_layer(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """he_setup: ring degree N, L limbs of 30-bit NTT primes, plaintext modulus t."""

    def __init__(self, N: int, L: int, t: int = 786433, primes: Optional[Sequence[int]] = None):
        lib = load_library()
        h = ctypes.c_void_p()
        parr = None if primes is None else (ctypes.c_uint32 * L)(*[int(p) for p in primes])
        _check(lib.he_setup(N, L, parr, t, ctypes.byref(h)), "he_setup")
        self.handle = h
        ps = (ctypes.c_uint32 * L)()
        ds = (ctypes.c_uint32 * L)()
        _check(lib.he_ctx_params(h, None, None, None, ps, ds), "he_ctx_params")
        self.N, self.L, self.t = N, L, t
        self.primes = [int(x) for x in ps]
        self.delta_l = [int(x) for x in ds]
        self._reserved = {}       # stream handle -> bytes reserved with he_workspace_reserve

    def reserve(self, nbytes: int, stream=None) -> None:
        """Grow the context workspace of `stream` to at least `nbytes` (he_workspace_reserve).  The
        layer calls below reserve what they need on first use; a caller that must not allocate later
        (graph capture, a serving loop) reserves up front."""
        h = _stream(stream)
        if self._reserved.get(h, 0) >= nbytes:
            return
        _check(load_library().he_workspace_reserve(self.handle, h, nbytes), "he_workspace_reserve")
        self._reserved[h] = nbytes

    def sync_check(self, stream=None) -> None:
        """Raise if a one-launch layer call on `stream` gave up a wait (he_sync_check)."""
        _check(load_library().he_sync_check(self.handle, _stream(stream)), "he_sync_check")

    def geometry(self, spec, flags: int = HE_PACK_CLASS_INTT) -> "LayerInfo":
        """The library's tiling of a layer description, before packing (he_layer_geometry)."""
        info = LayerInfo()
        _check(load_library().he_layer_geometry(self.handle, ctypes.byref(_desc(spec)), flags, ctypes.byref(info)),
               "he_layer_geometry")
        return info

    # ---------------------------------------------------------- packing
    def pack_conv(self, spec, weights: np.ndarray, rho: np.ndarray, flags: int = HE_PACK_CLASS_INTT) -> Layer:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.int8))
        if w.shape != (spec.c_o, spec.c_i, spec.f, spec.f):
            raise ValueError(f"weights shape {w.shape}")
        r = np.ascontiguousarray(np.asarray(rho, dtype=np.uint32))
        d = _desc(spec)
        info = self.geometry(spec, flags)
        if r.shape != (info.K_in, spec.c_o, self.N):
            raise ValueError(f"rho shape {r.shape}, expected {(info.K_in, spec.c_o, self.N)}")
        h = ctypes.c_void_p()
        _check(load_library().he_pack_filters(self.handle, ctypes.byref(d), w.ctypes.data, r.ctypes.data, None,
                                              flags, ctypes.byref(h)), "he_pack_filters")
        return Layer(self, h.value, HE_LAYER_CONV, spec.c_o)

    def pack_fc(self, spec, weights: np.ndarray, rho: np.ndarray, bias: Optional[np.ndarray] = None) -> Layer:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.int8))
        if w.shape != (spec.n_o, spec.n_i):
            raise ValueError(f"weights shape {w.shape}")
        r = np.ascontiguousarray(np.asarray(rho, dtype=np.uint32))
        b = None if bias is None else np.ascontiguousarray(np.asarray(bias, dtype=np.int32))
        d = _desc(spec)
        info = self.geometry(spec)
        if r.shape != (info.blocks, self.N):
            raise ValueError(f"rho shape {r.shape}, expected {(info.blocks, self.N)}")
        h = ctypes.c_void_p()
        _check(load_library().he_pack_filters(self.handle, ctypes.byref(d), w.ctypes.data, r.ctypes.data,
                                              None if b is None else b.ctypes.data, 0, ctypes.byref(h)),
               "he_pack_filters")
        layer = Layer(self, h.value, HE_LAYER_FC, 0)
        layer.rows = layer.info.blocks
        return layer

    def pack_operands(self, spec, a: np.ndarray, b: np.ndarray, flags: int = HE_PACK_CLASS_INTT) -> Layer:
        """A layer with resident operands NTT(a), NTT(b) (e.g. the client masks p1, p2).

        conv: a, b [K_in][c_o][L][N]; fc: [blocks][L][N]; u32 residues below each limb's prime.
        """
        a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
        b = np.ascontiguousarray(np.asarray(b, dtype=np.uint32))
        if a.shape != b.shape:
            raise ValueError("a and b must have the same shape")
        d = _desc(spec)
        kind = HE_LAYER_FC if isinstance(spec, FCSpec) else HE_LAYER_CONV
        h = ctypes.c_void_p()
        _check(load_library().he_pack_operands(self.handle, ctypes.byref(d), a.ctypes.data, b.ctypes.data, flags,
                                               ctypes.byref(h)), "he_pack_operands")
        layer = Layer(self, h.value, kind, spec.c_o if kind == HE_LAYER_CONV else 0)
        if kind == HE_LAYER_FC:
            layer.rows = layer.info.blocks
        return layer

    def client_masks(self, server: "Layer", b, e1, e2) -> "Layer":
        """The client's layer for `server` built on the device: masks p1 = rho b + e1 and
        p2 = Delta (fhat + rho) + e2.  b: device int32 [L][N] residues; e1, e2: device int32
        [K_in][c_o][N] (conv) or [blocks][N] (fc)."""
        i = server.info
        shp = (i.K_in, server.rows, self.N) if server.kind == HE_LAYER_CONV else (i.blocks, self.N)
        _check_dev(b, (self.L, self.N), "b")
        _check_dev(e1, shp, "e1")
        _check_dev(e2, shp, "e2")
        h = ctypes.c_void_p()
        _check(load_library().he_client_masks(self.handle, server.handle, _ptr(b), _ptr(e1), _ptr(e2),
                                              ctypes.byref(h)), "he_client_masks")
        return Layer(self, h.value, server.kind, server.rows)

    def encrypt_c0(self, v, b, msg, e0, out=None, stream=None):
        """out = -(v b + Delta msg + e0) per limb; v, e0 int32 [rows][N], b [L][N], msg [rows][N] < t."""
        import torch
        rows = v.shape[0]
        for name, t, shp in (("v", v, (rows, self.N)), ("b", b, (self.L, self.N)), ("msg", msg, (rows, self.N)),
                             ("e0", e0, (rows, self.N))):
            _check_dev(t, shp, name)
        if out is None:
            out = torch.empty((rows, self.L, self.N), dtype=torch.int32, device=v.device)
        _check_dev(out, (rows, self.L, self.N), "out")
        self.reserve(int(load_library().he_ctx_workspace_bytes(self.handle, rows)), stream)
        _check(load_library().he_encrypt_c0(self.handle, rows, _ptr(v), _ptr(b), _ptr(msg), _ptr(e0), _ptr(out),
                                            _stream(stream)), "he_encrypt_c0")
        return out

    def decrypt(self, x0, x1=None, out=None, stream=None):
        """Messages mod t of the share sums x0 + x1: x [rows][L][M] -> [rows][M] (M = N or a prefix length)."""
        import torch
        rows, M = x0.shape[0], x0.shape[-1]
        _check_dev(x0, (rows, self.L, M), "x0")
        _check_dev(x1, (rows, self.L, M), "x1", True)
        if out is None:
            out = torch.empty((rows, M), dtype=torch.int32, device=x0.device)
        _check_dev(out, (rows, M), "out")
        _check(load_library().he_decrypt(self.handle, rows, M, _ptr(x0), _ptr(x1), _ptr(out), _stream(stream)),
               "he_decrypt")
        return out

    # ---------------------------------------------------------- layer calls
    def conv_layer(self, layer: Layer, c0, sh=None, sh_next=None, out=None, stream=None, workspace=None):
        import torch
        B = c0.shape[0]
        i = layer.info
        _check_dev(c0, (B, i.K_in, self.L, self.N), "c0")
        _check_dev(sh, (B, i.K_in, self.N), "sh", True)
        _check_dev(sh_next, (B, i.K_out, self.N), "sh_next", True)
        if out is None:
            out = torch.empty((B, i.K_out, self.L, self.N), dtype=torch.int32, device=c0.device)
        _check_dev(out, (B, i.K_out, self.L, self.N), "out")
        lib = load_library()
        if workspace is None:
            self.reserve(layer.workspace_bytes(B), stream)
            rc = lib.he_conv_layer(self.handle, layer.handle, B, _ptr(c0), _ptr(sh), _ptr(sh_next), _ptr(out),
                                   _stream(stream))
        else:
            rc = lib.he_conv_layer_ws(self.handle, layer.handle, B, _ptr(c0), _ptr(sh), _ptr(sh_next), _ptr(out),
                                      _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream))
        _check(rc, "he_conv_layer")
        return out

    def conv_layer_noalloc(self, layer: Layer, c0, out, sh=None, sh_next=None, stream=None):
        """he_conv_layer_noalloc: the layer with the library's static device scratch as workspace."""
        B = c0.shape[0]
        i = layer.info
        _check_dev(c0, (B, i.K_in, self.L, self.N), "c0")
        _check_dev(sh, (B, i.K_in, self.N), "sh", True)
        _check_dev(sh_next, (B, i.K_out, self.N), "sh_next", True)
        _check_dev(out, (B, i.K_out, self.L, self.N), "out")
        rc = load_library().he_conv_layer_noalloc(self.handle, layer.handle, B, _ptr(c0), _ptr(sh), _ptr(sh_next),
                                                  _ptr(out), _stream(stream))
        _check(rc, "he_conv_layer_noalloc")
        return out

    def fc_layer(self, layer: Layer, c0, sh=None, sh_next=None, out=None, stream=None, workspace=None):
        import torch
        B = c0.shape[0]
        i = layer.info
        _check_dev(c0, (B, self.L, self.N), "c0")
        _check_dev(sh, (B, self.N), "sh", True)
        _check_dev(sh_next, (B, i.blocks, i.n_o_p), "sh_next", True)
        if out is None:
            out = torch.empty((B, i.blocks, self.L, i.n_o_p), dtype=torch.int32, device=c0.device)
        _check_dev(out, (B, i.blocks, self.L, i.n_o_p), "out")
        lib = load_library()
        if workspace is None:
            self.reserve(layer.workspace_bytes(B), stream)
            rc = lib.he_fc_layer(self.handle, layer.handle, B, _ptr(c0), _ptr(sh), _ptr(sh_next), _ptr(out),
                                 _stream(stream))
        else:
            rc = lib.he_fc_layer_ws(self.handle, layer.handle, B, _ptr(c0), _ptr(sh), _ptr(sh_next), _ptr(out),
                                    _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream))
        _check(rc, "he_fc_layer")
        return out

    # ---------------------------------------------------------- NTT-domain inputs (paper's protocol)
    def input_buffer(self, layer: Layer, B: int):
        """An NTT-domain input buffer [B][2 K_in][L][N] for `layer`."""
        import torch
        return torch.empty((B, 2 * layer.info.K_in, self.L, self.N), dtype=torch.int32, device="cuda")

    def inputs_ntt(self, layer: Layer, x, c0=None, sh=None, stream=None):
        """Forward NTTs of c0 and/or sh into x (he_layer_inputs_ntt); returns x."""
        B = x.shape[0]
        i = layer.info
        _check_dev(x, (B, 2 * i.K_in, self.L, self.N), "x")
        if layer.kind == HE_LAYER_CONV:
            _check_dev(c0, (B, i.K_in, self.L, self.N), "c0", True)
            _check_dev(sh, (B, i.K_in, self.N), "sh", True)
        else:
            _check_dev(c0, (B, self.L, self.N), "c0", True)
            _check_dev(sh, (B, self.N), "sh", True)
        _check(load_library().he_layer_inputs_ntt(self.handle, layer.handle, B, _ptr(c0), _ptr(sh), _ptr(x),
                                                  _stream(stream)), "he_layer_inputs_ntt")
        return x

    def layer_from_ntt(self, layer: Layer, x, has_sh: bool, sh_next=None, out=None, stream=None):
        """MAC, inverse and extraction of `layer` from NTT-domain inputs x (he_conv_layer_ntt /
        he_fc_layer_ntt)."""
        import torch
        B = x.shape[0]
        i = layer.info
        _check_dev(x, (B, 2 * i.K_in, self.L, self.N), "x")
        lib = load_library()
        if layer.kind == HE_LAYER_CONV:
            _check_dev(sh_next, (B, i.K_out, self.N), "sh_next", True)
            shape = (B, i.K_out, self.L, self.N)
            fn, name = lib.he_conv_layer_ntt, "he_conv_layer_ntt"
        else:
            _check_dev(sh_next, (B, i.blocks, i.n_o_p), "sh_next", True)
            shape = (B, i.blocks, self.L, i.n_o_p)
            fn, name = lib.he_fc_layer_ntt, "he_fc_layer_ntt"
        if out is None:
            out = torch.empty(shape, dtype=torch.int32, device=x.device)
        _check_dev(out, shape, "out")
        self.reserve(layer.workspace_bytes(B), stream)
        _check(fn(self.handle, layer.handle, B, _ptr(x), 1 if has_sh else 0, _ptr(sh_next), _ptr(out),
                  _stream(stream)), name)
        return out

    # ---------------------------------------------------------- primitives
    def ntt_forward(self, x, out=None, stream=None):
        import torch
        rows = x.shape[0]
        _check_dev(x, (rows, self.L, self.N), "x")
        out = torch.empty_like(x) if out is None else out
        _check(load_library().he_ntt_forward(self.handle, rows, _ptr(x), _ptr(out), _stream(stream)), "he_ntt_forward")
        return out

    def ntt_inverse(self, x, out=None, stream=None):
        import torch
        rows = x.shape[0]
        _check_dev(x, (rows, self.L, self.N), "x")
        out = torch.empty_like(x) if out is None else out
        _check(load_library().he_ntt_inverse(self.handle, rows, _ptr(x), _ptr(out), _stream(stream)), "he_ntt_inverse")
        return out

    def poly_mul(self, a, b, out=None, stream=None):
        import torch
        rows = a.shape[0]
        _check_dev(a, (rows, self.L, self.N), "a")
        _check_dev(b, (rows, self.L, self.N), "b")
        out = torch.empty_like(a) if out is None else out
        self.reserve(int(load_library().he_ctx_workspace_bytes(self.handle, rows)), stream)
        _check(load_library().he_poly_mul(self.handle, rows, _ptr(a), _ptr(b), _ptr(out), _stream(stream)),
               "he_poly_mul")
        return out

    # ---------------------------------------------------------- tuning
    def tune_force(self, knob: int, value: int) -> None:
        _check(load_library().he_tune_force(self.handle, knob, value), "he_tune_force")

    def autotune(self, layer: Layer, B: int, stream=None) -> None:
        _check(load_library().he_autotune_layer(self.handle, layer.handle, B, _stream(stream)), "he_autotune_layer")

    def tune_get(self, knob: int, key_size: int, key_rows: int) -> Optional[int]:
        v = ctypes.c_int32()
        rc = load_library().he_tune_get(self.handle, knob, key_size, key_rows, ctypes.byref(v))
        return int(v.value) if rc == HE_OK else None

    # ---------------------------------------------------------- kernel timing
    def profile_enable(self, kind_mask: int) -> None:
        _check(load_library().he_profile_enable(self.handle, kind_mask), "he_profile_enable")

    def profile_read(self, kind: int):
        n = ctypes.c_uint64()
        ms = ctypes.c_double()
        _check(load_library().he_profile_read(self.handle, kind, ctypes.byref(n), ctypes.byref(ms)),
               "he_profile_read")
        return int(n.value), float(ms.value)

    def profile_reset(self) -> None:
        _check(load_library().he_profile_reset(self.handle), "he_profile_reset")

    def free(self):
        if getattr(self, "handle", None):
            load_library().he_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def probe_rate(kind: int, iters: int = 4096):
    """he_probe_rate: (operations per second of the whole chip, ms of the timed launch)."""
    ops, ms = ctypes.c_double(), ctypes.c_double()
    _check(load_library().he_probe_rate(kind, iters, ctypes.byref(ops), ctypes.byref(ms)), "he_probe_rate")
    return ops.value, ms.value


class Sequence:
    """A recorded list of layer calls (he_seq_*): eager run, or hipGraph capture and replay.

    Keeps references to the layers and buffers it was given so they outlive it.
    """

    def __init__(self, ctx: Context):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(load_library().he_seq_create(ctx.handle, ctypes.byref(h)), "he_seq_create")
        self.handle = h
        self._keep = []

    def add(self, layer: Layer, c0, sh=None, sh_next=None, out=None):
        import torch
        B = c0.shape[0]
        i = layer.info
        if layer.kind == HE_LAYER_CONV:
            _check_dev(c0, (B, i.K_in, self.ctx.L, self.ctx.N), "c0")
            _check_dev(sh, (B, i.K_in, self.ctx.N), "sh", True)
            _check_dev(sh_next, (B, i.K_out, self.ctx.N), "sh_next", True)
            shape = (B, i.K_out, self.ctx.L, self.ctx.N)
        else:
            _check_dev(c0, (B, self.ctx.L, self.ctx.N), "c0")
            _check_dev(sh, (B, self.ctx.N), "sh", True)
            _check_dev(sh_next, (B, i.blocks, i.n_o_p), "sh_next", True)
            shape = (B, i.blocks, self.ctx.L, i.n_o_p)
        if out is None:
            out = torch.empty(shape, dtype=torch.int32, device=c0.device)
        _check_dev(out, shape, "out")
        _check(load_library().he_seq_add(self.handle, layer.handle, B, _ptr(c0), _ptr(sh), _ptr(sh_next),
                                         _ptr(out)), "he_seq_add")
        self._keep.append((layer, c0, sh, sh_next, out))
        return out

    def run(self, stream=None):
        _check(load_library().he_seq_run(self.handle, _stream(stream)), "he_seq_run")

    def capture(self, stream):
        _check(load_library().he_seq_capture(self.handle, _stream(stream)), "he_seq_capture")

    def replay(self, stream=None):
        _check(load_library().he_seq_replay(self.handle, _stream(stream)), "he_seq_replay")

    def __len__(self):
        return int(load_library().he_seq_length(self.handle))

    def free(self):
        if getattr(self, "handle", None):
            load_library().he_seq_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass



class Group:
    """Independent layer calls evaluated by one grouped launch (he_group_*).

    add() the calls (any layers of any contexts on one device), then build() once; run() is one
    launch.  Keeps references to the layers and buffers so they outlive it.
    """

    def __init__(self):
        self.handle = None
        self.chunk_log = 6
        self._calls = []
        self._keep = []

    def add(self, layer: Layer, c0, sh=None, sh_next=None, out=None):
        import torch
        if self.handle is not None:
            raise RuntimeError("Group: add after build")
        ctx = layer.ctx
        B = c0.shape[0]
        i = layer.info
        if layer.kind == HE_LAYER_CONV:
            _check_dev(c0, (B, i.K_in, ctx.L, ctx.N), "c0")
            _check_dev(sh, (B, i.K_in, ctx.N), "sh", True)
            _check_dev(sh_next, (B, i.K_out, ctx.N), "sh_next", True)
            shape = (B, i.K_out, ctx.L, ctx.N)
        else:
            _check_dev(c0, (B, ctx.L, ctx.N), "c0")
            _check_dev(sh, (B, ctx.N), "sh", True)
            _check_dev(sh_next, (B, i.blocks, i.n_o_p), "sh_next", True)
            shape = (B, i.blocks, ctx.L, i.n_o_p)
        if out is None:
            out = torch.empty(shape, dtype=torch.int32, device=c0.device)
        _check_dev(out, shape, "out")
        self._calls.append(LayerCall(ctx.handle, layer.handle, B, _ptr(c0), _ptr(sh), _ptr(sh_next), _ptr(out)))
        self._keep.append((ctx, layer, c0, sh, sh_next, out))
        return out

    def build(self, flags: int = HE_GROUP_MAC_AUTO):
        arr = (LayerCall * len(self._calls))(*self._calls)
        h = ctypes.c_void_p()
        _check(load_library().he_group_create(arr, len(self._calls), flags, ctypes.byref(h)), "he_group_create")
        self.handle = h
        return self

    def run(self, stream=None):
        _check(load_library().he_group_run(self.handle, _stream(stream)), "he_group_run")

    def check(self, stream=None):
        _check(load_library().he_group_check(self.handle, _stream(stream)), "he_group_check")

    def tune(self, stream=None) -> int:
        """he_group_tune: time each XCD chunk size, keep the fastest; returns its log2."""
        c = ctypes.c_uint32()
        _check(load_library().he_group_tune(self.handle, _stream(stream), ctypes.byref(c)), "he_group_tune")
        self.chunk_log = int(c.value)
        return self.chunk_log

    def set_chunk(self, chunk_log: int):
        _check(load_library().he_group_set_chunk(self.handle, chunk_log), "he_group_set_chunk")
        self.chunk_log = chunk_log

    def items(self):
        """(work items per phase (NTT, MAC, inverse), calls with image-tiled MAC, workspace bytes)."""
        it = (ctypes.c_uint32 * 3)()
        tiled, ws = ctypes.c_uint32(), ctypes.c_size_t()
        _check(load_library().he_group_items(self.handle, it, ctypes.byref(tiled), ctypes.byref(ws)),
               "he_group_items")
        return tuple(int(x) for x in it), int(tiled.value), int(ws.value)

    def __len__(self):
        return len(self._calls)

    def free(self):
        if getattr(self, "handle", None):
            load_library().he_group_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """he_server_*: continuous-batching server replaying a trace of layer requests."""

    def __init__(self, streams: int = 4, max_batch: int = 8, hbm_budget_bytes: int = 4 << 30,
                 timeout_s: float = 0.0):
        cfg = ServerConfig(streams, max_batch, hbm_budget_bytes, timeout_s)
        h = ctypes.c_void_p()
        _check(load_library().he_server_create(ctypes.byref(cfg), ctypes.byref(h)), "he_server_create")
        self.handle = h
        self._keep = []

    def add_layer(self, ctx: Context, layer: Layer) -> int:
        lid = ctypes.c_uint32()
        _check(load_library().he_server_add_layer(self.handle, ctx.handle, layer.handle, ctypes.byref(lid)),
               "he_server_add_layer")
        self._keep.append((ctx, layer))
        return int(lid.value)

    def add_request(self, layer_id: int, arrival_s: float, c0, sh, sh_next, out) -> None:
        """Buffers: one image's worth, laid out as for he_conv_layer / he_fc_layer (contiguous views)."""
        for name, t in (("c0", c0), ("out", out)):
            if t is None or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous device tensor")
        _check(load_library().he_server_add_request(self.handle, layer_id, float(arrival_s), _ptr(c0), _ptr(sh),
                                                    _ptr(sh_next), _ptr(out)), "he_server_add_request")

    def add_request_after(self, layer_id: int, arrival_s: float, after: int, c0, sh, sh_next, out) -> None:
        """A request held until request `after` (index of an earlier request, -1 = none) completes."""
        for name, t in (("c0", c0), ("out", out)):
            if t is None or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous device tensor")
        _check(load_library().he_server_add_request_after(self.handle, layer_id, float(arrival_s), int(after),
                                                          _ptr(c0), _ptr(sh), _ptr(sh_next), _ptr(out)),
               "he_server_add_request_after")

    def run(self) -> int:
        """Replay the trace; returns the first error code (0 when every request succeeded)."""
        return int(load_library().he_server_run(self.handle))

    def results(self):
        n = int(load_library().he_server_requests(self.handle))
        arr = np.zeros(n)
        dis = np.zeros(n)
        com = np.zeros(n)
        bat = np.zeros(n, dtype=np.uint32)
        st = np.zeros(n, dtype=np.int32)
        D = ctypes.POINTER(ctypes.c_double)
        _check(load_library().he_server_results(
            self.handle, arr.ctypes.data_as(D), dis.ctypes.data_as(D), com.ctypes.data_as(D),
            bat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
            "he_server_results")
        return dict(arrival=arr, dispatch=dis, complete=com, batch=bat, status=st)

    def free(self):
        if getattr(self, "handle", None):
            load_library().he_server_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
