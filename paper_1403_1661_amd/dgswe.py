"""ctypes binding of the dgswe C ABI (``include/dgswe.h``).

Argument marshalling only: every step of the solver runs in the HIP library
``libdgswe.so``; PyTorch is used for the device workspace and the stream.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgswe.so")

DG_OK = 0
ERRORS = {-1: "DG_EINVAL", -2: "DG_EMESH", -3: "DG_ENOMEM", -4: "DG_EDEVICE",
          -5: "DG_ENOTBOUND", -6: "DG_ENUMERIC", -7: "DG_ESTATE"}

DG_PLAIN_FP32, DG_FUSED_FP32, DG_FUSED_MFMA32, DG_FUSED_BF16X3, DG_FUSED_BF16X6 = 0, 1, 2, 3, 4
PRECISIONS = {"plain_fp32": DG_PLAIN_FP32, "fused_fp32": DG_FUSED_FP32,
              "fused_mfma32": DG_FUSED_MFMA32, "fused_bf16x3": DG_FUSED_BF16X3,
              "fused_bf16x6": DG_FUSED_BF16X6}
DG_LIMIT_PP, DG_LIMIT_TVB = 1, 2

# every symbol include/dgswe.h declares
EXPORTS = ["dg_default_params", "dg_create", "dg_destroy", "dg_last_error", "dg_query_sizes",
           "dg_bind", "dg_instance_elements", "dg_node_coords", "dg_reference",
           "dg_reference_nodes", "dg_set_bathymetry", "dg_set_state", "dg_prepare",
           "dg_advance", "dg_get_state", "dg_get_connectivity", "dg_get_levels",
           "dg_get_tvb_stencil", "dg_get_flags", "dg_get_diagnostics", "dg_checkpoint_bytes",
           "dg_get_checkpoint", "dg_set_checkpoint", "dg_set_profiling", "dg_kernel_timing",
           "dg_autotune", "dg_capture_graph", "dg_get_diagnostics_noalloc"]


class DGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("vx", C.POINTER(C.c_double)),
                ("vy", C.POINTER(C.c_double)), ("n_elements", C.c_int32),
                ("etov", C.POINTER(C.c_int32)), ("bc", C.POINTER(C.c_int8))]


class Params(C.Structure):
    _fields_ = [("N", C.c_int32), ("g", C.c_double), ("cfl", C.c_double), ("h0", C.c_double),
                ("eps", C.c_double), ("hvel", C.c_double), ("tvb_M", C.c_double), ("tvb_nu", C.c_double),
                ("limiter_mask", C.c_int32), ("max_levels", C.c_int32),
                ("precision", C.c_int32), ("dry_literal", C.c_int32), ("use_graph", C.c_int32),
                ("elems_per_block", C.c_int32), ("thin_cut", C.c_double), ("overint", C.c_int32),
                ("regroup_every", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("min_depth", C.c_double), ("time", C.c_double),
                ("steps", C.c_int64), ("negative_means", C.c_int64),
                ("pp_counts", C.c_int64 * 3), ("tvb_counts", C.c_int64 * 4)]


_lib = None

_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I32 = C.c_int32
_I64 = C.c_int64


def load_library(path: Optional[str] = None):
    """Load libdgswe.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime under the same soname; load it first so
    # that the library binds to the runtime torch's allocator and streams use
    import torch  # noqa: F401
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1403_1661_amd.build`")
    lib = C.CDLL(path)
    sig = {
        "dg_default_params": (_I32, [_I32, C.POINTER(Params)]),
        "dg_create": (_I32, [C.POINTER(MeshDesc), _I32, C.POINTER(Params), C.POINTER(_P)]),
        "dg_destroy": (None, [_P]),
        "dg_last_error": (C.c_char_p, []),
        "dg_query_sizes": (_I32, [_P, C.POINTER(_I64), C.POINTER(_I32), C.POINTER(_I32),
                                  C.POINTER(_I64)]),
        "dg_bind": (_I32, [_P, _P, _I64, _P]),
        "dg_instance_elements": (_I32, [_P, _I32, C.POINTER(_I32)]),
        "dg_node_coords": (_I32, [_P, _I32, _D, _D]),
        "dg_reference": (_I32, [_P, _I32, _D]),
        "dg_reference_nodes": (_I32, [_P, _D, _D]),
        "dg_set_bathymetry": (_I32, [_P, _I32, _D]),
        "dg_set_state": (_I32, [_P, _I32, _D, _D, _D, _P]),
        "dg_prepare": (_I32, [_P, _P]),
        "dg_advance": (_I32, [_P, _I32, _P]),
        "dg_get_state": (_I32, [_P, _I32, _D, _D, _D, _P]),
        "dg_get_connectivity": (_I32, [_P, _I32, C.POINTER(C.c_int32), C.POINTER(C.c_int8)]),
        "dg_get_levels": (_I32, [_P, _I32, C.POINTER(C.c_int8), _D]),
        "dg_get_tvb_stencil": (_I32, [_P, _I32, C.POINTER(C.c_int8), _D]),
        "dg_get_flags": (_I32, [_P, _I32, C.POINTER(C.c_uint8), _P]),
        "dg_get_diagnostics": (_I32, [_P, _I32, C.POINTER(Diag), _P]),
        "dg_checkpoint_bytes": (_I32, [_P, C.POINTER(_I64)]),
        "dg_get_checkpoint": (_I32, [_P, _P, _I64, _P]),
        "dg_set_checkpoint": (_I32, [_P, _P, _I64, _P]),
        "dg_set_profiling": (_I32, [_P, _I32]),
        "dg_kernel_timing": (_I32, [_P, _I32, _D, C.POINTER(_I64), C.POINTER(_I64)]),
        "dg_capture_graph": (_I32, [_P, _P]),
        "dg_get_diagnostics_noalloc": (_I32, [_P, _I32, _P, _P]),
        "dg_autotune": (_I32, [_P, _I32, _I32, C.POINTER(_I32), C.POINTER(_I32), _D, _P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != DG_OK:
        raise DGError(rc, _lib.dg_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def default_params(N: int, **kw) -> Params:
    lib = load_library()
    p = Params()
    _check(lib.dg_default_params(N, C.byref(p)))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class Solver:
    """One solver handle over one or more triangulated instances."""

    def __init__(self, meshes: Sequence, N: int, **params):
        self.lib = load_library()
        self.N = N
        self.params = default_params(N, **params)
        self._keep = []
        descs = (MeshDesc * len(meshes))()
        for i, mesh in enumerate(meshes):
            # (vx, vy, etov) or (vx, vy, etov, bc) with bc the (K, 3) face tags
            vx, vy, etov = mesh[:3]
            vx = np.ascontiguousarray(vx, dtype=np.float64)
            vy = np.ascontiguousarray(vy, dtype=np.float64)
            ev = np.ascontiguousarray(etov, dtype=np.int32)
            if ev.ndim != 2 or ev.shape[1] != 3:
                raise ValueError(f"mesh {i}: etov must be (K, 3), got {ev.shape}")
            if vx.shape != vy.shape:
                raise ValueError(f"mesh {i}: vx and vy differ in shape")
            self._keep += [vx, vy, ev]
            descs[i].n_vertices = vx.size
            descs[i].vx = _dptr(vx)
            descs[i].vy = _dptr(vy)
            descs[i].n_elements = ev.shape[0]
            descs[i].etov = ev.ctypes.data_as(C.POINTER(C.c_int32))
            if len(mesh) > 3 and mesh[3] is not None:
                bc = np.ascontiguousarray(mesh[3], dtype=np.int8)
                if bc.shape != ev.shape:
                    raise ValueError(f"mesh {i}: bc has shape {bc.shape}, etov {ev.shape}")
                self._keep.append(bc)
                descs[i].bc = bc.ctypes.data_as(C.POINTER(C.c_int8))
        h = C.c_void_p()
        _check(self.lib.dg_create(descs, len(meshes), C.byref(self.params), C.byref(h)))
        self.h = h
        self._keep = []
        self.n_inst = len(meshes)
        K, Np, Nfp, ws = _I64(), _I32(), _I32(), _I64()
        _check(self.lib.dg_query_sizes(self.h, C.byref(K), C.byref(Np), C.byref(Nfp), C.byref(ws)))
        self.K, self.Np, self.Nfp, self.workspace_bytes = K.value, Np.value, Nfp.value, ws.value
        self.Ks = []
        for i in range(self.n_inst):
            k = _I32()
            _check(self.lib.dg_instance_elements(self.h, i, C.byref(k)))
            self.Ks.append(k.value)
        self.workspace = None
        self.device = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.dg_destroy(h)
            self.h = None

    # -- device ---------------------------------------------------------
    @staticmethod
    def _stream(stream=None) -> int:
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        return int(s.cuda_stream)

    def bind(self, device="cuda:0", stream=None):
        import torch
        dev = torch.device(device)
        torch.cuda.set_device(dev)
        buf = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        off = (-buf.data_ptr()) % 256
        self.workspace = buf
        self._ws_ptr = buf.data_ptr() + off
        self.device = dev
        _check(self.lib.dg_bind(self.h, C.c_void_p(self._ws_ptr), self.workspace_bytes,
                                C.c_void_p(self._stream(stream))))
        return self

    # -- host setup data ------------------------------------------------
    def node_coords(self, inst=0):
        K = self.Ks[inst]
        x = np.empty((K, self.Np))
        y = np.empty((K, self.Np))
        _check(self.lib.dg_node_coords(self.h, inst, _dptr(x), _dptr(y)))
        return x, y

    def reference(self, which: int):
        q = (3 * self.N + 2) // 2
        nc = q * q
        shapes = {0: (self.Np, self.Np), 1: (self.Np, self.Np), 2: (self.Np, 3 * self.Nfp),
                  3: (self.Np, self.Np), 4: (self.Np,), 5: (3, self.Nfp), 6: (3, nc), 7: (nc, self.Np),
                  8: (self.Np, nc), 9: (self.Np, nc), 10: (self.Np, nc), 11: (2, q), 12: (q, self.Nfp),
                  13: (self.Np, 3 * q)}
        out = np.empty(shapes[which])
        _check(self.lib.dg_reference(self.h, which, _dptr(out)))
        return out

    def reference_nodes(self):
        r = np.empty(self.Np)
        s = np.empty(self.Np)
        _check(self.lib.dg_reference_nodes(self.h, _dptr(r), _dptr(s)))
        return r, s

    def connectivity(self, inst=0):
        K = self.Ks[inst]
        etoe = np.empty((K, 3), dtype=np.int32)
        etof = np.empty((K, 3), dtype=np.int8)
        _check(self.lib.dg_get_connectivity(self.h, inst, etoe.ctypes.data_as(C.POINTER(C.c_int32)),
                                            etof.ctypes.data_as(C.POINTER(C.c_int8))))
        return etoe, etof

    def levels(self, inst=0):
        K = self.Ks[inst]
        lev = np.empty(K, dtype=np.int8)
        dt = C.c_double()
        _check(self.lib.dg_get_levels(self.h, inst, lev.ctypes.data_as(C.POINTER(C.c_int8)),
                                      C.byref(dt)))
        return lev, dt.value

    def tvb_stencil(self, inst=0):
        K = self.Ks[inst]
        pair = np.empty((K, 3, 2), dtype=np.int8)
        alpha = np.empty((K, 3, 2))
        _check(self.lib.dg_get_tvb_stencil(self.h, inst, pair.ctypes.data_as(C.POINTER(C.c_int8)),
                                           _dptr(alpha)))
        return pair, alpha

    # -- state ----------------------------------------------------------
    def _check_nodal(self, inst, a):
        if not 0 <= inst < self.n_inst:
            raise IndexError(f"instance {inst} out of range 0..{self.n_inst - 1}")
        if a.shape != (self.Ks[inst], self.Np):
            raise ValueError(f"nodal array of instance {inst} must be {(self.Ks[inst], self.Np)}, "
                             f"got {a.shape}")

    def set_bathymetry(self, inst, B):
        B = np.ascontiguousarray(B, dtype=np.float64)
        self._check_nodal(inst, B)
        _check(self.lib.dg_set_bathymetry(self.h, inst, _dptr(B)))

    def set_state(self, inst, h, hu, hv, stream=None):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (h, hu, hv)]
        for a in arrs:
            self._check_nodal(inst, a)
        _check(self.lib.dg_set_state(self.h, inst, *[_dptr(a) for a in arrs],
                                     C.c_void_p(self._stream(stream))))

    def prepare(self, stream=None):
        _check(self.lib.dg_prepare(self.h, C.c_void_p(self._stream(stream))))

    def advance(self, n_steps: int, stream=None):
        _check(self.lib.dg_advance(self.h, int(n_steps), C.c_void_p(self._stream(stream))))

    def get_state(self, inst=0, stream=None):
        K = self.Ks[inst]
        out = [np.empty((K, self.Np)) for _ in range(3)]
        _check(self.lib.dg_get_state(self.h, inst, *[_dptr(a) for a in out],
                                     C.c_void_p(self._stream(stream))))
        return out

    def flags(self, inst=0, stream=None):
        f = np.empty(self.Ks[inst], dtype=np.uint8)
        _check(self.lib.dg_get_flags(self.h, inst, f.ctypes.data_as(C.POINTER(C.c_uint8)),
                                     C.c_void_p(self._stream(stream))))
        return f

    def diagnostics(self, inst=0, stream=None) -> dict:
        d = Diag()
        _check(self.lib.dg_get_diagnostics(self.h, inst, C.byref(d),
                                           C.c_void_p(self._stream(stream))))
        return {"mass": d.mass, "min_depth": d.min_depth, "time": d.time, "steps": d.steps,
                "negative_means": d.negative_means, "pp_counts": list(d.pp_counts),
                "tvb_counts": list(d.tvb_counts)}

    def diagnostics_noalloc(self, inst, out_device_ptr: int, stream=None):
        """Enqueue the diagnostics reductions into 9 doubles at a device
        address (mass, min depth, positivity and TVB code counts)."""
        _check(self.lib.dg_get_diagnostics_noalloc(self.h, inst, C.c_void_p(out_device_ptr),
                                                   C.c_void_p(self._stream(stream))))

    def checkpoint(self, stream=None) -> bytes:
        n = _I64()
        _check(self.lib.dg_checkpoint_bytes(self.h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(self.lib.dg_get_checkpoint(self.h, buf, n.value, C.c_void_p(self._stream(stream))))
        return buf.raw

    def restore(self, blob: bytes, stream=None):
        buf = C.create_string_buffer(blob, len(blob))
        _check(self.lib.dg_set_checkpoint(self.h, buf, len(blob), C.c_void_p(self._stream(stream))))

    def set_profiling(self, on: bool):
        _check(self.lib.dg_set_profiling(self.h, 1 if on else 0))

    def kernel_timing(self, which: int = 0):
        """(average us, launches, elements per launch) of the step kernel
        (which = 0) or the TVB kernel (which = 1) over the profiling region."""
        us = C.c_double()
        n = _I64()
        e = _I64()
        _check(self.lib.dg_kernel_timing(self.h, int(which), C.byref(us), C.byref(n), C.byref(e)))
        return us.value, n.value, e.value

    def capture_graph(self, stream=None):
        _check(self.lib.dg_capture_graph(self.h, C.c_void_p(self._stream(stream))))

    def autotune(self, reps: int = 10, stream=None):
        """Time each elements-per-block candidate of the step kernel on the
        current state and keep the fastest; returns [(elements, us), ...]."""
        n = _I32()
        epb = (_I32 * 8)()
        us = (C.c_double * 8)()
        _check(self.lib.dg_autotune(self.h, reps, 8, C.byref(n), epb,
                                    C.cast(us, _D), C.c_void_p(self._stream(stream))))
        return [(int(epb[i]), float(us[i])) for i in range(min(n.value, 8))]
