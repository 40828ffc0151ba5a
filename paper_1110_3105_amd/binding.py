"""ctypes binding of the C ABI declared in include/rs.h (argument marshalling only).

Every numerical step runs in the HIP library ``lib/librs.so``.  If that library is
missing the import fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "librs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                      "(run `python paper_1110_3105_amd/build.py`)")

# PyTorch ships its own HIP runtime with the same soname (libamdhip64.so.7).  Loading
# torch first makes the library bind to that copy, so that the process holds one HIP
# runtime shared by torch's allocator/streams and the library's kernels.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

RS_OK, RS_EINVAL, RS_ENOMEM, RS_ESINGULAR, RS_EDEVICE, RS_EBUSY, RS_ENOTSUP = range(7)
STATUS_NAMES = {0: "RS_OK", 1: "RS_EINVAL", 2: "RS_ENOMEM", 3: "RS_ESINGULAR",
                4: "RS_EDEVICE", 5: "RS_EBUSY", 6: "RS_ENOTSUP"}
KINDS = {"lap2d_sl": 1, "lap2d_dl": 2, "lap3d_sl": 3, "helm2d_cfie": 4, "helm3d_sl": 5}
LAUNCH = {"level": 0, "per_box": 1}

EXPORTED = ["rs_build_tree", "rs_tree_info", "rs_tree_export", "rs_tree_free", "rs_factor",
            "rs_factor_ex", "rs_solve", "rs_solve_ex", "rs_free", "rs_last_error",
            "rs_device_count", "rs_query", "rs_box_skeletons", "rs_box_export",
            "rs_profile_enable", "rs_profile_reset", "rs_profile_read", "rs_factor_batched",
            "rs_solve_batched", "rs_server_create", "rs_server_submit_factor",
            "rs_server_submit_solve", "rs_server_poll", "rs_server_release", "rs_server_query",
            "rs_server_reset_stats", "rs_server_destroy", "rs_plan_create", "rs_plan_launch",
            "rs_plan_free", "rs_autotune", "rs_tune_entries", "rs_tune_clear", "rs_tune_save",
            "rs_tune_load", "rs_solve_noalloc", "rs_matvec", "rs_query_levels",
            "rs_factor_estimate", "rs_factor_solve_ex"]
FAMILIES = ["assemble", "id", "factor", "sweep_up", "sweep_down", "permute"]


class rs_kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("identity", C.c_double),
                ("wavenumber", C.c_double), ("eta", C.c_double),
                ("normals", C.POINTER(C.c_double)), ("curvature", C.POINTER(C.c_double)),
                ("proxy_points", C.c_int32), ("proxy_ratio", C.c_double),
                ("id_mode", C.c_int32), ("oversample", C.c_int32), ("sketch_seed", C.c_uint64)]


ID_MODES = {"cpqr": 0, "sketch": 1}


class rs_options(C.Structure):
    _fields_ = [("launch_mode", C.c_int32), ("stream", C.c_void_p)]


class rs_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("nbox", C.c_int64), ("maxdepth", C.c_int32),
                ("dim", C.c_int32), ("root_size", C.c_int64), ("total_skeletons", C.c_int64),
                ("factor_doubles", C.c_int64), ("max_box_n", C.c_int64),
                ("max_box_m", C.c_int64), ("factor_ms", C.c_double), ("plan_ms", C.c_double),
                ("wait_ms", C.c_double), ("complex_values", C.c_int32), ("pad", C.c_int32)]


class rs_level_stats(C.Structure):
    _fields_ = [("depth", C.c_int32), ("boxes", C.c_int32), ("n_total", C.c_int64),
                ("k_total", C.c_int64), ("max_n", C.c_int32), ("max_m", C.c_int32),
                ("factor_doubles", C.c_int64), ("device_ms", C.c_double), ("plan_ms", C.c_double)]


class rs_server_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_batch_requests", C.c_int32),
                ("max_batch_rhs", C.c_int32)]


class rs_server_stats(C.Structure):
    _fields_ = [("solves_done", C.c_int64), ("rhs_done", C.c_int64), ("factors_done", C.c_int64),
                ("rejected", C.c_int64), ("batches", C.c_int64), ("resident_bytes", C.c_int64),
                ("queued_solves", C.c_int64), ("queued_factors", C.c_int64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("window_ms", C.c_double)]


_P = C.c_void_p
_PD = C.POINTER(C.c_double)
_PI64 = C.POINTER(C.c_int64)
_PI32 = C.POINTER(C.c_int32)

_sig = {
    "rs_build_tree": (C.c_int, [C.c_int32, C.c_int64, _PD, C.c_int32, C.POINTER(_P)]),
    "rs_tree_info": (C.c_int, [_P, _PI64, _PI32]),
    "rs_tree_export": (C.c_int, [_P, _PI64, _PI32, _PI32, _PI64, _PI64, _PD, _PD]),
    "rs_tree_free": (None, [_P]),
    "rs_factor": (C.c_int, [C.POINTER(rs_kernel), _P, _PD, _PD, C.c_double, C.POINTER(_P)]),
    "rs_factor_ex": (C.c_int, [C.POINTER(rs_kernel), _P, _PD, _PD, C.c_double,
                               C.POINTER(rs_options), C.POINTER(_P)]),
    "rs_factor_solve_ex": (C.c_int, [C.POINTER(rs_kernel), _P, _PD, _PD, C.c_double,
                                     C.POINTER(rs_options), _P, C.c_int64, C.c_int32,
                                     C.POINTER(_P)]),
    "rs_solve": (C.c_int, [_P, _P, C.c_int64, C.c_int32, _P]),
    "rs_solve_ex": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.POINTER(rs_options)]),
    "rs_solve_noalloc": (C.c_int, [_P, _P, C.c_int64, C.c_int32, _P]),
    "rs_matvec": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int64, C.c_int32, _P]),
    "rs_free": (C.c_int, [_P]),
    "rs_last_error": (C.c_char_p, []),
    "rs_device_count": (C.c_int32, []),
    "rs_query": (C.c_int, [_P, C.POINTER(rs_stats)]),
    "rs_factor_estimate": (C.c_int, [C.POINTER(rs_kernel), _P, C.c_double,
                                     C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "rs_query_levels": (C.c_int, [_P, C.POINTER(rs_level_stats), C.c_int32,
                                  C.POINTER(C.c_int32)]),
    "rs_box_skeletons": (C.c_int, [_P, _PI32, _PI64, C.c_int64, _PI64]),
    "rs_box_export": (C.c_int, [_P, C.c_int64, _PI32, _PI32, _PI64, _PD]),
    "rs_factor_batched": (C.c_int, [C.c_int32, C.POINTER(rs_kernel), C.POINTER(_P),
                                    C.POINTER(_PD), C.POINTER(_PD), _PD, C.POINTER(rs_options),
                                    C.POINTER(_P)]),
    "rs_solve_batched": (C.c_int, [C.c_int32, C.POINTER(_P), C.POINTER(C.c_void_p), _PI64,
                                   _PI32, C.POINTER(rs_options)]),
    "rs_server_create": (C.c_int, [C.POINTER(rs_server_opts), C.POINTER(_P)]),
    "rs_server_submit_factor": (C.c_int, [_P, C.POINTER(rs_kernel), _P, _PD, _PD, C.c_double,
                                          C.POINTER(C.c_uint64)]),
    "rs_server_submit_solve": (C.c_int, [_P, _P, C.c_void_p, C.c_int64, C.c_int32, _P,
                                         C.POINTER(C.c_uint64)]),
    "rs_server_poll": (C.c_int, [_P, C.c_uint64, C.c_int32, _PI32, _PI32, C.POINTER(_P)]),
    "rs_server_release": (C.c_int, [_P, _P]),
    "rs_server_query": (C.c_int, [_P, C.POINTER(rs_server_stats)]),
    "rs_server_reset_stats": (C.c_int, [_P]),
    "rs_server_destroy": (None, [_P]),
    "rs_plan_create": (C.c_int, [C.c_int32, C.POINTER(_P), C.POINTER(C.c_void_p), _PI64, _PI32,
                                 C.POINTER(_P)]),
    "rs_plan_launch": (C.c_int, [_P, _P]),
    "rs_plan_free": (C.c_int, [_P]),
    "rs_autotune": (C.c_int, [_P, _PI32, C.c_int32, C.c_int32, _P]),
    "rs_tune_entries": (C.c_int, [C.POINTER(C.c_uint32), _PI32, C.c_int32, _PI32]),
    "rs_tune_clear": (C.c_int, []),
    "rs_tune_save": (C.c_int, [C.c_char_p]),
    "rs_tune_load": (C.c_int, [C.c_char_p]),
    "rs_profile_enable": (C.c_int, [C.c_int32]),
    "rs_profile_reset": (C.c_int, []),
    "rs_profile_read": (C.c_int, [C.c_int32, _PI64, _PD, _PD, _PD, _PD]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


class RSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code: int):
    if code != RS_OK:
        raise RSError(code, _lib.rs_last_error().decode())


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_PD)


def device_count() -> int:
    return int(_lib.rs_device_count())


def profile_enable(on: bool = True):
    _check(_lib.rs_profile_enable(1 if on else 0))


def profile_reset():
    _check(_lib.rs_profile_reset())


def profile_read() -> dict:
    """Per kernel family: launches, total_ms, flops, bytes, entries since the last reset."""
    out = {}
    for i, name in enumerate(FAMILIES):
        n = C.c_int64()
        ms, fl, by, en = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        _check(_lib.rs_profile_read(i, C.byref(n), C.byref(ms), C.byref(fl), C.byref(by),
                                    C.byref(en)))
        out[name] = dict(launches=int(n.value), total_ms=ms.value, flops=fl.value,
                         bytes=by.value, entries=en.value)
    return out


class Tree:
    """Owning wrapper of an rs_tree."""

    def __init__(self, points: np.ndarray, leaf_size: int):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim != 2:
            raise ValueError("points must be (n, dim)")
        self.points = pts
        self.n, self.dim = pts.shape
        h = _P()
        _check(_lib.rs_build_tree(self.dim, self.n, _dptr(pts), int(leaf_size), C.byref(h)))
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            _lib.rs_tree_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self):
        nb, md = C.c_int64(), C.c_int32()
        _check(_lib.rs_tree_info(self._h, C.byref(nb), C.byref(md)))
        return int(nb.value), int(md.value)

    def export(self) -> dict:
        nb, _ = self.info()
        perm = np.empty(self.n, dtype=np.int64)
        depth = np.empty(nb, dtype=np.int32)
        parent = np.empty(nb, dtype=np.int32)
        begin = np.empty(nb, dtype=np.int64)
        end = np.empty(nb, dtype=np.int64)
        center = np.empty((nb, self.dim), dtype=np.float64)
        side = np.empty(nb, dtype=np.float64)
        _check(_lib.rs_tree_export(self._h, perm.ctypes.data_as(_PI64),
                                   depth.ctypes.data_as(_PI32), parent.ctypes.data_as(_PI32),
                                   begin.ctypes.data_as(_PI64), end.ctypes.data_as(_PI64),
                                   center.ctypes.data_as(_PD), side.ctypes.data_as(_PD)))
        return dict(perm=perm, depth=depth, parent=parent, begin=begin, end=end,
                    center=center, side=side)


def build_tree(points: np.ndarray, leaf_size: int) -> Tree:
    return Tree(points, leaf_size)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)      # torch.cuda.Stream


def _rhs_dtype(complex_values: bool):
    import torch
    return torch.complex128 if complex_values else torch.float64


class Handle:
    """Owning wrapper of an rs_handle (compressed inverse resident in device memory)."""

    def __init__(self, h, n: int, keep, server=None):
        self._h = h
        self.n = n
        self._keep = keep
        self._server = server
        self.is_complex = bool(self.stats()["complex_values"])

    @property
    def dtype(self):
        """torch dtype of right-hand sides: float64, or complex128 for Helmholtz."""
        return _rhs_dtype(self.is_complex)

    def __del__(self):
        try:
            self.free()
        except RSError as e:
            if e.code == RS_EBUSY and self._server is None:
                try:
                    import torch
                    torch.cuda.synchronize()
                    self.free()
                except Exception:
                    pass
        except Exception:
            pass

    def free(self):
        """Releases the factorization (RS_EBUSY while a solve on it is still queued or
        running on its stream: synchronize that stream first)."""
        if getattr(self, "_h", None):
            if self._server is not None:
                if self._server._s is not None:
                    _check(_lib.rs_server_release(self._server._s, self._h))
            else:
                _check(_lib.rs_free(self._h))
            self._h = None

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        s = rs_stats()
        _check(_lib.rs_query(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in rs_stats._fields_}

    def levels(self) -> list:
        """Per-level records of the factorization, finest level first and the root last."""
        cnt = C.c_int32(0)
        _check(_lib.rs_query_levels(self._h, None, 0, C.byref(cnt)))
        arr = (rs_level_stats * max(cnt.value, 1))()
        _check(_lib.rs_query_levels(self._h, arr, cnt.value, C.byref(cnt)))
        return [{f: getattr(arr[i], f) for f, _ in rs_level_stats._fields_}
                for i in range(cnt.value)]

    def solve_ptr(self, ptr: int, ldb: int, nrhs: int, stream=None, launch_mode: str = "level"):
        o = rs_options(LAUNCH[launch_mode], _stream_ptr(stream))
        _check(_lib.rs_solve_ex(self._h, C.c_void_p(ptr), int(ldb), int(nrhs), C.byref(o)))

    def solve(self, B, stream=None, launch_mode: str = "level"):
        """In-place B := A_eps^{-1} B for a CUDA tensor of shape (n,) or (n, nrhs), float64
        (complex128 for a Helmholtz handle)."""
        import torch
        if not (isinstance(B, torch.Tensor) and B.is_cuda and B.dtype == self.dtype):
            raise TypeError(f"B must be a {self.dtype} tensor on the HIP device")
        vec = B.dim() == 1
        X = B.unsqueeze(1) if vec else B
        if X.shape[0] != self.n:
            raise ValueError("B has the wrong number of rows")
        nrhs = X.shape[1]
        colmajor = X.stride(0) == 1 and (nrhs == 1 or X.stride(1) >= self.n)
        work = X if colmajor else X.t().contiguous().t()
        ldb = work.stride(1) if nrhs > 1 else self.n
        if stream is None:
            stream = torch.cuda.current_stream(B.device)
        self.solve_ptr(work.data_ptr(), ldb, nrhs, stream, launch_mode)
        if not colmajor:
            X.copy_(work)
        return B

    def matvec(self, X, stream=None):
        """Y = A_eps X (compressed forward operator) for a device tensor X of shape (n,) or
        (n, nrhs); returns a new column-major tensor."""
        import torch
        if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == self.dtype):
            raise TypeError(f"X must be a {self.dtype} tensor on the HIP device")
        vec = X.dim() == 1
        X2 = X.unsqueeze(1) if vec else X
        if X2.shape[0] != self.n:
            raise ValueError("X has the wrong number of rows")
        nrhs = X2.shape[1]
        if not (X2.stride(0) == 1 and (nrhs == 1 or X2.stride(1) >= self.n)):
            X2 = X2.t().contiguous().t()
        ldx = X2.stride(1) if nrhs > 1 else self.n
        Y = torch.empty(nrhs, self.n, dtype=X.dtype, device=X.device).t()
        if stream is None:
            stream = torch.cuda.current_stream(X.device)
        _check(_lib.rs_matvec(self._h, C.c_void_p(X2.data_ptr()), int(ldx),
                              C.c_void_p(Y.data_ptr()), self.n, int(nrhs), _stream_ptr(stream)))
        return Y[:, 0] if vec else Y

    def solve_noalloc(self, B, stream=None):
        """In-place solve through rs_solve_noalloc (workspace in the library's fixed
        per-device scratch; no device allocation).  B: column-major device tensor."""
        import torch
        if not (isinstance(B, torch.Tensor) and B.is_cuda and B.dtype == self.dtype):
            raise TypeError(f"B must be a {self.dtype} tensor on the HIP device")
        X = B.unsqueeze(1) if B.dim() == 1 else B
        if X.shape[0] != self.n or X.stride(0) != 1 or (X.shape[1] > 1 and X.stride(1) < self.n):
            raise ValueError("B must be column-major with n rows")
        ldb = X.stride(1) if X.shape[1] > 1 else self.n
        if stream is None:
            stream = torch.cuda.current_stream(B.device)
        _check(_lib.rs_solve_noalloc(self._h, C.c_void_p(X.data_ptr()), int(ldb),
                                     int(X.shape[1]), _stream_ptr(stream)))
        return B

    def solve_host(self, b: np.ndarray, stream=None) -> np.ndarray:
        """Synchronous solve of host right-hand sides (numpy, shape (n,) or (n, nrhs),
        float64 or complex128 to match the handle); returns a new array."""
        dt = np.complex128 if self.is_complex else np.float64
        X = np.array(b, dtype=dt, order="F", copy=True)
        vec = X.ndim == 1
        if vec:
            X = X.reshape(-1, 1, order="F")
        if X.shape[0] != self.n:
            raise ValueError("b has the wrong number of rows")
        self.solve_ptr(X.ctypes.data, self.n, X.shape[1], stream)
        return X[:, 0] if vec else X

    def box_skeletons(self):
        nb = self.stats()["nbox"]
        ks = np.empty(nb, dtype=np.int32)
        tot = C.c_int64()
        _check(_lib.rs_box_skeletons(self._h, ks.ctypes.data_as(_PI32), None, 0, C.byref(tot)))
        sk = np.empty(max(int(tot.value), 1), dtype=np.int64)
        _check(_lib.rs_box_skeletons(self._h, ks.ctypes.data_as(_PI32), sk.ctypes.data_as(_PI64),
                                     sk.size, C.byref(tot)))
        out, off = [], 0
        for k in ks:
            kk = max(int(k), 0)
            out.append(sk[off:off + kk].copy())
            off += kk
        return ks, out

    def box_export(self, b: int):
        n, k = C.c_int32(), C.c_int32()
        _check(_lib.rs_box_export(self._h, int(b), C.byref(n), C.byref(k), None, None))
        J = np.empty(max(n.value, 1), dtype=np.int64)
        T = np.empty(max(k.value * (n.value - k.value), 1),
                     dtype=np.complex128 if self.is_complex else np.float64)
        _check(_lib.rs_box_export(self._h, int(b), C.byref(n), C.byref(k),
                                  J.ctypes.data_as(_PI64), T.ctypes.data_as(_PD)))
        kk, nn = k.value, n.value
        return J[:nn], T[:kk * (nn - kk)].reshape((nn - kk, kk)).T if kk and nn - kk else \
            np.zeros((kk, nn - kk))


def factor(kind: str, tree: Tree, points: np.ndarray, weights: np.ndarray, eps: float,
           normals: Optional[np.ndarray] = None, curvature: Optional[np.ndarray] = None,
           identity: float = 0.0, proxy_points: int = 64, proxy_ratio: float = 1.5,
           launch_mode: str = "level", stream=None, wavenumber: float = 0.0,
           eta: float = 0.0, id_mode: str = "cpqr", sketch_seed: int = 0,
           oversample: int = 16) -> Handle:
    """Compress and factor (rs_factor_ex).  id_mode "sketch" compresses each box through
    its random row sketch (the randomized ID; seed and oversampling as in rs.h)."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    nrm = None if normals is None else np.ascontiguousarray(normals, dtype=np.float64)
    kap = None if curvature is None else np.ascontiguousarray(curvature, dtype=np.float64)
    if pts.shape[0] != w.shape[0]:
        raise ValueError("points and weights differ in length")
    k = _kernel_struct(kind, pts, nrm, kap, identity, proxy_points, proxy_ratio, wavenumber, eta,
                       id_mode, sketch_seed, oversample)
    o = rs_options(LAUNCH[launch_mode], _stream_ptr(stream))
    h = _P()
    _check(_lib.rs_factor_ex(C.byref(k), tree.handle, _dptr(pts), _dptr(w), float(eps),
                             C.byref(o), C.byref(h)))
    return Handle(h, pts.shape[0], keep=(tree,))


def factor_solve(kind: str, tree: Tree, points: np.ndarray, weights: np.ndarray, eps: float,
                 B, normals: Optional[np.ndarray] = None,
                 curvature: Optional[np.ndarray] = None, identity: float = 0.0,
                 proxy_points: int = 64, proxy_ratio: float = 1.5, launch_mode: str = "level",
                 stream=None, wavenumber: float = 0.0, eta: float = 0.0, id_mode: str = "cpqr",
                 sketch_seed: int = 0, oversample: int = 16) -> Handle:
    """Factor and solve in one call (rs_factor_solve_ex): B (a device tensor of shape (n,)
    or (n, nrhs), float64 or complex128 as the operator) is overwritten with the
    solution; the same bits as factor() followed by Handle.solve()."""
    import torch
    pts = np.ascontiguousarray(points, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    nrm = None if normals is None else np.ascontiguousarray(normals, dtype=np.float64)
    kap = None if curvature is None else np.ascontiguousarray(curvature, dtype=np.float64)
    if pts.shape[0] != w.shape[0]:
        raise ValueError("points and weights differ in length")
    dtype = torch.complex128 if kind in ("helm2d_cfie", "helm3d_sl") else torch.float64
    if not (isinstance(B, torch.Tensor) and B.is_cuda and B.dtype == dtype):
        raise TypeError(f"B must be a {dtype} tensor on the HIP device")
    X = B.unsqueeze(1) if B.dim() == 1 else B
    if X.shape[0] != pts.shape[0]:
        raise ValueError("B has the wrong number of rows")
    nrhs = X.shape[1]
    colmajor = X.stride(0) == 1 and (nrhs == 1 or X.stride(1) >= pts.shape[0])
    work = X if colmajor else X.t().contiguous().t()
    ldb = work.stride(1) if nrhs > 1 else pts.shape[0]
    if stream is None:
        stream = torch.cuda.current_stream(B.device)
    k = _kernel_struct(kind, pts, nrm, kap, identity, proxy_points, proxy_ratio, wavenumber, eta,
                       id_mode, sketch_seed, oversample)
    o = rs_options(LAUNCH[launch_mode], _stream_ptr(stream))
    h = _P()
    _check(_lib.rs_factor_solve_ex(C.byref(k), tree.handle, _dptr(pts), _dptr(w), float(eps),
                                   C.byref(o), C.c_void_p(work.data_ptr()), int(ldb), int(nrhs),
                                   C.byref(h)))
    if not colmajor:
        X.copy_(work)
    return Handle(h, pts.shape[0], keep=(tree,))


def factor_estimate(kind: str, tree: Tree, eps: float, proxy_points: int = 64,
                    wavenumber: float = 0.0) -> dict:
    """Device footprint of a factorization before it runs (rs_factor_estimate): bytes the
    handle keeps and bytes needed besides while it is factored."""
    pts = np.zeros((1, tree.dim), dtype=np.float64)
    k = _kernel_struct(kind, pts, None, None, 0.0, proxy_points, 1.5, wavenumber, 0.0)
    res, tr = C.c_size_t(), C.c_size_t()
    _check(_lib.rs_factor_estimate(C.byref(k), tree.handle, float(eps), C.byref(res),
                                   C.byref(tr)))
    return {"resident": res.value, "transient": tr.value}


def _kernel_struct(kind, pts, nrm, kap, identity, proxy_points, proxy_ratio, wavenumber=0.0,
                   eta=0.0, id_mode="cpqr", sketch_seed=0, oversample=16):
    return rs_kernel(KINDS[kind], pts.shape[1], float(identity), float(wavenumber), float(eta),
                     _dptr(nrm), _dptr(kap), int(proxy_points), float(proxy_ratio),
                     ID_MODES[id_mode], int(oversample), int(sketch_seed))


def factor_batched(problems, launch_mode: str = "level", stream=None):
    """Factors several problems with shared per-level launches.

    ``problems`` is a list of dicts with keys kind, tree, points, weights, eps and
    optionally normals, curvature, identity, proxy_points, proxy_ratio, wavenumber, eta.
    Returns one Handle per problem.
    """
    count = len(problems)
    keep, ks, trees, pts_p, w_p, eps = [], [], [], [], [], []
    for q in problems:
        pts = np.ascontiguousarray(q["points"], dtype=np.float64)
        w = np.ascontiguousarray(q["weights"], dtype=np.float64)
        nrm = q.get("normals")
        kap = q.get("curvature")
        nrm = None if nrm is None else np.ascontiguousarray(nrm, dtype=np.float64)
        kap = None if kap is None else np.ascontiguousarray(kap, dtype=np.float64)
        keep += [pts, w, nrm, kap]
        ks.append(_kernel_struct(q["kind"], pts, nrm, kap, q.get("identity", 0.0),
                                 q.get("proxy_points", 64), q.get("proxy_ratio", 1.5),
                                 q.get("wavenumber", 0.0), q.get("eta", 0.0),
                                 q.get("id_mode", "cpqr"), q.get("sketch_seed", 0),
                                 q.get("oversample", 16)))
        trees.append(q["tree"].handle)
        pts_p.append(_dptr(pts))
        w_p.append(_dptr(w))
        eps.append(float(q["eps"]))
    K = (rs_kernel * count)(*ks)
    T = (_P * count)(*trees)
    PP = (_PD * count)(*pts_p)
    WW = (_PD * count)(*w_p)
    E = (C.c_double * count)(*eps)
    out = (_P * count)()
    o = rs_options(LAUNCH[launch_mode], _stream_ptr(stream))
    _check(_lib.rs_factor_batched(count, K, T, PP, WW, E, C.byref(o), out))
    return [Handle(_P(out[i]), problems[i]["points"].shape[0], keep=(problems[i]["tree"],))
            for i in range(count)]


def solve_batched(handles, blocks, stream=None):
    """In place B_i := A_i^{-1} B_i for CUDA tensors (n_i,) or (n_i, nrhs_i) that are
    column-major (stride (1, ldb)), float64 (complex128 for Helmholtz handles); all
    requests share the per-level sweep launches."""
    import torch
    count = len(handles)
    if len(blocks) != count:
        raise ValueError("one block per handle")
    ptrs, ldbs, nrhs = _block_args(handles, blocks)
    H = (_P * count)(*[h.handle for h in handles])
    Bp = (C.c_void_p * count)(*ptrs)
    L = (C.c_int64 * count)(*ldbs)
    R = (C.c_int32 * count)(*nrhs)
    if stream is None:
        stream = torch.cuda.current_stream()
    o = rs_options(LAUNCH["level"], _stream_ptr(stream))
    _check(_lib.rs_solve_batched(count, H, Bp, L, R, C.byref(o)))


def _block_args(handles, blocks):
    """(pointers, ldb, nrhs) of column-major device blocks, checked against the handles."""
    import torch
    ptrs, ldbs, nrhs = [], [], []
    for h, B in zip(handles, blocks):
        if not (isinstance(B, torch.Tensor) and B.is_cuda and B.dtype == h.dtype):
            raise TypeError("each block must be a tensor of its handle's dtype on the device")
        X = B.unsqueeze(1) if B.dim() == 1 else B
        if X.shape[0] != h.n or X.stride(0) != 1 or (X.shape[1] > 1 and X.stride(1) < h.n):
            raise ValueError("each block must be column-major with n rows")
        ptrs.append(X.data_ptr())
        ldbs.append(X.stride(1) if X.shape[1] > 1 else h.n)
        nrhs.append(X.shape[1])
    return ptrs, ldbs, nrhs


class Plan:
    """A solve captured into a HIP graph (rs_plan_*): replaying it solves the current
    contents of the same device blocks in place, bitwise as rs_solve_batched."""

    def __init__(self, handles, blocks):
        if len(handles) != len(blocks) or not handles:
            raise ValueError("one block per handle, at least one")
        ptrs, ldbs, nrhs = _block_args(handles, blocks)
        count = len(handles)
        H = (_P * count)(*[h.handle for h in handles])
        Bp = (C.c_void_p * count)(*ptrs)
        L = (C.c_int64 * count)(*ldbs)
        R = (C.c_int32 * count)(*nrhs)
        p = _P()
        _check(_lib.rs_plan_create(count, H, Bp, L, R, C.byref(p)))
        self._p = p
        self._keep = (list(handles), list(blocks))

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(_lib.rs_plan_launch(self._p, _stream_ptr(stream)))

    def free(self):
        if getattr(self, "_p", None):
            _check(_lib.rs_plan_free(self._p))
            self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def autotune(handle: "Handle", nrhs_list=(1, 16, 64, 512), reps: int = 3, stream=None):
    """Times the sweep tile widths on the handle's levels and records the fastest per
    bucket in the library's process-wide table (speed only; results never change)."""
    import torch
    lst = (C.c_int32 * len(nrhs_list))(*[int(x) for x in nrhs_list])
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(_lib.rs_autotune(handle.handle, lst, len(nrhs_list), int(reps), _stream_ptr(stream)))


def tune_entries() -> dict:
    """{bucket: width} with buckets decoded as (mfma, complex, log2 nrhs, box bucket)."""
    cnt = C.c_int32()
    _check(_lib.rs_tune_entries(None, None, 0, C.byref(cnt)))
    n = cnt.value
    keys = (C.c_uint32 * max(n, 1))()
    widths = (C.c_int32 * max(n, 1))()
    _check(_lib.rs_tune_entries(keys, widths, max(n, 1), C.byref(cnt)))
    out = {}
    for i in range(cnt.value):
        k = keys[i]
        out[(bool(k & 1), bool(k & 2), (k >> 2) & 63, (k >> 8) & 255)] = widths[i]
    return out


def tune_clear():
    _check(_lib.rs_tune_clear())


def tune_save(path: str):
    _check(_lib.rs_tune_save(path.encode()))


def tune_load(path: str):
    _check(_lib.rs_tune_load(path.encode()))


class Server:
    """Request server (rs_server_*): resident factorizations, continuous batching of
    solve requests, factor requests admitted against a device-memory budget."""

    def __init__(self, hbm_budget: int, max_batch_requests: int = 64, max_batch_rhs: int = 4096):
        o = rs_server_opts(int(hbm_budget), int(max_batch_requests), int(max_batch_rhs))
        h = _P()
        _check(_lib.rs_server_create(C.byref(o), C.byref(h)))
        self._s = h
        self._pending = {}          # ticket -> objects kept alive until completion

    def close(self):
        if getattr(self, "_s", None):
            _lib.rs_server_destroy(self._s)
            self._s = None

    def __del__(self):
        self.close()

    def submit_factor(self, kind: str, tree: Tree, points, weights, eps: float, normals=None,
                      curvature=None, identity: float = 0.0, proxy_points: int = 64,
                      proxy_ratio: float = 1.5, wavenumber: float = 0.0, eta: float = 0.0) -> int:
        pts = np.ascontiguousarray(points, dtype=np.float64)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        nrm = None if normals is None else np.ascontiguousarray(normals, dtype=np.float64)
        kap = None if curvature is None else np.ascontiguousarray(curvature, dtype=np.float64)
        k = _kernel_struct(kind, pts, nrm, kap, identity, proxy_points, proxy_ratio, wavenumber,
                           eta)
        t = C.c_uint64()
        _check(_lib.rs_server_submit_factor(self._s, C.byref(k), tree.handle, _dptr(pts), _dptr(w),
                                            float(eps), C.byref(t)))
        self._pending[t.value] = ("factor", pts.shape[0], tree)
        return t.value

    def submit_solve(self, handle: Handle, B, stream=None) -> int:
        """Queues B := A^{-1} B for a device tensor B.  The request runs after the work
        queued on `stream` (default: the current torch stream of B's device) so far."""
        import torch
        if not (isinstance(B, torch.Tensor) and B.is_cuda):
            raise TypeError("B must be a tensor on the HIP device")
        if B.dtype != handle.dtype:
            raise TypeError(f"B must be {handle.dtype} for this handle")
        X = B.unsqueeze(1) if B.dim() == 1 else B
        if X.shape[0] != handle.n or X.stride(0) != 1 or (X.shape[1] > 1 and X.stride(1) < handle.n):
            raise ValueError("B must be column-major with n rows")
        ldb = X.stride(1) if X.shape[1] > 1 else handle.n
        if stream is None:
            stream = torch.cuda.current_stream(B.device)
        t = C.c_uint64()
        _check(_lib.rs_server_submit_solve(self._s, handle.handle, C.c_void_p(X.data_ptr()),
                                           int(ldb), int(X.shape[1]), _stream_ptr(stream),
                                           C.byref(t)))
        self._pending[t.value] = ("solve", B, handle)
        return t.value

    def poll(self, ticket: int, timeout_ms: int = 0):
        """(done, status, Handle-or-None); a completed ticket is forgotten."""
        done, st, h = C.c_int32(), C.c_int32(), _P()
        _check(_lib.rs_server_poll(self._s, C.c_uint64(ticket), int(timeout_ms), C.byref(done),
                                   C.byref(st), C.byref(h)))
        if not done.value:
            return False, None, None
        kind = self._pending.pop(ticket, (None,))
        handle = None
        if kind[0] == "factor" and st.value == RS_OK and h.value:
            handle = Handle(_P(h.value), kind[1], keep=(kind[2],), server=self)
        return True, st.value, handle

    def wait(self, ticket: int):
        done, st, h = self.poll(ticket, -1)
        if st != RS_OK:
            raise RSError(st, _lib.rs_last_error().decode())
        return h

    def stats(self) -> dict:
        s = rs_server_stats()
        _check(_lib.rs_server_query(self._s, C.byref(s)))
        return {f: getattr(s, f) for f, _ in rs_server_stats._fields_}

    def reset_stats(self):
        _check(_lib.rs_server_reset_stats(self._s))
