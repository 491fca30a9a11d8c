"""ctypes binding of libdi.so (argument marshalling only).

Every computation runs in the HIP library; this module converts numpy arrays or
torch tensors into pointers, and status codes into exceptions.  There is no CPU
fallback: importing the binding without the built library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdi.so")

DI_OK, DI_EINVAL, DI_ENOMEM, DI_EHIP, DI_ENOCONV, DI_ESTATE, DI_ENUMERIC = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "DI_OK", -1: "DI_EINVAL", -2: "DI_ENOMEM", -3: "DI_EHIP", -4: "DI_ENOCONV", -5: "DI_ESTATE",
                -6: "DI_ENUMERIC"}
LOOP_STREAM, LOOP_GRAPH = 0, 1
X_RAW, X_NORM, F, H, LAMBDA, X_PI, IN_PTR, IN_IDX, INV_S, FRONTIER, RESIDUALS, LEAKS, DONE_SWEEPS, \
    MASS_DEFECTS = range(14)
INFO_N, INFO_M, INFO_K, INFO_M_LOCAL, INFO_RANGE_LOG2, INFO_INNER_ROUNDS, INFO_FIXED_K, INFO_TOTAL_SWEEPS, \
    INFO_DEVICE_BYTES, INFO_KERNEL_NS, INFO_KERNEL_LAUNCHES, INFO_LOCAL_PUSHES, INFO_REMOTE_UPDATES, INFO_M_REMOTE, \
    INFO_NRANGES, INFO_N_INTERNAL, INFO_LIVE_ALLOCATIONS = range(17)

EXPORTED = ["di_init", "di_diffuse", "di_power", "di_power_noalloc", "di_adjoint", "di_read", "di_update",
            "di_set_sweep", "di_reset", "di_set_z", "di_save", "di_load", "di_info", "di_destroy", "di_last_error"]
NOALLOC_SCRATCH_BYTES = 32 << 20


class DIError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


class DiCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("out_ptr", ctypes.c_void_p),
                ("out_idx", ctypes.c_void_p), ("w", ctypes.c_void_p), ("on_device", ctypes.c_int)]


class DiOpts(ctypes.Structure):
    _fields_ = [("fluid_fp32", ctypes.c_int), ("theta", ctypes.c_double), ("max_sweeps", ctypes.c_int64),
                ("deterministic", ctypes.c_int), ("range_log2", ctypes.c_int), ("inner_rounds", ctypes.c_int),
                ("k", ctypes.c_int), ("n_graphs", ctypes.c_int64), ("graph_ptr", ctypes.c_void_p),
                ("loop_mode", ctypes.c_int), ("sweeps_per_sync", ctypes.c_int), ("normalized_stop", ctypes.c_int),
                ("timing", ctypes.c_int), ("range_cut", ctypes.c_int), ("stream", ctypes.c_void_p)]


class DiStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("edge_updates", ctypes.c_int64), ("node_updates", ctypes.c_int64),
                ("residual", ctypes.c_double), ("bound", ctypes.c_double), ("bound_norm", ctypes.c_double),
                ("leak", ctypes.c_double), ("mass_defect", ctypes.c_double), ("ms", ctypes.c_double),
                ("converged", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdi.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libdi.so not found at %s: run __graft_entry__.build() first" % path)
    # Load PyTorch's HIP runtime first when it is installed, so that the library and the
    # tensors handed to it share one runtime (and the runtime PyTorch was built against).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.di_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(DiCsr), dbl, vp, ctypes.POINTER(DiOpts)]
    lib.di_diffuse.argtypes = [vp, dbl, ctypes.POINTER(DiStats)]
    lib.di_power.argtypes = [vp, dbl, ctypes.POINTER(DiStats)]
    lib.di_power_noalloc.argtypes = [vp, dbl, vp, ctypes.POINTER(DiStats)]
    lib.di_adjoint.argtypes = [vp, vp, dbl, vp, vp, ci, ctypes.POINTER(DiStats)]
    lib.di_read.argtypes = [vp, ci, vp, ci]
    lib.di_update.argtypes = [vp, ctypes.POINTER(DiCsr)]
    lib.di_set_sweep.argtypes = [vp, dbl, ci]
    lib.di_reset.argtypes = [vp]
    lib.di_set_z.argtypes = [vp, vp]
    lib.di_save.argtypes = [vp, ctypes.c_char_p]
    lib.di_load.argtypes = [vp, ctypes.c_char_p]
    lib.di_info.argtypes = [vp, ci, ctypes.POINTER(i64)]
    lib.di_destroy.argtypes = [vp]
    lib.di_last_error.restype = ctypes.c_char_p
    lib.di_last_error.argtypes = []
    for name in EXPORTED:
        getattr(lib, name).restype = getattr(lib, name).restype if name == "di_last_error" else ci
    _lib = lib
    return lib


def _check(rc: int, allow=()):
    if rc != DI_OK and rc not in allow:
        raise DIError(rc, load_library().di_last_error().decode())
    return rc


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a, dtype=None):
    """(pointer, keepalive, on_device) of a numpy array or torch tensor."""
    if a is None:
        return None, None, 0
    if _is_torch(a):
        t = a.contiguous()
        return ctypes.c_void_p(t.data_ptr()), t, int(t.is_cuda)
    arr = np.ascontiguousarray(a, dtype=dtype)
    return ctypes.c_void_p(arr.ctypes.data), arr, 0


def current_stream_handle() -> Optional[int]:
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:  # torch missing or without a device: the null stream
        pass
    return None


class Solver:
    """One D-Iteration / power-iteration context on the device."""

    def __init__(self, n, out_ptr, out_idx, w=None, d: float = 0.85, Z=None, *, fluid_fp32: bool = False,
                 theta: float = 1.0, max_sweeps: int = 0, deterministic: bool = False, range_log2: int = 0,
                 inner_rounds: int = 0, k: int = 1, graph_ptr=None, loop_mode: int = LOOP_STREAM,
                 sweeps_per_sync: int = 0, normalized_stop: bool = False, timing: bool = False, range_cut: int = 0,
                 stream=None):
        lib = load_library()
        self._lib = lib
        self.n = int(n)
        self.d = float(d)
        self.k = int(k)
        p_ptr, k_ptr, dev0 = _ptr(out_ptr, np.int64)
        p_idx, k_idx, dev1 = _ptr(out_idx, np.int32)
        p_w, k_w, dev2 = _ptr(w, np.float32)
        self.m = int(k_idx.shape[0]) if k_idx is not None else 0
        if len({dev0, dev1} | ({dev2} if w is not None else set())) != 1:
            raise ValueError("graph arrays must all be on the host or all on the device")
        csr = DiCsr(self.n, self.m, p_ptr, p_idx, p_w, dev0)
        zptr, zkeep, zdev = _ptr(None if Z is None else np.asfortranarray(np.asarray(Z, dtype=np.float64)).ravel(order="F"),
                                 np.float64)
        if zdev:
            raise ValueError("Z must be a host array")
        gp, gkeep, _ = _ptr(graph_ptr, np.int64)
        opts = DiOpts()
        opts.fluid_fp32 = int(fluid_fp32)
        opts.theta = float(theta)
        opts.max_sweeps = int(max_sweeps)
        opts.deterministic = int(deterministic)
        opts.range_log2 = int(range_log2)
        opts.inner_rounds = int(inner_rounds)
        opts.k = int(k)
        opts.n_graphs = 1 if graph_ptr is None else len(gkeep) - 1
        opts.graph_ptr = gp
        opts.loop_mode = int(loop_mode)
        opts.sweeps_per_sync = int(sweeps_per_sync)
        opts.normalized_stop = int(normalized_stop)
        opts.timing = int(timing)
        opts.range_cut = int(range_cut)
        if stream is None:
            stream = current_stream_handle()
        opts.stream = ctypes.c_void_p(stream) if stream else None
        self.n_graphs = opts.n_graphs
        self.fluid_fp32 = bool(fluid_fp32)
        self._ctx = ctypes.c_void_p()
        _check(lib.di_init(ctypes.byref(self._ctx), ctypes.byref(csr), self.d, zptr, ctypes.byref(opts)))
        del k_ptr, k_idx, k_w, zkeep, gkeep

    # -- solves -------------------------------------------------------------
    def diffuse(self, tol: float, allow_noconv: bool = False) -> dict:
        st = DiStats()
        rc = self._lib.di_diffuse(self._ctx, float(tol), ctypes.byref(st))
        _check(rc, (DI_ENOCONV,) if allow_noconv else ())
        return st.as_dict()

    def power(self, tol: float) -> dict:
        st = DiStats()
        _check(self._lib.di_power(self._ctx, float(tol), ctypes.byref(st)))
        return st.as_dict()

    def power_noalloc(self, tol: float, x_out) -> dict:
        """Power iteration into x_out (a device tensor of n doubles) with no allocation
        in the library: its vectors live in the library's per-device scratch array."""
        if not (_is_torch(x_out) and x_out.is_cuda and x_out.is_contiguous()):
            raise ValueError("x_out must be a contiguous device tensor")
        st = DiStats()
        _check(self._lib.di_power_noalloc(self._ctx, float(tol), ctypes.c_void_p(x_out.data_ptr()), ctypes.byref(st)))
        return st.as_dict()

    def adjoint(self, g, tol_inf: float, want_dw: bool = True):
        """(dZ, dw, stats) for dL/dx = g; host arrays in, host arrays out (or device tensors)."""
        st = DiStats()
        if _is_torch(g):
            import torch
            gt = g.contiguous().to(torch.float64)
            dZ = torch.empty(self.n, dtype=torch.float64, device=gt.device)
            dw = torch.empty(self.m, dtype=torch.float64, device=gt.device) if want_dw else None
            _check(self._lib.di_adjoint(self._ctx, ctypes.c_void_p(gt.data_ptr()), float(tol_inf),
                                        ctypes.c_void_p(dZ.data_ptr()),
                                        ctypes.c_void_p(dw.data_ptr()) if dw is not None else None,
                                        int(gt.is_cuda), ctypes.byref(st)))
            return dZ, dw, st.as_dict()
        ga = np.ascontiguousarray(g, dtype=np.float64)
        dZ = np.empty(self.n)
        dw = np.empty(self.m) if want_dw else None
        _check(self._lib.di_adjoint(self._ctx, ctypes.c_void_p(ga.ctypes.data), float(tol_inf),
                                    ctypes.c_void_p(dZ.ctypes.data),
                                    ctypes.c_void_p(dw.ctypes.data) if dw is not None else None, 0,
                                    ctypes.byref(st)))
        return dZ, dw, st.as_dict()

    # -- results ------------------------------------------------------------
    def read(self, what: int, out=None):
        n, m, k = self.n, self.m, self.k
        if what in (X_RAW, X_NORM, F, H):
            shape, dt = ((n,) if k == 1 else (k, n)), np.float64
        elif what in (LAMBDA, X_PI, INV_S):
            shape, dt = (n,), np.float64
        elif what == IN_PTR:
            shape, dt = (n + 1,), np.int64
        elif what == IN_IDX:
            shape, dt = (m,), np.int32
        elif what == FRONTIER:
            buf = np.zeros(n + 2, dtype=np.int32)
            _check(self._lib.di_read(self._ctx, what, ctypes.c_void_p(buf.ctypes.data), 0))
            cnt = int(buf[:2].view(np.int64)[0])
            return buf[2:2 + cnt].copy()
        elif what in (RESIDUALS, LEAKS, MASS_DEFECTS):
            shape, dt = (max(k, self.n_graphs),), np.float64
        elif what == DONE_SWEEPS:
            shape, dt = (max(k, self.n_graphs),), np.int64
        else:
            raise ValueError("unknown read target %d" % what)
        if out is not None and _is_torch(out):
            t = out
            _check(self._lib.di_read(self._ctx, what, ctypes.c_void_p(t.data_ptr()), int(t.is_cuda)))
            return t
        arr = np.empty(shape, dtype=dt)
        if arr.size:
            _check(self._lib.di_read(self._ctx, what, ctypes.c_void_p(arr.ctypes.data), 0))
        return arr

    def update(self, out_ptr, out_idx, w=None):
        """Replace the graph (same n) and keep the D-Iteration state (Theorem 4)."""
        p_ptr, k_ptr, dev0 = _ptr(out_ptr, np.int64)
        p_idx, k_idx, dev1 = _ptr(out_idx, np.int32)
        p_w, k_w, dev2 = _ptr(w, np.float32)
        if len({dev0, dev1} | ({dev2} if w is not None else set())) != 1:
            raise ValueError("graph arrays must all be on the host or all on the device")
        m = int(k_idx.shape[0]) if k_idx is not None else 0
        csr = DiCsr(self.n, m, p_ptr, p_idx, p_w, dev0)
        _check(self._lib.di_update(self._ctx, ctypes.byref(csr)))
        self.m = m
        del k_ptr, k_idx, k_w

    def update_graph(self, g):
        self.update(g.out_ptr, g.out_idx, g.w)

    def set_options(self, theta: float, inner_rounds: int = 0):
        """New frontier scale (and local rounds, if > 0) for the following sweeps."""
        _check(self._lib.di_set_sweep(self._ctx, float(theta), int(inner_rounds)))

    def reset(self):
        _check(self._lib.di_reset(self._ctx))

    def set_z(self, Z=None):
        """New distribution(s) Z (n, or n x k) on the resident graph; resets the solve."""
        if Z is None:
            _check(self._lib.di_set_z(self._ctx, None))
            return
        z = np.asfortranarray(np.asarray(Z, dtype=np.float64)).ravel(order="F")
        if z.size != self.n * self.k:
            raise ValueError("Z must hold n * k = %d values" % (self.n * self.k))
        _check(self._lib.di_set_z(self._ctx, ctypes.c_void_p(z.ctypes.data)))

    def save(self, path: str):
        _check(self._lib.di_save(self._ctx, path.encode()))

    def load(self, path: str):
        _check(self._lib.di_load(self._ctx, path.encode()))

    def info(self, key: int) -> int:
        v = ctypes.c_int64()
        _check(self._lib.di_info(self._ctx, key, ctypes.byref(v)))
        return int(v.value)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            self._lib.di_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def live_allocations() -> int:
    """Device allocations the library holds in this process (all contexts)."""
    v = ctypes.c_int64(0)
    _check(load_library().di_info(None, INFO_LIVE_ALLOCATIONS, ctypes.byref(v)))
    return int(v.value)


def from_graph(g, **kw) -> Solver:
    """Solver for a graph object with n, out_ptr, out_idx, w attributes."""
    return Solver(g.n, g.out_ptr, g.out_idx, g.w, **kw)
