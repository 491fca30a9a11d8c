"""CPU reference ("oracle") for D-Iteration / power iteration on PageRank.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never imports it and shares no code with it.

Plain fp64 arithmetic in the paper's order (``di_oracle.c``), plus dense
solves of the closed form x = (1-d)(I - dP)^{-1} Z (Section 2.1) through
``numpy.linalg.solve`` for graphs of at most a few thousand nodes.

Pinned by ``tests/test_oracle.py`` against closed forms, brute force, the
paper's invariants and bounds, and finite differences.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build_library(force: bool = False) -> str:
    src = os.path.join(_HERE, "di_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # DI_ORACLE_LIB names another build of the same source (the sanitizer test uses it)
    path = os.environ.get("DI_ORACLE_LIB")
    if not path:
        if not os.path.exists(_LIB_PATH):
            build_library()
        path = _LIB_PATH
    lib = ctypes.CDLL(path)
    i64, dbl, vp, ci = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
    lib.or_build_in.argtypes = [i64, i64, vp, vp, vp, vp, vp]
    lib.or_inv_s.argtypes = [i64, vp, vp, vp]
    lib.or_inv_s.restype = None
    lib.or_fixed_scale.argtypes = [i64, vp]
    lib.or_fixed_scale.restype = ci
    lib.or_fixed_sum_abs.argtypes = [i64, vp, ci]
    lib.or_fixed_sum_abs.restype = dbl
    lib.or_fixed_sum_signed.argtypes = [i64, vp, ci, vp]
    lib.or_fixed_sum_signed.restype = dbl
    lib.or_fixed_value.argtypes = [vp, ci]
    lib.or_fixed_value.restype = dbl
    lib.or_di_sequential.argtypes = [i64, vp, vp, vp, vp, dbl, vp, vp, vp, ci, i64, dbl, vp]
    lib.or_di_sequential.restype = i64
    lib.or_di_sync.argtypes = [i64, vp, vp, vp, vp, vp, dbl, dbl, ci, ci, vp, vp, vp, dbl, i64, vp, vp, vp, vp]
    lib.or_di_sync.restype = i64
    lib.or_power.argtypes = [i64, vp, vp, vp, vp, dbl, vp, vp, dbl, i64, vp, vp]
    lib.or_power.restype = i64
    lib.or_gauss_seidel.argtypes = [i64, vp, vp, vp, vp, dbl, vp, vp, i64]
    lib.or_gauss_seidel.restype = None
    lib.or_adjoint_sync.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, ci, vp, vp, dbl, i64, vp]
    lib.or_adjoint_sync.restype = i64
    lib.or_edge_grad.argtypes = [i64, vp, vp, vp, vp, dbl, vp, vp, vp, vp]
    lib.or_edge_grad.restype = None
    lib.or_spmv_P.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    lib.or_spmv_P.restype = None
    lib.or_spmv_P_rows.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
    lib.or_spmv_P_rows.restype = None
    lib.or_num_threads.restype = ci
    _lib = lib
    return lib


def _p(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "arrays passed to the oracle must be contiguous"
    return ctypes.c_void_p(a.ctypes.data)


def num_threads() -> int:
    return int(_load().or_num_threads())


class OGraph:
    """Oracle-side graph: OUT as given, IN and 1/s_j built here."""

    def __init__(self, n, out_ptr, out_idx, w=None):
        self.n = int(n)
        self.out_ptr = np.ascontiguousarray(out_ptr, dtype=np.int64)
        self.out_idx = np.ascontiguousarray(out_idx, dtype=np.int32)
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
        self.m = int(self.out_ptr[-1])
        lib = _load()
        self.in_ptr = np.empty(self.n + 1, dtype=np.int64)
        self.in_idx = np.empty(self.m, dtype=np.int32)
        self.in_eid = np.empty(self.m, dtype=np.int64)
        if lib.or_build_in(self.n, self.m, _p(self.out_ptr), _p(self.out_idx), _p(self.in_ptr), _p(self.in_idx),
                           _p(self.in_eid)) != 0:
            raise MemoryError("or_build_in")
        self.in_w = None if self.w is None else np.ascontiguousarray(self.w[self.in_eid])
        self.inv_s = np.empty(self.n, dtype=np.float64)
        lib.or_inv_s(self.n, _p(self.out_ptr), _p(self.w), _p(self.inv_s))
        self.dangling = np.diff(self.out_ptr) == 0

    @classmethod
    def of(cls, g):
        return cls(g.n, g.out_ptr, g.out_idx, g.w)

    # dense P[i][j] = w(j->i)/s_j (Section 2.1, equation def-p); small graphs only
    def dense_P(self) -> np.ndarray:
        assert self.n <= 5000, "dense P only for small graphs"
        P = np.zeros((self.n, self.n))
        for j in range(self.n):
            for e in range(self.out_ptr[j], self.out_ptr[j + 1]):
                i = self.out_idx[e]
                P[i, j] += (float(self.w[e]) if self.w is not None else 1.0) * self.inv_s[j]
        return P

    def P_times(self, v: np.ndarray) -> np.ndarray:
        v = np.ascontiguousarray(v, dtype=np.float64)
        y = np.empty(self.n)
        _load().or_spmv_P(self.n, _p(self.in_ptr), _p(self.in_idx), _p(self.in_w), _p(self.inv_s), _p(v), _p(y))
        return y

    def P_times_rows(self, rows: np.ndarray, v: np.ndarray) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        y = np.empty(len(rows))
        _load().or_spmv_P_rows(len(rows), _p(rows), _p(self.in_ptr), _p(self.in_idx), _p(self.in_w),
                               _p(self.inv_s), _p(v), _p(y))
        return y


# --------------------------------------------------------------------------
# Closed form (Section 2.1): x = (1-d) (I - dP)^{-1} Z
# --------------------------------------------------------------------------
def dense_solve(og: OGraph, d: float, Z: np.ndarray) -> np.ndarray:
    P = og.dense_P()
    A = np.eye(og.n) - d * P
    return np.linalg.solve(A, (1.0 - d) * np.asarray(Z, dtype=np.float64))


def dense_adjoint(og: OGraph, d: float, g: np.ndarray) -> np.ndarray:
    """lambda = (I - d P^T)^{-1} g."""
    P = og.dense_P()
    return np.linalg.solve(np.eye(og.n) - d * P.T, np.asarray(g, dtype=np.float64))


def uniform_Z(n: int) -> np.ndarray:
    return np.full(n, 1.0 / n)


def fixed_scale(v: np.ndarray) -> int:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return int(_load().or_fixed_scale(len(v), _p(v)))


def fixed_sum_abs(v: np.ndarray, K: int) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return float(_load().or_fixed_sum_abs(len(v), _p(v), K))


def fixed_sum_signed(v: np.ndarray, K: int):
    """Exact signed sum of v on 2^-K: (value rounded once to double, [low, high] 64-bit
    words of the two's-complement 128-bit integer)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(2, dtype=np.uint64)
    val = float(_load().or_fixed_sum_signed(len(v), _p(v), K, _p(out)))
    return val, out


def update_fluid(og_old: "OGraph", og_new: "OGraph", d: float, H: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Theorem 4 (Section 3.5): after diffusions on P reached (H, F), D-Iteration on P'
    continues from H'_0 = H and F'_0 = F + d (P' - P) H.  (P' - P) H is evaluated as
    P' H - P H, each product a left fold over its IN rows (unchanged rows cancel exactly)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    return np.asarray(F, dtype=np.float64) + d * (og_new.P_times(H) - og_old.P_times(H))


def initial_fluid(d: float, Z: np.ndarray, fluid_fp32: bool = False) -> np.ndarray:
    """F_0 = (1-d) Z (Section 3.1), rounded to float when the fluid is stored in float."""
    F = (1.0 - d) * np.asarray(Z, dtype=np.float64)
    if fluid_fp32:
        F = F.astype(np.float32).astype(np.float64)
    return np.ascontiguousarray(F)


# --------------------------------------------------------------------------
# Sequential D-Iteration (Section 3.1, schedulers of Section 3.4)
# --------------------------------------------------------------------------
class SequentialDI:
    """Elementary diffusions one node at a time; sched 'cyc' or 'argmax'."""

    def __init__(self, og: OGraph, d: float, Z: np.ndarray, sched: str = "cyc"):
        self.og, self.d = og, float(d)
        self.F = initial_fluid(d, Z)
        self.F0 = self.F.copy()
        self.H = np.zeros(og.n)
        self.l = np.zeros(1)
        self.pos = np.zeros(1, dtype=np.int64)
        self.sched = {"cyc": 0, "argmax": 1}[sched]
        self.steps = 0

    def run(self, max_steps: int, tol: float = 0.0) -> int:
        og = self.og
        k = _load().or_di_sequential(og.n, _p(og.out_ptr), _p(og.out_idx), _p(og.w), _p(og.inv_s), self.d,
                                     _p(self.F), _p(self.H), _p(self.l), self.sched, int(max_steps), float(tol),
                                     _p(self.pos))
        self.steps += int(k)
        return int(k)

    @property
    def residual(self) -> float:
        return float(np.abs(self.F).sum())

    def update(self, og_new: "OGraph") -> None:
        """Switch to the matrix P' of og_new (same nodes) by Theorem 4: keep H, set
        F = F + d (P' - P) H (signed), and count as leaked the history at the nodes
        dangling in P' (the fluid those diffusions would have lost under P')."""
        assert og_new.n == self.og.n
        self.F = update_fluid(self.og, og_new, self.d, self.H, self.F)
        self.og = og_new
        self.l[0] = float(self.H[og_new.dangling].sum())


# --------------------------------------------------------------------------
# Synchronous-sweep D-Iteration (the GPU's deterministic sweep)
# --------------------------------------------------------------------------
class SyncDI:
    def __init__(self, og: OGraph, d: float, Z: np.ndarray, theta: float = 1.0, fluid_fp32: bool = False):
        self.og, self.d, self.theta, self.fp32 = og, float(d), float(theta), bool(fluid_fp32)
        self.F = initial_fluid(d, Z, fluid_fp32)
        self.F_init = self.F.copy()
        self.K = fixed_scale(self.F)
        self.H = np.zeros(og.n)
        self.l_fixed = np.zeros(2, dtype=np.uint64)
        self.sweeps = 0
        self.trace = []  # (R_t, |A_t|, edges) per sweep
        self.last_frontier = np.zeros(0, dtype=np.int32)
        self.converged = False

    def run(self, tol: float, max_sweeps: int = 1 << 40, record_frontier: bool = False) -> int:
        og = self.og
        cap = min(int(max_sweeps), 100000)
        tr = np.zeros(3 * max(cap, 1))
        fr = np.zeros(og.n, dtype=np.int32) if record_frontier else None
        flen = np.zeros(1, dtype=np.int64)
        conv = np.zeros(1, dtype=np.int32)
        t = _load().or_di_sync(og.n, _p(og.out_ptr), _p(og.in_ptr), _p(og.in_idx), _p(og.in_w), _p(og.inv_s),
                               self.d, self.theta, int(self.fp32), self.K, _p(self.F), _p(self.H),
                               _p(self.l_fixed), float(tol), cap, _p(tr), _p(fr), _p(flen), _p(conv))
        if t < 0:
            raise MemoryError("or_di_sync")
        self.sweeps += int(t)
        self.converged = bool(conv[0])
        self.trace.extend(tr[: 3 * t].reshape(-1, 3).tolist())
        if record_frontier and t > 0:
            self.last_frontier = fr[: int(flen[0])].copy()
        return int(t)

    def update(self, og_new: "OGraph") -> None:
        """Switch to the matrix P' of og_new (same nodes) by Theorem 4 (Section 3.5): keep H,
        set F = F + d (P' - P) H (signed; rounded once to float in the float-fluid mode),
        choose the fixed-point scale for the new fluid, and set the leak to the exact sum of
        H over the nodes dangling in P' (those diffusions lose their fluid under P')."""
        assert og_new.n == self.og.n
        F = update_fluid(self.og, og_new, self.d, self.H, self.F)
        if self.fp32:
            F = F.astype(np.float32).astype(np.float64)
        self.F = F
        self.og = og_new
        # the scale covers the new fluid and, as before, the starting fluid (which bounds
        # the leak: n max F_0 >= (1-d) |Z|_1 >= (1-d) l)
        self.K = fixed_scale(np.maximum(np.abs(F), np.abs(self.F_init)))
        self.l_fixed = fixed_sum_signed(self.H[og_new.dangling], self.K)[1]
        self.converged = False

    @property
    def R(self) -> float:
        return fixed_sum_abs(self.F, self.K)

    @property
    def l(self) -> float:
        return float(_load().or_fixed_value(_p(self.l_fixed), self.K))

    def x_norm(self) -> np.ndarray:
        """(1-d)/(1-d-d l) H (implicit completion, Section 3.3)."""
        return (1.0 - self.d) / (1.0 - self.d - self.d * self.l) * self.H


# --------------------------------------------------------------------------
# Power iteration (Section 2.2)
# --------------------------------------------------------------------------
def power(og: OGraph, d: float, Z: np.ndarray, tol: float, max_iters: int = 100000, x0=None):
    """Jacobi PI from x_0 = 0 (or x0); returns (x, iterations, residual trace)."""
    x = np.zeros(og.n) if x0 is None else np.array(x0, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    tr = np.zeros(max_iters)
    conv = np.zeros(1, dtype=np.int32)
    k = _load().or_power(og.n, _p(og.in_ptr), _p(og.in_idx), _p(og.in_w), _p(og.inv_s), float(d), _p(Z), _p(x),
                         float(tol), int(max_iters), _p(tr), _p(conv))
    if k < 0:
        raise MemoryError("or_power")
    return x, int(k), tr[:k].copy()


def gauss_seidel(og: OGraph, d: float, Z: np.ndarray, x0, sweeps: int) -> np.ndarray:
    """`sweeps` Gauss-Seidel rounds (Section 2.3) from x0: entries updated in place in
    index order, so row i reads the new values of the rows before it."""
    x = np.array(x0, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    _load().or_gauss_seidel(og.n, _p(og.in_ptr), _p(og.in_idx), _p(og.in_w), _p(og.inv_s), float(d), _p(Z), _p(x),
                            int(sweeps))
    return x


# --------------------------------------------------------------------------
# Adjoint: lambda = (I - d P^T)^{-1} g, and the gradients of L with dL/dx = g
# --------------------------------------------------------------------------
def adjoint(og: OGraph, d: float, g: np.ndarray, tol_inf: float, theta: float = 1.0, max_sweeps: int = 100000):
    F = np.ascontiguousarray(g, dtype=np.float64).copy()
    K = fixed_scale(F)
    H = np.zeros(og.n)
    conv = np.zeros(1, dtype=np.int32)
    t = _load().or_adjoint_sync(og.n, _p(og.out_ptr), _p(og.out_idx), _p(og.w), _p(og.inv_s), float(d),
                                float(theta), K, _p(F), _p(H), float(tol_inf), int(max_sweeps), _p(conv))
    if t < 0:
        raise MemoryError("or_adjoint_sync")
    return H, F, int(t), bool(conv[0])


def edge_grad(og: OGraph, d: float, x: np.ndarray, lam: np.ndarray):
    """(dL/dw in OUT order, dL/dZ) from x and lambda."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    dw = np.empty(og.m)
    dZ = np.empty(og.n)
    _load().or_edge_grad(og.n, _p(og.out_ptr), _p(og.out_idx), _p(og.w), _p(og.inv_s), float(d), _p(x), _p(lam),
                         _p(dw), _p(dZ))
    return dw, dZ


# --------------------------------------------------------------------------
# Checks that hold for any schedule (Section 3.2 and 3.3)
# --------------------------------------------------------------------------
def invariant_residual(og: OGraph, d: float, F0, H, F) -> float:
    """max |H + F - F_0 - d P H| (equation HnFn); sparse product, any size."""
    r = np.asarray(H) + np.asarray(F) - np.asarray(F0) - d * og.P_times(H)
    return float(np.max(np.abs(r))) if len(r) else 0.0


def invariant_residual_l1(og: OGraph, d: float, F0, H, F) -> float:
    """|H + F - F_0 - d P H|_1: by (I - dP)^{-1} it adds at most this / (1-d) to |x - H|_1."""
    r = np.asarray(H) + np.asarray(F) - np.asarray(F0) - d * og.P_times(H)
    return float(np.abs(r).sum())


def mass_defect(og: OGraph, d: float, Z, H, F, l: float) -> float:
    """sum F + (1-d) sum H + d l - (1-d) sum Z; zero in exact arithmetic.

    Follows from equation HnFn and 1^T P = 1^T - 1_D^T (dangling columns are null),
    with l the fluid diffused at dangling nodes (Section 3.3)."""
    return float(np.sum(F) + (1.0 - d) * np.sum(H) + d * l - (1.0 - d) * np.sum(Z))
