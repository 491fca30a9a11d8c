"""Autotuner for the sweep options of the HIP library.

The block-local sweep has three knobs whose best values depend on the graph: the frontier
scale theta (a node is taken when |F_i| >= theta |F|_1 / n), the local rounds per sweep,
and the range size 2^range_log2 (the k-column tile's range size is fixed by the LDS its
k columns need, so only theta and the rounds are tuned there; the adjoint diffusion runs on
the forward context's ranges, so it too tunes theta and the rounds only).  The tuner times complete
solves to the caller's tolerance on the caller's graph through the library (all arithmetic
runs in the HIP kernels; this module only chooses options and keeps a cache):

1. every candidate (theta, rounds) once per range size, fastest device time of the call;
2. the best few again, `repeats` times each; the lowest median wins.

Results are cached in a JSON file keyed by what decides them: n, m, a hash of the
out- and in-degree histograms (log2 buckets), the number of columns, the fluid precision,
whether the graph is weighted, d and the tolerance.  A later solve on a graph of the same
shape and degree structure reuses the choice without timing anything.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
from typing import Optional

import numpy as np

from . import binding as B

THETAS = (0.15, 0.2, 0.3, 0.5, 1.0)
ROUNDS = (4, 6, 8)
RANGE_LOG2 = (10, 11)
TILE_THETAS = (0.3, 0.5, 1.0)
TILE_ROUNDS = (2, 4, 6)
ADJ_THETAS = (0.5, 1.0)
ADJ_ROUNDS = (4, 6, 8)


def default_cache_path() -> str:
    base = os.environ.get("DI_TUNE_CACHE")
    if base:
        return base
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1501_06350_amd", "tune.json")


def graph_key(g, k: int, fp32: bool, d: float, tol: float) -> str:
    """Cache key: sizes, degree structure (log2 histograms of out- and in-degrees), the
    number of columns, the fluid precision, weights, d and the tolerance."""
    out_deg = np.diff(np.asarray(g.out_ptr, dtype=np.int64))
    in_deg = np.bincount(np.asarray(g.out_idx, dtype=np.int64), minlength=g.n)
    h = hashlib.sha256()
    for deg in (out_deg, in_deg):
        buckets = np.zeros(deg.size, dtype=np.int64)
        nz = deg > 0
        buckets[nz] = np.floor(np.log2(deg[nz])).astype(np.int64) + 1
        hist = np.bincount(buckets, minlength=40)
        # coarse shares (per mille), so that graphs drawn from one generator share a key
        h.update(np.round(1000.0 * hist / max(deg.size, 1)).astype(np.int64).tobytes())
    return "n=%d m=%d k=%d fp32=%d w=%d d=%g tol=%g deg=%s" % (
        g.n, int(out_deg.sum()), k, int(fp32), int(getattr(g, "w", None) is not None), d, tol, h.hexdigest()[:16])


class Tuner:
    def __init__(self, cache_path: Optional[str] = None, repeats: int = 3, finalists: int = 3, log=None):
        self.cache_path = cache_path or default_cache_path()
        self.repeats = repeats
        self.finalists = finalists
        self.log = log or (lambda *a: None)
        self.cache = {}
        try:
            with open(self.cache_path) as f:
                self.cache = json.load(f)
        except (OSError, ValueError):
            self.cache = {}

    def _save(self):
        try:
            os.makedirs(os.path.dirname(self.cache_path) or ".", exist_ok=True)
            tmp = self.cache_path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)
        except OSError:
            pass

    @staticmethod
    def _time(s, tol: float) -> float:
        """Device time (ms) of one solve from the starting state."""
        s.reset()
        st = s.diffuse(tol)
        if not st["converged"]:
            return float("inf")
        return float(st["ms"])

    def _first_pass(self, s, cands, tol):
        out = []
        for th, rd in cands:
            s.set_options(theta=th, inner_rounds=rd)
            self._time(s, tol)  # warm-up of this setting
            ms = self._time(s, tol)
            out.append((ms, th, rd))
            self.log("tune: theta=%g rounds=%d: %.2f ms" % (th, rd, ms))
        return out

    def _finalists(self, s, cands, tol):
        best = None
        for th, rd in cands:
            s.set_options(theta=th, inner_rounds=rd)
            med = statistics.median([self._time(s, tol) for _ in range(self.repeats)])
            self.log("tune: finalist theta=%g rounds=%d: median %.2f ms" % (th, rd, med))
            if best is None or med < best[0]:
                best = (med, th, rd)
        return best

    def _search(self, make, grid, tol):
        """Time every (range size, theta, rounds) of `grid` once, then the finalists again."""
        first = []
        for rb, cands in grid:
            with make(rb) as s:
                first += [(ms, rb, th, rd) for ms, th, rd in self._first_pass(s, cands, tol)]
        first.sort()
        by_rb = {}
        for ms, rb, th, rd in first[: self.finalists]:
            by_rb.setdefault(rb, []).append((th, rd))
        best = None
        for rb, cands in by_rb.items():
            with make(rb) as s:
                med, th, rd = self._finalists(s, cands, tol)
            if best is None or med < best[0]:
                best = (med, rb, th, rd)
        return best

    def tune_context(self, s, key: str, tol: float = 1e-8, thetas=THETAS, rounds=ROUNDS, force: bool = False) -> dict:
        """theta and rounds for a live single-column context s (its range size stays): the
        context is left with the chosen options and reset.  key names the workload in the
        cache (see graph_key)."""
        key = "context " + key
        if not force and key in self.cache:
            res = dict(self.cache[key], cached=True)
        else:
            first = sorted(self._first_pass(s, [(th, rd) for th in thetas for rd in rounds], tol))
            med, th, rd = self._finalists(s, [(th, rd) for _, th, rd in first[: self.finalists]], tol)
            res = {"theta": th, "inner_rounds": rd, "ms": round(med, 3)}
            self.cache[key] = res
            self._save()
            res = dict(res, cached=False)
        s.set_options(theta=res["theta"], inner_rounds=res["inner_rounds"])
        s.reset()
        return res

    def tune_single(self, g, d: float = 0.85, tol: float = 1e-8, fluid_fp32: bool = False, Z=None,
                    thetas=THETAS, rounds=ROUNDS, range_log2=RANGE_LOG2, force: bool = False) -> dict:
        """Sweep options for one right-hand side on g: {"theta", "inner_rounds", "range_log2", "ms"}."""
        key = "single " + graph_key(g, 1, fluid_fp32, d, tol)
        if not force and key in self.cache:
            return dict(self.cache[key], cached=True)
        rbs = [rb for rb in range_log2 if (1 << rb) * 256 <= max(g.n, 1 << 16) or rb == min(range_log2)]

        def make(rb):
            return B.Solver(g.n, g.out_ptr, g.out_idx, getattr(g, "w", None), d=d, Z=Z, fluid_fp32=fluid_fp32,
                            range_log2=rb)

        grid = [(rb, [(th, rd) for th in thetas for rd in rounds]) for rb in rbs]
        ms, rb, th, rd = self._search(make, grid, tol)
        res = {"theta": th, "inner_rounds": rd, "range_log2": rb, "ms": round(ms, 3)}
        self.cache[key] = res
        self._save()
        return dict(res, cached=False)

    def tune_tile(self, g, Z, d: float = 0.85, tol: float = 1e-8, fluid_fp32: bool = True,
                  thetas=TILE_THETAS, rounds=TILE_ROUNDS, force: bool = False) -> dict:
        """Sweep options of the k-column tile for the right-hand sides Z (n x k): {"theta",
        "inner_rounds", "ms"} (the tile's range size follows from k and the LDS)."""
        Z = np.asarray(Z, dtype=np.float64)
        k = Z.shape[1]
        key = "tile " + graph_key(g, k, fluid_fp32, d, tol)
        if not force and key in self.cache:
            return dict(self.cache[key], cached=True)

        def make(_rb):
            return B.Solver(g.n, g.out_ptr, g.out_idx, getattr(g, "w", None), d=d, Z=Z, k=k, fluid_fp32=fluid_fp32)

        grid = [(0, [(th, rd) for th in thetas for rd in rounds])]
        ms, _, th, rd = self._search(make, grid, tol)
        res = {"theta": th, "inner_rounds": rd, "ms": round(ms, 3)}
        self.cache[key] = res
        self._save()
        return dict(res, cached=False)

    def tune_adjoint(self, s, rhs, key: str, tol_inf: float = 1e-11, thetas=ADJ_THETAS, rounds=ADJ_ROUNDS,
                     force: bool = False) -> dict:
        """theta and rounds for the adjoint diffusion of a live context s whose forward solve
        has converged: complete di_adjoint calls for the right-hand side rhs, timed by their
        device clock.  The context is left with the chosen options (they also apply to its
        later forward sweeps).  key names the workload in the cache (see graph_key)."""
        key = "adjoint " + key
        if not force and key in self.cache:
            res = dict(self.cache[key], cached=True)
        else:
            def run():
                _, _, st = s.adjoint(rhs, tol_inf, want_dw=False)
                return float(st["ms"]) if st["converged"] else float("inf")

            first = []
            for th in thetas:
                for rd in rounds:
                    s.set_options(theta=th, inner_rounds=rd)
                    run()  # warm-up of this setting
                    ms = run()
                    first.append((ms, th, rd))
                    self.log("tune adjoint: theta=%g rounds=%d: %.2f ms" % (th, rd, ms))
            first.sort()
            best = None
            for _, th, rd in first[: self.finalists]:
                s.set_options(theta=th, inner_rounds=rd)
                med = statistics.median([run() for _ in range(self.repeats)])
                self.log("tune adjoint: finalist theta=%g rounds=%d: median %.2f ms" % (th, rd, med))
                if best is None or med < best[0]:
                    best = (med, th, rd)
            res = {"theta": best[1], "inner_rounds": best[2], "ms": round(best[0], 3)}
            self.cache[key] = res
            self._save()
            res = dict(res, cached=False)
        s.set_options(theta=res["theta"], inner_rounds=res["inner_rounds"])
        return res
