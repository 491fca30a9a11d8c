"""Pins of the CPU oracle against closed forms, brute force and the paper's theorems.

Every check here is independent of the oracle's own code path: hand-derived
fixtures (tests/golden), a matrix P assembled here with numpy, truncated Neumann
series, math.fsum / Fraction sums, numpy's stable argsort, and the paper's
identities and bounds.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as W

D = 0.85
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def P_numpy(g) -> np.ndarray:
    """P[i][j] = w(j->i) / s_j assembled with numpy (equation def-p)."""
    n = g.n
    src = np.repeat(np.arange(n), np.diff(g.out_ptr))
    dst = g.out_idx.astype(np.int64)
    w = np.ones(g.m) if g.w is None else g.w.astype(np.float64)
    s = np.zeros(n)
    np.add.at(s, src, w)
    P = np.zeros((n, n))
    np.add.at(P, (dst, src), w / s[src])
    return P


def random_graph(n, seed, weighted=False, p_dangling=0.2, loops=True):
    rng = np.random.default_rng(seed)
    deg = rng.integers(1, 6, size=n)
    deg[rng.random(n) < p_dangling] = 0
    src = np.repeat(np.arange(n), deg)
    dst = rng.integers(0, n, size=len(src))
    if not loops:
        dst = np.where(dst == src, (dst + 1) % n, dst)
    w = rng.lognormal(0.0, 1.0, size=len(src)).astype(np.float32) if weighted else None
    return W.from_edges(n, src, dst, w, "rand(%d,%d)" % (n, seed))


def golden_cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def case_graph(c):
    e = c["edges"]
    src = [a for a, _, _ in e]
    dst = [b for _, b, _ in e]
    w = [float(x) for _, _, x in e]
    weighted = any(x != 1 for x in w)
    return W.from_edges(c["n"], src, dst, w if weighted else None, c["name"])


# --------------------------------------------------------------------------
# Closed forms (hand-derived fixtures)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", golden_cases(), ids=lambda c: c["name"])
def test_closed_forms_all_solvers(case):
    g = case_graph(case)
    og = O.OGraph.of(g)
    d = float(Fraction(case["d"]))
    Z = np.array([float(Fraction(z)) for z in case["Z"]])
    x = np.array([float(Fraction(v)) for v in case["x"]])
    np.testing.assert_allclose(O.dense_solve(og, d, Z), x, rtol=0, atol=1e-15)
    for sched in ("cyc", "argmax"):
        s = O.SequentialDI(og, d, Z, sched)
        s.run(10 ** 6, tol=1e-14)
        np.testing.assert_allclose(s.H, x, rtol=0, atol=1e-13)
    for theta in (1.0, 0.0):
        y = O.SyncDI(og, d, Z, theta=theta)
        y.run(1e-14)
        assert y.converged
        np.testing.assert_allclose(y.H, x, rtol=0, atol=1e-13)
    xp, _, _ = O.power(og, d, Z, 1e-14)
    np.testing.assert_allclose(xp, x, rtol=0, atol=1e-13)


def test_closed_form_detects_transposed_matrix():
    """Planted mistake: feeding the reversed cycle must break the cycle3 fixture."""
    c = [c for c in golden_cases() if c["name"] == "cycle3_point_mass"][0]
    rev = dict(c, edges=[[b, a, w] for a, b, w in c["edges"]])
    og = O.OGraph.of(case_graph(rev))
    x = np.array([float(Fraction(v)) for v in c["x"]])
    assert np.abs(O.dense_solve(og, D, np.array([1.0, 0.0, 0.0])) - x).max() > 1e-2


def test_uniform_closed_forms():
    # complete graph with self-loops: P = J/n, x uniform
    n = 6
    src = np.repeat(np.arange(n), n)
    dst = np.tile(np.arange(n), n)
    og = O.OGraph.of(W.from_edges(n, src, dst))
    Z = np.full(n, 1.0 / n)
    np.testing.assert_allclose(O.dense_solve(og, D, Z), Z, atol=1e-15)
    # directed n-cycle, uniform Z
    n = 9
    og = O.OGraph.of(W.from_edges(n, np.arange(n), (np.arange(n) + 1) % n))
    y = O.SyncDI(og, D, np.full(n, 1.0 / n))
    y.run(1e-14)
    np.testing.assert_allclose(y.H, 1.0 / n, atol=1e-14)


def test_edgeless_converges_in_one_sweep():
    og = O.OGraph.of(W.from_edges(5, [], []))
    Z = np.array([0.1, 0.2, 0.3, 0.15, 0.25])
    y = O.SyncDI(og, D, Z, theta=0.0)  # every node with fluid is active
    y.run(1e-15)
    assert y.sweeps == 1 and y.converged
    np.testing.assert_array_equal(y.H, (1 - D) * Z)
    y = O.SyncDI(og, D, Z)  # theta = 1: the above-average nodes first, then the rest
    y.run(1e-15)
    assert y.sweeps == 2 and y.converged
    np.testing.assert_array_equal(y.H, (1 - D) * Z)


# --------------------------------------------------------------------------
# Dense solve against a truncated Neumann series (brute force)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("weighted", [False, True])
def test_dense_solve_vs_neumann_series(weighted):
    g = random_graph(40, 3, weighted)
    og = O.OGraph.of(g)
    P = P_numpy(g)
    Z = np.random.default_rng(1).random(g.n)
    Z /= Z.sum()
    term = (1 - D) * Z
    acc = term.copy()
    for _ in range(400):  # d^400 ~ 1e-28
        term = D * (P @ term)
        acc += term
    np.testing.assert_allclose(O.dense_solve(og, D, Z), acc, rtol=0, atol=1e-15)
    np.testing.assert_allclose(og.dense_P(), P, rtol=1e-15, atol=1e-16)


# --------------------------------------------------------------------------
# Graph preparation
# --------------------------------------------------------------------------
def test_transpose_matches_stable_argsort():
    g = W.tiny_zipf(3000, 5)
    og = O.OGraph.of(g)
    src = np.repeat(np.arange(g.n), np.diff(g.out_ptr)).astype(np.int32)
    order = np.argsort(g.out_idx, kind="stable")
    np.testing.assert_array_equal(og.in_idx, src[order])
    np.testing.assert_array_equal(og.in_eid, order)
    cnt = np.bincount(g.out_idx, minlength=g.n)
    np.testing.assert_array_equal(og.in_ptr, np.concatenate([[0], np.cumsum(cnt)]))


def _product_graphs():
    """Weighted and unweighted graphs with dangling nodes, self-loops and repeated edges."""
    out = []
    for weighted in (False, True):
        g = random_graph(300, 21 + weighted, weighted=weighted, p_dangling=0.25)
        src = np.repeat(np.arange(g.n), np.diff(g.out_ptr))
        assert (src == g.out_idx).any(), "the graph must hold a self-loop"
        pairs = src.astype(np.int64) * g.n + g.out_idx
        assert len(np.unique(pairs)) < len(pairs), "the graph must hold a repeated edge"
        assert (np.diff(g.out_ptr) == 0).any()
        out.append(g)
    # a graph with a hub receiving most edges (long IN row)
    rng = np.random.default_rng(5)
    src = np.repeat(np.arange(400), rng.integers(0, 6, size=400))
    dst = np.where(rng.random(len(src)) < 0.6, 7, rng.integers(0, 400, size=len(src)))
    out.append(W.from_edges(400, src, dst, rng.lognormal(0.0, 1.0, len(src)).astype(np.float32), "hub"))
    return out


@pytest.mark.parametrize("gi", [0, 1, 2])
def test_sparse_product_matches_dense_P(gi):
    """OGraph.P_times / P_times_rows (the checkers of the large-graph certificates) against
    P assembled here with numpy from the edge list (equation def-p)."""
    g = _product_graphs()[gi]
    og = O.OGraph.of(g)
    P = P_numpy(g)
    rng = np.random.default_rng(30 + gi)
    # two sums of the same terms in different orders differ by at most about
    # 2 (row length) eps times the sum of |terms|
    tol_rows = 2.0 * (np.diff(og.in_ptr) + 1) * np.finfo(float).eps
    for v in (rng.random(g.n), rng.standard_normal(g.n), np.eye(g.n)[3], np.ones(g.n)):
        ref = P @ v
        scale = np.abs(P) @ np.abs(v)
        assert np.all(np.abs(og.P_times(v) - ref) <= tol_rows * scale)
        rows = np.sort(rng.choice(g.n, size=60, replace=False))
        np.testing.assert_array_equal(og.P_times_rows(rows, v), og.P_times(v)[rows])
        assert np.all(np.abs(og.P_times_rows(rows, v) - ref[rows]) <= tol_rows[rows] * scale[rows])
    # column sums: 1 for every non-dangling column, 0 for a dangling one (Section 2.1)
    colsum = np.array([og.P_times(e).sum() for e in np.eye(g.n)[:50]])
    dang = np.diff(g.out_ptr)[:50] == 0
    np.testing.assert_allclose(colsum[~dang], 1.0, atol=1e-14)
    assert (colsum[dang] == 0.0).all()


def test_sparse_product_pin_detects_target_scaling():
    """Planted mistake: scaling each entry by 1/s of the target instead of the source must
    fail the comparison the pin above makes."""
    g = _product_graphs()[1]
    og = O.OGraph.of(g)
    v = np.random.default_rng(40).random(g.n)
    src = np.repeat(np.arange(g.n), np.diff(g.out_ptr))
    # y_i = sum over edges j -> i of w_e / s_i * v_j (the mutated oracle formula)
    bad = np.zeros(g.n)
    np.add.at(bad, g.out_idx, g.w.astype(np.float64) * og.inv_s[g.out_idx] * v[src])
    assert np.abs(bad - P_numpy(g) @ v).max() > 1e-3
    assert np.abs(og.P_times(v) - P_numpy(g) @ v).max() < 1e-13


def test_inv_s_left_fold():
    g = random_graph(50, 7, weighted=True)
    og = O.OGraph.of(g)
    for j in range(g.n):
        ws = g.w[g.out_ptr[j]:g.out_ptr[j + 1]]
        if len(ws) == 0:
            assert og.inv_s[j] == 0.0
            continue
        s = 0.0
        for v in ws:
            s += float(v)
        assert og.inv_s[j] == 1.0 / s


# --------------------------------------------------------------------------
# Fixed-point residual = correctly rounded sum
# --------------------------------------------------------------------------
def test_fixed_point_sum_is_correctly_rounded():
    rng = np.random.default_rng(0)
    for trial in range(20):
        n = int(rng.integers(1, 5000))
        v = rng.random(n) * np.exp2(rng.integers(-60, 0, size=n).astype(np.float64))
        K = O.fixed_scale(v)
        exact = math.fsum(np.abs(v))
        assert O.fixed_sum_abs(v, K) == exact
        # exact rational check on a few
        if trial < 3:
            fr = sum(Fraction(float(a)) for a in np.abs(v))
            assert O.fixed_sum_abs(v, K) == float(fr)
    # order independence
    v = rng.random(1000)
    K = O.fixed_scale(v)
    assert O.fixed_sum_abs(v, K) == O.fixed_sum_abs(v[::-1].copy(), K)


# --------------------------------------------------------------------------
# The paper's invariant, bounds and theorems on sequential DI
# --------------------------------------------------------------------------
@pytest.mark.parametrize("sched", ["cyc", "argmax"])
@pytest.mark.parametrize("weighted", [False, True])
def test_sequential_invariants(sched, weighted):
    g = random_graph(30, 11, weighted)
    og = O.OGraph.of(g)
    P = P_numpy(g)
    Z = np.random.default_rng(2).random(g.n)
    Z /= Z.sum()
    x = O.dense_solve(og, D, Z)
    s = O.SequentialDI(og, D, Z, sched)
    prevH = s.H.copy()
    prevR = s.residual
    dang = np.diff(g.out_ptr) == 0
    for step in range(600):
        s.run(1)
        # equation HnFn: H + F = F_0 + d P H
        assert np.abs(s.H + s.F - s.F0 - D * (P @ s.H)).max() < 1e-15
        # mass balance: sum F + (1-d) sum H + d l = (1-d) sum Z, l = fluid at dangling nodes
        l = s.H[dang].sum()
        assert abs(s.l[0] - l) < 1e-15
        assert abs(s.F.sum() + (1 - D) * s.H.sum() + D * l - (1 - D) * Z.sum()) < 1e-15
        # F >= 0, H non-decreasing (Section 3.1)
        assert (s.F >= 0).all() and (s.H >= prevH).all()
        # Theorem 1, equation SL
        R = s.F.sum()
        assert np.abs(x - s.H).sum() <= R / (1 - D) + 1e-15
        # implicit completion (Section 3.3): normalised result at exact distance
        xbar = x / x.sum()
        c = (1 - D) / (1 - D - D * l)
        assert abs(np.abs(xbar - c * s.H).sum() - R / (1 - D - D * l)) < 1e-14
        if sched == "argmax":  # one-step form of Theorem 3
            assert R <= (1 - (1 - D) / g.n) * prevR + 1e-16
        else:  # Theorem 2
            assert np.abs(x - s.H).sum() <= D ** ((step + 1) // g.n) + 1e-15
        prevH, prevR = s.H.copy(), R


@pytest.mark.parametrize("sched", ["cyc", "argmax"])
def test_sequential_stop_follows_the_exact_residual(sched):
    """The sequential solver keeps |F|_1 as a running fixed-point sum; it must stop at the
    first step whose full re-sum of |F| meets the tolerance (graph with self-loops, repeated
    edges, weights and dangling nodes)."""
    g0 = random_graph(50, 31, weighted=True)
    src = np.concatenate([np.repeat(np.arange(g0.n), np.diff(g0.out_ptr)), [3, 3, 7, 11]])
    dst = np.concatenate([g0.out_idx, [3, 3, 7, 11]])  # self-loops, one of them repeated
    w = np.concatenate([g0.w, np.array([0.5, 2.0, 1.0, 3.0], dtype=np.float32)])
    g = W.from_edges(g0.n, src, dst, w, "loops")
    og = O.OGraph.of(g)
    Z = np.random.default_rng(6).random(g.n)
    K = O.fixed_scale(O.initial_fluid(D, Z))
    for tol in (1e-3, 1e-6, 1e-9):
        s = O.SequentialDI(og, D, Z, sched)
        k = s.run(10 ** 6, tol=tol)
        assert 0 < k < 10 ** 6
        assert O.fixed_sum_abs(s.F, K) / (1 - D) <= tol
        t = O.SequentialDI(og, D, Z, sched)
        t.run(k - 1)
        assert O.fixed_sum_abs(t.F, K) / (1 - D) > tol


def test_bound_is_equality_without_dangling_nodes():
    g = random_graph(25, 4, weighted=True, p_dangling=0.0)
    og = O.OGraph.of(g)
    Z = np.full(g.n, 1.0 / g.n)
    x = O.dense_solve(og, D, Z)
    s = O.SequentialDI(og, D, Z, "cyc")
    for _ in range(40):
        s.run(7)
        assert abs(np.abs(x - s.H).sum() - s.F.sum() / (1 - D)) < 1e-14


# --------------------------------------------------------------------------
# Synchronous sweeps and power iteration
# --------------------------------------------------------------------------
@pytest.mark.parametrize("weighted", [False, True])
def test_sync_sweep_invariant_and_limit(weighted):
    g = random_graph(200, 8, weighted)
    og = O.OGraph.of(g)
    P = P_numpy(g)
    Z = np.full(g.n, 1.0 / g.n)
    x = O.dense_solve(og, D, Z)
    y = O.SyncDI(og, D, Z)
    F0 = y.F.copy()
    while not y.converged:
        y.run(1e-13, max_sweeps=1)
        assert np.abs(y.H + y.F - F0 - D * (P @ y.H)).max() < 1e-15
        assert np.abs(x - y.H).sum() <= y.R / (1 - D) + 1e-15
    assert np.abs(x - y.H).sum() <= 1e-13


def test_sync_theta0_is_power_iteration():
    g = random_graph(150, 9, weighted=True)
    og = O.OGraph.of(g)
    Z = np.random.default_rng(3).random(g.n)
    y = O.SyncDI(og, D, Z, theta=0.0)
    for t in range(1, 30):
        y.run(1e-300, max_sweeps=1)
        xt, _, _ = O.power(og, D, Z, tol=1e-300, max_iters=t)
        np.testing.assert_allclose(y.H, xt, rtol=1e-14, atol=1e-17)


def test_power_certificate():
    g = random_graph(120, 10)
    og = O.OGraph.of(g)
    Z = np.full(g.n, 1.0 / g.n)
    x = O.dense_solve(og, D, Z)
    xk = np.zeros(g.n)
    for k in range(1, 40):
        xk1, _, tr = O.power(og, D, Z, tol=1e-300, max_iters=k)
        xkm, _, _ = O.power(og, D, Z, tol=1e-300, max_iters=k - 1) if k > 1 else (np.zeros(g.n), 0, None)
        gap = np.abs(xk1 - xkm).sum()
        assert np.abs(x - xkm).sum() <= gap / (1 - D) + 1e-15
        assert np.abs(x - xk1).sum() <= D * gap / (1 - D) + 1e-15


@pytest.mark.parametrize("weighted", [False, True])
def test_gauss_seidel(weighted):
    """Gauss-Seidel (Section 2.3): with every edge pointing to a higher index, P is strictly
    lower triangular and one round is forward substitution, the exact solution; with every
    edge pointing to a lower index no row reads a new value, so one round is one power
    iteration; on a general graph the rounds converge to the dense solution."""
    rng = np.random.default_rng(17)
    n = 70
    src = rng.integers(0, n, size=300)
    dst = rng.integers(0, n, size=300)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    w = rng.lognormal(0, 1, size=len(src)).astype(np.float32) if weighted else None
    Z = rng.random(n)
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    up = O.OGraph.of(W.from_edges(n, lo, hi, w))  # j -> i with j < i
    x = O.dense_solve(up, D, Z)
    np.testing.assert_allclose(O.gauss_seidel(up, D, Z, np.zeros(n), 1), x, rtol=1e-13, atol=1e-16)
    down = O.OGraph.of(W.from_edges(n, hi, lo, w))  # j -> i with j > i
    x0 = rng.random(n)
    x1, _, _ = O.power(down, D, Z, tol=1e-300, max_iters=1, x0=x0)
    np.testing.assert_allclose(O.gauss_seidel(down, D, Z, x0, 1), x1, rtol=1e-14, atol=1e-17)
    og = O.OGraph.of(random_graph(120, 5, weighted))
    Zg = O.uniform_Z(og.n)
    xg = O.dense_solve(og, D, Zg)
    assert np.abs(O.gauss_seidel(og, D, Zg, np.zeros(og.n), 300) - xg).sum() <= 1e-14


def test_permutation_invariance():
    g = random_graph(80, 12, weighted=True)
    perm = np.random.default_rng(5).permutation(g.n)
    src = np.repeat(np.arange(g.n), np.diff(g.out_ptr))
    g2 = W.from_edges(g.n, perm[src], perm[g.out_idx], g.w)
    Z = np.random.default_rng(6).random(g.n)
    Z2 = np.empty_like(Z)
    Z2[perm] = Z
    x = O.dense_solve(O.OGraph.of(g), D, Z)
    y = O.SyncDI(O.OGraph.of(g2), D, Z2)
    y.run(1e-14)
    np.testing.assert_allclose(y.H[perm], x, atol=1e-14)


def test_fp32_fluid_sync_close_to_fp64():
    g = W.tiny_zipf(2000, 3)
    og = O.OGraph.of(g)
    Z = O.uniform_Z(g.n)
    x = O.dense_solve(og, D, Z)
    y = O.SyncDI(og, D, Z, fluid_fp32=True)
    y.run(1e-10)
    assert np.abs(y.H - x).sum() <= 1e-6 * np.abs(x).sum()
    # the fluid is float-representable after every sweep
    assert (y.F.astype(np.float32).astype(np.float64) == y.F).all()


def test_tiny_config_oracle_agrees_with_dense():
    g = W.tiny_zipf(2000, 1)
    og = O.OGraph.of(g)
    Z = O.uniform_Z(g.n)
    x = O.dense_solve(og, D, Z)
    for sched in ("cyc", "argmax"):
        s = O.SequentialDI(og, D, Z, sched)
        s.run(10 ** 8, tol=1e-11)
        assert np.abs(s.H - x).sum() <= 1e-11
    y = O.SyncDI(og, D, Z)
    y.run(1e-11)
    assert np.abs(y.H - x).sum() <= 1e-11


# --------------------------------------------------------------------------
# Adjoint and gradients
# --------------------------------------------------------------------------
@pytest.mark.parametrize("weighted", [False, True])
def test_adjoint_vs_dense_and_duality(weighted):
    g = random_graph(120, 13, weighted)
    og = O.OGraph.of(g)
    P = P_numpy(g)
    Z = np.random.default_rng(4).random(g.n)
    Z /= Z.sum()
    c = np.random.default_rng(5).standard_normal(g.n)
    lam_dense = np.linalg.solve(np.eye(g.n) - D * P.T, c)
    lam, F, sweeps, conv = O.adjoint(og, D, c, tol_inf=1e-14)
    assert conv
    assert np.abs(lam - lam_dense).max() <= 1e-13 * np.abs(lam_dense).max()
    # L-infinity certificate (|P^T|_inf <= 1)
    assert np.abs(lam - lam_dense).max() <= np.abs(F).max() / (1 - D) + 1e-15
    x = O.dense_solve(og, D, Z)
    assert abs(c @ x - (1 - D) * Z @ lam) < 1e-14


@pytest.mark.parametrize("weighted", [False, True])
def test_gradients_vs_finite_differences(weighted):
    g = random_graph(30, 14, weighted=True)
    if not weighted:
        g = W.Graph(g.n, g.out_ptr, g.out_idx, np.ones(g.m, dtype=np.float32), g.name)
    og = O.OGraph.of(g)
    Z = np.random.default_rng(6).random(g.n)
    Z /= Z.sum()
    c = np.random.default_rng(7).standard_normal(g.n)
    x = O.dense_solve(og, D, Z)
    lam = O.dense_adjoint(og, D, c)
    dw, dZ = O.edge_grad(og, D, x, lam)

    def loss(w, Zv):
        gg = W.Graph(g.n, g.out_ptr, g.out_idx, w.astype(np.float32), "")
        return c @ O.dense_solve(O.OGraph.of(gg), D, Zv)

    # weights are float32: perturb in float32 and divide by the realised step
    for e in range(g.m):
        w0 = g.w.copy()
        wp, wm = w0.copy(), w0.copy()
        wp[e] = np.float32(float(w0[e]) * (1 + 2.0 ** -8))
        wm[e] = np.float32(float(w0[e]) * (1 - 2.0 ** -8))
        fd = (loss(wp, Z) - loss(wm, Z)) / (float(wp[e]) - float(wm[e]))
        assert abs(fd - dw[e]) <= 1e-4 * max(abs(dw[e]), 1e-3)
    for i in range(g.n):
        h = 1e-6
        Zp, Zm = Z.copy(), Z.copy()
        Zp[i] += h
        Zm[i] -= h
        fd = (loss(g.w, Zp) - loss(g.w, Zm)) / (2 * h)
        assert abs(fd - dZ[i]) <= 1e-7 + 1e-6 * abs(dZ[i])


# --------------------------------------------------------------------------
# Graph update (Section 3.5, Theorem 4)
# --------------------------------------------------------------------------
def rewired(g, seed, frac=0.08, weighted=False):
    """g with a share of its edges moved to new targets, some edges dropped (sources may
    become dangling) and edges added at dangling nodes: same nodes, another matrix P'."""
    rng = np.random.default_rng(seed)
    src = np.repeat(np.arange(g.n), np.diff(g.out_ptr))
    dst = g.out_idx.astype(np.int64).copy()
    w = None if g.w is None else g.w.copy()
    move = rng.random(len(dst)) < frac
    dst[move] = rng.integers(0, g.n, size=int(move.sum()))
    keep = rng.random(len(dst)) >= frac / 2
    src, dst = src[keep], dst[keep]
    w = None if w is None else w[keep]
    dang = np.flatnonzero(np.diff(g.out_ptr) == 0)
    new_src = rng.choice(dang, size=max(1, len(dang) // 3), replace=False) if len(dang) else np.zeros(0, int)
    src = np.concatenate([src, new_src])
    dst = np.concatenate([dst, rng.integers(0, g.n, size=len(new_src))])
    if w is not None:
        w = np.concatenate([w, rng.lognormal(0, 1, size=len(new_src)).astype(np.float32)])
    return W.from_edges(g.n, src, dst, w, g.name + "'")


def test_update_hand_fixture():
    case = json.load(open(GOLDEN))["updates"][0]
    fr = lambda a: np.array([float(Fraction(v)) for v in a])
    d = float(Fraction(case["d"]))
    Z = fr(case["Z"])

    def graph(key):
        e = case[key]
        return O.OGraph.of(W.from_edges(case["n"], [a for a, _, _ in e], [b for _, b, _ in e], None, key))

    a, b = graph("edges_before"), graph("edges_after")
    s = O.SequentialDI(a, d, Z, "cyc")
    s.run(case["steps_before"])
    np.testing.assert_allclose(s.H, fr(case["H_before"]), rtol=0, atol=1e-16)
    np.testing.assert_allclose(s.F, fr(case["F_before"]), rtol=0, atol=1e-16)
    s.update(b)
    np.testing.assert_allclose(s.F, fr(case["F_after"]), rtol=0, atol=1e-16)
    assert s.F.min() < 0  # the update brings negative fluid (remark after Theorem 4)
    s.run(10 ** 5, tol=1e-15)
    np.testing.assert_allclose(s.H, fr(case["x_after"]), rtol=0, atol=1e-14)
    np.testing.assert_allclose(O.dense_solve(b, d, Z), fr(case["x_after"]), rtol=0, atol=1e-15)
    # the synchronous sweep, updated at another point, reaches the same fixed point
    y = O.SyncDI(a, d, Z)
    y.run(1e-300, max_sweeps=3)
    y.update(b)
    y.run(1e-15)
    assert y.converged
    np.testing.assert_allclose(y.H, fr(case["x_after"]), rtol=0, atol=1e-14)


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("sched", ["cyc", "argmax", "sync"])
def test_update_invariants_and_limit(weighted, sched):
    """After the update: equation HnFn holds for P' (with the original F_0), |F|_1 never
    grows, Theorem 1's certificate holds for the signed fluid, the mass balance holds with
    the leak reset to the history at P'-dangling nodes, and H reaches the dense solution of
    x' = d P' x' + (1-d) Z."""
    g = random_graph(60, 21, weighted)
    g2 = rewired(g, 5, weighted=weighted)
    oa, ob = O.OGraph.of(g), O.OGraph.of(g2)
    assert ob.dangling.sum() != oa.dangling.sum() or (ob.dangling != oa.dangling).any()
    P2 = P_numpy(g2)
    Z = np.random.default_rng(4).random(g.n)
    Z /= Z.sum()
    x2 = O.dense_solve(ob, D, Z)
    F0 = O.initial_fluid(D, Z)
    dang2 = np.diff(g2.out_ptr) == 0
    if sched == "sync":
        s = O.SyncDI(oa, D, Z)
        s.run(1e-300, max_sweeps=4)
    else:
        s = O.SequentialDI(oa, D, Z, sched)
        s.run(150)
    s.update(ob)
    assert s.F.min() < 0
    R_prev = np.inf
    for _ in range(400):
        assert np.abs(s.H + s.F - F0 - D * (P2 @ s.H)).max() < 1e-15
        R = np.abs(s.F).sum()
        assert R <= R_prev * (1 + 1e-15) + 1e-17
        assert np.abs(x2 - s.H).sum() <= R / (1 - D) + 1e-15
        l = s.l if sched == "sync" else s.l[0]
        assert abs(l - s.H[dang2].sum()) < 1e-15
        assert abs(s.F.sum() + (1 - D) * s.H.sum() + D * l - (1 - D) * Z.sum()) < 1e-15
        R_prev = R
        if sched == "sync":
            s.run(1e-14, max_sweeps=1)
            if s.converged:
                break
        else:
            s.run(30)
    if sched != "sync":
        s.run(10 ** 6, tol=1e-14)
    assert np.abs(x2 - s.H).sum() <= 1e-13


def test_update_to_the_same_graph_changes_nothing():
    g = random_graph(80, 3, weighted=True)
    og, og2 = O.OGraph.of(g), O.OGraph.of(g)
    y = O.SyncDI(og, D, O.uniform_Z(g.n))
    y.run(1e-300, max_sweeps=5)
    F, H = y.F.copy(), y.H.copy()
    y.update(og2)
    np.testing.assert_array_equal(y.F, F)
    np.testing.assert_array_equal(y.H, H)


def test_update_pin_detects_a_wrong_sign():
    """Injecting d (P - P') H instead of d (P' - P) H (a plausible slip) misses x'."""
    g = random_graph(60, 21)
    og, og2 = O.OGraph.of(g), O.OGraph.of(rewired(g, 5))
    Z = O.uniform_Z(g.n)
    x2 = O.dense_solve(og2, D, Z)
    s = O.SequentialDI(og, D, Z, "cyc")
    s.run(150)
    s.F = O.update_fluid(og2, og, D, s.H, s.F)  # operands swapped
    s.og = og2
    s.run(10 ** 6, tol=1e-14)
    assert np.abs(x2 - s.H).sum() > 1e-3
