"""GPU results against the CPU oracle (HIP library through the C ABI).

Bit-exact: IN adjacency, 1/s_j, and the deterministic sweep (frontier, residual,
F and H after every sweep).  Tolerance: the default block-local sweep and power
iteration, |dx|_1 <= 1e-9 |x|_1 with double fluid and <= 1e-6 with float fluid.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
D = 0.85


def say(*a):
    print(*a, flush=True)


def small_graphs():
    rng = np.random.default_rng(21)
    n = 3000
    deg = rng.integers(0, 9, size=n)
    src = np.repeat(np.arange(n), deg)
    dst = rng.integers(0, n, size=len(src))
    wts = rng.lognormal(0, 1, size=len(src)).astype(np.float32)
    return {
        "tiny10k": W.tiny_zipf(10_000, 1),
        "web20k": W.webgen(20_000, 7),
        "rand3k_w": W.from_edges(n, src, dst, wts, "rand3k_w"),
    }


GRAPHS = small_graphs()


@pytest.fixture(scope="module")
def oracle_graphs():
    return {k: O.OGraph.of(g) for k, g in GRAPHS.items()}


# --------------------------------------------------------------------------
# Graph construction: bit-exact
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("rb", [8, 13])
@pytest.mark.parametrize("cut", [-1, 0])
def test_in_adjacency_bit_exact(gpu, oracle_graphs, name, rb, cut):
    """IN, 1/s and the local/cross-range split; with cut-aligned ranges (cut = 0) IN and 1/s
    are read back through the relabelling and must still equal the oracle's."""
    g, og = GRAPHS[name], oracle_graphs[name]
    say("graph build", name, "rb", rb, "cut", cut)
    with gpu.from_graph(g, range_log2=rb, range_cut=cut) as s:
        np.testing.assert_array_equal(s.read(gpu.IN_PTR), og.in_ptr)
        np.testing.assert_array_equal(s.read(gpu.IN_IDX), og.in_idx)
        np.testing.assert_array_equal(s.read(gpu.INV_S), og.inv_s)
        m_loc, m_rem = s.info(gpu.INFO_M_LOCAL), s.info(gpu.INFO_M_REMOTE)
        assert m_loc + m_rem == g.m
        assert s.info(gpu.INFO_N) == g.n
        if cut == -1:
            src = np.repeat(np.arange(g.n), np.diff(g.out_ptr))
            assert m_loc == int(((src >> rb) == (g.out_idx.astype(np.int64) >> rb)).sum())
        else:  # ranges end at the caller's cut points: no range exceeds 2^rb caller nodes
            assert g.n <= s.info(gpu.INFO_N_INTERNAL) <= 2 * g.n + (1 << rb)


# --------------------------------------------------------------------------
# Deterministic sweep: bit-exact against the oracle's synchronous sweep
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("fp32", [False, True])
def test_deterministic_sweeps_bit_exact(gpu, oracle_graphs, name, fp32):
    g, og = GRAPHS[name], oracle_graphs[name]
    Z = O.uniform_Z(g.n) if name != "rand3k_w" else np.random.default_rng(3).random(g.n)
    say("deterministic", name, "fp32", fp32)
    y = O.SyncDI(og, D, Z, fluid_fp32=fp32)
    with gpu.from_graph(g, d=D, Z=None if name != "rand3k_w" else Z, deterministic=True, fluid_fp32=fp32,
                        max_sweeps=1) as s:
        assert s.info(gpu.INFO_FIXED_K) == y.K
        for t in range(60):
            st = s.diffuse(1e-12, allow_noconv=True)
            y.run(1e-12, max_sweeps=1, record_frontier=True)
            if y.converged:
                assert st["converged"]
                break
            np.testing.assert_array_equal(s.read(gpu.FRONTIER), y.last_frontier)
            np.testing.assert_array_equal(s.read(gpu.H), y.H)
            np.testing.assert_array_equal(s.read(gpu.F), y.F)
            assert s.read(gpu.RESIDUALS)[0] == y.R
            assert s.read(gpu.LEAKS)[0] == y.l


def test_deterministic_full_solve_matches_oracle(gpu, oracle_graphs):
    g, og = GRAPHS["tiny10k"], oracle_graphs["tiny10k"]
    Z = O.uniform_Z(g.n)
    tol = 1e-10 / (1 - D)  # remaining L1 fluid <= 1e-10
    y = O.SyncDI(og, D, Z)
    y.run(tol)
    with gpu.from_graph(g, d=D, deterministic=True) as s:
        st = s.diffuse(tol)
        assert st["converged"] and st["sweeps"] == y.sweeps
        np.testing.assert_array_equal(s.read(gpu.H), y.H)
        assert st["residual"] == y.R


# --------------------------------------------------------------------------
# Block-local sweep and power iteration: tolerance parity
# --------------------------------------------------------------------------
def reference_x(og, Z):
    y = O.SyncDI(og, D, Z)
    y.run(1e-14)
    return y.H


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("rb", [8, 0, 10, "max"])
def test_block_local_solve(gpu, oracle_graphs, name, fp32, rb):
    # rb "max" = the largest range (13, for either fluid type): the kernel that
    # reads the local adjacency from global memory; smaller ranges stage it in LDS
    if rb == "max":
        rb = 13
    g, og = GRAPHS[name], oracle_graphs[name]
    Z = O.uniform_Z(g.n)
    x = reference_x(og, Z)
    rel = 1e-6 if fp32 else 1e-9
    say("block-local", name, "fp32", fp32, "rb", rb)
    with gpu.from_graph(g, d=D, fluid_fp32=fp32, range_log2=rb, max_sweeps=5000) as s:
        st = s.diffuse(1e-11)
        assert st["converged"]
        H = s.read(gpu.H)
        F = s.read(gpu.F)
        assert np.abs(H - x).sum() <= rel * np.abs(x).sum()
        # certificate (Theorem 1); with float fluid the library recomputes F = F_0 + dPH - H
        # in double before it stops, so only the rounding of that F to float (2^-24) remains
        assert np.abs(H - x).sum() <= st["bound"] * (1 + 1e-7) + 1e-14
        # mass balance: sum F + (1-d) sum H + d l = (1-d) sum Z, on the host and as the
        # library reports it (exact sums on the device)
        l = s.read(gpu.LEAKS)[0]
        defect = O.mass_defect(og, D, Z, H, F, l)
        assert abs(defect) <= (1e-6 if fp32 else 1e-13)
        assert abs(st["mass_defect"] - defect) <= (1e-7 * st["residual"] if fp32 else 0) + 1e-14
        assert s.read(gpu.MASS_DEFECTS)[0] == st["mass_defect"]
        # invariant H + F = F_0 + d P H (equation HnFn) with the exact F_0 = (1-d) Z, P
        # applied by the oracle; with float fluid its L1 defect is the rounding of the
        # recomputed fluid to float
        F0 = O.initial_fluid(D, Z, False)
        if fp32:
            assert O.invariant_residual_l1(og, D, F0, H, F) <= 1e-7 * st["residual"] + 1e-15
        else:
            assert O.invariant_residual(og, D, F0, H, F) <= 1e-15


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("fp32", [False, True])
def test_power_iteration(gpu, oracle_graphs, name, fp32):
    g, og = GRAPHS[name], oracle_graphs[name]
    Z = O.uniform_Z(g.n)
    say("power", name, "fp32", fp32)
    xo, k, _ = O.power(og, D, Z, 1e-11)
    with gpu.from_graph(g, d=D, fluid_fp32=fp32) as s:
        st = s.power(1e-11)
        xg = s.read(gpu.X_PI)
        rel = 1e-6 if fp32 else 1e-9
        assert np.abs(xg - xo).sum() <= rel * np.abs(xo).sum()
        if not fp32:  # same iteration count up to a stop decision at the rounding boundary
            assert abs(st["sweeps"] - k) <= 1


@pytest.mark.parametrize("kw", [{"deterministic": True}, {"range_cut": -1}, {}])
def test_set_z_back_to_uniform(gpu, kw):
    """A context built with an explicit Z and then given Z = NULL solves the uniform
    problem: power iteration and D-Iteration equal a fresh uniform-Z context's results
    (bit for bit in deterministic mode)."""
    g = GRAPHS["web20k"]
    Zr = np.random.default_rng(4).random(g.n)
    say("set_z(None)", kw)
    with gpu.from_graph(g, d=D, **kw) as fresh:
        st0 = fresh.diffuse(1e-11)
        H0 = fresh.read(gpu.H)
        p0 = fresh.power(1e-11)
        X0 = fresh.read(gpu.X_PI)
    with gpu.from_graph(g, d=D, Z=Zr, **kw) as s:
        s.diffuse(1e-11)
        s.power(1e-11)
        s.set_z(None)
        st1 = s.diffuse(1e-11)
        H1 = s.read(gpu.H)
        p1 = s.power(1e-11)
        X1 = s.read(gpu.X_PI)
    assert p1["converged"] and p1["sweeps"] == p0["sweeps"] > 1
    np.testing.assert_array_equal(X1, X0)
    if kw.get("deterministic"):
        assert st1["sweeps"] == st0["sweeps"]
        np.testing.assert_array_equal(H1, H0)
    else:
        x = np.abs(H0).sum()
        assert np.abs(H1 - H0).sum() <= st0["bound"] + st1["bound"] + 1e-15 * x


def test_deterministic_theta0_matches_power_iterates(gpu, oracle_graphs):
    g, og = GRAPHS["web20k"], oracle_graphs["web20k"]
    xo, _, _ = O.power(og, D, O.uniform_Z(g.n), tol=1e-300, max_iters=15)
    with gpu.from_graph(g, d=D, deterministic=True, theta=0.0, max_sweeps=15) as s:
        s.diffuse(1e-300, allow_noconv=True)
        np.testing.assert_allclose(s.read(gpu.H), xo, rtol=1e-13, atol=1e-20)


def test_dense_reference_small(gpu):
    g = W.tiny_zipf(2000, 1)
    og = O.OGraph.of(g)
    Z = np.random.default_rng(9).random(g.n)
    Z /= Z.sum()
    x = O.dense_solve(og, D, Z)
    xbar = x / x.sum()  # completion by Z (Section 3.3) rescales x into a distribution
    for kw in ({}, {"fluid_fp32": True}, {"deterministic": True}, {"range_log2": 8}):
        with gpu.from_graph(g, d=D, Z=Z, **kw) as s:
            s.diffuse(1e-12)
            rel = 1e-6 if kw.get("fluid_fp32") else 1e-9
            assert np.abs(s.read(gpu.H) - x).sum() <= rel * np.abs(x).sum(), kw
            assert np.abs(s.read(gpu.X_NORM) - xbar).sum() <= rel * np.abs(xbar).sum(), kw


# --------------------------------------------------------------------------
# Edge cases
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["single_loop", "edgeless", "all_dangling", "unsorted_rows", "multi_edges",
                                  "single_dangling"])
def test_edge_cases(gpu, case):
    if case == "single_loop":
        g = W.from_edges(1, [0], [0])
    elif case == "single_dangling":
        g = W.from_edges(1, [], [])
    elif case == "edgeless":
        g = W.from_edges(7, [], [])
    elif case == "all_dangling":
        g = W.from_edges(300, [], [])
    elif case == "multi_edges":
        g = W.from_edges(5, [0, 0, 0, 1, 2, 3, 3], [1, 1, 1, 2, 0, 3, 3])
    else:
        g0 = W.tiny_zipf(500, 2)
        rng = np.random.default_rng(1)
        idx = g0.out_idx.copy()
        for i in range(g0.n):
            b, e = g0.out_ptr[i], g0.out_ptr[i + 1]
            idx[b:e] = rng.permutation(idx[b:e])
        g = W.Graph(g0.n, g0.out_ptr, idx, None, "unsorted")
    og = O.OGraph.of(g)
    Z = np.random.default_rng(2).random(g.n) + 0.1
    x = O.dense_solve(og, D, Z)
    for kw in ({}, {"deterministic": True}, {"fluid_fp32": True}):
        with gpu.from_graph(g, d=D, Z=Z, **kw) as s:
            st = s.diffuse(1e-13 if not kw.get("fluid_fp32") else 1e-9)
            assert st["converged"]
            rel = 1e-6 if kw.get("fluid_fp32") else 1e-11
            assert np.abs(s.read(gpu.H) - x).sum() <= rel * np.abs(x).sum() + 1e-15, (case, kw)
            s.power(1e-13)
            assert np.abs(s.read(gpu.X_PI) - x).sum() <= rel * np.abs(x).sum() + 1e-15


def test_device_inputs(gpu):
    import torch
    g = W.webgen(5000, 3, weighted=True)
    og = O.OGraph.of(g)
    x = reference_x(og, O.uniform_Z(g.n))
    dev = torch.device("cuda:0")
    s = gpu.Solver(g.n, torch.from_numpy(g.out_ptr).to(dev), torch.from_numpy(g.out_idx).to(dev),
                   torch.from_numpy(g.w).to(dev), d=D)
    s.diffuse(1e-12)
    out = torch.empty(g.n, dtype=torch.float64, device=dev)
    s.read(gpu.H, out=out)
    assert np.abs(out.cpu().numpy() - x).sum() <= 1e-9 * np.abs(x).sum()
    s.close()


def test_device_graph_is_checked_on_the_device(gpu):
    """A graph given in device memory is checked there with the host check's rules and
    messages, and solves bit for bit like the same graph given on the host (sorted rows are
    copied device to device; unsorted rows are sorted on the host first)."""
    import torch
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    g = W.webgen(5000, 3, weighted=True)
    m = len(g.out_idx)
    rng = np.random.default_rng(5)
    rows = np.nonzero(np.diff(g.out_ptr) >= 3)[0]
    shuffled = g.out_idx.copy()
    for r in rows[:50]:
        b, e = g.out_ptr[r], g.out_ptr[r + 1]
        shuffled[b:e] = shuffled[b:e][rng.permutation(e - b)]
    for idx in (g.out_idx, shuffled):  # the same arrays on the host and on the device
        hs = {}
        for where in ("host", "device"):
            arrs = (g.out_ptr, idx, g.w) if where == "host" else (T(g.out_ptr), T(idx), T(g.w))
            with gpu.Solver(g.n, *arrs, d=D, deterministic=True) as s:
                s.diffuse(1e-12)
                hs[where] = s.read(gpu.H)
        assert np.array_equal(hs["host"], hs["device"])
    base = gpu.live_allocations()
    p_bad_first = g.out_ptr.copy(); p_bad_first[0] = 1
    p_bad_last = g.out_ptr.copy(); p_bad_last[-1] = m - 1
    r = int(rows[10])
    p_bad_mid = g.out_ptr.copy(); p_bad_mid[r] = p_bad_mid[r + 1] + 1
    i_big = g.out_idx.copy(); i_big[123] = g.n
    i_neg = g.out_idx.copy(); i_neg[7] = -1
    w_zero = g.w.copy(); w_zero[99] = 0.0
    w_nan = g.w.copy(); w_nan[5] = np.nan
    cases = [(p_bad_first, g.out_idx, g.w), (p_bad_last, g.out_idx, g.w), (p_bad_mid, g.out_idx, g.w),
             (g.out_ptr, i_big, g.w), (g.out_ptr, i_neg, g.w), (g.out_ptr, g.out_idx, w_zero),
             (g.out_ptr, g.out_idx, w_nan)]
    for arrs in cases:
        msgs = []
        for on_dev in (False, True):
            with pytest.raises(gpu.DIError) as e:
                gpu.Solver(g.n, *[T(a) if on_dev else a for a in arrs], d=D)
            assert e.value.code == gpu.DI_EINVAL
            msgs.append(str(e.value))
        say(msgs[1])
        assert msgs[0] == msgs[1]
        assert gpu.live_allocations() == base


def test_error_paths(gpu):
    g = W.tiny_zipf(300, 3)
    with gpu.from_graph(g, d=D, max_sweeps=2) as s:
        with pytest.raises(gpu.DIError) as e:
            s.diffuse(0.0)
        assert e.value.code == gpu.DI_EINVAL
        with pytest.raises(gpu.DIError) as e:
            s.adjoint(np.ones(g.n), 1e-10)
        assert e.value.code == gpu.DI_ESTATE
        with pytest.raises(gpu.DIError) as e:
            s.diffuse(1e-14)
        assert e.value.code == gpu.DI_ENOCONV
        # the state is kept: later calls continue to convergence
        for _ in range(200):
            st = s.diffuse(1e-14, allow_noconv=True)
            if st["converged"]:
                break
        assert st["converged"]


def test_checkpoint_resume(gpu, tmp_path):
    g = GRAPHS["web20k"]
    path = str(tmp_path / "ck.bin")
    with gpu.from_graph(g, d=D, deterministic=True, max_sweeps=7) as a:
        a.diffuse(1e-12, allow_noconv=True)
        a.save(path)
        a.diffuse(1e-12, allow_noconv=True)
        a.diffuse(1e-12, allow_noconv=True)
        ref_H, ref_F = a.read(gpu.H), a.read(gpu.F)
    with gpu.from_graph(g, d=D, deterministic=True, max_sweeps=7) as b:
        b.load(path)
        b.diffuse(1e-12, allow_noconv=True)
        b.diffuse(1e-12, allow_noconv=True)
        np.testing.assert_array_equal(b.read(gpu.H), ref_H)
        np.testing.assert_array_equal(b.read(gpu.F), ref_F)
    with gpu.from_graph(g, d=0.8, deterministic=True) as c:
        with pytest.raises(gpu.DIError):
            c.load(path)


def test_graph_loop_mode_matches_stream(gpu):
    g = GRAPHS["web20k"]
    res = []
    for lm in (gpu.LOOP_STREAM, gpu.LOOP_GRAPH):
        with gpu.from_graph(g, d=D, deterministic=True, loop_mode=lm, sweeps_per_sync=4) as s:
            st = s.diffuse(1e-11)
            res.append((st["sweeps"], s.read(gpu.H)))
            s.power(1e-11)
            res.append((0, s.read(gpu.X_PI)))
    assert res[0][0] == res[2][0]
    np.testing.assert_array_equal(res[0][1], res[2][1])
    np.testing.assert_array_equal(res[1][1], res[3][1])


@pytest.mark.parametrize("fp32", [False, True])
def test_graph_loop_mode_fast_sweeps(gpu, oracle_graphs, fp32):
    """Fast block-local sweeps (and the float fluid's recomputation) under HIP-graph
    capture: every replay of the captured chunk, with eager work and synchronisation
    between replays, meets the certificate against the oracle; the sweep count stays near
    the stream-mode one (fast sweeps are not reproducible bit for bit)."""
    g, og = GRAPHS["web20k"], oracle_graphs["web20k"]
    Z = O.uniform_Z(g.n)
    x = reference_x(og, Z)
    rel = 1e-6 if fp32 else 1e-9
    sweeps = {}
    for lm in (gpu.LOOP_STREAM, gpu.LOOP_GRAPH):
        say("fast sweeps, loop mode", lm, "fp32", fp32)
        with gpu.from_graph(g, d=D, fluid_fp32=fp32, loop_mode=lm, sweeps_per_sync=4) as s:
            for rep in range(3):
                s.reset()
                st = s.diffuse(1e-11)
                H = s.read(gpu.H)
                assert st["converged"], (lm, rep)
                err = np.abs(H - x).sum()
                assert err <= st["bound"] * (1 + 1e-6) + 1e-14, (lm, rep, err, st["bound"])
                assert err <= rel * np.abs(x).sum()
                s.power(1e-11)  # eager work between replays
            sweeps[lm] = st["sweeps"]
    assert abs(sweeps[gpu.LOOP_STREAM] - sweeps[gpu.LOOP_GRAPH]) <= 3
