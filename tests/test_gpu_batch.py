"""Several right-hand sides (n x k tile) and unions of independent graphs on the GPU.

Deterministic mode: every column of the tile, and every graph of a union, must equal the
oracle's synchronous sweep run on that column / graph alone, bit for bit (history,
fluid, residual, leak and the sweep at which it stopped), with the oracle's fixed-point
scale set to the one the library reports.  Fast mode: each column / graph must meet
its own certificate |x - H|_1 <= |F|_1 / (1-d) against an exact reference (a dense
solve, or the oracle run far past the tolerance).  With float fluid the library
recomputes the fluid from H in double before it stops, so the certificate holds there
too, up to the rounding of that fluid to float (2^-24 relative).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
D = 0.85


def say(*a):
    print(*a, flush=True)


def oracle_column(og, Z, K, tol, fp32=False):
    y = O.SyncDI(og, D, Z, fluid_fp32=fp32)
    y.K = K
    y.run(tol)
    assert y.converged
    return y


def exact(og, Z):
    if og.n <= 2000:
        return O.dense_solve(og, D, Z)
    y = O.SyncDI(og, D, Z)
    y.run(1e-14)
    return y.H


def rand_weighted(n, seed):
    rng = np.random.default_rng(seed)
    deg = rng.integers(0, 8, size=n)
    src = np.repeat(np.arange(n), deg)
    dst = rng.integers(0, n, size=len(src))
    w = rng.lognormal(0, 1, size=len(src)).astype(np.float32)
    return W.from_edges(n, src, dst, w, "rand%d" % n)


def hub_graph(n, seed, weighted):
    """Random sparse graph plus three hubs with 2500-5000 in-edges each (IN rows longer
    than one segment of the float tile's fluid recomputation)."""
    rng = np.random.default_rng(seed)
    deg = rng.integers(0, 6, size=n)
    src = [np.repeat(np.arange(n), deg)]
    dst = [rng.integers(0, n, size=int(deg.sum()))]
    for hub, cnt in ((3, 5000), (n // 2, 2600), (n - 5, 4100)):
        src.append(rng.choice(n, size=cnt, replace=False))
        dst.append(np.full(cnt, hub))
    src, dst = np.concatenate(src), np.concatenate(dst)
    w = rng.lognormal(0, 1, size=len(src)).astype(np.float32) if weighted else None
    return W.from_edges(n, src, dst, w, "hubs%d" % n)


# ---------------------------------------------------------------------------
# n x k tile
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["web20k_k64_f64", "web20k_k64_f32", "rand3k_w_k5_f64", "zipf5k_k33_f32"])
def test_tile_deterministic_bit_exact(gpu, case):
    g = {"web20k": lambda: W.webgen(20_000, 8), "rand3k": lambda: rand_weighted(3000, 5),
         "zipf5k": lambda: W.tiny_zipf(5000, 3)}[case.split("_")[0]]()
    k = int([t for t in case.split("_") if t.startswith("k")][0][1:])
    fp32 = case.endswith("f32")
    tol = 1e-7 if fp32 else 1e-11
    say("tile det", case, "n=%d m=%d k=%d" % (g.n, g.m, k))
    og = O.OGraph.of(g)
    Z = W.ppr_Z(g.n, k, 16, seed=4)
    with gpu.from_graph(g, d=D, Z=Z, k=k, deterministic=True, fluid_fp32=fp32) as s:
        st = s.diffuse(tol)
        assert st["converged"]
        K = s.info(gpu.INFO_FIXED_K)
        H = s.read(gpu.H)
        F = s.read(gpu.F)
        R = s.read(gpu.RESIDUALS)
        L = s.read(gpu.LEAKS)
        done = s.read(gpu.DONE_SWEEPS)
    assert H.shape == (k, g.n)
    for c in range(k):
        y = oracle_column(og, Z[:, c], K, tol, fp32)
        np.testing.assert_array_equal(H[c], y.H, err_msg="H column %d" % c)
        np.testing.assert_array_equal(F[c], y.F, err_msg="F column %d" % c)
        assert R[c] == y.R and L[c] == y.l, c
        assert done[c] == y.sweeps, (c, done[c], y.sweeps)
    assert st["sweeps"] == done.max()


@pytest.mark.parametrize("case", ["rand1500_w_f64", "rand1500_w_f32", "web50k_f32", "web50k_f64", "hubs6k_f32",
                                  "hubs6k_w_f32"])
def test_tile_fast_certificates(gpu, case):
    if case.startswith("rand"):
        g = rand_weighted(1500, 9)
    elif case.startswith("hubs"):
        g = hub_graph(6000, 12, "_w_" in case)
    else:
        g = W.webgen(50_000, 6)
    fp32 = case.endswith("f32")
    k = 64
    og = O.OGraph.of(g)
    Z = W.ppr_Z(g.n, k, 16, seed=7)
    tol = 1e-8
    say("tile fast", case)
    with gpu.from_graph(g, d=D, Z=Z, k=k, fluid_fp32=fp32) as s:
        st = s.diffuse(tol)
        assert st["converged"]
        H = s.read(gpu.H)
        F = s.read(gpu.F)
        R = s.read(gpu.RESIDUALS)
        Xn = s.read(gpu.X_NORM)
        L = s.read(gpu.LEAKS)
        done = s.read(gpu.DONE_SWEEPS)
        MD = s.read(gpu.MASS_DEFECTS)
    assert (done >= 1).all() and done.max() == st["sweeps"]
    assert len(MD) == k and st["mass_defect"] == MD[np.argmax(np.abs(MD))]
    for c in range(0, k, 9 if g.n > 2000 else 1):
        # the leak is the history at the dangling nodes (Section 3.3)
        assert abs(L[c] - H[c][og.dangling].sum()) <= 1e-14, (c, L[c], H[c][og.dangling].sum())
        md = O.mass_defect(og, D, Z[:, c], H[c], F[c], L[c])
        slack = 1e-7 * R[c] if fp32 else 0.0
        assert abs(MD[c] - md) <= slack + 1e-14, (c, MD[c], md)
        assert abs(MD[c]) <= slack + 1e-13, (c, MD[c], md, R[c])
        x = exact(og, Z[:, c])
        assert R[c] / (1 - D) <= tol
        assert np.abs(H[c] - x).sum() <= R[c] / (1 - D) * (1 + 1e-7) + 1e-12, c
        assert np.abs(F[c]).sum() <= R[c] * (1 + 1e-12) + 1e-300
        # equation HnFn: H + F = F_0 + d P H, per column
        d_inv = O.invariant_residual_l1(og, D, O.initial_fluid(D, Z[:, c], False), H[c], F[c])
        assert d_inv <= 1e-7 * R[c] + 1e-14, (c, d_inv)
        scale = (1 - D) / (1 - D - D * L[c] / Z[:, c].sum())
        np.testing.assert_allclose(Xn[c], scale * H[c], rtol=1e-14, atol=0)


def test_tile_columns_match_single_solves(gpu):
    """Uniform Z in every column (Z = NULL): each column is the one-column solve."""
    g = W.webgen(30_000, 2)
    with gpu.from_graph(g, d=D, k=3, deterministic=True) as s:
        s.diffuse(1e-12)
        H = s.read(gpu.H)
    with gpu.from_graph(g, d=D, deterministic=True) as s1:
        s1.diffuse(1e-12)
        h1 = s1.read(gpu.H)
    for c in range(3):
        np.testing.assert_array_equal(H[c], h1)


def test_tile_graph_loop_and_continuation(gpu):
    g = W.webgen(20_000, 3)
    Z = W.ppr_Z(g.n, 8, 16, seed=2)
    with gpu.from_graph(g, d=D, Z=Z, k=8, deterministic=True) as s:
        s.diffuse(1e-10)
        ref = s.read(gpu.H)
        s.reset()
        # a budget too small: DI_ENOCONV keeps the state; the next call continues it
        with gpu.from_graph(g, d=D, Z=Z, k=8, deterministic=True, max_sweeps=5) as s2:
            st = s2.diffuse(1e-10, allow_noconv=True)
            assert not st["converged"] and st["sweeps"] == 5
            for _ in range(100):
                st = s2.diffuse(1e-10, allow_noconv=True)
                if st["converged"]:
                    break
            np.testing.assert_array_equal(s2.read(gpu.H), ref)
    with gpu.from_graph(g, d=D, Z=Z, k=8, deterministic=True, loop_mode=gpu.LOOP_GRAPH, sweeps_per_sync=3) as s3:
        s3.diffuse(1e-10)
        np.testing.assert_array_equal(s3.read(gpu.H), ref)
        # a second call with a smaller tolerance continues; reset starts over
        s3.diffuse(1e-12)
        assert (s3.read(gpu.RESIDUALS) / (1 - D) <= 1e-12).all()
        s3.reset()
        s3.diffuse(1e-10)
        np.testing.assert_array_equal(s3.read(gpu.H), ref)


def test_tile_edge_cases(gpu):
    # edgeless graph: one sweep moves all fluid to H and out through the dangling nodes
    n = 100
    g = W.from_edges(n, [], [], None, "edgeless")
    Z = W.ppr_Z(n, 4, 16, seed=1)
    with gpu.from_graph(g, d=D, Z=Z, k=4) as s:
        st = s.diffuse(1e-12)
        assert st["converged"]
        np.testing.assert_allclose(s.read(gpu.H), (1 - D) * Z.T, rtol=0, atol=0)
        np.testing.assert_allclose(s.read(gpu.LEAKS), (1 - D) * np.ones(4), rtol=1e-15)
        np.testing.assert_allclose(s.read(gpu.X_NORM), Z.T, rtol=1e-14)
    # one node with a self-loop: x = (1-d) z / (1-d) = z
    g1 = W.from_edges(1, [0], [0], None, "loop")
    with gpu.from_graph(g1, d=D, k=2) as s:
        s.diffuse(1e-13)
        np.testing.assert_allclose(s.read(gpu.H), [[1.0], [1.0]], rtol=0, atol=1e-13 / (1 - D) * 1.01)
    # a column concentrated on one dangling node and one on a hub
    g2 = W.tiny_zipf(3000, 5)
    og = O.OGraph.of(g2)
    dang = int(np.flatnonzero(np.diff(g2.out_ptr) == 0)[0])
    hub = int(np.argmax(np.diff(g2.out_ptr)))
    Z2 = np.zeros((g2.n, 2), order="F")
    Z2[dang, 0] = 1.0
    Z2[hub, 1] = 1.0
    with gpu.from_graph(g2, d=D, Z=Z2, k=2, fluid_fp32=True) as s:
        s.diffuse(1e-9)
        H = s.read(gpu.H)
        R = s.read(gpu.RESIDUALS)
    for c in range(2):
        x = exact(og, Z2[:, c])
        assert np.abs(H[c] - x).sum() <= R[c] / (1 - D) * (1 + 1e-7) + 1e-12


def test_tile_k64_ppr_workload(gpu):
    """Personalized PageRank workload: web-like graph n=4M, k=64 columns of 16 seeds, FP32 fluid."""
    g = W.webgen(4_000_000, 4)
    Z = W.ppr_Z(g.n, 64, 16, seed=4)
    say("k=64 tile on n=%d m=%d" % (g.n, g.m))
    with gpu.from_graph(g, d=D, Z=Z, k=64, fluid_fp32=True) as s:
        st = s.diffuse(1e-8)
        assert st["converged"]
        R = s.read(gpu.RESIDUALS)
        H = s.read(gpu.H)
    say("tile: %d sweeps, %.1f ms" % (st["sweeps"], st["ms"]))
    assert (R / (1 - D) <= 1e-8).all()
    cols = [0, 17, 40, 63]
    for c in cols:
        with gpu.from_graph(g, d=D, Z=np.ascontiguousarray(Z[:, c])) as s1:
            s1.diffuse(1e-12)
            x = s1.read(gpu.H)
        err = np.abs(H[c] - x).sum()
        assert err <= R[c] / (1 - D) * (1 + 1e-7) + 1e-12 / (1 - D), (c, err)


# ---------------------------------------------------------------------------
# union of graphs
# ---------------------------------------------------------------------------
def small_union(seed=0):
    sizes = [1000, 255, 256, 257, 3000, 1, 2, 7000, 513, 12_000]
    graphs = []
    for q, n in enumerate(sizes):
        if n == 1:
            graphs.append(W.from_edges(1, [], [], None, "one"))
        elif n == 2:
            graphs.append(W.from_edges(2, [0, 1, 1], [1, 0, 1], None, "two"))
        elif n < 1000:
            graphs.append(W.tiny_zipf(n, 20 + q))
        else:
            graphs.append(W.webgen(n, 30 + q))
    return graphs


@pytest.mark.parametrize("fp32", [False, True])
def test_union_deterministic_bit_exact(gpu, fp32):
    graphs = small_union()
    u, gp = W.union(graphs)
    tol = 1e-7 if fp32 else 1e-11
    say("union det fp32=%s n=%d graphs=%d" % (fp32, u.n, len(graphs)))
    with gpu.Solver(u.n, u.out_ptr, u.out_idx, None, d=D, graph_ptr=gp, deterministic=True, fluid_fp32=fp32) as s:
        st = s.diffuse(tol)
        assert st["converged"]
        K = s.info(gpu.INFO_FIXED_K)
        assert s.info(gpu.INFO_N) == u.n and s.info(gpu.INFO_N_INTERNAL) >= u.n
        H = s.read(gpu.H)
        F = s.read(gpu.F)
        R = s.read(gpu.RESIDUALS)
        L = s.read(gpu.LEAKS)
        done = s.read(gpu.DONE_SWEEPS)
        fr = s.read(gpu.FRONTIER)
    assert len(R) == len(graphs)
    last = None
    for q, gq in enumerate(graphs):
        og = O.OGraph.of(gq)
        y = oracle_column(og, np.full(gq.n, 1.0 / gq.n), K, tol, fp32)
        sl = slice(gp[q], gp[q + 1])
        np.testing.assert_array_equal(H[sl], y.H, err_msg="graph %d" % q)
        np.testing.assert_array_equal(F[sl], y.F, err_msg="graph %d" % q)
        assert R[q] == y.R and L[q] == y.l and done[q] == y.sweeps, (q, done[q], y.sweeps)
    assert st["sweeps"] == done.max()
    # the frontier of the last sweep lies in the graphs still running then
    running = [q for q in range(len(graphs)) if done[q] == done.max()]
    assert len(fr) > 0
    owner = np.searchsorted(gp, fr, side="right") - 1
    assert set(owner.tolist()) <= set(running)


@pytest.mark.parametrize("fp32", [False, True])
def test_union_fast_certificates(gpu, fp32):
    graphs = small_union()
    u, gp = W.union(graphs)
    tol = 1e-8
    with gpu.Solver(u.n, u.out_ptr, u.out_idx, None, d=D, graph_ptr=gp, fluid_fp32=fp32) as s:
        st = s.diffuse(tol)
        assert st["converged"]
        H = s.read(gpu.H)
        F = s.read(gpu.F)
        R = s.read(gpu.RESIDUALS)
        Xn = s.read(gpu.X_NORM)
        L = s.read(gpu.LEAKS)
        done = s.read(gpu.DONE_SWEEPS)
        MD = s.read(gpu.MASS_DEFECTS)
    assert (done >= 0).all()
    assert len(MD) == len(graphs) and st["mass_defect"] == MD[np.argmax(np.abs(MD))]
    for q, gq in enumerate(graphs):
        og = O.OGraph.of(gq)
        Zq = np.full(gq.n, 1.0 / gq.n)
        x = exact(og, Zq)
        sl = slice(gp[q], gp[q + 1])
        md = O.mass_defect(og, D, Zq, H[sl], F[sl], L[q])
        slack = 1e-7 * R[q] if fp32 else 0.0
        assert abs(MD[q]) <= slack + 1e-13 and abs(MD[q] - md) <= slack + 1e-14, (q, MD[q], md)
        assert R[q] / (1 - D) <= tol
        assert np.abs(H[sl] - x).sum() <= R[q] / (1 - D) * (1 + 1e-7) + 1e-12, q
        d_inv = O.invariant_residual_l1(og, D, O.initial_fluid(D, Zq, False), H[sl], F[sl])
        assert d_inv <= 1e-7 * R[q] + 1e-14, (q, d_inv)
        np.testing.assert_allclose(Xn[sl], (1 - D) / (1 - D - D * L[q] / Zq.sum()) * H[sl], rtol=1e-12, atol=0)


def test_union_second_call_and_reset(gpu):
    graphs = small_union()
    u, gp = W.union(graphs)
    with gpu.Solver(u.n, u.out_ptr, u.out_idx, None, d=D, graph_ptr=gp, deterministic=True) as s:
        s.diffuse(1e-10)
        ref = s.read(gpu.H)
        s.diffuse(1e-12)  # frozen graphs start again under the smaller tolerance
        R = s.read(gpu.RESIDUALS)
        assert (R / (1 - D) <= 1e-12).all()
        s.reset()
        s.diffuse(1e-10)
        np.testing.assert_array_equal(s.read(gpu.H), ref)
    with gpu.Solver(u.n, u.out_ptr, u.out_idx, None, d=D, graph_ptr=gp, fluid_fp32=True) as s:
        s.diffuse(1e-7)
        s.diffuse(1e-9)
        R = s.read(gpu.RESIDUALS)
        assert (R / (1 - D) <= 1e-9).all()
        with pytest.raises(gpu.DIError):
            s.power(1e-8)
        with pytest.raises(gpu.DIError):
            s.read(gpu.IN_PTR)


def test_union_256_graph_workload(gpu):
    """256 independent web-like graphs of log-uniform size 1k..200k, uniform Z each, FP32 fluid."""
    u, gp = W.multigraph_batch(256, 4)
    say("union of 256: n=%d m=%d" % (u.n, u.m))
    with gpu.Solver(u.n, u.out_ptr, u.out_idx, None, d=D, graph_ptr=gp, fluid_fp32=True) as s:
        st = s.diffuse(1e-8)
        assert st["converged"]
        R = s.read(gpu.RESIDUALS)
        H = s.read(gpu.H)
    say("union: %d sweeps, %.1f ms" % (st["sweeps"], st["ms"]))
    assert len(R) == 256 and (R / (1 - D) <= 1e-8).all()
    rng = np.random.default_rng(1)
    for q in sorted(rng.choice(256, 6, replace=False).tolist()):
        lo, hi = int(gp[q]), int(gp[q + 1])
        ptr = u.out_ptr[lo:hi + 1] - u.out_ptr[lo]
        idx = u.out_idx[u.out_ptr[lo]:u.out_ptr[hi]] - lo
        with gpu.Solver(hi - lo, ptr, idx, None, d=D) as s1:
            s1.diffuse(1e-12)
            x = s1.read(gpu.H)
        err = np.abs(H[lo:hi] - x).sum()
        assert err <= R[q] / (1 - D) * (1 + 1e-7) + 1e-12 / (1 - D), (q, err)
        # the oracle's exact residual of the graph's history certifies it on its own
        og = O.OGraph(hi - lo, ptr, idx)
        Hq = H[lo:hi]
        Rq = float(np.abs((1 - D) / (hi - lo) + D * og.P_times(Hq) - Hq).sum())
        assert Rq / (1 - D) <= 1e-8 * (1 + 1e-6), (q, Rq)


# ---------------------------------------------------------------------------
# new right-hand sides on a resident graph
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["single", "tile", "union"])
def test_set_z_matches_fresh_context(gpu, kind):
    if kind == "union":
        graphs = small_union()
        g, gp = W.union(graphs)
        kw = {"graph_ptr": gp}
        Z1 = np.random.default_rng(1).random(g.n)
        Z2 = np.random.default_rng(2).random(g.n)
    else:
        g = W.webgen(30_000, 9)
        kw = {"k": 8} if kind == "tile" else {}
        k = kw.get("k", 1)
        Z1 = W.ppr_Z(g.n, k, 16, seed=11)
        Z2 = W.ppr_Z(g.n, k, 16, seed=12)
        if k == 1:
            Z1, Z2 = Z1[:, 0].copy(), Z2[:, 0].copy()
    with gpu.Solver(g.n, g.out_ptr, g.out_idx, None, d=D, Z=Z2, deterministic=True, **kw) as fresh:
        fresh.diffuse(1e-10)
        ref = fresh.read(gpu.H)
        ref_sw = fresh.read(gpu.DONE_SWEEPS)
    with gpu.Solver(g.n, g.out_ptr, g.out_idx, None, d=D, Z=Z1, deterministic=True, **kw) as s:
        s.diffuse(1e-10)
        s.set_z(Z2)
        s.diffuse(1e-10)
        np.testing.assert_array_equal(s.read(gpu.H), ref)
        np.testing.assert_array_equal(s.read(gpu.DONE_SWEEPS), ref_sw)
        with pytest.raises(gpu.DIError):
            s.set_z(-np.ones_like(Z2))
        np.testing.assert_array_equal(s.read(gpu.H), ref)  # a rejected Z changes nothing


@pytest.mark.parametrize("kind", ["tile", "union"])
def test_graph_loop_mode_fast_batched(gpu, kind):
    """The fast tile (float fluid) and the fast union of graphs under HIP-graph capture:
    replays with eager work between them meet every column's / graph's certificate."""
    if kind == "tile":
        g = W.webgen(20_000, 3)
        Z = W.ppr_Z(g.n, 8, 16, seed=2)
        og = O.OGraph.of(g)
        refs = [exact(og, Z[:, c]) for c in range(8)]
        make = lambda lm: gpu.from_graph(g, d=D, Z=Z, k=8, fluid_fp32=True, loop_mode=lm, sweeps_per_sync=3)
    else:
        graphs = small_union()
        g, gp = W.union(graphs)
        refs = [exact(O.OGraph.of(q), np.full(q.n, 1.0 / q.n)) for q in graphs]
        make = lambda lm: gpu.Solver(g.n, g.out_ptr, g.out_idx, None, d=D, graph_ptr=gp, loop_mode=lm,
                                     sweeps_per_sync=3)
    for lm in (gpu.LOOP_STREAM, gpu.LOOP_GRAPH):
        say("fast", kind, "loop mode", lm)
        with make(lm) as s:
            for rep in range(3):
                s.reset()
                st = s.diffuse(1e-9)
                assert st["converged"], (lm, rep)
                H = s.read(gpu.H)
                R = s.read(gpu.RESIDUALS)
                for q, xr in enumerate(refs):
                    h = H[q] if kind == "tile" else H[gp[q]:gp[q + 1]]
                    assert np.abs(h - xr).sum() <= R[q] / (1 - D) * (1 + 1e-6) + 1e-13, (lm, rep, q)
                s.read(gpu.X_NORM)  # eager work between replays
            # new options and a new tolerance: the captured chunks must not be reused
            s.reset()
            s.set_options(theta=0.5, inner_rounds=3)
            st = s.diffuse(1e-10)
            assert st["converged"], lm
            H = s.read(gpu.H)
            R = s.read(gpu.RESIDUALS)
            assert R.max() / (1 - D) <= 1e-10
            for q, xr in enumerate(refs):
                h = H[q] if kind == "tile" else H[gp[q]:gp[q + 1]]
                assert np.abs(h - xr).sum() <= R[q] / (1 - D) * (1 + 1e-6) + 1e-13, (lm, "new options", q)
