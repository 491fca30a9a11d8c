"""Graph update (Section 3.5, Theorem 4) on the GPU against the oracle.

A context diffuses on P for a while, di_update swaps in P' (edited edges, weights and
dangling nodes on the same node set: H' = H, F' = F + d (P' - P) H, the leak reset to the
history at the nodes dangling in P'), and D-Iteration continues with signed fluid.

Deterministic mode: bit for bit against the oracle's synchronous sweep updated the same
way (F, H, fixed-point scale, residual and leak right after the update, then frontier, F,
H, residual and leak after every sweep to convergence), in double and float fluid.
Fast mode: the result meets |x' - H|_1 <= 1e-9 |x'|_1 (double; 1e-6 with float fluid)
against x' from the oracle on P', and the certificate |x' - H|_1 <= |F|_1 / (1-d) holds.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
D = 0.85


def say(*a):
    print(*a, flush=True)


def weighted_rand(n, seed):
    rng = np.random.default_rng(seed)
    deg = rng.integers(0, 8, size=n)
    src = np.repeat(np.arange(n), deg)
    dst = rng.integers(0, n, size=len(src))
    return W.from_edges(n, src, dst, rng.lognormal(0, 1, size=len(src)).astype(np.float32), "rand%d_w" % n)


CASES = {
    "tiny10k": lambda: W.tiny_zipf(10_000, 1),
    "web20k": lambda: W.webgen(20_000, 7),
    "rand3k_w": lambda: weighted_rand(3000, 21),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("fp32", [False, True])
def test_update_deterministic_bit_exact(gpu, name, fp32):
    g = CASES[name]()
    g2 = W.edit_graph(g, 3, 0.01)
    oa, ob = O.OGraph.of(g), O.OGraph.of(g2)
    Z = O.uniform_Z(g.n)
    say("update deterministic", name, "fp32", fp32, "m", g.m, "->", g2.m)
    y = O.SyncDI(oa, D, Z, fluid_fp32=fp32)
    y.run(1e-300, max_sweeps=6)
    with gpu.from_graph(g, d=D, deterministic=True, fluid_fp32=fp32, max_sweeps=1) as s:
        for _ in range(6):
            s.diffuse(1e-300, allow_noconv=True)
        np.testing.assert_array_equal(s.read(gpu.H), y.H)
        s.update_graph(g2)
        y.update(ob)
        assert s.info(gpu.INFO_FIXED_K) == y.K
        assert s.info(gpu.INFO_M) == g2.m
        np.testing.assert_array_equal(s.read(gpu.F), y.F)
        np.testing.assert_array_equal(s.read(gpu.H), y.H)
        assert s.read(gpu.LEAKS)[0] == y.l
        assert y.F.min() < 0  # the update injects negative fluid
        for t in range(200):
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
        assert y.converged
        np.testing.assert_array_equal(s.read(gpu.H), y.H)


def reference(og, Z):
    if og.n <= 2000:
        return O.dense_solve(og, D, Z)
    y = O.SyncDI(og, D, Z)
    y.run(1e-14)
    return y.H


@pytest.mark.parametrize("name", ["web20k", "rand3k_w", "web1m"])
@pytest.mark.parametrize("fp32", [False, True])
def test_update_fast_tolerance(gpu, name, fp32):
    g = W.webgen(1_000_000, 2) if name == "web1m" else CASES[name]()
    g2 = W.edit_graph(g, 4, 0.01)
    ob = O.OGraph.of(g2)
    Z = O.uniform_Z(g.n)
    x2 = reference(ob, Z)
    xn = float(np.abs(x2).sum())
    rel = 1e-6 if fp32 else 1e-9
    say("update fast", name, "fp32", fp32)
    with gpu.from_graph(g, d=D, fluid_fp32=fp32) as s:
        s.diffuse(1e-6)
        s.update_graph(g2)
        st = s.diffuse(1e-11)
        assert st["converged"]
        H = s.read(gpu.H)
        F = s.read(gpu.F)
        l = s.read(gpu.LEAKS)[0]
    err = float(np.abs(H - x2).sum())
    say("  %d sweeps after the update, |H - x'|_1 = %.3e, bound %.3e" % (st["sweeps"], err, st["bound"]))
    assert err <= rel * xn
    assert err <= st["bound"] * (1 + 1e-6) + 1e-13 * xn
    # invariant for P' with the original F_0, and the mass balance with the reset leak
    F0 = O.initial_fluid(D, Z, False)
    inv = O.invariant_residual_l1(ob, D, F0, H, F)
    assert inv <= (1e-7 * st["residual"] if fp32 else 1e-13 * xn) + 1e-15
    md = O.mass_defect(ob, D, Z, H, F, l)
    assert abs(st["mass_defect"] - md) <= (1e-7 * st["residual"] if fp32 else 0) + 1e-13
    assert abs(md) <= (1e-7 * st["residual"] if fp32 else 0) + 1e-13


def test_update_edge_cases(gpu):
    import torch
    g = W.webgen(20_000, 7)
    g2 = W.edit_graph(g, 5, 0.01)
    Z = O.uniform_Z(g.n)
    x = reference(O.OGraph.of(g), Z)
    x2 = reference(O.OGraph.of(g2), Z)
    with gpu.from_graph(g, d=D) as s:
        s.diffuse(1e-11)
        # the same graph again: nothing to correct, the call converges at once
        s.update_graph(g)
        st = s.diffuse(1e-11)
        assert st["converged"] and st["sweeps"] == 0
        assert np.abs(s.read(gpu.H) - x).sum() <= 1e-9 * np.abs(x).sum()
        # device arrays; then back to the first graph
        dev = torch.device("cuda:0")
        s.update(torch.from_numpy(g2.out_ptr).to(dev), torch.from_numpy(g2.out_idx).to(dev))
        st = s.diffuse(1e-11)
        assert st["converged"] and np.abs(s.read(gpu.H) - x2).sum() <= 1e-9 * np.abs(x2).sum()
        s.update_graph(g)
        s.diffuse(1e-11)
        assert np.abs(s.read(gpu.H) - x).sum() <= 1e-9 * np.abs(x).sum()
        # power iteration runs on the new graph
        s.power(1e-11)
        assert np.abs(s.read(gpu.X_PI) - x).sum() <= 1e-9 * np.abs(x).sum()
        # another node count is refused and leaves the context as it was
        g3 = W.tiny_zipf(500, 2)
        with pytest.raises(gpu.DIError) as e:
            s.update(g3.out_ptr, g3.out_idx)
        assert e.value.code == gpu.DI_EINVAL
        assert np.abs(s.read(gpu.H) - x).sum() <= 1e-9 * np.abs(x).sum()
    Zk = W.ppr_Z(g.n, 4, 16, seed=3)
    with gpu.from_graph(g, d=D, Z=Zk, k=4) as s:
        with pytest.raises(gpu.DIError):
            s.update_graph(g2)
