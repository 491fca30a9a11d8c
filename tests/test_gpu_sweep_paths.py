"""Paths of the single-column block-local sweep's local rounds, against the CPU oracle.

The graph is built so that every path of the local rounds runs:
- a 64-node chunk whose nodes carry 300 local edges each (19,200 edge slots, more than one
  push list holds) and a single node with 1,500 local edges: the oversized-chunk path,
  where the chunk's nodes push one at a time with the whole wave striding over each
  node's edges (one node or many);
- chunks of 64 nodes with 12 edges each (768 slots): lists that fill on edge slots;
- chunks of 64 nodes with one edge each: lists that fill on nodes;
- dangling nodes and a sparse background with 80% short edges.
Frontier scale 0.05 makes most sources send in most sweeps (the gather then reads the
in-flight values directly), scale 4 leaves most idle (the gather tests the bitmap first);
1, 6 and 12 local rounds; double and float fluid; cut-aligned and plain ranges.

Checks: the solve converges; |H - x|_1 <= rel |x|_1 (x from the oracle's synchronous
D-Iteration run to 1e-14), and within the certified bound (Theorem 1); double fluid stays
nonnegative (two waves may take from one node in different local rounds; float fluid is
recomputed in double before the stop, a residual signed at the rounding level); mass balance
sum F + (1-d) sum H + d l = (1-d) sum Z with the leak l the library reports (about 12% of
the nodes are dangling); the invariant H + F = F_0 + d P H (equation HnFn) with P applied
by the oracle.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
D = 0.85


def say(*a):
    print(*a, flush=True)


def chunky_graph(n=24_000, seed=31):
    rng = np.random.default_rng(seed)
    deg = rng.integers(0, 8, size=n)
    deg[0:64] = 300
    deg[200] = 1500
    deg[4096:4096 + 3 * 64] = 12
    deg[8192:8192 + 4 * 64] = 1
    deg[12000:12100] = 0
    src = np.repeat(np.arange(n), deg)
    near = np.clip(src + rng.integers(-400, 401, size=len(src)), 0, n - 1)
    far = rng.integers(0, n, size=len(src))
    dst = np.where(rng.random(len(src)) < 0.8, near, far)
    heavy = (src < 64) | (src == 200)
    dst[heavy] = rng.integers(0, 1000, size=int(heavy.sum()))  # inside the first range
    return W.from_edges(n, src, dst, None, "chunky24k")


@pytest.fixture(scope="module")
def chunky():
    g = chunky_graph()
    og = O.OGraph.of(g)
    Z = O.uniform_Z(g.n)
    ref = O.SyncDI(og, D, Z)
    ref.run(1e-14)
    assert ref.converged
    return g, og, Z, ref.H


CASES = [(th, r, fp32, 0) for th in (0.05, 1.0, 4.0) for r in (1, 6, 12) for fp32 in (False, True)]
CASES += [(th, 6, False, -1) for th in (0.05, 1.0, 4.0)]


@pytest.mark.parametrize("theta,rounds,fp32,cut", CASES)
def test_local_round_paths(gpu, chunky, theta, rounds, fp32, cut):
    g, og, Z, x = chunky
    say("chunky24k theta", theta, "rounds", rounds, "fp32", fp32, "range_cut", cut)
    rel = 1e-6 if fp32 else 1e-9
    with gpu.from_graph(g, d=D, fluid_fp32=fp32, theta=theta, inner_rounds=rounds, range_cut=cut,
                        max_sweeps=20000) as s:
        st = s.diffuse(1e-11)
        assert st["converged"]
        H = s.read(gpu.H)
        F = s.read(gpu.F)
        leak = s.read(gpu.LEAKS)[0]
    err = float(np.abs(H - x).sum())
    say("  %d sweeps, bound %.3e, |H - x|_1 = %.3e" % (st["sweeps"], st["bound"], err))
    assert err <= rel * float(np.abs(x).sum())
    assert err <= st["bound"] * (1 + 1e-7) + 1e-14
    if not fp32:
        assert np.all(F >= 0)
    defect = F.sum() + (1 - D) * H.sum() + D * leak - (1 - D) * Z.sum()
    assert abs(defect) <= (1e-6 if fp32 else 1e-13)
    F0 = O.initial_fluid(D, Z, False)
    if fp32:
        assert O.invariant_residual_l1(og, D, F0, H, F) <= 1e-7 * st["residual"] + 1e-15
    else:
        assert O.invariant_residual(og, D, F0, H, F) <= 1e-15
