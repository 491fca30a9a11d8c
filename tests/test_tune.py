"""The autotuner: its cache key on the CPU; the search on the GPU (options that solve to
the tolerance, a cache hit on a second call, di_set_sweep on a live context)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1501_06350_amd import tune

D = 0.85


def test_graph_key_separates_what_decides_the_options():
    g = W.webgen(30_000, 3)
    k0 = tune.graph_key(g, 1, False, D, 1e-8)
    assert k0 == tune.graph_key(g, 1, False, D, 1e-8)
    assert k0 != tune.graph_key(g, 64, False, D, 1e-8)
    assert k0 != tune.graph_key(g, 1, True, D, 1e-8)
    assert k0 != tune.graph_key(g, 1, False, D, 1e-10)
    assert k0 != tune.graph_key(W.webgen(40_000, 3), 1, False, D, 1e-8)
    assert k0 != tune.graph_key(W.tiny_zipf(30_000, 3), 1, False, D, 1e-8)


@pytest.mark.gpu
def test_tuner_single_and_tile(gpu, tmp_path):
    g = W.webgen(30_000, 9)
    path = str(tmp_path / "tune.json")
    t = tune.Tuner(path, repeats=2, finalists=2)
    r = t.tune_single(g, D, 1e-8, thetas=(0.2, 1.0), rounds=(4, 6), range_log2=(8, 9))
    assert not r["cached"] and r["theta"] in (0.2, 1.0) and r["inner_rounds"] in (4, 6) and r["range_log2"] in (8, 9)
    assert r["ms"] > 0
    r2 = tune.Tuner(path).tune_single(g, D, 1e-8)
    assert r2["cached"] and r2["theta"] == r["theta"]
    # the chosen options solve to the tolerance
    og = O.OGraph.of(g)
    y = O.SyncDI(og, D, O.uniform_Z(g.n))
    y.run(1e-14)
    with gpu.from_graph(g, d=D, theta=r["theta"], inner_rounds=r["inner_rounds"], range_log2=r["range_log2"]) as s:
        st = s.diffuse(1e-8)
        assert np.abs(s.read(gpu.H) - y.H).sum() <= st["bound"] + 1e-13
    Z = W.ppr_Z(g.n, 8, 16, seed=2)
    rt = t.tune_tile(g, Z, D, 1e-8, thetas=(0.5, 1.0), rounds=(2, 4))
    assert rt["theta"] in (0.5, 1.0) and rt["inner_rounds"] in (2, 4)


@pytest.mark.gpu
def test_set_sweep_on_a_live_context(gpu):
    g = W.webgen(30_000, 9)
    og = O.OGraph.of(g)
    y = O.SyncDI(og, D, O.uniform_Z(g.n))
    y.run(1e-14)
    with gpu.from_graph(g, d=D, max_sweeps=3) as s:
        s.diffuse(1e-11, allow_noconv=True)
        s.set_options(0.3, 7)
        assert s.info(gpu.INFO_INNER_ROUNDS) == 7
        for _ in range(100):
            st = s.diffuse(1e-11, allow_noconv=True)
            if st["converged"]:
                break
        assert st["converged"]
        assert np.abs(s.read(gpu.H) - y.H).sum() <= 1e-9 * np.abs(y.H).sum()
        with pytest.raises(gpu.DIError):
            s.set_options(-1.0, 4)
        with pytest.raises(gpu.DIError):
            s.set_options(1.0, 65)


@pytest.mark.gpu
def test_tuner_adjoint(gpu, tmp_path):
    g = W.webgen(30_000, 9, weighted=True)
    c = W.normal_vector(g.n, 4)
    path = str(tmp_path / "tune.json")
    key = tune.graph_key(g, 1, False, D, 1e-11)
    og = O.OGraph.of(g)
    lam_o, _, _, conv = O.adjoint(og, D, c, tol_inf=1e-14)
    assert conv
    with gpu.from_graph(g, d=D) as s:
        s.diffuse(1e-11)
        r = tune.Tuner(path, repeats=2, finalists=2).tune_adjoint(s, c, key, 1e-11, thetas=(0.5, 1.0), rounds=(4, 6))
        assert not r["cached"] and r["theta"] in (0.5, 1.0) and r["inner_rounds"] in (4, 6) and r["ms"] > 0
        assert s.info(gpu.INFO_INNER_ROUNDS) == r["inner_rounds"]
        r2 = tune.Tuner(path).tune_adjoint(s, c, key, 1e-11)
        assert r2["cached"] and r2["theta"] == r["theta"] and r2["inner_rounds"] == r["inner_rounds"]
        # the chosen options reach the tolerance
        _, _, st = s.adjoint(c, 1e-11)
        assert st["converged"] and np.abs(s.read(gpu.LAMBDA) - lam_o).max() <= st["bound"] + 2e-14
