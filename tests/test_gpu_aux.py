"""Auxiliary behaviour of the HIP library through the C ABI: the DI_LOG records of a solve
(checked sweep by sweep against the oracle's synchronous sweep in deterministic mode), and
injected device-allocation failures (DI_FAIL_ALLOC_AT) at every allocation of a context's
life: each failing call returns DI_ENOMEM, frees what it had allocated, and a retry of the
same call succeeds with the oracle's result."""
import gc
import json

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
D = 0.85


def say(*a):
    print(*a, flush=True)


def read_log(path):
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]


def test_log_records_every_sweep_of_a_deterministic_solve(gpu, tmp_path, monkeypatch):
    g = W.webgen(20_000, 7)
    og = O.OGraph.of(g)
    tol = 1e-9
    y = O.SyncDI(og, D, O.uniform_Z(g.n))
    y.run(tol)
    path = str(tmp_path / "di.jsonl")
    monkeypatch.setenv("DI_LOG", path)
    with gpu.from_graph(g, d=D, deterministic=True, sweeps_per_sync=1) as s:
        st = s.diffuse(tol)
        s.power(1e-9)
    monkeypatch.delenv("DI_LOG")
    recs = read_log(path)
    sync = [r for r in recs if r["call"] == "diffuse" and r["event"] == "sync"]
    end = [r for r in recs if r["call"] == "diffuse" and r["event"] == "end"]
    say("%d diffuse records, %d oracle sweeps" % (len(sync), len(y.trace)))
    assert len(end) == 1 and end[0]["status"] == 0 and end[0]["converged"] == 1
    assert end[0]["sweeps"] == st["sweeps"] == len(sync) == len(y.trace)
    assert end[0]["edge_updates"] == st["edge_updates"]
    # the oracle's trace holds the residual as each sweep begins; a record, as it ends
    after = [tr[0] for tr in y.trace[1:]] + [y.R]
    nodes = edges = 0
    for t, (r, (_, act, ne), R) in enumerate(zip(sync, y.trace, after)):
        nodes += int(act)
        edges += int(ne)
        assert r["sweep"] == t + 1 and r["sweeps"] == t + 1
        assert r["residual"] == R  # the exact fixed-point residual, printed with 17 digits
        assert r["node_updates"] == nodes and r["edge_updates"] == edges
        assert r["bound"] == R / (1 - D)
        assert r["rounds"] == pytest.approx(nodes / g.n, rel=1e-5)
    assert end[0]["residual"] == y.R
    # power iteration: one record per iteration and the end record
    psync = [r for r in recs if r["call"] == "power" and r["event"] == "sync"]
    pend = [r for r in recs if r["call"] == "power" and r["event"] == "end"]
    assert len(pend) == 1 and pend[0]["converged"] == 1 and len(psync) == pend[0]["sweeps"]
    assert all(a["residual"] >= b["residual"] for a, b in zip(psync, psync[1:]))


def test_log_records_adjoint_and_union(gpu, tmp_path, monkeypatch):
    """The adjoint's records carry its L-infinity bound (the last one meets the tolerance);
    a union of graphs logs its sweeps and its end record like a single graph."""
    path = str(tmp_path / "di.jsonl")
    monkeypatch.setenv("DI_LOG", path)
    g = W.webgen(20_000, 14, weighted=True)
    c = W.normal_vector(g.n, 8)
    with gpu.from_graph(g, d=D, sweeps_per_sync=2) as s:
        s.diffuse(1e-11)
        _, _, sta = s.adjoint(c, 1e-11)
    u, gp = W.union([W.webgen(3000, 21), W.tiny_zipf(700, 22), W.from_edges(1, [], [])])
    with gpu.Solver(u.n, u.out_ptr, u.out_idx, None, d=D, graph_ptr=gp, sweeps_per_sync=1) as su:
        stu = su.diffuse(1e-9)
    monkeypatch.delenv("DI_LOG")
    recs = read_log(path)
    adj = [r for r in recs if r["call"] == "adjoint"]
    aend = [r for r in adj if r["event"] == "end"]
    assert len(aend) == 1 and aend[0]["converged"] == 1 and aend[0]["sweeps"] == sta["sweeps"]
    assert aend[0]["bound"] == sta["bound"] and aend[0]["bound"] <= 1e-11
    asyncs = [r for r in adj if r["event"] == "sync"]
    assert len(asyncs) >= 1 and all(r["call"] == "adjoint" for r in asyncs)
    # the union's records follow the adjoint's end record (a freed context's address may be
    # reused, so the ctx field alone does not tell the two contexts apart)
    after = recs[recs.index(aend[0]) + 1:]
    diff = [r for r in after if r["call"] == "diffuse"]
    uend = diff[-1]
    assert uend["event"] == "end" and uend["converged"] == 1 and uend["sweeps"] == stu["sweeps"]
    usync = [r for r in diff if r["event"] == "sync"]
    assert len(usync) == stu["sweeps"]
    assert all(r["sweeps"] == t + 1 for t, r in enumerate(usync))


def test_log_is_off_when_unset(gpu, tmp_path, monkeypatch):
    monkeypatch.delenv("DI_LOG", raising=False)
    g = W.tiny_zipf(2000, 3)
    with gpu.from_graph(g, d=D) as s:
        s.diffuse(1e-8)
    monkeypatch.setenv("DI_LOG", str(tmp_path / "none" / "x.jsonl"))  # unopenable: never an error
    with gpu.from_graph(g, d=D) as s:
        assert s.diffuse(1e-8)["converged"]


def test_injected_allocation_failures_free_everything(gpu, monkeypatch):
    """Walk k over every device allocation of a context's life (build, diffuse, power,
    adjoint): the k-th fails; the failing call returns DI_ENOMEM, the same call succeeds
    once the injection is off, and closing the context leaves no device allocation of the
    library behind."""
    g = W.webgen(20_000, 14, weighted=True)
    og = O.OGraph.of(g)
    Z = O.uniform_Z(g.n)
    y = O.SyncDI(og, D, Z)
    y.run(1e-13)
    c = W.normal_vector(g.n, 2)
    lam_o, _, _, conv = O.adjoint(og, D, c, tol_inf=1e-14)
    assert conv
    gc.collect()  # contexts other tests left to the collector are closed before the count is taken
    base = gpu.live_allocations()
    failures = {}
    for k in range(1, 1000):
        monkeypatch.setenv("DI_FAIL_ALLOC_AT", str(k))
        try:
            s = gpu.from_graph(g, d=D)
        except gpu.DIError as e:
            assert e.code == gpu.DI_ENOMEM, str(e)
            assert gpu.live_allocations() == base, "k=%d: init left allocations behind" % k
            failures["init"] = failures.get("init", 0) + 1
            continue
        failed = None
        with s:
            calls = [("diffuse", lambda: s.diffuse(1e-10)), ("power", lambda: s.power(1e-10)),
                     ("adjoint", lambda: s.adjoint(c, 1e-11))]
            out = {}
            for name, call in calls:
                try:
                    out[name] = call()
                except gpu.DIError as e:
                    assert e.code == gpu.DI_ENOMEM, "k=%d %s: %s" % (k, name, e)
                    assert failed is None
                    failed = name
                    monkeypatch.delenv("DI_FAIL_ALLOC_AT")
                    out[name] = call()  # the retry allocates what the failed call did not keep
            monkeypatch.delenv("DI_FAIL_ALLOC_AT", raising=False)
            st = out["diffuse"]
            assert st["converged"] and np.abs(s.read(gpu.H) - y.H).sum() <= st["bound"] + 1e-13
            assert out["power"]["converged"]
            assert np.abs(s.read(gpu.X_PI) - y.H).sum() <= 1e-9
            _, _, sta = out["adjoint"]
            assert sta["converged"] and np.abs(s.read(gpu.LAMBDA) - lam_o).max() <= sta["bound"] + 2e-14
        assert gpu.live_allocations() == base, "k=%d: the context's close left allocations behind" % k
        if failed is None:
            break  # k beyond every allocation of the sequence
        failures[failed] = failures.get(failed, 0) + 1
    say("allocations failed per call:", failures)
    assert failures.get("init", 0) > 10 and failures.get("power", 0) > 0 and failures.get("adjoint", 0) > 0
