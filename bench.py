#!/usr/bin/env python3
"""Benchmark: D-Iteration vs power iteration to a certified L1 distance of 1e-8 on the
50M-node web-like graph (float fluid, double history and residual), one MI355X.

One step = one D-Iteration solve from F_0 = (1-d) Z to |F|_1 / (1-d) <= 1e-8
(di_reset + di_diffuse).  K power-iteration solves to the same certified tolerance
are timed after the K steps.  Graph generation, upload and the device-side graph
build happen before the timed region; inputs are resident in HBM when it starts.

Prints one JSON line (rank 0).  See DESIGN.md for the byte model behind "roofline".
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
D = 0.85
TOL = 1e-8


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=50_000_000)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--fp64", action="store_true", help="double fluid instead of float")
    ap.add_argument("--no-batched", action="store_true", help="skip the k=64 and 256-graph legs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=4)
    ap.add_argument("--range-log2", type=int, default=0)
    ap.add_argument("--rounds", type=int, default=0)
    ap.add_argument("--theta", type=float, default=1.0)
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for rocprofv3 --pmc runs: a copy of known size, then one DI solve")
    ap.add_argument("--batched-only", action="store_true",
                    help="for profiling: run only the k=64 and 256-graph legs and print their figures")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every box here has a single MI355X, and the multi-GPU "
              "partitioning of the sweep is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_1501_06350_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    fp32 = not args.fp64
    if args.traffic_probe:
        traffic_probe(args, fp32)
        return
    if args.batched_only:
        print(json.dumps({"batched": bench_batched(fp32), "union": bench_union(fp32), "adjoint": bench_adjoint()}),
              flush=True)
        return
    t0 = time.time()
    g = W.webgen(args.n, args.seed)
    log("graph webgen(n=%d, seed=%d): m=%d generated in %.1fs" % (g.n, args.seed, g.m, time.time() - t0))
    t0 = time.time()
    s = B.from_graph(g, d=D, fluid_fp32=fp32, timing=True, range_log2=args.range_log2, inner_rounds=args.rounds,
                     theta=args.theta)
    log("di_init (upload + IN build + block-local split) %.1fs, device bytes %.2f GB" %
        (time.time() - t0, s.info(B.INFO_DEVICE_BYTES) / 1e9))
    n, m = g.n, g.m

    def di_step():
        s.reset()
        return s.diffuse(TOL)

    for _ in range(args.warmup):
        st = di_step()
        log("warmup DI: sweeps=%d ms=%.2f bound=%.3e" % (st["sweeps"], st["ms"], st["bound"]))
    torch.cuda.synchronize()
    stats = []
    kern_ns, kern_launch = 0, 0
    local_pushes = 0
    t_start = time.perf_counter()
    for _ in range(args.steps):
        st = di_step()
        stats.append(st)
        kern_ns += s.info(B.INFO_KERNEL_NS)
        kern_launch += s.info(B.INFO_KERNEL_LAUNCHES)
        local_pushes += s.info(B.INFO_LOCAL_PUSHES)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = 1e3 * wall / args.steps
    edges = sum(x["edge_updates"] for x in stats) / args.steps
    sweeps = sum(x["sweeps"] for x in stats) / args.steps
    diffusions = sum(x["node_updates"] for x in stats) / args.steps
    di_ms = sum(x["ms"] for x in stats) / args.steps
    assert all(x["converged"] for x in stats)
    geups = edges / (ms_per_step * 1e-3) / 1e9
    log("DI: %.2f ms/step (device %.2f ms), sweeps %.1f, edge updates %.3e, rounds %.2f, GEUPS %.1f" %
        (ms_per_step, di_ms, sweeps, edges, edges / m, geups))

    # roofline of the dominant kernel (the block-local sweep)
    T = 4 if fp32 else 8
    m_rem = s.info(B.INFO_M_REMOTE)
    nr = s.info(B.INFO_NRANGES)
    per_sweep = n * 3 * T + m_rem * (6 + T) + nr * 16
    alg_bytes = sweeps * args.steps * per_sweep + diffusions * args.steps * 48 + local_pushes * 2
    avg_ns = kern_ns / max(kern_launch, 1)
    bytes_per_launch = alg_bytes / max(kern_launch, 1)
    achieved = bytes_per_launch / avg_ns  # GB/s (bytes per ns)
    log("block-local sweep kernel: %d launches, avg %.1f us, %.3f GB/launch -> %.0f GB/s" %
        (kern_launch, avg_ns / 1e3, bytes_per_launch / 1e9, achieved))

    # power iteration to the same certified tolerance
    pi = []
    s.power(TOL)  # warm-up (allocates and builds row blocks)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pk_ns, pk_l = 0, 0
    for _ in range(args.steps):
        p = s.power(TOL)
        pi.append(p)
        pk_ns += s.info(B.INFO_KERNEL_NS)
        pk_l += s.info(B.INFO_KERNEL_LAUNCHES)
    torch.cuda.synchronize()
    pi_ms = 1e3 * (time.perf_counter() - t1) / args.steps
    pi_iters = pi[-1]["sweeps"]
    pi_geups = pi_iters * m / (pi_ms * 1e-3) / 1e9
    pi_bytes_iter = m * (4 + T) + n * (8 + 8 + 8 + T + 8)  # idx+gather per edge; ptr,x,x_new,xt,inv_s per node
    pi_achieved = pi_bytes_iter / (pk_ns / max(pk_l, 1))
    xd, xp = s.read(B.H), s.read(B.X_PI)
    di_pi_l1 = float(np.abs(xd - xp).sum())
    used_rb, used_rounds = s.info(B.INFO_RANGE_LOG2), s.info(B.INFO_INNER_ROUNDS)
    log("PI (f32 x/s): %.2f ms/solve, %d iterations, GEUPS %.1f, kernel avg %.1f us -> %.0f GB/s; |x_DI - x_PI|_1 = %.2e" %
        (pi_ms, pi_iters, pi_geups, pk_ns / max(pk_l, 1) / 1e3, pi_achieved, di_pi_l1))
    s.close()
    del xp

    # The certificate of power iteration holds for exact iterates; with x/s rounded to float
    # each iterate carries rounding of the order of the tolerance, so that variant can stop
    # farther than 1e-8 from x (its distance to the certified D-Iteration result gives a
    # lower bound on its error, reported below).  The comparator is power iteration with
    # double x/s, on a double context.
    s64 = B.from_graph(g, d=D, fluid_fp32=False, timing=True)
    s64.power(TOL)  # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p64_ns, p64_l, p64 = 0, 0, None
    for _ in range(args.steps):
        p64 = s64.power(TOL)
        p64_ns += s64.info(B.INFO_KERNEL_NS)
        p64_l += s64.info(B.INFO_KERNEL_LAUNCHES)
    torch.cuda.synchronize()
    pi64_ms = 1e3 * (time.perf_counter() - t1) / args.steps
    pi64_iters = p64["sweeps"]
    pi64_geups = pi64_iters * m / (pi64_ms * 1e-3) / 1e9
    pi64_bytes_iter = m * (4 + 8) + n * (8 + 8 + 8 + 8 + 8)
    pi64_achieved = pi64_bytes_iter / (p64_ns / max(p64_l, 1))
    xp64 = s64.read(B.X_PI)
    di_pi64_l1 = float(np.abs(xd - xp64).sum())
    s64.close()
    del xp64
    log("PI (f64 x/s): %.2f ms/solve, %d iterations, GEUPS %.1f, kernel avg %.1f us -> %.0f GB/s; |x_DI - x_PI|_1 = %.2e" %
        (pi64_ms, pi64_iters, pi64_geups, p64_ns / max(p64_l, 1) / 1e3, pi64_achieved, di_pi64_l1))

    result = {
        "metric": "GEUPS + time-to-L1 1e-8, DI vs power iter, 50M nodes; k=64 batched PPR",
        "value": round(geups, 3),
        "unit": "GEUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": "webgen n=%d m=%d seed=%d, d=0.85, uniform Z, L1 tol 1e-8, %s fluid + f64 history" %
                               (n, m, args.seed, "f32" if fp32 else "f64"),
                   "range_log2": used_rb, "inner_rounds": used_rounds,
                   "theta": args.theta},
        "time_to_tol_ms": {"di": round(ms_per_step, 3), "pi": round(pi64_ms, 3)},
        "di_vs_pi_speedup": round(pi64_ms / ms_per_step, 3),
        "di": {"sweeps": sweeps, "edge_updates": edges, "diffusions": diffusions, "rounds": round(edges / m, 3),
               "device_ms": round(di_ms, 3), "bound": stats[-1]["bound"]},
        "pi": {"x_over_s": "f64", "iterations": pi64_iters, "geups": round(pi64_geups, 3),
               "l1_diff_to_di": di_pi64_l1,
               "roofline": {"bound": "hbm", "achieved": round(pi64_achieved, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(pi64_achieved / HBM_PEAK_GBS, 4)}},
        "pi_f32_gather": {"ms": round(pi_ms, 3), "iterations": pi_iters, "geups": round(pi_geups, 3),
                          "l1_diff_to_di": di_pi_l1,
                          # |x_PI - x|_1 >= |x_PI - x_DI|_1 - |x_DI - x|_1 (D-Iteration's certified bound)
                          "l1_error_at_least": max(0.0, di_pi_l1 - stats[-1]["bound"]),
                          "roofline": {"bound": "hbm", "achieved": round(pi_achieved, 1), "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": round(pi_achieved / HBM_PEAK_GBS, 4)}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": "k_bld2_sweep", "launches": kern_launch, "avg_us": round(avg_ns / 1e3, 2)},
    }
    del xd

    if not args.no_batched:
        for key, fn in (("batched_k64", lambda: bench_batched(fp32)), ("union_256", lambda: bench_union(fp32)),
                        ("adjoint_2m", bench_adjoint)):
            try:
                result[key] = fn()
            except Exception as e:  # reported, not fatal: the headline is the single solve
                result[key] = {"error": str(e)[:300]}
            log("%s: %s" % (key, json.dumps(result[key])))

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(g, args.cpu_sweeps)
    print(json.dumps(result), flush=True)


COPY_BYTES = 1 << 30
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_k_bld2_sweep_webgen50m.md")


def sweep_source_hash():
    import hashlib
    with open(os.path.join(ROOT, "paper_1501_06350_amd", "csrc", "sweep.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the block-local sweep from the committed counter profile,
    or None when the kernel source changed since the counters were taken."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("- "):
            key, val = line[2:].split(":", 1)
            vals[key.strip()] = val.strip().strip("`")
    if vals.get("sweep.hip sha256") != sweep_source_hash():
        return None
    try:
        return float(vals["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def traffic_probe(args, fp32):
    """Three copies of a known size (the counter scale), then one D-Iteration solve on the
    headline graph; run under rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE."""
    import torch
    import workloads as W
    from paper_1501_06350_amd import binding as B
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    g = W.webgen(args.n, args.seed)
    with B.from_graph(g, d=D, fluid_fp32=fp32) as s:
        st = s.diffuse(TOL)
    torch.cuda.synchronize()
    log("traffic probe: copies of %d bytes, then %d sweeps, sweep.hip sha256 %s" %
        (COPY_BYTES, st["sweeps"], sweep_source_hash()))


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, 1e3 * (time.perf_counter() - t)


def bench_batched(fp32):
    """Personalized PageRank, webgen(4M, seed 4), k=64 columns of 16 seeds each, L1 tol 1e-8
    per column: one k=64 tile solve vs 64 single-column solves on the same resident graph
    (di_set_z between them, outside the timed calls)."""
    import numpy as np
    import workloads as W
    from paper_1501_06350_amd import binding as B
    g = W.webgen(4_000_000, 4)
    Z = W.ppr_Z(g.n, 64, 16, 4)
    out = {"workload": "webgen n=%d m=%d seed=4, k=64 x 16 seeds, %s fluid" % (g.n, g.m, "f32" if fp32 else "f64")}
    singles, single_sweeps = 0.0, 0
    with B.from_graph(g, d=D, Z=np.ascontiguousarray(Z[:, 0]), fluid_fp32=fp32) as sc:
        sc.diffuse(TOL)  # warm-up
        for c in range(64):
            sc.set_z(np.ascontiguousarray(Z[:, c]))
            st, ms = _timed(lambda: sc.diffuse(TOL))
            singles += ms
            single_sweeps += st["sweeps"]
    out["single_total_ms"] = round(singles, 3)
    out["single_mean_sweeps"] = round(single_sweeps / 64, 2)
    with B.from_graph(g, d=D, Z=Z, k=64, fluid_fp32=fp32) as sb:
        sb.diffuse(TOL)  # warm-up
        sb.reset()
        st, ms = _timed(lambda: sb.diffuse(TOL))
        assert st["converged"]
    out["batched_ms"] = round(ms, 3)
    out["speedup"] = round(singles / ms, 3)
    out["batched_sweeps"] = st["sweeps"]
    out["edge_column_updates"] = st["edge_updates"]
    out["geups_edge_columns"] = round(st["edge_updates"] / (ms * 1e-3) / 1e9, 3)
    # byte model of the k-column push: per edge x column (4 + 2 k T) / k bytes (the target's
    # index once per row, its fluid entry read and written), per taken row k (2T + 16) (own
    # fluid and history), per sweep a scan of F; over the whole solve (every kernel)
    k, T = 64, (4 if fp32 else 8)
    alg = st["edge_updates"] * (4 + 2 * k * T) / k + st["node_updates"] * k * (2 * T + 16) + \
        st["sweeps"] * g.n * k * T
    ach = alg / (ms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4), "scope": "whole k=64 solve"}
    return out


def bench_union(fp32):
    """256 independent webgen graphs of log-uniform size 1k..200k (seed 4), uniform Z each,
    L1 tol 1e-8 per graph: one union solve vs 256 separate solves (all graphs resident)."""
    import numpy as np
    import workloads as W
    from paper_1501_06350_amd import binding as B
    u, gp = W.multigraph_batch(256, 4)
    out = {"workload": "256 webgen graphs, n=%d m=%d, %s fluid" % (u.n, u.m, "f32" if fp32 else "f64")}
    ctxs = []
    try:
        for q in range(256):
            lo, hi = int(gp[q]), int(gp[q + 1])
            ptr = u.out_ptr[lo:hi + 1] - u.out_ptr[lo]
            idx = u.out_idx[u.out_ptr[lo]:u.out_ptr[hi]] - lo
            s = B.Solver(hi - lo, ptr, idx, None, d=D, fluid_fp32=fp32)
            s.diffuse(TOL)  # warm-up
            s.reset()
            ctxs.append(s)
        sep = 0.0
        for s in ctxs:
            st, ms = _timed(lambda: s.diffuse(TOL))
            sep += ms
    finally:
        for s in ctxs:
            s.close()
    out["separate_total_ms"] = round(sep, 3)
    with B.Solver(u.n, u.out_ptr, u.out_idx, None, d=D, graph_ptr=gp, fluid_fp32=fp32) as su:
        su.diffuse(TOL)
        su.reset()
        st, ms = _timed(lambda: su.diffuse(TOL))
        assert st["converged"]
        done = su.read(B.DONE_SWEEPS)
    out["union_ms"] = round(ms, 3)
    out["speedup"] = round(sep / ms, 3)
    out["union_sweeps"] = st["sweeps"]
    out["graph_sweeps_min_max"] = [int(done.min()), int(done.max())]
    # push byte model: per edge update 4 + 2T, per diffusion 40, per sweep a scan of F
    T = 4 if fp32 else 8
    alg = st["edge_updates"] * (4 + 2 * T) + st["node_updates"] * 40 + st["sweeps"] * u.n * T
    ach = alg / (ms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4), "scope": "whole union solve"}
    return out


def bench_adjoint():
    """Adjoint diffusion and edge gradients on the weighted webgen(2M, seed 5), double
    arithmetic: forward to a certified 1e-11, then di_adjoint for c ~ N(0, 1) to a certified
    L-infinity 1e-11 (timed: the transposed diffusion and the per-edge gradient)."""
    import numpy as np
    import workloads as W
    from paper_1501_06350_amd import binding as B
    g = W.webgen(2_000_000, 5, weighted=True)
    c = W.normal_vector(g.n, 5)
    out = {"workload": "webgen n=%d m=%d seed=5, LogNormal(0,1) weights, c ~ N(0,1), f64" % (g.n, g.m)}
    with B.from_graph(g, d=D) as s:
        s.diffuse(1e-11)
        s.adjoint(c, 1e-11)  # warm-up
        (dZ, dw, st), ms = _timed(lambda: s.adjoint(c, 1e-11))
    out["adjoint_ms"] = round(ms, 3)
    out["sweeps"] = st["sweeps"]
    out["edge_updates"] = st["edge_updates"]
    out["bound_inf"] = st["bound"]
    # byte model: per edge update 4 (index) + 4 (weight) + 16 (double fluid read and write),
    # per diffusion 40, per sweep a scan of F (8 n); the gradient once: per edge 4 + 4 + 8 + 8
    # (index, weight, lambda gather, gradient write), per node 32
    alg = st["edge_updates"] * 24 + st["node_updates"] * 40 + st["sweeps"] * g.n * 8 + g.m * 24 + g.n * 32
    ach = alg / (ms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4), "scope": "whole adjoint call"}
    return out


def cpu_baseline(g, sweeps):
    """The oracle's synchronous sweep on the same graph, a bounded number of sweeps."""
    import oracle as O
    t0 = time.time()
    og = O.OGraph.of(g)
    log("oracle graph build %.1fs" % (time.time() - t0))
    y = O.SyncDI(og, D, O.uniform_Z(g.n), fluid_fp32=True)
    t = time.perf_counter()
    y.run(TOL, max_sweeps=sweeps)
    dt = time.perf_counter() - t
    edges = sum(tr[2] for tr in y.trace)
    return {"value": round(edges / dt / 1e9, 5), "unit": "GEUPS", "cores": 1, "kind": "oracle",
            "sample": "first %d synchronous sweeps of the oracle's D-Iteration (float fluid) on the same "
                      "webgen graph, %.3e edge updates in %.1f s" % (sweeps, edges, dt)}


if __name__ == "__main__":
    main()
