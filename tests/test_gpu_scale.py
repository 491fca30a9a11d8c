"""Parity at the sizes the bench measures (HIP library through the C ABI, oracle on the CPU).

webgen(1M, 2): the library's D-Iteration and power iteration against the oracle's
synchronous D-Iteration run to a certified 1e-11, element by element (|dx|_1 <= 1e-9 |x|_1
with double arithmetic, <= 1e-6 |x|_1 with float fluid or float x/s).

webgen(50M, 3), the headline configuration (frontier scale 0.2, 6 local rounds, tol
1e-8, double fluid and float fluid): the oracle recomputes, in double, the exact residual F = F_0 + d P H - H of the
history the library returns, over all rows and row by row on a sample, and checks the
certificate |x - H|_1 <= |F|_1 / (1-d) <= tol (Theorem 1) without the library's own residual;
power iteration with double x/s must land within the two certified bounds of it.

k = 64 columns on webgen(4M, 4): the oracle's exact residual of sampled columns certifies them.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
D = 0.85


def say(*a):
    print(*a, flush=True)


def test_webgen_1m_against_oracle(gpu):
    g = W.webgen(1_000_000, 2)
    og = O.OGraph.of(g)
    Z = O.uniform_Z(g.n)
    ref = O.SyncDI(og, D, Z)
    ref.run(1e-11)
    assert ref.converged
    xb = ref.R / (1 - D)  # |x - H_ref|_1 <= xb
    x = ref.H
    xn = float(np.abs(x).sum())
    say("oracle: %d sweeps, bound %.3e" % (ref.sweeps, xb))
    for fp32, tol, rel in ((False, 1e-11, 1e-9), (True, 1e-8, 1e-6)):
        with gpu.from_graph(g, d=D, fluid_fp32=fp32) as s:
            st = s.diffuse(tol)
            assert st["converged"] and st["bound"] <= tol
            H = s.read(gpu.H)
            err = float(np.abs(H - x).sum())
            say("DI fp32=%d: %d sweeps, bound %.3e, |H - x_ref|_1 = %.3e" % (fp32, st["sweeps"], st["bound"], err))
            assert err <= st["bound"] * (1 + 1e-6) + xb + 1e-15 * xn
            assert err <= rel * xn
            # mass balance reported by the library against the oracle's sums of the result
            md = O.mass_defect(og, D, Z, H, s.read(gpu.F), s.read(gpu.LEAKS)[0])
            say("mass defect: library %.3e, oracle %.3e" % (st["mass_defect"], md))
            assert abs(st["mass_defect"]) <= (1e-7 * st["residual"] if fp32 else 0) + 1e-13 * Z.sum()
            assert abs(st["mass_defect"] - md) <= (1e-7 * st["residual"] if fp32 else 0) + 1e-13 * Z.sum()
            p = s.power(tol)
            xp = s.read(gpu.X_PI)
            errp = float(np.abs(xp - x).sum())
            say("PI fp32=%d: %d iterations, |x_PI - x_ref|_1 = %.3e" % (fp32, p["sweeps"], errp))
            assert errp <= rel * xn


def exact_residual_l1(og, F0, H):
    """|F_0 + d P H - H|_1 in double, P applied by the oracle."""
    return float(np.abs(F0 + D * og.P_times(H) - H).sum())


@pytest.fixture(scope="module")
def web50m():
    g = W.webgen(50_000_000, 3)
    return g, O.OGraph.of(g)


@pytest.mark.parametrize("fp32", [False, True])
def test_headline_50m_certificate(gpu, web50m, fp32):
    g, og = web50m
    say("webgen(50M, 3): n=%d m=%d, float fluid %d" % (g.n, g.m, fp32))
    Z = O.uniform_Z(g.n)
    F0 = (1 - D) * Z
    with gpu.from_graph(g, d=D, fluid_fp32=fp32, theta=0.2, inner_rounds=6) as s:
        st = s.diffuse(1e-8)
        assert st["converged"] and st["bound"] <= 1e-8
        H = s.read(gpu.H)
        Fg = s.read(gpu.F)
        lg = s.read(gpu.LEAKS)[0]
    say("DI: %d sweeps, bound %.3e" % (st["sweeps"], st["bound"]))
    # mass balance at the full size: the library's exact device sums against the oracle's
    md = O.mass_defect(og, D, Z, H, Fg, lg)
    say("mass defect: library %.3e, oracle %.3e" % (st["mass_defect"], md))
    slack = 1e-7 * st["residual"] if fp32 else 0.0
    assert abs(st["mass_defect"]) <= slack + 1e-13 * Z.sum()
    assert abs(st["mass_defect"] - md) <= slack + 1e-13 * Z.sum()
    assert np.all(H >= 0)
    # every row: the certificate from the oracle's own residual
    R = exact_residual_l1(og, F0, H)
    say("oracle residual |F|_1 / (1-d) = %.4e" % (R / (1 - D)))
    assert R / (1 - D) <= 1e-8 * (1 + 1e-6)
    # row by row on a sample: the fluid the library returns is that residual.  Float fluid
    # was recomputed from H at the end: the two sides sum a row's terms in different orders
    # (allow the rounding of a sum of in-degree + 2 nonnegative terms), then the result was
    # rounded to float.  Double fluid was never recomputed: it carries the rounding of the
    # pushes it received (far below 1e-11 of the row's terms).
    rows = np.sort(np.random.default_rng(5).choice(g.n, size=4096, replace=False))
    PH = og.P_times_rows(rows, H)
    Fr = F0[rows] + D * PH - H[rows]
    terms = F0[rows] + D * PH + H[rows]
    gap = np.abs(Fg[rows] - Fr)
    if fp32:
        indeg = (og.in_ptr[rows + 1] - og.in_ptr[rows]).astype(np.float64)
        allow = np.abs(Fr) * 2.0 ** -23 + (indeg + 3) * 2.0 ** -52 * terms
    else:
        allow = 1e-11 * terms
    assert np.all(gap <= allow), float(np.max(gap - allow))
    # power iteration with double x/s on the same graph
    with gpu.from_graph(g, d=D, fluid_fp32=False) as s64:
        p = s64.power(1e-8)
        xp = s64.read(gpu.X_PI)
    diff = float(np.abs(xp - H).sum())
    say("PI: %d iterations, |x_PI - H|_1 = %.3e" % (p["sweeps"], diff))
    # |x - x_PI|_1 <= d/(1-d) |x_{k+1} - x_k|_1 <= d tol (the returned iterate is x_{k+1})
    assert diff <= R / (1 - D) * (1 + 1e-6) + D * 1e-8 + 1e-12


def test_tile_k64_columns_certified_by_oracle(gpu):
    g = W.webgen(4_000_000, 4)
    Z = W.ppr_Z(g.n, 64, 16, seed=4)
    with gpu.from_graph(g, d=D, Z=Z, k=64, fluid_fp32=True) as s:
        st = s.diffuse(1e-8)
        assert st["converged"]
        H = s.read(gpu.H)
        F = s.read(gpu.F)
        leaks, res, mds = s.read(gpu.LEAKS), s.read(gpu.RESIDUALS), s.read(gpu.MASS_DEFECTS)
    og = O.OGraph.of(g)
    assert st["mass_defect"] == mds[np.argmax(np.abs(mds))]
    for c in (0, 9, 31, 63):
        R = exact_residual_l1(og, (1 - D) * Z[:, c], H[c])
        say("column %d: oracle residual bound %.4e" % (c, R / (1 - D)))
        assert R / (1 - D) <= 1e-8 * (1 + 1e-6)
        md = O.mass_defect(og, D, Z[:, c], H[c], F[c], leaks[c])
        say("column %d: mass defect library %.3e, oracle %.3e" % (c, mds[c], md))
        assert abs(mds[c]) <= 1e-7 * res[c] + 1e-13
        assert abs(mds[c] - md) <= 1e-7 * res[c] + 1e-13
