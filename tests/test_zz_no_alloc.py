"""di_power_noalloc (power iteration with its vectors in the library's static per-device
scratch array) against di_power on the same context, through the C ABI: the same
iterates bit for bit and the same iteration count, on two calls in a row where the second
runs on a smaller graph (the scratch keeps the first call's contents), with cut-aligned and
plain ranges and with double and float x/s; graphs beyond the scratch are refused."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
D = 0.85


def say(*a):
    print(*a, flush=True)


def run_pair(gpu, g, **kw):
    import torch
    with gpu.from_graph(g, d=D, **kw) as s:
        ref = s.power(1e-11)
        xr = s.read(gpu.X_PI)
        x = torch.full((g.n,), np.nan, dtype=torch.float64, device="cuda")
        st = s.power_noalloc(1e-11, x)
        torch.cuda.synchronize()
        # the context's own result is untouched by the no-allocation call
        np.testing.assert_array_equal(s.read(gpu.X_PI), xr)
        xa = x.cpu().numpy()
    assert st["converged"] and ref["converged"]
    assert st["sweeps"] == ref["sweeps"]
    assert st["residual"] == ref["residual"]
    np.testing.assert_array_equal(xa, xr)
    return st


@pytest.mark.parametrize("kw", [{}, {"range_cut": -1}, {"fluid_fp32": True}, {"deterministic": True}])
def test_noalloc_power_matches_power_two_calls(gpu, kw):
    big = W.webgen(400_000, 8)
    small = W.tiny_zipf(20_000, 5)
    say("noalloc power", kw, "n", big.n, "then", small.n)
    run_pair(gpu, big, **kw)
    run_pair(gpu, small, **kw)


def test_noalloc_power_refuses_graphs_beyond_the_scratch(gpu):
    import torch
    n = 1_100_000  # above the 1,048,544 nodes the scratch holds with double x/s
    g = W.from_edges(n, np.arange(n - 1), np.arange(1, n))
    say("noalloc refusal, n", n)
    with gpu.from_graph(g, d=D, range_cut=-1) as s:
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        with pytest.raises(gpu.DIError) as e:
            s.power_noalloc(1e-8, x)
        assert e.value.code == gpu.DI_EINVAL
        # the context stays usable
        assert s.power(1e-8)["converged"]


def test_noalloc_power_edge_inputs(gpu):
    import torch
    lib = gpu.load_library()
    g = W.tiny_zipf(500, 3)
    with gpu.from_graph(g, d=D, k=2) as s:  # two right-hand sides: refused
        x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        with pytest.raises(gpu.DIError):
            s.power_noalloc(1e-8, x)
    with gpu.from_graph(g, d=D) as s:
        st = gpu.DiStats()
        assert lib.di_power_noalloc(s._ctx, 1e-8, None, ctypes.byref(st)) == gpu.DI_EINVAL
        x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        assert lib.di_power_noalloc(s._ctx, 0.0, ctypes.c_void_p(x.data_ptr()), ctypes.byref(st)) == gpu.DI_EINVAL
    assert lib.di_power_noalloc(None, 1e-8, None, None) == gpu.DI_EINVAL
