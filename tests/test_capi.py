"""C ABI: the library loads, exports every entry point declared in include/di.h, and
rejects invalid arguments before touching the device (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "di.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(di_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1501_06350_amd import binding
    return binding.load_library()


def test_header_and_binding_agree():
    from paper_1501_06350_amd import binding
    assert declared_functions() == sorted(binding.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_codes_match_header():
    from paper_1501_06350_amd import binding
    src = open(os.path.join(ROOT, "include", "di.h")).read()
    for name, val in re.findall(r"#define (DI_E\w+|DI_OK) \(?(-?\d+)\)?", src):
        assert getattr(binding, name) == int(val)


def test_read_and_info_keys_match_header():
    from paper_1501_06350_amd import binding
    src = open(os.path.join(ROOT, "include", "di.h")).read()
    found = 0
    for name, val in re.findall(r"#define DI_(\w+) (\d+)\b", src):
        if name.startswith("LOOP_"):
            assert getattr(binding, name) == int(val)
        elif hasattr(binding, name):
            assert getattr(binding, name) == int(val), name
            found += 1
        elif name.startswith("INFO_"):
            raise AssertionError("binding lacks %s" % name)
    assert found >= 28


def _csr(n, ptr, idx, w=None):
    from paper_1501_06350_amd import binding
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    keep = [ptr, idx]
    wp = None
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float32)
        keep.append(w)
        wp = ctypes.c_void_p(w.ctypes.data)
    c = binding.DiCsr(n, len(idx), ctypes.c_void_p(ptr.ctypes.data), ctypes.c_void_p(idx.ctypes.data), wp, 0)
    return c, keep


def _init(lib, csr, d=0.85, Z=None, opts=None):
    from paper_1501_06350_amd import binding
    ctx = ctypes.c_void_p()
    zp = None
    if Z is not None:
        Z = np.ascontiguousarray(Z, dtype=np.float64)
        zp = ctypes.c_void_p(Z.ctypes.data)
    rc = lib.di_init(ctypes.byref(ctx), ctypes.byref(csr), d, zp, ctypes.byref(opts) if opts else None)
    return rc, ctx


@pytest.mark.parametrize("case", [
    "d_zero", "d_one", "bad_first_ptr", "ptr_decreasing", "idx_out_of_range", "idx_negative", "w_zero",
    "w_nan", "Z_negative", "Z_zero_sum", "k_too_big", "range_log2", "theta_negative", "n_zero"])
def test_validation_rejects(lib, case):
    from paper_1501_06350_amd import binding
    n = 4
    ptr, idx, w, d, Z, opts = [0, 1, 2, 3, 4], [1, 2, 3, 0], None, 0.85, None, None
    if case == "d_zero":
        d = 0.0
    elif case == "d_one":
        d = 1.0
    elif case == "bad_first_ptr":
        ptr = [1, 1, 2, 3, 4]
    elif case == "ptr_decreasing":
        ptr, idx = [0, 2, 1, 3, 4], [1, 2, 3, 0]
    elif case == "idx_out_of_range":
        idx = [1, 2, 4, 0]
    elif case == "idx_negative":
        idx = [1, -1, 3, 0]
    elif case == "w_zero":
        w = [1.0, 0.0, 1.0, 1.0]
    elif case == "w_nan":
        w = [1.0, float("nan"), 1.0, 1.0]
    elif case == "Z_negative":
        Z = [0.5, -0.1, 0.3, 0.3]
    elif case == "Z_zero_sum":
        Z = [0.0, 0.0, 0.0, 0.0]
    elif case in ("k_too_big", "range_log2", "theta_negative"):
        opts = binding.DiOpts()
        opts.theta = 1.0
        opts.k = 65 if case == "k_too_big" else 1
        opts.range_log2 = 20 if case == "range_log2" else 0
        if case == "theta_negative":
            opts.theta = -1.0
    csr, keep = _csr(n, ptr, idx, w)
    if case == "n_zero":
        csr.n = 0
    rc, ctx = _init(lib, csr, d, Z, opts)
    assert rc == binding.DI_EINVAL, (case, rc)
    assert ctx.value is None
    assert len(lib.di_last_error()) > 0


@pytest.mark.parametrize("case", ["edge_leaves_graph", "graph_ptr_end", "graph_ptr_flat", "k_with_union",
                                  "union_zero_Z", "union_no_ptr"])
def test_union_validation_rejects(lib, case):
    """A union of graphs (n_graphs > 1) is checked on the host before any device call."""
    from paper_1501_06350_amd import binding
    n = 6
    ptr, idx = [0, 1, 2, 3, 4, 5, 6], [1, 2, 0, 4, 5, 3]  # two 3-cycles
    gp = [0, 3, 6]
    Z = None
    opts = binding.DiOpts()
    opts.theta = 1.0
    opts.k = 1
    if case == "edge_leaves_graph":
        idx = [1, 2, 3, 4, 5, 3]
    elif case == "graph_ptr_end":
        gp = [0, 3, 5]
    elif case == "graph_ptr_flat":
        gp = [0, 3, 3, 6]
    elif case == "k_with_union":
        opts.k = 2
    elif case == "union_zero_Z":
        Z = [0.5, 0.25, 0.25, 0.0, 0.0, 0.0]
    gpa = np.ascontiguousarray(gp, dtype=np.int64)
    opts.n_graphs = len(gp) - 1
    opts.graph_ptr = None if case == "union_no_ptr" else ctypes.c_void_p(gpa.ctypes.data)
    csr, keep = _csr(n, ptr, idx)
    rc, ctx = _init(lib, csr, 0.85, Z, opts)
    assert rc == binding.DI_EINVAL, (case, rc)
    assert ctx.value is None
    assert len(lib.di_last_error()) > 0


def test_null_arguments(lib):
    from paper_1501_06350_amd import binding
    assert lib.di_init(None, None, 0.85, None, None) == binding.DI_EINVAL
    assert lib.di_diffuse(None, 1e-8, None) == binding.DI_EINVAL
    assert lib.di_power(None, 1e-8, None) == binding.DI_EINVAL
    assert lib.di_read(None, 0, None, 0) == binding.DI_EINVAL
    assert lib.di_set_z(None, None) == binding.DI_EINVAL
    assert lib.di_reset(None) == binding.DI_EINVAL
    assert lib.di_adjoint(None, None, 1e-8, None, None, 0, None) == binding.DI_EINVAL
    assert lib.di_info(None, 0, None) == binding.DI_EINVAL
    assert lib.di_save(None, None) == binding.DI_EINVAL
    assert lib.di_load(None, None) == binding.DI_EINVAL
    assert lib.di_destroy(None) == binding.DI_OK


def test_live_allocations_needs_no_context(lib):
    """The process-wide allocation count is the one info key that takes a NULL context
    (and touches no device: nothing has been allocated in this process)."""
    import ctypes
    from paper_1501_06350_amd import binding
    v = ctypes.c_int64(-1)
    assert lib.di_info(None, binding.INFO_LIVE_ALLOCATIONS, ctypes.byref(v)) == binding.DI_OK
    assert v.value == 0
    assert lib.di_info(None, binding.INFO_N, ctypes.byref(v)) == binding.DI_EINVAL
