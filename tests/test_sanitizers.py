"""The oracle and the input generator under AddressSanitizer and UndefinedBehaviorSanitizer.

Both C sources are rebuilt with -fsanitize=address,undefined and the oracle's own test file
runs against those builds in a child process (the sanitizer runtimes preloaded, as the
interpreter itself is not instrumented); any invalid access or undefined operation ends
that run with an error.  A copy of the oracle with a planted off-by-one read shows that
the sanitizers are live in that set-up.  CPU only.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def build(src, out, extra):
    subprocess.check_call(["gcc", *SAN, *extra, "-fopenmp", "-fPIC", "-shared", "-o", out, src, "-lm"])


def run_oracle_tests(tmp, oracle_lib, webgen_lib, select=None):
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": runtime("libasan.so") + ":" + runtime("libubsan.so"),
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=23",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=24",
        "DI_ORACLE_LIB": oracle_lib,
        "DI_WEBGEN_LIB": webgen_lib,
        "OMP_NUM_THREADS": "2",
    })
    cmd = [sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle.py"), "-q", "-x", "-s", "-m", "not gpu",
           "-p", "no:cacheprovider"]
    if select:
        cmd += ["-k", select]
    return subprocess.run(cmd, cwd=tmp, env=env, capture_output=True, text=True, timeout=600)


@pytest.fixture(scope="module")
def san_libs(tmp_path_factory):
    if not shutil.which("gcc") or not runtime("libasan.so") or not runtime("libubsan.so"):
        pytest.skip("gcc sanitizer runtimes not installed")
    tmp = str(tmp_path_factory.mktemp("san"))
    oracle_flags = ["-std=c11", "-ffp-contract=off", "-fno-fast-math"]
    ol = os.path.join(tmp, "liboracle_san.so")
    wl = os.path.join(tmp, "libwebgen_san.so")
    build(os.path.join(ROOT, "oracle", "di_oracle.c"), ol, oracle_flags)
    build(os.path.join(ROOT, "workloads", "webgen.c"), wl, [])
    return tmp, ol, wl, oracle_flags


def test_oracle_suite_is_clean_under_sanitizers(san_libs):
    tmp, ol, wl, _ = san_libs
    r = run_oracle_tests(tmp, ol, wl)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out
    assert " passed" in out


def test_a_planted_out_of_bounds_read_is_caught(san_libs):
    tmp, _, wl, flags = san_libs
    src = open(os.path.join(ROOT, "oracle", "di_oracle.c")).read()
    good = "int64_t b = out_ptr[j], e = out_ptr[j + 1];"
    assert good in src
    bad_src = os.path.join(tmp, "di_oracle_planted.c")
    with open(bad_src, "w") as f:  # reads one entry past the end of out_ptr for the last row
        f.write(src.replace(good, good + " { volatile int64_t past = out_ptr[j + 2]; (void)past; }"))
    bad = os.path.join(tmp, "liboracle_planted.so")
    build(bad_src, bad, flags)
    r = run_oracle_tests(tmp, bad, wl)
    out = r.stdout + r.stderr
    assert r.returncode != 0 and "heap-buffer-overflow" in out, out[-3000:]
