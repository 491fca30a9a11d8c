"""bench.py's bookkeeping, on the CPU: the lookup of the measured HBM traffic (keyed on the
sources that decide the sweep's traffic and on the sweep options), the roofline fields, and
the refusal of more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_lookup_keyed_on_sources_and_options(tmp_path, monkeypatch):
    prof = tmp_path / "traffic.md"
    prof.write_text("# summary\n\n- source sha256: `abc`\n- options: `%s`\n- traffic bytes per launch: `1.5e+10`\n"
                    % bench.traffic_options(0.2, 0, 6))
    monkeypatch.setattr(bench, "traffic_profile", lambda prec: str(prof))
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: "abc")
    assert bench.measured_traffic("f64", 0.2, 0, 6) == 1.5e10
    assert bench.measured_traffic("f64", 0.3, 0, 6) is None
    assert bench.measured_traffic("f64", 0.2, -1, 6) is None
    assert bench.measured_traffic("f64", 0.2, 0, 4) is None
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: "def")
    assert bench.measured_traffic("f64", 0.2, 0, 6) is None
    monkeypatch.setattr(bench, "traffic_profile", lambda prec: str(tmp_path / "missing.md"))
    assert bench.measured_traffic("f64", 0.2, 0, 6) is None


def test_committed_traffic_profile_is_well_formed():
    vals = {}
    for line in open(bench.traffic_profile("f64")).read().splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    assert len(vals["source sha256"]) == 64
    assert vals["options"].startswith("theta=")
    assert float(vals["traffic bytes per launch"]) > 0


def test_roofline_fields():
    r = bench.roofline(1600.0, traffic=None)
    assert (r["bound"], r["unit"], r["peak"]) == ("hbm", "GB/s", 8000.0)
    assert abs(r["frac"] - 0.2) < 1e-12 and r["traffic"] is None


def test_more_than_one_gpu_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr
