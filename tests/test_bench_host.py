"""Host logic of bench.py (no GPU): which stored oracle records a run is compared with,
and how counter-measured traffic is looked up."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as W  # noqa: E402


def test_stored_records_only_for_the_weak_exact_workload():
    """The stored records are the oracle's weak-coupling, exact-field-step Lambda run: a
    strongly coupled or Cayley run of the same grid is a different model and is not
    compared with them; nor is a shorter run."""
    prob = W.lambda3()
    got = bench.stored_lambda3_records(prob)
    assert got is not None
    recs, stride = got
    assert stride > 0
    assert set(recs) == {r["name"] for r in prob["records"]}
    assert len({len(np.asarray(v)) for v in recs.values()}) == 1
    for key, value in (("coupling", "strong"), ("field_step", "cayley")):
        other = W.lambda3()
        other[key] = value
        assert bench.stored_lambda3_records(other) is None
    short = W.lambda3()
    short["n_steps"] = 1000
    assert bench.stored_lambda3_records(short) is None


def test_traffic_records_match_kernel_workload_and_sources(tmp_path, monkeypatch):
    """A traffic-record line is used only for its own kernel, workload, depth and steps,
    and only while the device sources hash to the recorded value."""
    src = "0123456789abcdef"
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.md").write_text(
        "text\n"
        f"traffic-record: kernel=kA workload=w/nx8 depth=16 steps=100 source={src} bytes_per_launch=1234\n"
        "traffic-record: kernel=kB workload=w/nx8 depth=16 steps=100 source=0000000000000000 bytes_per_launch=99\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: src)
    assert bench.measured_traffic("kA", "w/nx8", 16, 100) == 1234.0
    assert bench.measured_traffic("kA", "w/nx8", 32, 100) is None
    assert bench.measured_traffic("kA", "w/nx16", 16, 100) is None
    assert bench.measured_traffic("kB", "w/nx8", 16, 100) is None  # other sources
