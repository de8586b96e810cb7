"""Host checks of bench.py that need no GPU: one GPU only, and the traffic record is read
only for the layout and kernel sources it was measured with."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_matches_layout_and_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    from paper_2211_02435_amd.rocprof_summary import kernel_source_hash
    for storage in ("f32", "f64"):
        rec = os.path.join(ROOT, "profiles", "traffic_d3q27_cumulant_512_%s.json" % storage)
        t = json.load(open(rec))
        if t["kernel_source_sha"] == kernel_source_hash():
            assert bench.measured_traffic("d3q27_cumulant_512", t["layout"], storage) == t["bytes_per_launch"]
        other = "planes" if t["layout"] == "rows" else "rows"
        assert bench.measured_traffic("d3q27_cumulant_512", other, storage) is None
        assert bench.measured_traffic("no_such_workload", t["layout"], storage) is None
    assert bench.measured_traffic("d3q27_cumulant_512", "rows", "f16") is None


def test_traffic_hash_covers_runtime_and_build_flags():
    sys.path.insert(0, ROOT)
    from paper_2211_02435_amd import rocprof_summary as R
    files = R.kernel_sources()
    for needed in ("paper_2211_02435_amd/csrc/lbm_runtime.hip", "paper_2211_02435_amd/csrc/lbm_instantiate.inc",
                   "paper_2211_02435_amd/csrc/k_d3q27_f32.hip", "paper_2211_02435_amd/build.py"):
        assert needed in files


def test_cpu_baseline_record_on_a_tiny_sample():
    """The oracle legs of the CPU baseline (all usable cores, one core, the D2Q9 run) on tiny
    copies: the record carries every field the bench line states."""
    sys.path.insert(0, ROOT)
    import bench
    import lbm_workloads as W
    r = bench.cpu_baseline(W.WORKLOADS["d3q27_cumulant_512"], n_all=8, steps_all=1, n_one=6, steps_one=1,
                           d2q9_steps=2)
    assert r["kind"] == "oracle" and r["unit"] == "MLUPS" and r["value"] > 0
    assert 1 <= r["cores"] <= 16
    assert r["single_core"]["cores"] == 1 and r["single_core"]["value"] > 0
    assert r["d2q9_central_64"]["value"] > 0
    assert r["cpu_model"] and r["nproc"] >= 1 and r["usable_cores"] >= 1
