"""CPU checks of bench.py's command line: more than one GPU is refused with
a message (the benchmark measures one GPU), every extension workload name is
one bench.py knows how to run, and a committed traffic figure is reported
only for the sources, workload and configuration it was taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_extension_workloads_are_listed():
    sys.path.insert(0, ROOT)
    import bench
    assert len(set(bench.EXTENSIONS)) == len(bench.EXTENSIONS)
    for name in ("expectations_clements_m20_n5_b512", "threshold_clements_m20_n5_b512",
                 "sample_clements_m20_n5_b512_s1024", "unbunched_haar_m24_n8_b16", "superposition_m6_n3_g1024",
                 "superposition_shared_m8_n4_g4096", "fidelity_m6_n4_b1024"):
        assert name in bench.EXTENSIONS
        assert os.path.exists(os.path.join(ROOT, "profiles", "bench_%s.json" % name))


def test_traffic_figure_applies_only_to_its_sources_workload_and_configuration(tmp_path, monkeypatch):
    import json
    sys.path.insert(0, ROOT)
    import bench
    (tmp_path / "profiles").mkdir()
    with open(tmp_path / "profiles" / "traffic_k.json", "w") as f:
        json.dump({"bytes_per_launch": 5.0, "src_sha256": "abc", "workload": "w", "config": "fused/768"}, f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_sha256", lambda: "abc")
    assert bench.load_traffic("k", "w", "fused/768") == 5.0
    assert bench.load_traffic("k", "w") == 5.0  # no autotuned configuration to match
    assert bench.load_traffic("k", "w", "fused/1024") is None
    assert bench.load_traffic("k", "other", "fused/768") is None
    assert bench.load_traffic("missing", "w") is None
    monkeypatch.setattr(bench, "sources_sha256", lambda: "changed")
    assert bench.load_traffic("k", "w", "fused/768") is None
