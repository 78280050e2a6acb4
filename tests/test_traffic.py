"""CPU test of the HBM-traffic summariser: calibration by the copy probe and
attribution to the kernel instance with the most dispatches (the same one in
both counter runs)."""
import json
import os
import sqlite3

from paper_2602_11092_amd import traffic


def _db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real, dispatch_id int)")
    for name, vals in rows.items():
        for i, v in enumerate(vals):
            con.execute("insert into counters_collection values (?, ?, ?, ?)", (name, counter, v, hash(name) % 1000 * 100 + i))
    con.commit()
    con.close()


def test_calibrated_traffic_of_the_most_dispatched_instance(tmp_path):
    probe = "void at::native::neg_kernel_stub"
    chosen = "void slos::fused_bwd_kernel<768, 12, 20>(int)"
    other = "void slos::fused_bwd_kernel<512, 18, 20>(int)"
    # the probe reads 1 GiB but the counter shows half of it; writes read true
    _db(tmp_path / "f.db", "FETCH_SIZE", {probe: [512 * 1024.0], chosen: [100.0, 100.0, 100.0], other: [7.0]})
    _db(tmp_path / "w.db", "WRITE_SIZE", {probe: [1024 * 1024.0], chosen: [10.0, 10.0, 10.0], other: [9.0]})
    traffic.main(str(tmp_path / "f.db"), str(tmp_path / "w.db"), str(tmp_path), "w1", "cmd")
    d = json.load(open(tmp_path / "traffic_fock_probs_backward.json"))
    assert d["kernel"] == chosen
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    assert d["read_bytes_per_launch"] == 100.0 * 1024 * 2.0
    assert d["write_bytes_per_launch"] == 10.0 * 1024
    assert d["bytes_per_launch"] == d["read_bytes_per_launch"] + d["write_bytes_per_launch"]
    assert os.path.exists(tmp_path / "traffic_fock_probs_backward.txt")
    assert d["config"] == "fused/768" and d["workload"] == "w1"


def test_runs_that_timed_different_instances_are_refused(tmp_path):
    probe = "void at::native::neg_kernel_stub"
    a = "void slos::fused_pairs_fwd_kernel<1024, 1, 2>(int)"
    b = "void slos::fused_pairs_fwd_kernel<1024, 1, 4>(int)"
    _db(tmp_path / "f.db", "FETCH_SIZE", {probe: [1.0], a: [5.0] * 6, b: [6.0] * 40})
    _db(tmp_path / "w.db", "WRITE_SIZE", {probe: [1.0], a: [5.0] * 40, b: [6.0] * 6})
    try:
        traffic.main(str(tmp_path / "f.db"), str(tmp_path / "w.db"), str(tmp_path), "w1", "cmd")
    except SystemExit as e:
        assert "different instances" in str(e)
    else:
        raise AssertionError("mixed instances were accepted")
    assert not os.path.exists(tmp_path / "traffic_fock_probs.json")


def test_configuration_names_from_kernel_symbols():
    assert traffic.config_of("void slos::(anonymous namespace)::fused_pairs_fwd_kernel<1024, 1, 4>(int, x)") == \
        "fused-pairs/1024/4"
    assert traffic.config_of("void slos::(anonymous namespace)::fused_fwd_kernel<512, 0>(int, x)") == "fused/512"
    assert traffic.config_of("void slos::(anonymous namespace)::fused_bwd_kernel<1024, 10, 20, false>(int)") == \
        "fused/1024"
    assert traffic.config_of("slos::(anonymous namespace)::mesh_apply_kernel(int, float const*)") is None
