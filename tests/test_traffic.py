"""CPU test of the HBM-traffic summariser: calibration by the copy probe and
attribution to the kernel instance with the most dispatches."""
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
    traffic.main(str(tmp_path / "f.db"), str(tmp_path / "w.db"), str(tmp_path), "cmd")
    d = json.load(open(tmp_path / "traffic_fock_probs_backward.json"))
    assert d["kernel"] == chosen
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    assert d["read_bytes_per_launch"] == 100.0 * 1024 * 2.0
    assert d["write_bytes_per_launch"] == 10.0 * 1024
    assert d["bytes_per_launch"] == d["read_bytes_per_launch"] + d["write_bytes_per_launch"]
    assert os.path.exists(tmp_path / "traffic_fock_probs_backward.txt")
