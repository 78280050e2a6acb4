"""HBM traffic per launch of the library's kernels from two rocprofv3 counter
runs of the benchmark (one with FETCH_SIZE, one with WRITE_SIZE, both with
the benchmark's --copy-probe), scaled by what the same counters read for the
probe's elementwise kernel of known size (1 GiB read, 1 GiB written).

    python -m paper_2602_11092_amd.traffic FETCH_DB WRITE_DB OUT_DIR WORKLOAD "<command>"

writes OUT_DIR/traffic_<entry point>.json (read by bench.py while the kernel
sources are unchanged and it times the same workload and configuration) and
OUT_DIR/traffic_<entry point>.txt.  Both runs must time the same kernel
instance (give them the same --autotune-cache, written by a plain benchmark
run): counter collection serialises the launches, so an autotuner timing
under it may pick another instance.
"""
import hashlib
import json
import os
import re
import sqlite3
import sys

# C-ABI entry point -> symbol fragments of the kernels it may launch
KERNELS = {
    "fock_probs": ("fused_fwd_kernel", "fused_pairs_fwd_kernel"),
    "fock_probs_backward": ("fused_bwd_kernel",),
    "mesh_to_unitary": ("mesh_apply_kernel", "mesh_apply_shared_kernel"),
    "mesh_to_unitary_backward": ("mesh_bwd_sweep_kernel",),
}
PROBE = "neg_kernel"
PROBE_BYTES = float(1 << 30)


def config_of(symbol):
    """The autotuner's name of a SLOS kernel instance ('variant/block' or
    'fused-pairs/block/tile'), read from its template arguments; None for
    other kernels."""
    mt = re.search(r"(fused_pairs_fwd_kernel|fused_fwd_kernel|fused_bwd_kernel)<(\d+), (\d+)(?:, (\d+))?", symbol)
    if not mt:
        return None
    if mt.group(1) == "fused_pairs_fwd_kernel":
        return "fused-pairs/%s/%s" % (mt.group(2), mt.group(4))
    return "fused/%s" % mt.group(2)


def dominant(counts, frags):
    """(name, (mean KiB, dispatches)) of the instance with the most dispatches
    among the kernels whose names hold one of `frags`, or None."""
    cands = sorted(((k, v) for k, v in counts.items() if any(f in k for f in frags)), key=lambda kv: -kv[1][1])
    return cands[0] if cands else None


def per_dispatch_kib(db, counter):
    """{kernel name: mean counter value per dispatch (KiB)} from a rocpd database."""
    con = sqlite3.connect(db)
    out = {}
    for name, val, n in con.execute(
            "select kernel_name, sum(value), count(distinct dispatch_id) from counters_collection "
            "where counter_name = ? group by kernel_name", (counter,)):
        out[name] = (val / max(n, 1), n)
    return out


def sources_sha256(root):
    h = hashlib.sha256()
    csrc = os.path.join(root, "paper_2602_11092_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def main(fetch_db, write_db, out_dir, workload, command):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fetch = per_dispatch_kib(fetch_db, "FETCH_SIZE")
    write = per_dispatch_kib(write_db, "WRITE_SIZE")
    probe_f = [v for k, v in fetch.items() if PROBE in k]
    probe_w = [v for k, v in write.items() if PROBE in k]
    if not probe_f or not probe_w:
        raise SystemExit("copy probe kernel not found in the counter runs")
    kf = PROBE_BYTES / (probe_f[0][0] * 1024.0)
    kw = PROBE_BYTES / (probe_w[0][0] * 1024.0)
    sha = sources_sha256(root)
    for entry, frags in KERNELS.items():
        # the instance the timed step runs: the one with the most dispatches
        # (the autotuner launches the others a few times each)
        fs, ws = dominant(fetch, frags), dominant(write, frags)
        if not fs or not ws:
            continue
        if fs[0] != ws[0]:
            raise SystemExit("%s: the counter runs timed different instances (%s / %s); give both the same "
                             "--autotune-cache" % (entry, fs[0], ws[0]))
        f_kib, nf = fs[1]
        w_kib, nw = ws[1]
        rd = f_kib * 1024.0 * kf
        wr = w_kib * 1024.0 * kw
        d = {"kernel": fs[0], "config": config_of(fs[0]), "workload": workload, "entry_point": entry, "fetch_kib_raw": f_kib, "write_kib_raw": w_kib,
             "fetch_scale": kf, "write_scale": kw, "read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
             "bytes_per_launch": rd + wr, "dispatches": [nf, nw], "src_sha256": sha, "command": command}
        with open(os.path.join(out_dir, "traffic_%s.json" % entry), "w") as f:
            json.dump(d, f, indent=1)
        with open(os.path.join(out_dir, "traffic_%s.txt" % entry), "w") as f:
            f.write("HBM traffic of %s (%s), per launch, workload %s\n" % (entry, fs[0][:90], workload))
            if d["config"]:
                f.write("configuration: %s\n" % d["config"])
            f.write("command: %s\n" % command)
            f.write("FETCH_SIZE %.1f KiB raw x %.4f (probe calibration) = %.3f MB read\n" % (f_kib, kf, rd / 1e6))
            f.write("WRITE_SIZE %.1f KiB raw x %.4f (probe calibration) = %.3f MB written\n" % (w_kib, kw, wr / 1e6))
            f.write("dispatches averaged: %d (fetch run), %d (write run)\n" % (nf, nw))
        print(entry, "read %.3f MB write %.3f MB per launch" % (rd / 1e6, wr / 1e6))


if __name__ == "__main__":
    main(*sys.argv[1:6])
