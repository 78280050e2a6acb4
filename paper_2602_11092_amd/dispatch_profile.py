"""Per-dispatch profile of one forward + adjoint of a workload, for the
layered kernels whose per-layer launches differ by orders of magnitude.

    python paper_2602_11092_amd/dispatch_profile.py run WORKLOAD [FWD_BLOCK] [BWD_BLOCK]
        one warm-up pair, then one fock_probs + fock_probs_backward (layered
        variant), dL/dp = the workload's loss weights or ones
    python paper_2602_11092_amd/dispatch_profile.py summarize TRACE_DIR FETCH_DIR OUT_TXT "<command>"
        joins a rocprofv3 --kernel-trace run and a --pmc FETCH_SIZE run of
        `run` dispatch by dispatch (the last fwd + bwd): duration, L2-to-fabric
        bytes (FETCH_SIZE KiB x 2, the copy-probe factor of the traffic
        summaries) and the rate they imply.
"""
import csv
import glob
import os
import sys

FETCH_SCALE = 2.0  # FETCH_SIZE KiB -> bytes factor measured with the copy probe (traffic summaries)


def run(workload, fwd_block=512, bwd_block=256):
    import torch

    import workloads as W
    from paper_2602_11092_amd import _binding as B

    wl = W.make(workload)
    dev = "cuda:0"
    U = torch.from_numpy(wl.U).to(dev) if wl.U is not None else None
    if U is None:
        U = B.mesh_to_unitary(torch.from_numpy(wl.theta).to(dev), torch.from_numpy(wl.x).to(dev), wl.enc_scale)
    n_max = int(wl.occ.sum(1).max())
    batch = B.Batch(B.Plan(wl.m, n_max), wl.occ)
    batch.set_config(B.OP_PROBS, B.VARIANT_LAYERED, fwd_block)
    batch.set_config(B.OP_PROBS_BACKWARD, B.VARIANT_LAYERED, bwd_block)
    p = torch.empty(batch.out_len, device=dev)
    gp = torch.ones(batch.out_len, device=dev)
    gU = torch.empty_like(U)
    for _ in range(2):
        B.fock_probs(batch, U, out=p)
        B.fock_probs_backward(batch, U, gp, out=gU)
    torch.cuda.synchronize()
    print("done", workload, flush=True)


def _rows(d, pattern):
    out = []
    for path in glob.glob(os.path.join(d, "**", pattern), recursive=True):
        out += list(csv.DictReader(open(path)))
    return out


def summarize(trace_dir, fetch_dir, out_txt, command):
    kt = sorted(_rows(trace_dir, "*kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"]))
    kt = [r for r in kt if "slos" in r["Kernel_Name"]]
    fetch = {}
    for r in _rows(fetch_dir, "*counter_collection.csv"):
        if r["Counter_Name"] == "FETCH_SIZE":
            key = int(r["Dispatch_Id"])
            fetch.setdefault(key, [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
    fs = [v for k, v in sorted(fetch.items()) if "slos" in v[0]]
    half = len(kt) // 2  # the second fwd + bwd pair
    kt, fs = kt[half:], fs[len(fs) // 2:]
    lines = ["per-dispatch profile: one layered fock_probs + fock_probs_backward", "command: %s" % command,
             "FETCH_SIZE from a separate --pmc run of the same command, x %.1f (copy-probe factor)" % FETCH_SCALE, "",
             "%-62s %9s %11s %9s" % ("kernel (grid)", "us", "fetch MB", "TB/s")]
    total_us = total_mb = 0.0
    for i, r in enumerate(kt):
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        mb = fs[i][1] * 1024 * FETCH_SCALE / 1e6 if i < len(fs) and fs[i][0] == r["Kernel_Name"] else float("nan")
        name = r["Kernel_Name"].replace("slos::(anonymous namespace)::", "").replace("void ", "")
        name = name.split("(")[0][:44] + " (%s)" % r["Grid_Size_X"]
        lines.append("%-62s %9.1f %11.1f %9.2f" % (name, us, mb, mb / us if us > 0 else 0.0))  # MB/us = TB/s
        total_us += us
        total_mb += mb if mb == mb else 0.0
    lines.append("%-62s %9.1f %11.1f" % ("total", total_us, total_mb))
    text = "\n".join(lines) + "\n"
    with open(out_txt, "w") as f:
        f.write(text)
    print(text, end="")


if __name__ == "__main__":
    # run as a file (python3 .../dispatch_profile.py): the repository root holds the package and workloads.py
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    if sys.argv[1] == "run":
        run(sys.argv[2], *(int(v) for v in sys.argv[3:5]))
    else:
        summarize(*sys.argv[2:6])
