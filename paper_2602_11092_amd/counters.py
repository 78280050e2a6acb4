"""Hardware-counter summary of the library's SLOS kernels from rocprofv3
counter runs (CSV output), one run per counter set:

    python -m paper_2602_11092_amd.counters OUT_TXT "<command>" RUN_DIR [RUN_DIR ...]

For the instance of each kernel family with the most dispatches it averages
every counter per dispatch and derives: VALU instructions per FP32 FMA
instruction, VALU and LDS instructions per CU, the VALU issue share of the
kernel's duration (one wave instruction per clock per CU), the share of wave
time spent waiting, and LDS bank-conflict cycles per LDS-active cycle.
"""
import collections
import csv
import glob
import os
import sys

FAMILIES = {
    "fock_probs (one sample per workgroup)": "fused_fwd_kernel",
    "fock_probs (two samples per workgroup)": "fused_pairs_fwd_kernel",
    "fock_probs_backward": "fused_bwd_kernel",
}
NUM_CU = 256


def load(run_dirs):
    """{kernel name: {counter: mean per dispatch}}, {kernel name: dispatches}."""
    sums = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    for d in run_dirs:
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(path)):
                sums[r["Kernel_Name"]][r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    means, disp = {}, {}
    for k, cs in sums.items():
        means[k] = {c: sum(v.values()) / len(v) for c, v in cs.items()}
        disp[k] = max(len(v) for v in cs.values())
    return means, disp


def derive(c):
    """Derived figures from one kernel's mean counters (missing ones skipped)."""
    out = {}
    if "SQ_INSTS_VALU" in c and c.get("SQ_INSTS_VALU_FMA_F32"):
        out["VALU instructions per FP32 FMA instruction"] = c["SQ_INSTS_VALU"] / c["SQ_INSTS_VALU_FMA_F32"]
    if "SQ_INSTS_VALU" in c:
        out["VALU wave instructions per CU"] = c["SQ_INSTS_VALU"] / NUM_CU
    if "SQ_INSTS_LDS" in c:
        out["LDS wave instructions per CU"] = c["SQ_INSTS_LDS"] / NUM_CU
    if "SQ_INSTS_SALU" in c:
        out["SALU wave instructions per CU"] = c["SQ_INSTS_SALU"] / NUM_CU
    if "SQ_INSTS_VALU" in c and c.get("GRBM_GUI_ACTIVE"):
        # GRBM_GUI_ACTIVE is summed over the 8 XCDs: clocks of the kernel = value / 8
        out["VALU issue share of the kernel's clocks"] = c["SQ_INSTS_VALU"] / NUM_CU / (c["GRBM_GUI_ACTIVE"] / 8)
    if c.get("SQ_WAVE_CYCLES") and "SQ_WAIT_ANY" in c:
        out["share of wave time waiting (any)"] = c["SQ_WAIT_ANY"] / c["SQ_WAVE_CYCLES"]
    if c.get("SQ_WAVE_CYCLES") and "SQ_WAIT_INST_LDS" in c:
        out["share of wave time waiting to issue LDS"] = c["SQ_WAIT_INST_LDS"] / c["SQ_WAVE_CYCLES"]
    if c.get("SQ_LDS_IDX_ACTIVE") and "SQ_LDS_BANK_CONFLICT" in c:
        out["LDS bank-conflict cycles per LDS-active cycle"] = c["SQ_LDS_BANK_CONFLICT"] / c["SQ_LDS_IDX_ACTIVE"]
    return out


def main(out_txt, command, *run_dirs):
    means, disp = load(run_dirs)
    lines = ["Hardware counters of the SLOS kernels, mean per dispatch (rocprofv3 --pmc, one run per counter set)",
             "command: %s" % command, ""]
    for title, frag in FAMILIES.items():
        cands = [k for k in means if frag in k]
        if not cands:
            continue
        k = max(cands, key=lambda n: disp[n])
        lines.append("%s: %s (%d dispatches)" % (title, k[:110], disp[k]))
        for name, v in sorted(means[k].items()):
            lines.append("  %-28s %14.4g" % (name, v))
        for name, v in derive(means[k]).items():
            lines.append("  > %-52s %10.4g" % (name, v))
        lines.append("")
    with open(out_txt, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main(*sys.argv[1:])
