#!/usr/bin/env python3
"""Benchmark of the strong-simulation hot path on one MI355X.

One step = mesh -> U (per-sample angle encoding), fused Fock-space forward to
probabilities, fused adjoint to dL/dU, mesh adjoint to dL/dtheta and dL/dx,
for the 512-sample m=20, n=5 workload (Fock dimension 42504, input photons in
modes 0,4,8,12,16).  dL/dp comes from the workload's linear readout and mean
cross-entropy, evaluated once before timing; the readout itself is timed
separately (train_step_ms) since it is ordinary PyTorch, not this path.

Prints ONE JSON line.  Usage:
    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-plain]
"""
import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Fock amplitudes/sec, batched fwd+bwd (m=20,n=5); % of HBM peak; max |Δp|"
HBM_PEAK_GBS = 8000.0
# FP32 FMA on the vector ALUs without packed (dual) FP32 math, which this
# build keeps disabled: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz.
ALU_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="clements_m20_n5_b512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--eager", action="store_true", help="launch the step eagerly instead of replaying a HIP graph")
    ap.add_argument("--autotune-cache", default=None,
                    help="JSON file of autotuner choices to reuse and extend (default: $SLOS_AUTOTUNE_CACHE, else none)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration under rocprofv3 --pmc)")
    return ap.parse_args()


VARIANT_NAMES = {1: "fused", 2: "layered", 3: "fused-pairs"}


def cfg_name(r):
    """'variant/block' (or 'variant/block/tile') of an autotune report entry."""
    s = "%s/%d" % (VARIANT_NAMES[r["variant"]], r["block"])
    return s + ("/%d" % r["tile"] if r.get("tile") else "")


def replay_percentiles(run, stream, n=100):
    """Median, 10th and 90th percentile (ms) of n single replays, each
    bracketed by its own HIP events on the launch stream."""
    import numpy as np
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        run()
        b.record(stream)
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"n": n, "median_ms": round(float(np.median(t)), 5), "p10_ms": round(float(np.percentile(t, 10)), 5),
            "p90_ms": round(float(np.percentile(t, 90)), 5)}


def roofline_of(kernel, avg_ms, flops, nbytes, workload, config=None):
    """Roofline entry of one kernel from its algorithmic flops and HBM bytes
    per launch: the bound is the resource it comes closer to saturating
    (FP32 vector ALUs without packed math, or HBM).  `config` is the
    autotuned configuration that was timed on `workload`, if any."""
    alu = flops / (avg_ms * 1e-3) / 1e12
    hbm = nbytes / (avg_ms * 1e-3) / 1e9
    fa, fh = alu / ALU_PEAK_TFLOPS, hbm / HBM_PEAK_GBS
    r = {"kernel": kernel, "avg_us": round(avg_ms * 1e3, 3), "algorithmic_flop": flops, "algorithmic_bytes": nbytes,
         "alu_tflops": round(alu, 3), "alu_frac": round(fa, 4), "hbm_gbs": round(hbm, 1), "hbm_frac": round(fh, 4)}
    if fa >= fh:
        r.update({"bound": "alu", "achieved": round(alu, 3), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                  "frac": round(fa, 4)})
    else:
        r.update({"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(fh, 4)})
    r["traffic"] = load_traffic(kernel, workload, config)
    return r


def time_region(fn, iters, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(iters):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / iters  # ms


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(the work would shard by samples, with one all-reduce of dL/dtheta). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_2602_11092_amd import _binding as B
    from paper_2602_11092_amd.autotune import autotune

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.workload in EXTENSIONS or re.fullmatch(FIDELITY_NAME, args.workload):
        return bench_extension(args, dev)
    wl = W.make(args.workload)
    if wl.theta is None or not wl.backward or not (wl.n == wl.n.max()).all():
        return bench_other(args, wl, dev)
    m, Bn = wl.m, wl.B
    n = int(wl.n.max())
    N = math.comb(m + n - 1, n)

    # ---- inputs resident in HBM
    theta = torch.from_numpy(wl.theta).to(dev)
    x = torch.from_numpy(wl.x).to(dev)
    Wr = torch.from_numpy(wl.readout_W).to(dev)
    br = torch.from_numpy(wl.readout_b).to(dev)
    labels = torch.from_numpy(wl.labels).to(dev)
    t0 = time.time()
    plan = B.Plan(m, n)
    batch = B.Batch(plan, wl.occ)
    log("plan+batch %.2fs, out_len %d, fwd cfg %s, bwd cfg %s" % (
        time.time() - t0, batch.out_len, batch.get_config(B.OP_PROBS), batch.get_config(B.OP_PROBS_BACKWARD)))

    U = torch.empty(Bn, m, m, dtype=torch.complex64, device=dev)
    p = torch.empty(batch.out_len, dtype=torch.float32, device=dev)
    gU = torch.empty_like(U)
    gt = torch.empty_like(theta)
    gx = torch.empty_like(x)
    mws = B.mesh_workspace(m, Bn, dev)
    B.mesh_to_unitary(theta, x, wl.enc_scale, out=U, ws=mws)
    # kernel variant and workgroup size per op, picked by timing on this batch
    tuned = autotune(batch, U, ops=(B.OP_PROBS, B.OP_PROBS_BACKWARD), warmup=3, iters=10, cache=args.autotune_cache)
    names = VARIANT_NAMES
    tuned_cfg = {op_name: cfg_name(tuned[op])
                 for op, op_name in ((B.OP_PROBS, "fock_probs"), (B.OP_PROBS_BACKWARD, "fock_probs_backward"))}
    log("autotune: %s" % json.dumps({k: [(names[v], b, t, round(us, 1)) for v, b, t, us in tuned[op]["timings"]]
                                      for op, k in ((B.OP_PROBS, "fwd"), (B.OP_PROBS_BACKWARD, "bwd"))}))
    fws = batch.workspace(B.OP_PROBS, dev)
    bws = batch.workspace(B.OP_PROBS_BACKWARD, dev)

    # dL/dp from the readout + cross-entropy of the workload (once)
    B.fock_probs(batch, U, out=p, ws=fws)
    pv = p.detach().clone().view(Bn, N).requires_grad_(True)
    loss = torch.nn.functional.cross_entropy(pv @ Wr.t() + br, labels)
    (gp,) = torch.autograd.grad(loss, pv)
    gp = gp.contiguous().view(-1)
    torch.cuda.synchronize()

    def step():
        B.mesh_to_unitary(theta, x, wl.enc_scale, out=U, ws=mws)
        B.fock_probs(batch, U, out=p, ws=fws)
        B.fock_probs_backward(batch, U, gp, out=gU, ws=bws)
        B.mesh_to_unitary_backward(theta, x, wl.enc_scale, gU, ws=mws, out_theta=gt, out_x=gx)

    step()
    torch.cuda.synchronize()
    if args.eager:
        run = step
    else:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        run = graph.replay
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    # ---- timed region: exactly K steps between two synchronisations
    t_start = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_start) * 1e3
    ms_per_step = e0.elapsed_time(e1) / args.steps
    replays = replay_percentiles(run, stream)
    amps_per_step = Bn * N
    value = amps_per_step / (ms_per_step * 1e-3)
    log("step %.4f ms (wall %.4f ms/step), %.3e amps/s" % (ms_per_step, wall_ms / args.steps, value))

    # ---- per-kernel averages (HIP events on the launch stream)
    kiters = max(20, min(200, args.steps))
    k_fwd = time_region(lambda: B.fock_probs(batch, U, out=p, ws=fws), kiters, stream)
    k_bwd = time_region(lambda: B.fock_probs_backward(batch, U, gp, out=gU, ws=bws), kiters, stream)
    k_mesh = time_region(lambda: B.mesh_to_unitary(theta, x, wl.enc_scale, out=U, ws=mws), kiters, stream)
    k_meshb = time_region(lambda: B.mesh_to_unitary_backward(theta, x, wl.enc_scale, gU, ws=mws, out_theta=gt,
                                                             out_x=gx), kiters, stream)
    kernels_us = {"fock_probs": k_fwd * 1e3, "fock_probs_backward": k_bwd * 1e3,
                  "mesh_to_unitary": k_mesh * 1e3, "mesh_to_unitary_backward": k_meshb * 1e3}
    log("kernels (us): %s" % json.dumps({k: round(v, 2) for k, v in kernels_us.items()}))

    # algorithmic traffic per sample: U in (8 m^2) and p out (4 N) forward;
    # U in, dL/dp in (4 N) and dL/dU out (8 m^2) backward
    u_bytes = 8 * m * m
    fwd_bytes = Bn * (u_bytes + 4 * N)
    bwd_bytes = Bn * (u_bytes + 4 * N + u_bytes)
    step_bytes = fwd_bytes + bwd_bytes + 2 * Bn * (4 * m + u_bytes)  # + mesh in/out
    # complex multiply-adds per sample: forward = every edge of every layer
    # once (n * N); adjoint = recompute layers 1..n-1, recompute the last
    # layer, two per edge in the last layer's pull and the lower pulls
    edges_top = m * math.comb(m + n - 2, n - 1)
    edges_all = n * N
    edges_low = edges_all - edges_top
    cmac_fwd = edges_all
    cmac_bwd = edges_low + edges_top + 2 * edges_top + 2 * edges_low
    flop_bwd = 8.0 * cmac_bwd * Bn
    flop_fwd = 8.0 * cmac_fwd * Bn
    dominant = "fock_probs_backward" if k_bwd >= k_fwd else "fock_probs"
    if dominant == "fock_probs_backward":
        dur, flops, nbytes = k_bwd, flop_bwd, bwd_bytes
    else:
        dur, flops, nbytes = k_fwd, flop_fwd, fwd_bytes
    roofline = roofline_of(dominant, dur, flops, nbytes, args.workload, tuned_cfg.get(dominant))
    hbm_frac_step = step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS

    # ---- readout + cross-entropy + its backward, for the full training step
    def readout_step():
        pv2 = p.view(Bn, N).detach().requires_grad_(True)
        l2 = torch.nn.functional.cross_entropy(pv2 @ Wr.t() + br, labels)
        (g2,) = torch.autograd.grad(l2, pv2)
        gp.copy_(g2.view(-1))
    readout_ms = time_region(readout_step, 20, stream)

    # ---- unbatched per-sample plain path on the same GPU
    plain = None
    if not args.no_plain:
        plain = plain_path(B, wl, theta, x, gp, plan, N, dev, stream, ms_per_step)

    # ---- copy probe for counter calibration: an elementwise kernel of its own
    # name that reads 1 GiB and writes 1 GiB
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()

    # ---- achievable HBM bandwidth on this machine: a STREAM-like elementwise copy
    # (torch.neg, 1 GiB read + 1 GiB written), HIP events over 10 calls
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        torch.neg(src, out=dst)
    copy_ms = time_region(lambda: torch.neg(src, out=dst), 10, stream)
    copy_gbs = 2.0 * (1 << 30) / (copy_ms * 1e-3) / 1e9
    del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        run()  # U, p and dL/dU of one step, for the comparison with the oracle
        torch.cuda.synchronize()
        cpu = cpu_baseline(wl, U, p, gp, gU, N)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Fock amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "batch": Bn, "fock_dim": N,
                   "pass": "mesh fwd + fock_probs + fock_probs_backward + mesh bwd",
                   "launch": "eager" if args.eager else "hip_graph", "autotuned": tuned_cfg},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "replays": replays,
        "hbm_frac_step": round(hbm_frac_step, 4),
        "hbm_copy_gbs": round(copy_gbs, 1),  # achievable: a 1 GiB elementwise copy on this machine
        "hbm_frac_step_of_copy": round(hbm_frac_step * HBM_PEAK_GBS / copy_gbs, 4),
        "kernels_us": {k: round(v, 3) for k, v in kernels_us.items()},
        "train_step_ms": round(ms_per_step + readout_ms, 4),
        "readout_ms": round(readout_ms, 4),
        "plain_path": plain,
        "max_abs_dp": cpu.get("max_abs_dp") if cpu else None,
        "grad_rel_err": cpu.get("grad_rel_err") if cpu else None,
    }
    print(json.dumps(out), flush=True)


def plain_path(B, wl, theta, x, gp, plan, N, dev, stream, ms_batched):
    """Per-sample calls (B = 1, one launch per photon layer, no graph) of the
    same four entry points; returns the time for the whole batch."""
    import numpy as np
    import torch
    m, Bn = wl.m, wl.B
    batch1 = B.Batch(plan, wl.occ[:1])
    batch1.set_config(B.OP_PROBS, B.VARIANT_LAYERED)
    batch1.set_config(B.OP_PROBS_BACKWARD, B.VARIANT_LAYERED)
    fws = batch1.workspace(B.OP_PROBS, dev)
    bws = batch1.workspace(B.OP_PROBS_BACKWARD, dev)
    mws = B.mesh_workspace(m, 1, dev)
    U1 = torch.empty(1, m, m, dtype=torch.complex64, device=dev)
    p1 = torch.empty(N, dtype=torch.float32, device=dev)
    g1 = torch.empty_like(U1)
    gt = torch.zeros_like(theta)
    gt1 = torch.empty_like(theta)
    gx1 = torch.empty(1, m, dtype=torch.float32, device=dev)

    def one(b):
        xb = x[b:b + 1]
        B.mesh_to_unitary(theta, xb, wl.enc_scale, out=U1, ws=mws)
        B.fock_probs(batch1, U1, out=p1, ws=fws)
        B.fock_probs_backward(batch1, U1, gp[b * N:(b + 1) * N], out=g1, ws=bws)
        B.mesh_to_unitary_backward(theta, xb, wl.enc_scale, g1, ws=mws, out_theta=gt1, out_x=gx1)
        gt.add_(gt1)

    for b in range(4):
        one(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(Bn):
        one(b)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    return {"ms_per_step": round(ms, 3), "speedup_of_batched_fused": round(ms / ms_batched, 1),
            "variant": "layered, B=1 per call, eager: about 13 kernel launches per sample, so the factor is "
                       "mostly launch overhead"}


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def omp_threads(n):
    """Sets the OpenMP thread count of the calling thread's next parallel
    regions (the oracle's C code runs in libgomp); False where libgomp
    cannot be loaded."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except (OSError, AttributeError):
        return False


def cpu_baseline(wl, U, p, gp, gU, N):
    """The FP64 oracle (Ryser permanents and minor permanents) timed on the
    host for a bounded sample of the workload's samples; also the largest
    |p_gpu - p| and the relative error of dL/dU over the sampled samples."""
    import numpy as np
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    U64 = U.cpu().numpy().astype(np.complex128)
    pn = p.cpu().numpy()
    gpn = gp.cpu().numpy().astype(np.float64)
    gUn = gU.cpu().numpy().astype(np.complex128)
    worst = 0.0
    gerr = [0.0, 0.0]

    def one(b):
        a = O.amplitudes(U64[b], wl.occ[b])
        g = O.probs_grad(U64[b], wl.occ[b], gpn[b * N:(b + 1) * N])
        gerr[0] += float(np.linalg.norm(gUn[b] - g) ** 2)
        gerr[1] += float(np.linalg.norm(g) ** 2)
        return float(np.abs(np.abs(a) ** 2 - pn[b * N:(b + 1) * N]).max())

    O.build(force=False)
    t0 = time.perf_counter()
    worst = max(worst, one(0))
    t1 = time.perf_counter() - t0
    S = int(max(1, min(wl.B - 1, 20.0 / max(t1, 1e-3))))  # about 15-20 s of CPU work
    t0 = time.perf_counter()
    for b in range(1, 1 + S):
        worst = max(worst, one(b))
    dt = time.perf_counter() - t0
    # the same work for one more sample on one thread
    single = None
    b1 = min(S + 1, wl.B - 1)
    if omp_threads(1):
        try:
            t0 = time.perf_counter()
            O.amplitudes(U64[b1], wl.occ[b1])
            O.probs_grad(U64[b1], wl.occ[b1], gpn[b1 * N:(b1 + 1) * N])
            single = N / (time.perf_counter() - t0)
        finally:
            omp_threads(threads)
    return {"value": S * N / dt, "unit": "Fock amplitudes/s", "cores": threads, "kind": "oracle",
            "sample": "%d of %d samples, forward amplitudes + minor-permanent gradient, FP64 Ryser, OpenMP" % (
                S, wl.B),
            "seconds": round(dt, 2), "cpu_model": cpu_model(), "single_thread_value": single,
            "max_abs_dp": worst, "grad_rel_err": math.sqrt(gerr[0] / max(gerr[1], 1e-300)),
            "grad_samples": S + 1}


def bench_other(args, wl, dev):
    """The metric's other configurations, each as a line of its own: m=6 n=3
    B=64 and m=16 n=6 B=256 (Haar unitaries, forward), m=12 Clements mesh
    with n in 2..6 mixed in one batch of 4096 (mesh + forward), m=24 n=8 B=16
    (Haar, forward + adjoint of L = sum_b sum_t w_t p_bt, layers recomputed).
    One step is [mesh forward] + fock_probs [+ fock_probs_backward], replayed
    as a HIP graph.  The line carries the headline's fields: roofline of the
    dominant kernel, the oracle timed beside it, max |dp|, the gradient error
    where there is an adjoint, replay percentiles and device memory."""
    import numpy as np
    import torch

    from paper_2602_11092_amd import _binding as B
    from paper_2602_11092_amd.autotune import autotune

    stream = torch.cuda.current_stream()
    m, Bn = wl.m, wl.B
    torch.cuda.reset_peak_memory_stats()
    plan = B.Plan(m, int(wl.n.max()))
    batch = B.Batch(plan, wl.occ)
    if wl.U is not None:
        U = torch.from_numpy(wl.U).to(dev)
        theta = x = mws = None
    else:
        theta = torch.from_numpy(wl.theta).to(dev)
        x = torch.from_numpy(wl.x).to(dev)
        U = torch.empty(Bn, m, m, dtype=torch.complex64, device=dev)
        mws = B.mesh_workspace(m, Bn, dev)
        B.mesh_to_unitary(theta, x, wl.enc_scale, out=U, ws=mws)
    ops = (B.OP_PROBS, B.OP_PROBS_BACKWARD) if wl.backward else (B.OP_PROBS,)
    tuned = autotune(batch, U, ops=ops, warmup=1, iters=2, cache=args.autotune_cache)
    p = torch.empty(batch.out_len, dtype=torch.float32, device=dev)
    gU = torch.empty_like(U)
    fws = batch.workspace(B.OP_PROBS, dev)
    bws = batch.workspace(B.OP_PROBS_BACKWARD, dev) if wl.backward else None
    gp = None
    if wl.backward:  # L = sum_b sum_t w_t p_bt: dL/dp = w for every sample
        gp = torch.from_numpy(np.tile(wl.loss_w, Bn)).to(dev)

    def step():
        if theta is not None:
            B.mesh_to_unitary(theta, x, wl.enc_scale, out=U, ws=mws)
        B.fock_probs(batch, U, out=p, ws=fws)
        if wl.backward:
            B.fock_probs_backward(batch, U, gp, out=gU, ws=bws)

    step()
    torch.cuda.synchronize()
    if args.eager:
        run = step
    else:
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        run = graph.replay
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(args.steps):
        run()
    b.record(stream)
    b.synchronize()
    ms = a.elapsed_time(b) / args.steps
    replays = replay_percentiles(run, stream)
    free, total = torch.cuda.mem_get_info(dev)
    memory = {"torch_peak_gb": round(torch.cuda.max_memory_allocated(dev) / 1e9, 3),
              "device_used_gb": round((total - free) / 1e9, 3)}
    amps = int(batch.out_len)
    log("%s: step %.4f ms, %.3e amps/s" % (wl.name, ms, amps / (ms * 1e-3)))

    # per-kernel times and the dominant kernel's roofline (algorithmic work:
    # n_b * N_b complex MACs per forward sample, three times that per adjoint
    # sample with recomputation; U in and p out, plus dL/dp in and dL/dU out)
    kiters = max(10, min(100, args.steps))
    kernels = {"fock_probs": time_region(lambda: B.fock_probs(batch, U, out=p, ws=fws), kiters, stream)}
    if wl.backward:
        kernels["fock_probs_backward"] = time_region(lambda: B.fock_probs_backward(batch, U, gp, out=gU, ws=bws),
                                                     kiters, stream)
    if theta is not None:
        kernels["mesh_to_unitary"] = time_region(lambda: B.mesh_to_unitary(theta, x, wl.enc_scale, out=U, ws=mws),
                                                 kiters, stream)
    edges = float(sum(int(n) * math.comb(m + int(n) - 1, int(n)) for n in wl.n))
    u_bytes = 8 * m * m * Bn
    work = {"fock_probs": (8.0 * edges, u_bytes + 4 * amps),
            "fock_probs_backward": (8.0 * 3 * edges, 2 * u_bytes + 4 * amps)}
    dominant = max((k for k in kernels if k in work), key=lambda k: kernels[k])
    dom_op = {"fock_probs": B.OP_PROBS, "fock_probs_backward": B.OP_PROBS_BACKWARD}[dominant]
    roofline = roofline_of(dominant, kernels[dominant], *work[dominant], args.workload,
                           config=cfg_name(tuned[dom_op]) if dom_op in tuned else None)
    torch.cuda.synchronize()
    cpu = None if args.no_cpu_baseline else cpu_baseline_other(wl, U, p, gU, gp)
    out = {"metric": "Fock amplitudes/sec, batched %s (%s)" % ("fwd+bwd" if wl.backward else "fwd", wl.name),
           "value": amps / (ms * 1e-3), "unit": "Fock amplitudes/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "c64", "data": "synthetic",
           "config": {"workload": wl.name, "m": m, "n": sorted(set(int(v) for v in wl.n)), "batch": Bn,
                      "outputs_per_step": amps, "launch": "eager" if args.eager else "hip_graph",
                      "pass": ("mesh fwd + " if theta is not None else "") + "fock_probs" +
                              (" + fock_probs_backward" if wl.backward else ""),
                      "autotuned": {str(op): cfg_name(t) for op, t in tuned.items()}},
           "roofline": roofline, "cpu_baseline": cpu, "replays": replays, "memory": memory,
           "kernels_us": {k: round(v * 1e3, 3) for k, v in kernels.items()},
           "max_abs_dp": cpu.get("max_abs_dp") if cpu else None,
           "grad_rel_err": cpu.get("grad_rel_err") if cpu else None}
    print(json.dumps(out), flush=True)


def cpu_baseline_other(wl, U, p, gU, gp):
    """The FP64 oracle beside the GPU for the other configurations, on a
    bounded sample: every output of as many samples as about 12 s allow, or
    for the m=24, n=8 workload 300 seeded outputs per sample (its samples have
    7.9 million outputs each).  Where there is an adjoint: the relative error
    of <dL/dU, V> against FP64 central differences (h = 1e-6) of the oracle
    loss, for two directions V on one output mode's row of sample 0 each (the
    outputs with t_j = 0 do not change along such a V and drop out)."""
    import numpy as np
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    O.build(force=False)
    U64 = U.cpu().numpy().astype(np.complex128)
    pn = p.cpu().numpy()
    off = np.concatenate([[0], np.cumsum([math.comb(wl.m + int(n) - 1, int(n)) for n in wl.n])])
    rng = np.random.default_rng(31)
    worst, done, units = 0.0, 0, 0
    t0 = time.perf_counter()
    big = off[1] - off[0] > 1_000_000
    while done < wl.B and time.perf_counter() - t0 < 12.0:
        b = done
        n = int(wl.n[b])
        if big:
            ranks = np.unique(rng.integers(0, off[b + 1] - off[b], 300))
            outs = np.stack([O.fock_unrank(wl.m, n, int(r)) for r in ranks])
            ref = O.probabilities(U64[b], wl.occ[b], outputs=outs)
            got = pn[off[b] + ranks]
        else:
            ref = O.probabilities(U64[b], wl.occ[b])
            got = pn[off[b]:off[b + 1]]
        worst = max(worst, float(np.abs(got - ref).max()))
        units += ref.size
        done += 1
    dt = time.perf_counter() - t0
    res = {"value": units / dt, "unit": "Fock amplitudes/s", "cores": threads, "cpu_model": cpu_model(),
           "kind": "oracle",
           "sample": ("%d of %d samples, 300 seeded outputs each" if big else "%d of %d samples, every output") % (
               done, wl.B) + ", FP64 Ryser, OpenMP", "seconds": round(dt, 2), "max_abs_dp": worst}
    if gp is not None:
        w = wl.loss_w.astype(np.float64)
        basis = O.fock_basis(wl.m, int(wl.n[0]))
        G = gU.cpu().numpy().astype(np.complex128)
        got, fd = [], []
        h = 1e-6
        for j in (3, 17):
            V = np.zeros((wl.m, wl.m), np.complex128)
            V[j, :] = rng.standard_normal(wl.m) + 1j * rng.standard_normal(wl.m)
            sel = basis[:, j] >= 1
            Lp = float(w[sel] @ O.probabilities(U64[0] + h * V, wl.occ[0], basis[sel]))
            Lm = float(w[sel] @ O.probabilities(U64[0] - h * V, wl.occ[0], basis[sel]))
            fd.append((Lp - Lm) / (2 * h))
            got.append(float(np.real(np.sum(np.conj(G[0]) * V))))
        res["grad_rel_err"] = float(np.linalg.norm(np.array(got) - fd) / np.linalg.norm(fd))
        res["grad_check"] = "sample 0, two row directions, FP64 central differences of the oracle loss"
    return res


# Workloads of the measurement, encoding and kernel extensions (one line each).
EXTENSIONS = ("expectations_clements_m20_n5_b512", "threshold_clements_m20_n5_b512",
              "sample_clements_m20_n5_b512_s1024", "unbunched_haar_m24_n8_b16", "unbunched_train_clements_m20_n5_b512",
              "superposition_m6_n3_g1024", "superposition_shared_m8_n4_g4096", "fidelity_m6_n4_b1024")
# fidelity kernels of other shapes: fidelity_m<modes>_n<photons>_b<Gram size>, photons in the first n modes
FIDELITY_NAME = r"fidelity_m(\d+)_n(\d+)_b(\d+)"
FP32_MFMA_PEAK = 157.3  # TFLOP/s, MI355X dense FP32 matrix-core rate
FP64_PEAK = 78.6  # TFLOP/s, MI355X vector FP64 (equal to its unpacked FP32 rate)


def slos_fwd_flop(m, n, flags=0, B=None):
    """Algorithmic flops of one forward: sum_k k N_k complex MACs (8 flops)."""
    from paper_2602_11092_amd import _binding as Bd
    return 8.0 * sum(k * Bd.slos_space_dim(m, k, flags) for k in range(1, n + 1))


def bench_extension(args, dev):
    """One line per extension workload: HIP-event time of its entry point on
    the launch stream, an ALU roofline from its algorithmic flops, and the
    FP64 oracle timed on a bounded sample beside it."""
    import numpy as np
    import torch

    import workloads as W
    from oracle import oracle as O
    from paper_2602_11092_amd import _binding as B

    name = args.workload
    stream = torch.cuda.current_stream()
    oracle_units = None  # units of `unit` one oracle call covers (default: one sample's share)
    rng = np.random.default_rng(2602)
    cpu_budget = 0.0 if args.no_cpu_baseline else 8.0  # seconds of oracle work
    if name.endswith("clements_m20_n5_b512") or name.startswith("sample_clements"):
        wl = W.make("clements_m20_n5_b512")
        m, n, Bn, occ = 20, 5, wl.B, wl.occ
        U64 = O.encoded_unitaries(wl.theta.astype(np.float64), wl.x.astype(np.float64), wl.enc_scale)
    elif name == "unbunched_haar_m24_n8_b16":
        wl = W.make("haar_m24_n8_b16")
        m, n, Bn, occ = 24, 8, wl.B, wl.occ
        U64 = wl.U.astype(np.complex128)
    elif name == "superposition_shared_m8_n4_g4096":
        m, n, Bn = 8, 4, 4096
        U64 = W.haar_unitaries(rng, 1, m)
        occ = None
    elif name == "superposition_m6_n3_g1024":
        m, n, Bn = 6, 3, 1024
        basis = O.fock_basis(m, n)
        occ = np.tile(basis, (Bn, 1)).astype(np.int32)
        U64 = W.haar_unitaries(rng, Bn, m)
    else:  # fidelity_m<m>_n<n>_b<B> (fidelity_m6_n4_b1024: the paper's kernel example shape)
        m, n, Bn = (int(v) for v in re.fullmatch(FIDELITY_NAME, name).groups())
        occ = np.zeros(m, dtype=np.int32)
        occ[:n] = 1
        U64 = W.haar_unitaries(rng, Bn, m)
    U = torch.from_numpy(U64.astype(np.complex64)).to(dev)
    Uh = U.cpu().numpy().astype(np.complex128)

    if name.startswith("expectations"):
        batch = B.Batch(B.Plan(m, n), occ)
        out = torch.empty((Bn, m), dtype=torch.float32, device=dev)
        ws = batch.workspace(B.OP_MODE_EXPECTATIONS, dev)
        step = lambda: B.fock_mode_expectations(batch, U, out=out, ws=ws)
        work, unit = Bn * math.comb(m + n - 1, n), "Fock states/s"
        flop = Bn * slos_fwd_flop(m, n)
        oracle_one = lambda b: O.mode_expectations(Uh[b], occ[b])
        check = lambda b, r: float(np.abs(out[b].cpu().numpy() - r).max())
        cfg = "fused last-layer epilogue, p never written"
    elif name.startswith("threshold"):
        batch = B.Batch(B.Plan(m, n, threshold=True), occ)
        out = torch.empty(batch.threshold_len, dtype=torch.float32, device=dev)
        ws = batch.workspace(B.OP_THRESHOLD_PROBS, dev)
        step = lambda: B.fock_threshold_probs(batch, U, out=out, ws=ws)
        work, unit = Bn * math.comb(m + n - 1, n), "Fock states/s"
        flop = Bn * slos_fwd_flop(m, n)
        oracle_one = lambda b: O.threshold_probs(Uh[b], occ[b])
        toff = batch.threshold_offsets
        check = lambda b, r: float(np.abs(out[toff[b]:toff[b + 1]].cpu().numpy() - r).max())
        cfg = ("fused forward summing whole click patterns in LDS (p never written)"
               if batch.get_config(B.OP_THRESHOLD_PROBS)[0] == B.VARIANT_FUSED
               else "probabilities, then per-pattern gather")
    elif name.startswith("sample"):
        S = 1024
        batch = B.Batch(B.Plan(m, n), occ)
        u = torch.from_numpy(rng.random((Bn, S)).astype(np.float32)).to(dev)
        out = torch.empty((Bn, S), dtype=torch.int32, device=dev)
        ws = batch.workspace(B.OP_SAMPLE, dev)
        step = lambda: B.fock_sample(batch, U, u, out=out, ws=ws)
        work, unit = Bn * S, "shots/s"
        flop = Bn * slos_fwd_flop(m, n)
        uh = u.cpu().numpy().astype(np.float64)
        oracle_one = lambda b: O.sample_shots(Uh[b], occ[b], uh[b])
        check = lambda b, r: float(np.mean(out[b].cpu().numpy() != r))  # fraction differing (boundary ties)
        cfg = "probabilities, FP64 cumulative sums, binary search; 1024 shots per sample"
    elif name.startswith("unbunched_train"):
        # forward + adjoint on the unbunched space (the fused adjoint's restricted instances)
        batch = B.Batch(B.Plan(m, n, unbunched=True), occ)
        out = torch.empty(batch.out_len, dtype=torch.float32, device=dev)
        gp = torch.from_numpy(rng.standard_normal(batch.out_len).astype(np.float32)).to(dev)
        gU = torch.empty_like(U)
        ws_f, ws_b = batch.workspace(B.OP_PROBS, dev), batch.workspace(B.OP_PROBS_BACKWARD, dev)

        def step():
            B.fock_probs(batch, U, out=out, ws=ws_f)
            B.fock_probs_backward(batch, U, gp, out=gU, ws=ws_b)
        work, unit = batch.out_len, "Fock amplitudes/s"
        flop = 4 * Bn * slos_fwd_flop(m, n, B.PLAN_UNBUNCHED)  # forward + the adjoint's three products
        outs = np.zeros((math.comb(m, n), m), dtype=np.int32)
        for r, c in enumerate(__import__("itertools").combinations(range(m), n)):
            outs[r, list(c)] = 1
        gph = gp.cpu().numpy().astype(np.float64)
        N = len(outs)
        oracle_one = lambda b: O.probs_grad(Uh[b], occ[b], gph[b * N:(b + 1) * N], outputs=outs)
        check = lambda b, r: float(np.abs(gU[b].cpu().numpy() - r).max() / np.abs(r).max())
        cfg = "unbunched space, probabilities + adjoint (%s/%s); error: max relative gradient error" % tuple(
            {B.VARIANT_FUSED: "fused", B.VARIANT_LAYERED: "layered"}.get(batch.get_config(op)[0], "?")
            for op in (B.OP_PROBS, B.OP_PROBS_BACKWARD))
    elif name.startswith("unbunched"):
        batch = B.Batch(B.Plan(m, n, unbunched=True), occ)
        out = torch.empty(batch.out_len, dtype=torch.float32, device=dev)
        ws = batch.workspace(B.OP_PROBS, dev)
        step = lambda: B.fock_probs(batch, U, out=out, ws=ws)
        work, unit = batch.out_len, "Fock amplitudes/s"
        flop = Bn * slos_fwd_flop(m, n, B.PLAN_UNBUNCHED)
        outs = np.zeros((math.comb(m, n), m), dtype=np.int32)
        for r, c in enumerate(__import__("itertools").combinations(range(m), n)):
            outs[r, list(c)] = 1
        pick = rng.integers(0, len(outs), 64)
        N = len(outs)
        oracle_one = lambda b: O.probabilities(Uh[b], occ[b], outs[pick])
        check = lambda b, r: float(np.abs(out[b * N + pick].cpu().numpy() - r).max())
        cfg = "unbunched space, probabilities (oracle on 64 sampled outputs per sample)"
        oracle_units = 64
    elif name.startswith("superposition_shared"):
        ss = B.SharedSuperposition(B.Plan(m, n), n)
        N = ss.N
        Uone = U[0].contiguous()
        X = torch.from_numpy(((rng.standard_normal((Bn, N)) + 1j * rng.standard_normal((Bn, N))) / np.sqrt(2 * N))
                             .astype(np.complex64)).to(dev)
        out = torch.empty((Bn, N), dtype=torch.complex64, device=dev)
        step = lambda: B.fock_shared_superposition_amplitudes(ss, Uone, X, out=out)
        work, unit = Bn * N, "output amplitudes/s"
        gemm_flop = 8.0 * Bn * N * N
        flop = gemm_flop + N * slos_fwd_flop(m, n)
        basis = O.fock_basis(m, n)
        A_ref = {}

        def oracle_one(b):
            if "A" not in A_ref:  # Uhat's rows, built once like the kernel's
                A_ref["A"] = np.stack([O.amplitudes(Uh[0], basis[c]) for c in range(N)])
            return X[b].cpu().numpy().astype(np.complex128) @ A_ref["A"]
        check = lambda b, r: float(np.abs(out[b].cpu().numpy() - r).max())
        cfg = "one U for every input: Uhat built by %d SLOS runs, then one complex GEMM (rocBLAS cgemm)" % N
    elif name.startswith("superposition"):
        N = math.comb(m + n - 1, n)
        batch = B.Batch(B.Plan(m, n), occ)
        sup = B.Superposition(batch, np.arange(Bn + 1) * N)
        Ug = U
        x = torch.from_numpy((rng.standard_normal(Bn * N) + 1j * rng.standard_normal(Bn * N)).astype(np.complex64)).to(dev)
        out = torch.empty(sup.out_len, dtype=torch.complex64, device=dev)
        ws = sup.workspace(False, dev)
        step = lambda: B.fock_superposition_amplitudes(sup, Ug, x, out=out, ws=ws)
        work, unit = Bn * N, "output amplitudes/s"
        flop = Bn * N * (slos_fwd_flop(m, n) + 8.0 * N)  # one SLOS per component + the weighted combine
        xh = x.cpu().numpy().astype(np.complex128)
        oracle_one = lambda b: O.superposition_amplitudes(Uh[b], occ[b * N:(b + 1) * N], xh[b * N:(b + 1) * N])
        check = lambda b, r: float(np.abs(out[b * N:(b + 1) * N].cpu().numpy() - r).max())
        cfg = "dense inputs: every basis state a component; one SLOS per component + combine"
    else:
        out = torch.empty((Bn, Bn), dtype=torch.float32, device=dev)
        step = lambda: B.fock_fidelity_kernel(occ, U, out=out)
        work, unit = Bn * Bn, "kernel entries/s"
        flop = Bn * Bn * (8.0 * n * n * m + (2 ** n) * (2 * n + 6 * (n - 1)))
        oracle_one = lambda b: np.array([O.fidelity(Uh[b], Uh[c], occ) for c in range(32)])
        check = lambda b, r: float(np.abs(out[b, :32].cpu().numpy() - r).max())
        cfg = "thread per pair, FP64 Ryser with unrolled Gray code (oracle: 32 entries per sampled row)"
        oracle_units = 32

    for _ in range(args.warmup):
        step()
    ms = time_region(step, args.steps, stream)
    achieved = flop / (ms * 1e-3) / 1e12
    line = {"metric": "%s throughput (%s)" % (name.split("_")[0], name), "value": work / (ms * 1e-3), "unit": unit,
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64" if name.startswith("fidelity") else "c64",
            "data": "synthetic", "config": {"workload": name, "m": m, "n": n, "batch": Bn, "path": cfg,
                                            "launch": "eager"},
            "roofline": ({"bound": "mfma", "achieved": round(achieved, 3), "peak": FP32_MFMA_PEAK, "unit": "TFLOP/s",
                          "frac": round(achieved / FP32_MFMA_PEAK, 4), "traffic": None, "algorithmic_flop": flop}
                         if name.startswith("superposition_shared") else
                         {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK, "unit": "TFLOP/s",
                          "frac": round(achieved / FP64_PEAK, 4), "traffic": None,
                          "algorithmic_flop": flop}),
            "cpu_baseline": None}
    if cpu_budget > 0:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        torch.cuda.synchronize()
        O.build(force=False)
        t0 = time.perf_counter()
        done, worst = 0, 0.0
        while done < Bn and time.perf_counter() - t0 < cpu_budget:
            worst = max(worst, check(done, oracle_one(done)))
            done += 1
        dt = time.perf_counter() - t0
        per = oracle_units or work / Bn
        line["cpu_baseline"] = {"value": done * per / dt, "unit": unit, "cores": threads, "cpu_model": cpu_model(),
                                "kind": "oracle",
                                "sample": "%d of %d samples (rows), %d %s each" % (done, Bn, per, unit.split("/")[0]),
                                "seconds": round(dt, 2),
                                "max_diff_vs_gpu": worst}
    print(json.dumps(line), flush=True)


def load_traffic(kernel, workload, config=None):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources, on the same workload and (for an autotuned
    op) on the configuration being timed (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        if d.get("src_sha256") != sources_sha256():
            return None
        if d.get("workload") != workload or (config is not None and d.get("config") != config):
            return None
        return d.get("bytes_per_launch")
    except Exception:
        return None


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2602_11092_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


if __name__ == "__main__":
    main()
