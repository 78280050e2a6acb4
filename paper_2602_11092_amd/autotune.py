"""Autotuner for the batched SLOS calls.

For each requested operation it times every (kernel variant, workgroup size)
that the library accepts for the batch (`slos_batch_set_config`), on the
caller's own inputs and stream, with HIP events, and keeps the fastest.  The
choice is stored in the batch, so later calls (and HIP-graph captures made
after tuning) use it.

    report = autotune(batch, U, ops=(OP_PROBS, OP_PROBS_BACKWARD))

Candidates that the library rejects for this batch (for instance the fused
variant when a sample's photon layers do not fit in LDS) are skipped; the
report lists every timed candidate.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Optional, Tuple

import torch

from . import _binding as B

# (variant, workgroup size) candidates per direction
FORWARD_CANDIDATES = [(B.VARIANT_FUSED, 256), (B.VARIANT_FUSED, 512), (B.VARIANT_FUSED, 1024),
                      (B.VARIANT_LAYERED, 128), (B.VARIANT_LAYERED, 256), (B.VARIANT_LAYERED, 512)]
BACKWARD_CANDIDATES = [(B.VARIANT_FUSED, 256), (B.VARIANT_FUSED, 512), (B.VARIANT_FUSED, 768), (B.VARIANT_FUSED, 1024),
                       (B.VARIANT_LAYERED, 128), (B.VARIANT_LAYERED, 256), (B.VARIANT_LAYERED, 512)]
_BACKWARD = (B.OP_AMPLITUDES_BACKWARD, B.OP_PROBS_BACKWARD, B.OP_MODE_EXPECTATIONS_BACKWARD,
             B.OP_THRESHOLD_PROBS_BACKWARD)


def _runner(batch: B.Batch, U: torch.Tensor, op: int):
    """A closure that runs `op` once on fixed buffers (allocated here, before timing)."""
    dev = U.device
    n = batch.out_len
    ws = batch.workspace(op, dev)
    if op == B.OP_PROBS:
        out = torch.empty(n, dtype=torch.float32, device=dev)
        return lambda: B.fock_probs(batch, U, out=out, ws=ws)
    if op == B.OP_AMPLITUDES:
        out = torch.empty(n, dtype=torch.complex64, device=dev)
        return lambda: B.fock_amplitudes(batch, U, out=out, ws=ws)
    if op == B.OP_MODE_EXPECTATIONS:
        out = torch.empty((batch.B, batch.m), dtype=torch.float32, device=dev)
        return lambda: B.fock_mode_expectations(batch, U, out=out, ws=ws)
    if op == B.OP_THRESHOLD_PROBS:
        out = torch.empty(batch.threshold_len, dtype=torch.float32, device=dev)
        return lambda: B.fock_threshold_probs(batch, U, out=out, ws=ws)
    if op == B.OP_SAMPLE:
        u = torch.rand((batch.B, 64), device=dev)
        out = torch.empty((batch.B, 64), dtype=torch.int32, device=dev)
        return lambda: B.fock_sample(batch, U, u, out=out, ws=ws)
    gU = torch.empty_like(U)
    if op == B.OP_PROBS_BACKWARD:
        g = torch.ones(n, dtype=torch.float32, device=dev)
        return lambda: B.fock_probs_backward(batch, U, g, out=gU, ws=ws)
    if op == B.OP_MODE_EXPECTATIONS_BACKWARD:
        g = torch.ones((batch.B, batch.m), dtype=torch.float32, device=dev)
        return lambda: B.fock_mode_expectations_backward(batch, U, g, out=gU, ws=ws)
    if op == B.OP_THRESHOLD_PROBS_BACKWARD:
        g = torch.ones(batch.threshold_len, dtype=torch.float32, device=dev)
        return lambda: B.fock_threshold_probs_backward(batch, U, g, out=gU, ws=ws)
    g = torch.ones(n, dtype=torch.complex64, device=dev)
    return lambda: B.fock_amplitudes_backward(batch, U, g, out=gU, ws=ws)


def _time_us(fn, warmup: int, iters: int) -> float:
    for _ in range(warmup):
        fn()
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(iters):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) * 1e3 / iters


def autotune(batch: B.Batch, U: torch.Tensor, ops: Iterable[int] = (B.OP_PROBS, B.OP_PROBS_BACKWARD),
             warmup: int = 2, iters: int = 5,
             candidates: Optional[Dict[int, List[Tuple[int, int]]]] = None) -> Dict[int, dict]:
    """Times the supported configurations of each op on `batch` and keeps the fastest.

    Returns {op: {"variant", "block", "us", "timings": [(variant, block, us), ...]}}.
    """
    report = {}
    for op in ops:
        cands = (candidates or {}).get(op) or (BACKWARD_CANDIDATES if op in _BACKWARD else FORWARD_CANDIDATES)
        before = batch.get_config(op)
        timings = []
        for variant, block in cands:
            try:
                batch.set_config(op, variant, block)
            except B.SlosError:
                continue  # not supported for this batch
            fn = _runner(batch, U, op)
            try:
                us = _time_us(fn, warmup, iters)
            except B.SlosError:
                continue
            timings.append((variant, block, us))
        if not timings:
            batch.set_config(op, *before)
            raise RuntimeError("autotune: no configuration runs op %d on this batch" % op)
        variant, block, us = min(timings, key=lambda r: r[2])
        batch.set_config(op, variant, block)
        report[op] = {"variant": variant, "block": block, "us": us, "timings": timings}
    return report
