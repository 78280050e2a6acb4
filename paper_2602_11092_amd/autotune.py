"""Autotuner for the batched SLOS calls.

For each requested operation it considers every (kernel variant, workgroup
size, tile) that the library accepts for the batch (`slos_batch_set_config_ex`),
and for each candidate:

1. a parity gate: on a small seeded batch of the same plan (two samples for
   each photon number of the batch, Haar-random unitaries drawn from a fixed
   seed), the candidate's outputs must agree with those of the reference
   configuration, the layered variant (one launch per photon layer), within
   1e-6 for amplitudes and probabilities, 1e-5 for per-mode and threshold
   sums, relative 1e-5 for gradients, and identical shots for all but 2% of
   the draws (a shot whose uniform falls on a cumulative-sum boundary may go
   either way);
2. timing on the caller's own inputs and stream, with HIP events.

The fastest candidate that passed is stored in the batch, so later calls (and
HIP-graph captures made after tuning) use it.  With a cache path (argument
or the SLOS_AUTOTUNE_CACHE environment variable) the choice is also kept in a
JSON file keyed by (m, plan flags, photon-number multiset, B, GPU
architecture, library build); a later call with the same key reuses it
without timing.

    report = autotune(batch, U, ops=(OP_PROBS, OP_PROBS_BACKWARD), cache="tune.json")
"""
from __future__ import annotations

import collections
import hashlib
import json
import os
from typing import Dict, Iterable, List, Optional, Tuple

import numpy as np
import torch

from . import _binding as B

# (variant, workgroup size, tile) candidates per direction
FORWARD_CANDIDATES = [(B.VARIANT_FUSED_PAIRS, 1024, 2), (B.VARIANT_FUSED_PAIRS, 1024, 4),
                      (B.VARIANT_FUSED_PAIRS, 1024, 8), (B.VARIANT_FUSED_PAIRS, 512, 4),
                      (B.VARIANT_FUSED, 256, 0), (B.VARIANT_FUSED, 512, 0), (B.VARIANT_FUSED, 1024, 0),
                      (B.VARIANT_LAYERED, 128, 0), (B.VARIANT_LAYERED, 256, 0), (B.VARIANT_LAYERED, 512, 0),
                      (B.VARIANT_LAYERED, 1024, 0)]
BACKWARD_CANDIDATES = [(B.VARIANT_FUSED, 256, 0), (B.VARIANT_FUSED, 512, 0), (B.VARIANT_FUSED, 768, 0),
                       (B.VARIANT_FUSED, 1024, 0), (B.VARIANT_LAYERED, 128, 0), (B.VARIANT_LAYERED, 256, 0),
                       (B.VARIANT_LAYERED, 512, 0), (B.VARIANT_LAYERED, 1024, 0)]
REFERENCE = (B.VARIANT_LAYERED, 256, 0)
_BACKWARD = (B.OP_AMPLITUDES_BACKWARD, B.OP_PROBS_BACKWARD, B.OP_MODE_EXPECTATIONS_BACKWARD,
             B.OP_THRESHOLD_PROBS_BACKWARD)
GATE_SEED = 20260211
GATE_SHOTS = 64


def _runner(batch: B.Batch, U: torch.Tensor, op: int, grad=None):
    """(fn, out): a closure running `op` once on fixed buffers (allocated
    here, before timing) and the tensor it writes."""
    dev = U.device
    n = batch.out_len
    ws = batch.workspace(op, dev)
    if op == B.OP_PROBS:
        out = torch.empty(n, dtype=torch.float32, device=dev)
        return (lambda: B.fock_probs(batch, U, out=out, ws=ws)), out
    if op == B.OP_AMPLITUDES:
        out = torch.empty(n, dtype=torch.complex64, device=dev)
        return (lambda: B.fock_amplitudes(batch, U, out=out, ws=ws)), out
    if op == B.OP_MODE_EXPECTATIONS:
        out = torch.empty((batch.B, batch.m), dtype=torch.float32, device=dev)
        return (lambda: B.fock_mode_expectations(batch, U, out=out, ws=ws)), out
    if op == B.OP_THRESHOLD_PROBS:
        out = torch.empty(batch.threshold_len, dtype=torch.float32, device=dev)
        return (lambda: B.fock_threshold_probs(batch, U, out=out, ws=ws)), out
    if op == B.OP_SAMPLE:
        u = grad if grad is not None else torch.rand((batch.B, GATE_SHOTS), device=dev)
        out = torch.empty((batch.B, u.shape[1]), dtype=torch.int32, device=dev)
        return (lambda: B.fock_sample(batch, U, u, out=out, ws=ws)), out
    gU = torch.empty_like(U)
    if op == B.OP_PROBS_BACKWARD:
        g = grad if grad is not None else torch.ones(n, dtype=torch.float32, device=dev)
        return (lambda: B.fock_probs_backward(batch, U, g, out=gU, ws=ws)), gU
    if op == B.OP_MODE_EXPECTATIONS_BACKWARD:
        g = grad if grad is not None else torch.ones((batch.B, batch.m), dtype=torch.float32, device=dev)
        return (lambda: B.fock_mode_expectations_backward(batch, U, g, out=gU, ws=ws)), gU
    if op == B.OP_THRESHOLD_PROBS_BACKWARD:
        g = grad if grad is not None else torch.ones(batch.threshold_len, dtype=torch.float32, device=dev)
        return (lambda: B.fock_threshold_probs_backward(batch, U, g, out=gU, ws=ws)), gU
    g = grad if grad is not None else torch.ones(n, dtype=torch.complex64, device=dev)
    return (lambda: B.fock_amplitudes_backward(batch, U, g, out=gU, ws=ws)), gU


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


# ------------------------------------------------------------------ parity gate

class _Gate:
    """A small seeded batch of the plan (two samples per photon number of the
    batch being tuned) with fixed inputs, and each op's reference outputs
    from the layered variant."""

    def __init__(self, batch: B.Batch, device):
        rng = np.random.default_rng(GATE_SEED)
        occ = []
        for n in sorted(set(int(v) for v in batch.n), reverse=True):
            rows = batch.occ[batch.n == n]
            occ += [rows[0], rows[-1]]
        self.batch = B.Batch(batch.plan, np.asarray(occ, dtype=np.int32))
        m, G = batch.m, len(occ)
        z = (rng.standard_normal((G, m, m)) + 1j * rng.standard_normal((G, m, m))) / np.sqrt(2.0)
        q, r = np.linalg.qr(z)
        d = np.diagonal(r, axis1=1, axis2=2)
        U = q * (d / np.abs(d))[:, None, :]
        self.U = torch.from_numpy(U.astype(np.complex64)).to(device)
        self.inputs = {}
        self.ref = {}
        self.device = device

    def _input(self, op: int):
        if op not in self.inputs:
            rng = np.random.default_rng(GATE_SEED + 1 + op)
            bt = self.batch
            if op in (B.OP_PROBS_BACKWARD,):
                v = rng.uniform(0, 1, bt.out_len).astype(np.float32)
            elif op == B.OP_AMPLITUDES_BACKWARD:
                v = (rng.standard_normal(bt.out_len) + 1j * rng.standard_normal(bt.out_len)).astype(np.complex64)
            elif op == B.OP_MODE_EXPECTATIONS_BACKWARD:
                v = rng.uniform(0, 1, (bt.B, bt.m)).astype(np.float32)
            elif op == B.OP_THRESHOLD_PROBS_BACKWARD:
                v = rng.uniform(0, 1, bt.threshold_len).astype(np.float32)
            elif op == B.OP_SAMPLE:
                v = rng.uniform(0, 1, (bt.B, GATE_SHOTS)).astype(np.float32)
            else:
                v = None
            self.inputs[op] = None if v is None else torch.from_numpy(v).to(self.device)
        return self.inputs[op]

    def _run(self, op: int, cfg) -> np.ndarray:
        self.batch.set_config(op, *cfg)
        fn, out = _runner(self.batch, self.U, op, self._input(op))
        fn()
        torch.cuda.synchronize()
        return out.cpu().numpy()

    def passes(self, op: int, cfg) -> bool:
        if op not in self.ref:
            self.ref[op] = self._run(op, REFERENCE)
        try:
            got = self._run(op, cfg)
        except B.SlosError:
            return False
        return agrees(op, got, self.ref[op])


def agrees(op: int, got: np.ndarray, ref: np.ndarray) -> bool:
    """The gate's test of a candidate's outputs against the reference's."""
    if got.shape != ref.shape or not np.all(np.isfinite(got)):
        return False
    if op in _BACKWARD:
        return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)) <= 1e-5
    if op == B.OP_SAMPLE:
        return float(np.mean(got != ref)) <= 0.02 if got.size else True
    tol = 1e-6 if op in (B.OP_PROBS, B.OP_AMPLITUDES) else 1e-5
    return float(np.abs(got - ref).max(initial=0.0)) <= tol


# ------------------------------------------------------------------ cache

_lib_digest = None


def _library_digest() -> str:
    global _lib_digest
    if _lib_digest is None:
        h = hashlib.sha256()
        with open(B.LIB_PATH, "rb") as f:
            for chunk in iter(lambda: f.read(1 << 20), b""):
                h.update(chunk)
        _lib_digest = h.hexdigest()[:16]
    return _lib_digest


def cache_key(batch: B.Batch, device) -> str:
    """(m, plan flags, photon-number multiset, B, GPU architecture, library build)."""
    counts = collections.Counter(int(v) for v in batch.n)
    multiset = ",".join("%dx%d" % (n, c) for n, c in sorted(counts.items(), reverse=True))
    arch = torch.cuda.get_device_properties(torch.device(device)).gcnArchName
    flags = B.space_flags(batch.plan.unbunched, batch.plan.dual_rail) | (B.PLAN_THRESHOLD if batch.plan.threshold else 0)
    return "m%d|flags%d|n%s|B%d|%s|lib%s" % (batch.m, flags, multiset, batch.B, arch, _library_digest())


def _load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path: str, key: str, op: int, entry: dict) -> None:
    data = _load_cache(path)
    data.setdefault(key, {})[str(op)] = entry
    tmp = "%s.tmp%d" % (path, os.getpid())
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


# ------------------------------------------------------------------ tuner

def autotune(batch: B.Batch, U: torch.Tensor, ops: Iterable[int] = (B.OP_PROBS, B.OP_PROBS_BACKWARD),
             warmup: int = 2, iters: int = 5,
             candidates: Optional[Dict[int, List[Tuple[int, int, int]]]] = None,
             cache: Optional[str] = None) -> Dict[int, dict]:
    """Picks a configuration per op for `batch` (see the module docstring).

    Returns {op: {"variant", "block", "tile", "us", "cached", "timings": [(variant, block, tile, us)],
    "rejected": [(variant, block, tile)]}}: `timings` lists the candidates timed, `rejected`
    those that failed the parity gate.
    """
    cache = cache if cache is not None else os.environ.get("SLOS_AUTOTUNE_CACHE") or None
    key = cache_key(batch, U.device) if cache else None
    stored = _load_cache(cache).get(key, {}) if cache else {}
    gate = None
    report = {}
    for op in ops:
        hit = stored.get(str(op))
        if hit is not None:
            try:
                batch.set_config(op, hit["variant"], hit["block"], hit.get("tile", 0))
                report[op] = {"variant": hit["variant"], "block": hit["block"], "tile": hit.get("tile", 0),
                              "us": hit["us"], "cached": True, "timings": [], "rejected": []}
                continue
            except B.SlosError:
                pass  # the stored choice no longer applies: tune again
        cands = (candidates or {}).get(op) or (BACKWARD_CANDIDATES if op in _BACKWARD else FORWARD_CANDIDATES)
        before = batch.get_config_ex(op)
        timings, rejected = [], []
        for variant, block, tile in cands:
            try:
                batch.set_config(op, variant, block, tile)
            except B.SlosError:
                continue  # not supported for this batch
            if gate is None:
                gate = _Gate(batch, U.device)
            if not gate.passes(op, (variant, block, tile)):
                rejected.append((variant, block, tile))
                continue
            fn, _ = _runner(batch, U, op)
            try:
                us = _time_us(fn, warmup, iters)
            except B.SlosError:
                continue
            timings.append((variant, block, tile, us))
        if not timings:
            batch.set_config(op, *before)
            raise RuntimeError("autotune: no configuration runs op %d on this batch" % op)
        variant, block, tile, us = min(timings, key=lambda r: r[3])
        batch.set_config(op, variant, block, tile)
        report[op] = {"variant": variant, "block": block, "tile": tile, "us": us, "cached": False,
                      "timings": timings, "rejected": rejected}
        if cache:
            _store_cache(cache, key, op, {"variant": variant, "block": block, "tile": tile, "us": us})
    return report
