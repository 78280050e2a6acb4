"""Seeded synthetic inputs for the strong-simulation workloads.

This module only draws random inputs (unitaries, phases, features, photon
counts, readout weights, labels, loss weights).  It holds none of the
method's arithmetic, and it is the one module that both the GPU path and the
FP64 oracle are fed from.

Recipe (every draw is float64 on the host, then cast to the GPU's types;
the oracle is given the cast values widened back to float64):

* seeds: numpy SeedSequence(1000 + index).spawn(6), children used in the
  fixed order  unitaries/phases, features, photon counts/modes, labels,
  readout weights, loss weights;
* Haar unitaries: Z = (A + iB)/sqrt 2 with A, B ~ N(0,1), Q, R = qr(Z),
  U = Q diag(R_ii/|R_ii|), cast to complex64;
* mesh phases ~ U[0, 2 pi) (one theta and one phi per MZI), float32;
* features ~ N(0,1), float32, encoded as phases pi * x;
* mixed photon counts n_b ~ U{lo..hi}, photons in modes 0..n_b-1;
* readout: Xavier-uniform W (gain 1), zero bias, labels ~ U{0..classes-1};
* weighted-sum loss weights ~ U[0,1), float32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

PI = math.pi


def haar_unitaries(rng: np.random.Generator, B: int, m: int) -> np.ndarray:
    """B Haar-random m x m unitaries (complex128) by QR with R-diagonal phases fixed."""
    Z = (rng.standard_normal((B, m, m)) + 1j * rng.standard_normal((B, m, m))) / math.sqrt(2.0)
    out = np.empty((B, m, m), dtype=np.complex128)
    for b in range(B):
        Q, R = np.linalg.qr(Z[b])
        d = np.diag(R)
        out[b] = Q * (d / np.abs(d))[None, :]
    return out


def occupation_first_modes(B: int, m: int, n) -> np.ndarray:
    """Occupation vectors with one photon in each of modes 0..n_b-1."""
    n = np.broadcast_to(np.asarray(n, dtype=np.int64), (B,))
    occ = np.zeros((B, m), dtype=np.int32)
    for b in range(B):
        occ[b, : n[b]] = 1
    return occ


def occupation_modes(B: int, m: int, modes) -> np.ndarray:
    occ = np.zeros((B, m), dtype=np.int32)
    for j in modes:
        occ[:, j] += 1
    return occ


def num_mzi_phases(m: int) -> int:
    """Two phases per MZI of a rectangular mesh with m(m-1)/2 MZIs."""
    return m * (m - 1)


@dataclass
class Workload:
    name: str
    m: int
    B: int
    occ: np.ndarray                     # [B, m] int32 input occupations
    U: Optional[np.ndarray] = None      # [B, m, m] complex64 (Haar workloads)
    theta: Optional[np.ndarray] = None  # [m(m-1)] float32 mesh phases
    x: Optional[np.ndarray] = None      # [B, m] float32 features
    enc_scale: float = PI
    backward: bool = False
    loss: str = "none"                  # "none" | "readout_ce" | "weighted_sum"
    readout_W: Optional[np.ndarray] = None
    readout_b: Optional[np.ndarray] = None
    labels: Optional[np.ndarray] = None
    loss_w: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> np.ndarray:
        return self.occ.sum(axis=1)


def _children(index: int):
    ss = np.random.SeedSequence(1000 + index)
    return [np.random.default_rng(c) for c in ss.spawn(6)]


def _fock_dim(m: int, n: int) -> int:
    return math.comb(m + n - 1, n)


def make(name: str, B: Optional[int] = None) -> Workload:
    """Build one of the named workloads.  `B` overrides the batch size (the
    draws for the first B samples are not the same as the full batch's)."""
    if name == "haar_m6_n3_b64":
        r = _children(0)
        B = B or 64
        m = 6
        U = haar_unitaries(r[0], B, m).astype(np.complex64)
        return Workload(name, m, B, occupation_first_modes(B, m, 3), U=U)
    if name == "haar_m16_n6_b256":
        r = _children(1)
        B = B or 256
        m = 16
        U = haar_unitaries(r[0], B, m).astype(np.complex64)
        return Workload(name, m, B, occupation_first_modes(B, m, 6), U=U)
    if name == "clements_m12_n2to6_b4096":
        r = _children(2)
        B = B or 4096
        m = 12
        theta = r[0].uniform(0.0, 2 * PI, num_mzi_phases(m)).astype(np.float32)
        x = r[1].standard_normal((B, m)).astype(np.float32)
        n = r[2].integers(2, 7, size=B)
        return Workload(name, m, B, occupation_first_modes(B, m, n), theta=theta, x=x)
    if name == "clements_m20_n5_b512":
        r = _children(3)
        B = B or 512
        m = 20
        theta = r[0].uniform(0.0, 2 * PI, num_mzi_phases(m)).astype(np.float32)
        x = r[1].standard_normal((B, m)).astype(np.float32)
        occ = occupation_modes(B, m, [0, 4, 8, 12, 16])
        N = _fock_dim(m, 5)
        classes = 10
        labels = r[3].integers(0, classes, size=B).astype(np.int64)
        a = math.sqrt(6.0 / (N + classes))
        W = r[4].uniform(-a, a, (classes, N)).astype(np.float32)
        return Workload(name, m, B, occ, theta=theta, x=x, backward=True, loss="readout_ce",
                        readout_W=W, readout_b=np.zeros(classes, np.float32), labels=labels)
    if name == "haar_m24_n8_b16":
        r = _children(4)
        B = B or 16
        m = 24
        U = haar_unitaries(r[0], B, m).astype(np.complex64)
        N = _fock_dim(m, 8)
        w = r[5].uniform(0.0, 1.0, N).astype(np.float32)
        return Workload(name, m, B, occupation_first_modes(B, m, 8), U=U, backward=True,
                        loss="weighted_sum", loss_w=w)
    raise KeyError(name)


WORKLOADS = ("haar_m6_n3_b64", "haar_m16_n6_b256", "clements_m12_n2to6_b4096",
             "clements_m20_n5_b512", "haar_m24_n8_b16")
