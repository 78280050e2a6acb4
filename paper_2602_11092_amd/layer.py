"""A thin trainable layer: angle-encoded rectangular mesh followed by the
Fock-space simulation (the quantum layer of arXiv 2602.11092, Sec. II-B,
with the encoding of Sec. II-C-1, U(x, theta) = W2 S(x) W1)."""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np
import torch
from torch import nn

from . import _binding as B
from .autograd import (fock_amplitudes, fock_mode_expectations, fock_probs, fock_shared_superposition_amplitudes,
                       fock_threshold_probs, mesh_to_unitary, probs_from_amplitudes)


class QuantumLayer(nn.Module):
    """x [batch, m] float32 -> probabilities [batch, C(m+n-1, n)] (or
    complex amplitudes with measurement="amplitudes", the per-mode photon
    number expectations [batch, m] with measurement="mode_expectations", or
    threshold-detector click probabilities with measurement="threshold_probs")
    for one input Fock state.  Trainable parameters: the m(m-1) mesh phases.

    computation_space="unbunched" keeps only the output states with at most
    one photon per mode (C(m, n) of them, in the same relative order);
    "dual_rail" keeps those with at most one photon per mode pair (2g, 2g+1)
    (the 2^n logical states when n = m/2).  Their adjoint runs in the
    layered kernels.  detector="threshold" turns mode_expectations into
    per-mode click probabilities P(t_j > 0)."""

    def __init__(self, m: int, input_state: Sequence[int], enc_scale: float = math.pi,
                 measurement: str = "probs", seed: int = 0, computation_space: str = "fock",
                 detector: str = "pnr"):
        super().__init__()
        occ = np.asarray(input_state, dtype=np.int32)
        if occ.shape != (m,):
            raise ValueError("input_state must have m entries")
        if measurement not in ("probs", "amplitudes", "mode_expectations", "threshold_probs"):
            raise ValueError("measurement must be 'probs', 'amplitudes', 'mode_expectations' or 'threshold_probs'")
        if detector not in ("pnr", "threshold"):
            raise ValueError("detector must be 'pnr' or 'threshold'")
        self.detector = detector
        if computation_space not in ("fock", "unbunched", "dual_rail"):
            raise ValueError("computation_space must be 'fock', 'unbunched' or 'dual_rail'")
        if computation_space == "unbunched" and int(occ.sum()) > m:
            raise ValueError("the unbunched space needs at most m photons")
        if computation_space == "dual_rail" and (m % 2 or 2 * int(occ.sum()) > m):
            raise ValueError("the dual-rail space needs an even m and at most m/2 photons")
        self.m = m
        self.n = int(occ.sum())
        self.occ = occ
        self.enc_scale = float(enc_scale)
        self.measurement = measurement
        self.computation_space = computation_space
        g = torch.Generator().manual_seed(seed)
        self.theta = nn.Parameter(torch.rand(m * (m - 1), generator=g) * (2 * math.pi))
        self._plan = None
        self._batches: Dict[int, B.Batch] = {}

    @property
    def output_size(self) -> int:
        if self.measurement == "mode_expectations":
            return self.m
        if self.measurement == "threshold_probs":
            return B.slos_threshold_dim(self.m, self.n)
        return B.slos_space_dim(self.m, self.n, self._flags())

    def _flags(self) -> int:
        return B.space_flags(self.computation_space == "unbunched", self.computation_space == "dual_rail")

    def _batch(self, nb: int) -> B.Batch:
        if self._plan is None:
            self._plan = B.Plan(self.m, max(self.n, 1), unbunched=self.computation_space == "unbunched",
                                dual_rail=self.computation_space == "dual_rail",
                                threshold=self.measurement == "threshold_probs")
        bt = self._batches.get(nb)
        if bt is None:
            bt = B.Batch(self._plan, np.tile(self.occ, (nb, 1)))
            self._batches[nb] = bt
        return bt

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        U = mesh_to_unitary(self.theta, x.to(torch.float32), self.enc_scale, self.m)
        bt = self._batch(x.shape[0])
        if self.measurement == "probs":
            return fock_probs(U, bt).view(x.shape[0], -1)
        if self.measurement == "mode_expectations":
            return fock_mode_expectations(U, bt, self.detector)
        if self.measurement == "threshold_probs":
            return fock_threshold_probs(U, bt).view(x.shape[0], -1)
        return fock_amplitudes(U, bt).view(x.shape[0], -1)


class AmplitudeEncodedLayer(nn.Module):
    """Amplitude encoding (Sec. II-C-2): X [batch, C(m+n-1, n)] complex64, each
    row an n-photon state in basis order, goes through the trainable mesh
    W2 W1 (no feature phases).  Returns the output amplitudes, or their
    squared moduli with measurement="probs".  One interferometer for the
    whole batch: its n-photon representation is built once per call and the
    batch goes through one complex GEMM."""

    def __init__(self, m: int, n: int, measurement: str = "amplitudes", seed: int = 0):
        super().__init__()
        if measurement not in ("amplitudes", "probs"):
            raise ValueError("measurement must be 'amplitudes' or 'probs'")
        self.m = m
        self.n = n
        self.measurement = measurement
        g = torch.Generator().manual_seed(seed)
        self.theta = nn.Parameter(torch.rand(m * (m - 1), generator=g) * (2 * math.pi))
        self._shared = None

    @property
    def state_size(self) -> int:
        return B.slos_fock_dim(self.m, self.n)

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        if self._shared is None:
            self._shared = B.SharedSuperposition(B.Plan(self.m, max(self.n, 1)), self.n)
        U = mesh_to_unitary(self.theta, None, 0.0, self.m)[0]
        out = fock_shared_superposition_amplitudes(U, X.to(torch.complex64), self._shared)
        return out if self.measurement == "amplitudes" else probs_from_amplitudes(out)


class FidelityKernel:
    """Fidelity kernel k(x1, x2) = |<phi(x1)|phi(x2)>|^2 with |phi(x)> =
    U(x, theta)|s> (Sec. III-A), for kernel methods with a precomputed Gram
    matrix: K = kernel(X) or kernel(X_test, X_train).  Features x (up to m
    per sample) drive the angle-encoding phases of the mesh; fewer features
    than modes leave the remaining phases at zero.  numpy inputs give a numpy
    Gram matrix (float64), torch inputs a float32 device tensor."""

    def __init__(self, m: int, input_state: Sequence[int], enc_scale: float = math.pi, seed: int = 0,
                 device: str = "cuda"):
        occ = np.asarray(input_state, dtype=np.int32)
        if occ.shape != (m,):
            raise ValueError("input_state must have m entries")
        self.m = m
        self.occ = occ
        self.enc_scale = float(enc_scale)
        self.device = device
        g = torch.Generator().manual_seed(seed)
        self.theta = (torch.rand(m * (m - 1), generator=g) * (2 * math.pi)).to(device)

    def _unitaries(self, X: torch.Tensor) -> torch.Tensor:
        X = X.to(self.device, torch.float32)
        if X.dim() != 2 or X.shape[1] > self.m:
            raise ValueError("features must be [batch, <= m]")
        if X.shape[1] < self.m:
            X = torch.cat([X, X.new_zeros(X.shape[0], self.m - X.shape[1])], dim=1)
        return B.mesh_to_unitary(self.theta, X.contiguous(), self.enc_scale)

    def __call__(self, X1, X2=None):
        as_numpy = isinstance(X1, np.ndarray)
        t1 = torch.as_tensor(np.asarray(X1, dtype=np.float32)) if as_numpy else X1
        U1 = self._unitaries(t1)
        if X2 is None:
            K = B.fock_fidelity_kernel(self.occ, U1)
        else:
            t2 = torch.as_tensor(np.asarray(X2, dtype=np.float32)) if isinstance(X2, np.ndarray) else X2
            K = B.fock_fidelity_kernel(self.occ, U1, self._unitaries(t2))
        return K.cpu().numpy().astype(np.float64) if as_numpy else K
