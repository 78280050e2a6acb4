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
from .autograd import fock_amplitudes, fock_probs, mesh_to_unitary


class QuantumLayer(nn.Module):
    """x [batch, m] float32 -> probabilities [batch, C(m+n-1, n)] (or
    complex amplitudes with measurement="amplitudes") for one input Fock
    state.  Trainable parameters: the m(m-1) mesh phases."""

    def __init__(self, m: int, input_state: Sequence[int], enc_scale: float = math.pi,
                 measurement: str = "probs", seed: int = 0):
        super().__init__()
        occ = np.asarray(input_state, dtype=np.int32)
        if occ.shape != (m,):
            raise ValueError("input_state must have m entries")
        if measurement not in ("probs", "amplitudes"):
            raise ValueError("measurement must be 'probs' or 'amplitudes'")
        self.m = m
        self.n = int(occ.sum())
        self.occ = occ
        self.enc_scale = float(enc_scale)
        self.measurement = measurement
        g = torch.Generator().manual_seed(seed)
        self.theta = nn.Parameter(torch.rand(m * (m - 1), generator=g) * (2 * math.pi))
        self._plan = None
        self._batches: Dict[int, B.Batch] = {}

    @property
    def output_size(self) -> int:
        return B.slos_fock_dim(self.m, self.n)

    def _batch(self, nb: int) -> B.Batch:
        if self._plan is None:
            self._plan = B.Plan(self.m, max(self.n, 1))
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
        return fock_amplitudes(U, bt).view(x.shape[0], -1)
