"""Shared helpers of the GPU parity tests."""
import math
import sys

import numpy as np
import torch

from paper_2602_11092_amd import _binding as B

DEV = "cuda:0"
P_TOL = 1e-5       # max |p_gpu - p_oracle|, absolute
A_TOL = 1e-5       # max |a_gpu - a_oracle|, absolute
G_RTOL = 1e-4      # ||g - g*|| / ||g*||


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev_c64(U: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(U.astype(np.complex64))).to(DEV)


def widen(U_c64: np.ndarray) -> np.ndarray:
    return U_c64.astype(np.complex128)


def run_forward(batch: B.Batch, U_dev: torch.Tensor, amplitudes: bool):
    out = B.fock_amplitudes(batch, U_dev) if amplitudes else B.fock_probs(batch, U_dev)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def rel_err(g: np.ndarray, ref: np.ndarray) -> float:
    return float(np.linalg.norm((g - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def fock_dim(m, n):
    return math.comb(m + n - 1, n)
