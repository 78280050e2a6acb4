"""The extension entry points at the library's limits (32 modes, 16 photons)
and on empty batches, against the oracle or exact properties."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import oracle as O
from paper_2602_11092_amd import _binding as B
from tests.gpu_util import DEV, say, to_dev_c64, widen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", [B.VARIANT_FUSED, B.VARIANT_LAYERED])
def test_expectations_and_threshold_at_32_modes(variant):
    m, n = 32, 2
    rng = np.random.default_rng(90)
    U = W.haar_unitaries(rng, 6, m).astype(np.complex64)
    occ = np.zeros((6, m), dtype=np.int32)
    occ[:, 0] = 1
    occ[np.arange(6), 5 + 4 * np.arange(6)] += 1
    occ[5, 0] = 2
    occ[5, 25] = 0
    batch = B.Batch(B.Plan(m, n, threshold=True), occ)
    for op in (B.OP_MODE_EXPECTATIONS, B.OP_THRESHOLD_PROBS):
        batch.set_config(op, variant, 256)
    Ud = to_dev_c64(U)
    say("limits m32 variant", variant)
    e = B.fock_mode_expectations(batch, Ud).cpu().numpy()
    P = B.fock_threshold_probs(batch, Ud).cpu().numpy()
    toff = batch.threshold_offsets
    assert toff[1] - toff[0] == 32 + math.comb(32, 2)
    for b in range(6):
        assert np.abs(e[b] - O.mode_expectations(widen(U[b]), occ[b])).max() <= 2e-5
        assert np.abs(P[toff[b]:toff[b + 1]] - O.threshold_probs(widen(U[b]), occ[b])).max() <= 2e-5


def test_sampling_at_32_modes():
    m, n = 32, 3
    rng = np.random.default_rng(91)
    U = W.haar_unitaries(rng, 4, m).astype(np.complex64)
    occ = np.zeros((4, m), dtype=np.int32)
    occ[:, [0, 15, 31]] = 1
    batch = B.Batch(B.Plan(m, n), occ)
    Ud = to_dev_c64(U)
    u = torch.from_numpy(rng.random((4, 512)).astype(np.float32)).to(DEV)
    shots = B.fock_sample(batch, Ud, u).cpu().numpy()
    p = B.fock_probs(batch, Ud).cpu().numpy().reshape(4, -1)
    uh = u.cpu().numpy().astype(np.float64)
    for b in range(4):
        cdf = np.cumsum(p[b].astype(np.float64))
        want = np.minimum(np.searchsorted(cdf, uh[b] * cdf[-1], side="right"), p.shape[1] - 1)
        assert (shots[b] == want).mean() >= 0.99


def test_fidelity_at_32_modes_16_photons():
    # 2^16 Ryser subsets per pair on the wave kernel; exact properties
    m, n = 32, 16
    occ = np.zeros(m, dtype=np.int32)
    occ[::2] = 1
    rng = np.random.default_rng(92)
    U = W.haar_unitaries(rng, 2, m).astype(np.complex64)
    D = np.exp(1j * rng.uniform(0, 2 * np.pi, m)).astype(np.complex64)
    say("fidelity m32 n16")
    K = B.fock_fidelity_kernel(occ, to_dev_c64(U), to_dev_c64((U * D[None, None, :]).astype(np.complex64)))
    assert np.abs(np.diag(K.cpu().numpy()) - 1).max() <= 1e-4
    P = np.arange(m)
    P[[0, 1]] = P[[1, 0]]  # an occupied mode and an empty one: orthogonal states
    K0 = B.fock_fidelity_kernel(occ, to_dev_c64(U), to_dev_c64(U[:, :, P].copy()))
    assert np.abs(np.diag(K0.cpu().numpy())).max() <= 1e-4


def test_empty_batches():
    plan = B.Plan(6, 3, threshold=True)
    batch = B.Batch(plan, np.zeros((0, 6), dtype=np.int32))
    U = torch.zeros((0, 6, 6), dtype=torch.complex64, device=DEV)
    assert B.fock_mode_expectations(batch, U).shape == (0, 6)
    assert B.fock_threshold_probs(batch, U).shape == (0,)
    assert B.fock_sample(batch, U, torch.zeros((0, 8), device=DEV)).shape == (0, 8)
    assert B.fock_fidelity_kernel([1, 1, 0, 0, 0, 0], U).shape == (0, 0)
