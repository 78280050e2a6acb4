"""GPU parity of the fidelity kernel K[a][b] = |<phi(U1_a)|phi(U2_b)>|^2
against the FP64 oracle (inner product of the two full output vectors), on
the GPU's own complex64 inputs, plus properties that hold at any size.

Tolerance: the kernel computes in FP64 and rounds once to FP32, so
|K_gpu - K| <= 1e-6 (FP32 rounding of a value <= 1, with margin)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import oracle as O
from paper_2602_11092_amd import _binding as B
from tests.gpu_util import DEV, say, to_dev_c64, widen

pytestmark = pytest.mark.gpu

K_TOL = 1e-6


def _haar(seed, B_, m):
    return W.haar_unitaries(np.random.default_rng(seed), B_, m).astype(np.complex64)


def _run(occ, U1, U2=None):
    K = B.fock_fidelity_kernel(occ, to_dev_c64(U1), None if U2 is None else to_dev_c64(U2))
    torch.cuda.synchronize()
    return K.cpu().numpy()


@pytest.mark.parametrize("occ", [[1, 0, 0, 0], [1, 1, 0, 0], [2, 0, 1, 0, 0], [1, 1, 1, 1, 0, 0],
                                 [0, 3, 0, 1, 0, 0], [1, 0, 1, 0, 1, 0, 1, 0], [2, 2, 1, 0, 0, 0, 0],
                                 # n >= 7: lanes walk several Gray-code steps
                                 [1, 1, 1, 1, 1, 1, 1, 0], [2, 2, 2, 1, 1, 0, 0, 0]])
def test_fidelity_against_oracle(occ):
    m = len(occ)
    say("fidelity", occ)
    U1, U2 = _haar(1, 5, m), _haar(2, 7, m)
    K = _run(occ, U1, U2)
    assert K.shape == (5, 7)
    ref = np.array([[O.fidelity(widen(U1[a]), widen(U2[b]), occ) for b in range(7)] for a in range(5)])
    assert np.abs(K - ref).max() <= K_TOL, np.abs(K - ref).max()


def test_gram_matrix_symmetric_with_unit_diagonal():
    occ = [1, 1, 1, 1, 0, 0]
    U = _haar(3, 33, 6)
    K = _run(occ, U)
    assert K.shape == (33, 33)
    assert np.abs(K - K.T).max() <= K_TOL
    assert np.abs(np.diag(K) - 1).max() <= K_TOL
    assert K.min() >= -K_TOL and K.max() <= 1 + K_TOL
    for a, b in [(0, 1), (5, 20), (32, 7)]:
        assert abs(K[a, b] - O.fidelity(widen(U[a]), widen(U[b]), occ)) <= K_TOL


@pytest.mark.parametrize("m,n", [(12, 8), (16, 12), (16, 16), (20, 10)])
def test_fidelity_large_n_properties(m, n):
    # U2 = U1 D (input-side phases): the same state up to a global phase, K = 1;
    # U2 = U1 P with P moving one photon to an empty mode: orthogonal, K = 0;
    # U2 = U1 P with P permuting occupied modes among equal counts: K = 1
    occ = np.zeros(m, dtype=np.int32)
    occ[:n if n <= m else m] = 1
    if n > m:
        occ[0] += n - m
    rng = np.random.default_rng(n)
    U1 = _haar(n + m, 3, m)
    D = np.exp(1j * rng.uniform(0, 2 * np.pi, m)).astype(np.complex64)
    U_phase = (U1 * D[None, None, :]).astype(np.complex64)
    say("fidelity properties m", m, "n", n)
    assert np.abs(np.diag(_run(occ, U1, U_phase)) - 1).max() <= 1e-5
    if n < m:
        P = np.arange(m)
        P[[0, m - 1]] = P[[m - 1, 0]]  # mode 0 (occupied) <-> mode m-1 (empty)
        assert np.abs(np.diag(_run(occ, U1, U1[:, :, P].copy()))).max() <= 1e-5
    P = np.arange(m)
    P[[0, 1]] = P[[1, 0]]  # both occupied once
    assert np.abs(np.diag(_run(occ, U1, U1[:, :, P].copy())) - 1).max() <= 1e-5


def test_fidelity_large_n_sampled_against_permanent():
    # n = 9 in m = 11: the oracle's Fock vectors (C(19, 9) states) for two pairs
    occ = [1] * 9 + [0, 0]
    U1, U2 = _haar(40, 2, 11), _haar(41, 2, 11)
    K = _run(occ, U1, U2)
    for a, b in [(0, 0), (1, 0)]:
        assert abs(K[a, b] - O.fidelity(widen(U1[a]), widen(U2[b]), occ)) <= K_TOL


def test_fidelity_edge_cases():
    # vacuum: every state is the same, K = 1; HOM: |1,1> through a 50:50
    # splitter is orthogonal to |1,1>; empty batches return at once
    U = _haar(5, 3, 4)
    assert np.abs(_run([0, 0, 0, 0], U) - 1).max() <= K_TOL
    bs = (np.array([[1, 1j], [1j, 1]]) / np.sqrt(2)).astype(np.complex64)[None]
    eye = np.eye(2, dtype=np.complex64)[None]
    assert abs(_run([1, 1], eye, bs)[0, 0]) <= K_TOL
    out = B.fock_fidelity_kernel([1, 0, 0, 0], to_dev_c64(U[:0]), to_dev_c64(U))
    assert out.shape == (0, 3)
    with pytest.raises(B.SlosError):
        B.fock_fidelity_kernel([17] + [0] * 3, to_dev_c64(U))


def test_fidelity_kernel_gram_from_features():
    # the paper's example shape: 4 features, 6 modes, 4 photons; a train Gram and a test-by-train block
    from paper_2602_11092_amd import FidelityKernel
    kern = FidelityKernel(6, [1, 1, 1, 1, 0, 0], seed=3)
    rng = np.random.default_rng(9)
    Xtr = rng.standard_normal((12, 4))
    Xte = rng.standard_normal((5, 4))
    Ktr = kern(Xtr)
    Kte = kern(Xte, Xtr)
    assert isinstance(Ktr, np.ndarray) and Ktr.shape == (12, 12) and Kte.shape == (5, 12)
    # U comes from the FP32 mesh, unitary to ~1e-7 per entry, so K(x, x) = |phi(x)|^4 is 1 to ~1e-6
    assert np.abs(Ktr - Ktr.T).max() <= K_TOL and np.abs(np.diag(Ktr) - 1).max() <= 1e-5
    th = kern.theta.cpu().numpy().astype(np.float64)
    pad = lambda X: np.concatenate([X, np.zeros((X.shape[0], 2))], axis=1).astype(np.float32).astype(np.float64)
    Utr = O.encoded_unitaries(th, pad(Xtr), math.pi)
    Ute = O.encoded_unitaries(th, pad(Xte), math.pi)
    occ = [1, 1, 1, 1, 0, 0]
    for a, b in [(0, 1), (3, 7), (11, 2)]:
        assert abs(Ktr[a, b] - O.fidelity(Utr[a], Utr[b], occ)) <= 1e-5
    for a, b in [(0, 0), (4, 9)]:
        assert abs(Kte[a, b] - O.fidelity(Ute[a], Utr[b], occ)) <= 1e-5
