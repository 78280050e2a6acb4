"""Invariants of the method checked on the GPU at sizes where the full
oracle is too slow: facts that hold for any unitary and any input, so a
mistake anywhere in the recursion (a dropped predecessor, a wrong
coefficient, a wrong norm) breaks them.

- Per-mode marginals (Sec. II-B measurements): sum_t t_j p_t equals
  sum_i s_i |U_ji|^2 for a unitary U, checked at m = 24, n = 8 (7,888,725
  outputs per sample) through the expectation epilogue.
- Phase invariance: diagonal phases on either side of U change no output
  probability (a global phase per output state), at m = 24, n = 8.
- Angle-encoding spectrum (Sec. II-C-1): with one encoded phase phi swept
  over 16 equispaced points, every output probability is a trigonometric
  polynomial in phi of degree at most n, so the discrete Fourier
  coefficients of order n+1..8 vanish, at the m = 20, n = 5 mesh.

Tolerances: the marginals sum up to 7.9M FP32 probabilities (expected
relative rounding ~1e-6 on a value <= n): 1e-4 absolute; per-output
probabilities 1e-5 absolute as everywhere; the Fourier coefficients of a
16-point DFT of values each within 1e-6 of exact: 1e-6 absolute."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from paper_2602_11092_amd import _binding as B
from tests.gpu_util import DEV, P_TOL, fock_dim, say, to_dev_c64

pytestmark = pytest.mark.gpu


def _marginals(U, occ):
    # sum_i s_i |U_ji|^2 in FP64
    return (np.abs(U.astype(np.complex128)) ** 2) @ occ.astype(np.float64)


def test_c5_marginals_through_the_expectation_epilogue():
    wl = W.make("haar_m24_n8_b16")
    say("marginals m24 n8 b16")
    m, n = 24, 8
    batch = B.Batch(B.Plan(m, n), wl.occ)
    U = to_dev_c64(wl.U)
    ex = B.fock_mode_expectations(batch, U)
    p = B.fock_probs(batch, U)
    torch.cuda.synchronize()
    ex = ex.cpu().numpy()
    for b in range(16):
        assert np.abs(ex[b] - _marginals(wl.U[b], wl.occ[b])).max() <= 1e-4, b
    # sum_j <n_j> = n, and the probabilities the same forward produces sum to 1
    assert np.abs(ex.sum(axis=1) - n).max() <= 1e-3
    pb = p.reshape(16, fock_dim(m, n)).double()
    assert float((pb.sum(dim=1) - 1).abs().max()) <= 1e-4


def test_c5_phase_invariance():
    wl = W.make("haar_m24_n8_b16")
    say("phase invariance m24 n8")
    m, n = 24, 8
    rng = np.random.default_rng(17)
    Ub = wl.U[:4]
    occ = wl.occ[:4]
    d1 = np.exp(2j * np.pi * rng.random((4, m)))
    d2 = np.exp(2j * np.pi * rng.random((4, m)))
    Up = (d1[:, :, None] * Ub.astype(np.complex128) * d2[:, None, :]).astype(np.complex64)
    batch = B.Batch(B.Plan(m, n), occ)
    p0 = B.fock_probs(batch, to_dev_c64(Ub))
    p1 = B.fock_probs(batch, to_dev_c64(Up))
    torch.cuda.synchronize()
    assert float((p0 - p1).abs().max()) <= P_TOL
    assert abs(float(p0.double().sum()) - 4.0) <= 4e-4


def test_c4_encoded_phase_spectrum():
    # one encoded phase swept over 16 points through the m = 20 mesh; the
    # probabilities of every output (42504 per point) must have no Fourier
    # component of order above n = 5
    wl = W.make("clements_m20_n5_b512")
    say("encoded phase spectrum m20 n5")
    m, n, K = 20, 5, 16
    theta = torch.from_numpy(wl.theta).to(DEV)
    x = np.repeat(wl.x[:1], K, axis=0).astype(np.float32)
    x[:, 7] = (2.0 * np.arange(K) / K).astype(np.float32)  # phase pi * x = 2 pi k / K
    U = B.mesh_to_unitary(theta, torch.from_numpy(x).to(DEV), wl.enc_scale)
    occ = np.repeat(wl.occ[:1], K, axis=0)
    batch = B.Batch(B.Plan(m, n), occ)
    p = B.fock_probs(batch, U)
    torch.cuda.synchronize()
    P = p.reshape(K, -1).double().cpu().numpy()
    F = np.fft.fft(P, axis=0) / K
    high = np.abs(F[n + 1:K - n]).max()  # orders n+1 .. K-n-1 (i.e. 6..10 with K = 16)
    low = np.abs(F[1:n + 1]).max()
    assert high <= 1e-6, high
    assert low > 100 * max(high, 1e-9)  # the phase does change the output distribution
    assert math.isclose(float(P.sum(axis=1).mean()), 1.0, abs_tol=1e-4)
