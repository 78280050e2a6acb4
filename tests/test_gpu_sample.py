"""GPU parity of inverse-transform shot sampling.  The shot is an integer
decided by floating point, so the exact check uses the decision in the
kernel's own precision: cumulative sums, in FP64, of the kernel's own
probabilities, rebuilt on the host.  Against the FP64 oracle, shots must
agree wherever the target u * sum(p) lies farther than 1e-4 from every CDF
boundary, and many shots must follow the oracle's p (chi-square)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import oracle as O
from paper_2602_11092_amd import _binding as B
from tests.gpu_util import DEV, say, to_dev_c64, widen

pytestmark = pytest.mark.gpu

VARIANTS = [B.VARIANT_FUSED, B.VARIANT_LAYERED]


def _run(batch, U, u, variant):
    batch.set_config(B.OP_SAMPLE, variant, 0)
    batch.set_config(B.OP_PROBS, variant, 0)
    Ud = to_dev_c64(U)
    shots = B.fock_sample(batch, Ud, torch.from_numpy(u).to(DEV))
    p = B.fock_probs(batch, Ud)
    torch.cuda.synchronize()
    return shots.cpu().numpy(), p.cpu().numpy()


def _check_own_precision(batch, p, u, shots):
    # the kernel's decision: first t with cdf[t] > u * cdf[-1], cdf in FP64 over the kernel's p
    near = 0
    for b in range(batch.B):
        o0, o1 = batch.offsets[b], batch.offsets[b + 1]
        cdf = np.cumsum(p[o0:o1].astype(np.float64))
        tgt = u[b].astype(np.float64) * cdf[-1]
        want = np.minimum(np.searchsorted(cdf, tgt, side="right"), o1 - o0 - 1)
        # summation order differs from the kernel's only by FP64 rounding
        ok = (shots[b] == want) | (np.abs(cdf[np.minimum(want, o1 - o0 - 1)] - tgt) < 1e-9)
        assert ok.all(), b
        near += int((shots[b] != want).sum())
    assert near <= 2


@pytest.mark.parametrize("variant", VARIANTS)
def test_sample_matches_its_own_cdf_and_the_oracle(variant):
    rng = np.random.default_rng(7)
    m, B_ = 6, 24
    U = W.haar_unitaries(rng, B_, m).astype(np.complex64)
    occ = np.zeros((B_, m), dtype=np.int32)
    for b in range(B_):
        np.add.at(occ[b], rng.choice(m, size=int(rng.integers(1, 5)), replace=True), 1)
    occ[5] = 0  # a vacuum sample
    u = rng.random((B_, 500)).astype(np.float32)
    batch = B.Batch(B.Plan(m, int(occ.sum(1).max())), occ)
    say("sample m6 variant", variant)
    shots, p = _run(batch, U, u, variant)
    assert shots.shape == (B_, 500) and shots.dtype == np.int32
    assert np.all(shots[5] == 0)
    _check_own_precision(batch, p, u, shots)
    for b in range(B_):
        n = int(occ[b].sum())
        ref = O.sample_shots(widen(U[b]), occ[b], u[b].astype(np.float64))
        cdf = np.cumsum(O.probabilities(widen(U[b]), occ[b]))
        tgt = u[b].astype(np.float64) * cdf[-1]
        far = np.abs(tgt[:, None] - cdf[None, :]).min(axis=1) > 1e-4
        assert np.all(shots[b][far] == ref[far]), b
        assert np.all((shots[b] >= 0) & (shots[b] < math.comb(m + n - 1, n)))


def test_sample_distribution_chi_square():
    rng = np.random.default_rng(8)
    m, s = 5, [1, 1, 1, 0, 0]
    U = W.haar_unitaries(rng, 1, m).astype(np.complex64)
    S = 200000
    u = rng.random((1, S)).astype(np.float32)
    batch = B.Batch(B.Plan(m, 3), np.array([s], dtype=np.int32))
    shots, _ = _run(batch, U, u, B.VARIANT_FUSED)
    p = O.probabilities(widen(U[0]), s)
    counts = np.bincount(shots[0], minlength=p.size)
    keep = p * S > 5
    chi2 = (((counts - p * S) ** 2) / (p * S))[keep].sum()
    dof = int(keep.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)


def test_sample_identity_and_edges():
    m = 5
    occ = np.array([[0, 2, 0, 1, 0], [1, 0, 0, 0, 1]], dtype=np.int32)
    U = np.stack([np.eye(m, dtype=np.complex64)] * 2)
    batch = B.Batch(B.Plan(m, 3), occ)
    u = np.random.default_rng(1).random((2, 64)).astype(np.float32)
    u[:, 0] = 0.0
    u[:, 1] = np.nextafter(np.float32(1), np.float32(0))
    for variant in VARIANTS:
        shots, _ = _run(batch, U, u, variant)
        assert np.all(shots[0] == O.fock_rank(m, 3, occ[0]))
        assert np.all(shots[1] == O.fock_rank(m, 2, occ[1]))
    empty = B.fock_sample(batch, to_dev_c64(U), torch.zeros((2, 0), device=DEV))
    assert empty.shape == (2, 0)


@pytest.mark.parametrize("variant", VARIANTS)
def test_sample_clements_m20_n5_b512(variant):
    wl = W.make("clements_m20_n5_b512")
    U = O.encoded_unitaries(wl.theta.astype(np.float64), wl.x.astype(np.float64), math.pi).astype(np.complex64)
    u = np.random.default_rng(2).random((512, 64)).astype(np.float32)
    batch = B.Batch(B.Plan(20, 5), wl.occ)
    say("sample clements_m20_n5_b512 variant", variant)
    shots, p = _run(batch, U, u, variant)
    _check_own_precision(batch, p, u, shots)


def test_sample_m24_n8_layered():
    # C(31, 8) = 7.9e6 states per sample: each sample spans hundreds of scan chunks
    wl = W.make("haar_m24_n8_b16", B=4)
    u = np.random.default_rng(3).random((4, 256)).astype(np.float32)
    batch = B.Batch(B.Plan(24, 8), wl.occ)
    say("sample haar_m24_n8 B=4")
    shots, p = _run(batch, wl.U, u, B.VARIANT_LAYERED)
    _check_own_precision(batch, p, u, shots)
