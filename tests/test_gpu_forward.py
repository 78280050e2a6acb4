"""GPU forward parity: amplitudes and probabilities from the HIP kernels
(fused and layered variants) against the FP64 Ryser oracle, element by
element, on the GPU's own complex64 inputs widened to FP64."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import oracle as O
from paper_2602_11092_amd import _binding as B
from tests.gpu_util import A_TOL, DEV, P_TOL, fock_dim, run_forward, say, to_dev_c64, widen

pytestmark = pytest.mark.gpu

VARIANTS = [B.VARIANT_FUSED, B.VARIANT_LAYERED]


def _haar(rng, B_, m):
    return W.haar_unitaries(rng, B_, m).astype(np.complex64)


def _check_against_oracle(batch, U64, occ, out, amplitudes, samples=None, tol=None):
    samples = range(batch.B) if samples is None else samples
    worst = 0.0
    for b in samples:
        o0, o1 = batch.offsets[b], batch.offsets[b + 1]
        ref = O.amplitudes(widen(U64[b]), occ[b]) if amplitudes else O.probabilities(widen(U64[b]), occ[b])
        assert o1 - o0 == ref.size
        worst = max(worst, float(np.abs(out[o0:o1] - ref).max()))
    assert worst <= (tol or (A_TOL if amplitudes else P_TOL)), worst
    return worst


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("amplitudes", [False, True])
def test_haar_m6_n3_b64_full(variant, amplitudes):
    wl = W.make("haar_m6_n3_b64")
    say("haar_m6_n3_b64", variant, amplitudes)
    plan = B.Plan(wl.m, 3)
    batch = B.Batch(plan, wl.occ)
    op = B.OP_AMPLITUDES if amplitudes else B.OP_PROBS
    batch.set_config(op, variant)
    out = run_forward(batch, to_dev_c64(wl.U), amplitudes)
    worst = _check_against_oracle(batch, wl.U, wl.occ, out, amplitudes)
    say("  max err", worst)


@pytest.mark.parametrize("variant", VARIANTS)
def test_haar_m16_n6_b256(variant):
    wl = W.make("haar_m16_n6_b256")
    say("haar_m16_n6_b256", variant)
    plan = B.Plan(wl.m, 6)
    batch = B.Batch(plan, wl.occ)
    batch.set_config(B.OP_PROBS, variant)
    batch.set_config(B.OP_AMPLITUDES, variant)
    U = to_dev_c64(wl.U)
    p = run_forward(batch, U, False)
    a = run_forward(batch, U, True)
    N = fock_dim(16, 6)
    assert p.size == 256 * N
    # full oracle comparison on a spread of samples
    _check_against_oracle(batch, wl.U, wl.occ, p, False, samples=[0, 1, 77, 128, 200, 255])
    _check_against_oracle(batch, wl.U, wl.occ, a, True, samples=[3, 254])
    # invariants on every sample
    pb = p.reshape(256, N)
    assert np.abs(pb.sum(axis=1) - 1).max() < 2e-5
    assert np.abs(np.abs(a.reshape(256, N)) ** 2 - pb).max() < 1e-6


@pytest.mark.parametrize("variant", VARIANTS)
def test_mixed_photon_numbers_clements_m12(variant):
    wl = W.make("clements_m12_n2to6_b4096")
    say("clements_m12_n2to6_b4096", variant)
    theta = torch.from_numpy(wl.theta).to(DEV)
    x = torch.from_numpy(wl.x).to(DEV)
    U = B.mesh_to_unitary(theta, x, wl.enc_scale)
    plan = B.Plan(wl.m, 6)
    batch = B.Batch(plan, wl.occ)
    batch.set_config(B.OP_PROBS, variant)
    p = run_forward(batch, U, False)
    assert p.size == sum(fock_dim(12, int(n)) for n in wl.n)
    U64 = U.cpu().numpy()
    picks = []
    for n in range(2, 7):
        idx = np.nonzero(wl.n == n)[0]
        picks += list(idx[:3]) + list(idx[-2:])
    _check_against_oracle(batch, U64, wl.occ, p, False, samples=picks)
    for b in range(wl.B):
        o0, o1 = batch.offsets[b], batch.offsets[b + 1]
        assert abs(p[o0:o1].sum() - 1) < 2e-5


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("m,occ", [
    (2, [1, 1]),                     # Hong-Ou-Mandel
    (5, [0, 0, 3, 0, 0]),            # all photons in one mode
    (6, [2, 0, 1, 0, 0, 1]),         # bunched input
    (7, [0, 0, 0, 0, 0, 0, 1]),      # one photon
    (3, [0, 0, 0]),                  # vacuum
    (32, [1, 0, 1] + [0] * 29),      # widest mode count
    (3, [5, 6, 5]),                  # many photons, few modes
    (9, [1, 1, 1, 1, 1, 1, 1, 1, 1]),
])
def test_edge_cases(variant, m, occ):
    say("edge", variant, m, occ)
    rng = np.random.default_rng(m * 31 + sum(occ))
    n = sum(occ)
    Bn = 3
    U = _haar(rng, Bn, m)
    if m == 2:
        U[0] = (np.array([[1, 1j], [1j, 1]]) / math.sqrt(2)).astype(np.complex64)
    plan = B.Plan(m, max(n, 1))
    batch = B.Batch(plan, np.tile(np.array(occ, np.int32), (Bn, 1)))
    for amplitudes in (False, True):
        op = B.OP_AMPLITUDES if amplitudes else B.OP_PROBS
        batch.set_config(op, variant)
        out = run_forward(batch, to_dev_c64(U), amplitudes)
        _check_against_oracle(batch, U, batch.occ, out, amplitudes)
    if m == 2:
        p = run_forward(batch, to_dev_c64(U), False)
        assert abs(p[1]) < 1e-7  # coincidence suppressed


@pytest.mark.parametrize("variant", VARIANTS)
def test_ragged_batch_with_every_photon_number(variant):
    m = 8
    rng = np.random.default_rng(5)
    occ = []
    for n in [0, 1, 5, 2, 0, 4, 3, 1, 6, 5]:
        o = np.zeros(m, np.int32)
        for j in rng.integers(0, m, n):
            o[j] += 1
        occ.append(o)
    occ = np.array(occ)
    U = _haar(rng, len(occ), m)
    plan = B.Plan(m, 6)
    batch = B.Batch(plan, occ)
    batch.set_config(B.OP_AMPLITUDES, variant)
    out = run_forward(batch, to_dev_c64(U), True)
    assert out.size == sum(fock_dim(m, int(n)) for n in occ.sum(1))
    _check_against_oracle(batch, U, occ, out, True)


def test_fused_and_layered_agree_and_are_deterministic():
    wl = W.make("haar_m16_n6_b256", B=40)
    plan = B.Plan(wl.m, 6)
    batch = B.Batch(plan, wl.occ)
    U = to_dev_c64(wl.U)
    batch.set_config(B.OP_AMPLITUDES, B.VARIANT_FUSED)
    a1 = run_forward(batch, U, True)
    a2 = run_forward(batch, U, True)
    assert np.array_equal(a1, a2)  # bitwise: no atomics
    batch.set_config(B.OP_AMPLITUDES, B.VARIANT_LAYERED)
    a3 = run_forward(batch, U, True)
    assert np.abs(a1 - a3).max() < 1e-6


def test_large_state_m24_n8_sampled():
    wl = W.make("haar_m24_n8_b16")
    say("haar_m24_n8_b16 forward")
    plan = B.Plan(wl.m, 8)
    batch = B.Batch(plan, wl.occ)
    assert batch.get_config(B.OP_PROBS)[0] == B.VARIANT_LAYERED  # a photon layer exceeds LDS
    U = to_dev_c64(wl.U)
    p = run_forward(batch, U, False)
    N = fock_dim(24, 8)
    assert p.size == 16 * N
    pb = p.reshape(16, N)
    assert np.abs(pb.sum(axis=1, dtype=np.float64) - 1).max() < 1e-4
    rng = np.random.default_rng(2)
    for b in [0, 7, 15]:
        ranks = np.unique(np.r_[0, N - 1, rng.integers(0, N, 300), np.argsort(pb[b])[-20:]])
        outs = np.stack([O.fock_unrank(24, 8, int(r)) for r in ranks])
        ref = O.probabilities(widen(wl.U[b]), wl.occ[b], outputs=outs)
        assert np.abs(pb[b, ranks] - ref).max() <= P_TOL


def test_hip_graph_replay_matches_eager():
    wl = W.make("haar_m6_n3_b64")
    plan = B.Plan(wl.m, 3)
    batch = B.Batch(plan, wl.occ)
    U = to_dev_c64(wl.U)
    eager = run_forward(batch, U, False)
    out = torch.empty(batch.out_len, dtype=torch.float32, device=DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.fock_probs(batch, U, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.fock_probs(batch, U, out=out)
    for rep in range(4):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), rep


@pytest.mark.parametrize("variant,block", [(B.VARIANT_FUSED, 256), (B.VARIANT_FUSED, 512),
                                           (B.VARIANT_FUSED, 1024), (B.VARIANT_LAYERED, 0)])
def test_clements_m20_n5_b512(variant, block):
    """The benchmark's own shape (m=20 Clements mesh with per-sample angle
    encoding, n=5 in modes 0,4,8,12,16, B=512): mesh -> U, then amplitudes and
    probabilities of the whole batch in one launch, compared element by
    element with the oracle on 9 samples, the first and last of the work order
    among them, at every fused workgroup size and in the layered variant."""
    wl = W.make("clements_m20_n5_b512")
    say("clements_m20_n5_b512 forward", variant, block)
    theta = torch.from_numpy(wl.theta).to(DEV)
    x = torch.from_numpy(wl.x).to(DEV)
    U = B.mesh_to_unitary(theta, x, wl.enc_scale)
    batch = B.Batch(B.Plan(wl.m, 5), wl.occ)
    for op in (B.OP_AMPLITUDES, B.OP_PROBS):
        batch.set_config(op, variant, block)
    a = run_forward(batch, U, True)
    p = run_forward(batch, U, False)
    N = fock_dim(20, 5)
    assert a.size == p.size == wl.B * N
    U64 = U.cpu().numpy()
    # every sample has 5 photons, so the largest-first work order is 0..511
    picks = [0, 1, 2, 63, 64, 255, 256, 510, 511]
    worst_a = _check_against_oracle(batch, U64, wl.occ, a, True, samples=picks)
    worst_p = _check_against_oracle(batch, U64, wl.occ, p, False, samples=picks)
    say("  max |da|", worst_a, "max |dp|", worst_p)
    # invariants on every sample: the norm, and p = |a|^2 from the two launches
    pb = p.reshape(wl.B, N)
    assert np.abs(pb.sum(axis=1, dtype=np.float64) - 1).max() < 2e-5
    assert np.abs(np.abs(a.reshape(wl.B, N)) ** 2 - pb).max() < 1e-6


# ------------------------------------------------ two samples per workgroup

@pytest.mark.parametrize("block", [512, 1024])
def test_pairs_variant_clements_m20_n5_b512(block):
    """The two-sample kernel at the benchmark's shape (its two largest layers
    overlap in LDS, so the held-state path runs): oracle on the first and last
    samples of the work order and on pairs' both halves, equal to the
    one-sample kernel on every output."""
    wl = W.make("clements_m20_n5_b512")
    say("pairs variant clements_m20_n5_b512", block)
    U = B.mesh_to_unitary(torch.from_numpy(wl.theta).to(DEV), torch.from_numpy(wl.x).to(DEV), wl.enc_scale)
    batch = B.Batch(B.Plan(wl.m, 5), wl.occ)
    ref = {}
    for op, amp in ((B.OP_PROBS, False), (B.OP_AMPLITUDES, True)):
        batch.set_config(op, B.VARIANT_FUSED, 1024)
        ref[amp] = run_forward(batch, U, amp)
        batch.set_config(op, B.VARIANT_FUSED_PAIRS, block)
        assert batch.get_config(op) == (B.VARIANT_FUSED_PAIRS, block)
    p = run_forward(batch, U, False)
    a = run_forward(batch, U, True)
    U64 = U.cpu().numpy()
    picks = [0, 1, 2, 3, 254, 255, 510, 511]
    worst_p = _check_against_oracle(batch, U64, wl.occ, p, False, samples=picks)
    worst_a = _check_against_oracle(batch, U64, wl.occ, a, True, samples=picks)
    say("  max |dp|", worst_p, "max |da|", worst_a)
    assert np.abs(p - ref[False]).max() <= 1e-7
    assert np.abs(a - ref[True]).max() <= 1e-7


def test_pairs_variant_mixed_batch_with_lone_samples():
    """Mixed photon numbers (odd counts leave samples without a partner),
    vacua, bunched inputs, and pairs whose two samples have different input
    modes: every sample against the oracle."""
    rng = np.random.default_rng(77)
    m = 9
    occ = []
    for n in [4, 4, 4, 3, 0, 2, 2, 5, 0, 3, 1]:
        o = np.zeros(m, np.int32)
        for j in rng.integers(0, m, n):
            o[j] += 1
        occ.append(o)
    occ = np.array(occ)
    U = _haar(rng, len(occ), m)
    batch = B.Batch(B.Plan(m, 5), occ)
    for op in (B.OP_PROBS, B.OP_AMPLITUDES):
        batch.set_config(op, B.VARIANT_FUSED_PAIRS, 512)
    Ud = to_dev_c64(U)
    for amp in (False, True):
        out = run_forward(batch, Ud, amp)
        _check_against_oracle(batch, U, occ, out, amp)


def test_pairs_variant_unsupported_and_measurement_forwards():
    # layers of two samples that do not fit LDS are refused; measurement forwards built on probabilities use it
    big = B.Batch(B.Plan(16, 6), np.tile(np.array([1] * 6 + [0] * 10, np.int32), (2, 1)))
    with pytest.raises(B.SlosError):
        big.set_config(B.OP_PROBS, B.VARIANT_FUSED_PAIRS, 1024)
    with pytest.raises(B.SlosError):
        big.set_config(B.OP_PROBS_BACKWARD, B.VARIANT_FUSED_PAIRS, 1024)
    rng = np.random.default_rng(5)
    m, Bn = 8, 9
    U = _haar(rng, Bn, m)
    occ = np.zeros((Bn, m), np.int32)
    occ[:, :3] = 1
    batch = B.Batch(B.Plan(m, 3, threshold=True), occ)
    Ud = to_dev_c64(U)
    batch.set_config(B.OP_THRESHOLD_PROBS, B.VARIANT_FUSED)
    ref = B.fock_threshold_probs(batch, Ud).cpu().numpy()
    batch.set_config(B.OP_THRESHOLD_PROBS, B.VARIANT_FUSED_PAIRS)
    got = B.fock_threshold_probs(batch, Ud).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-7
