"""GPU adjoint parity: dL/dU from the hand-written backward kernels against
the oracle's minor-permanent gradient, the closed form of d(sum p)/dU, and
FP64 central finite differences through the whole chain theta, x -> U -> p ->
readout cross-entropy."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import oracle as O
from paper_2602_11092_amd import _binding as B
from tests.gpu_util import DEV, G_RTOL, fock_dim, rel_err, say, to_dev_c64, widen

pytestmark = pytest.mark.gpu

VARIANTS = [B.VARIANT_FUSED, B.VARIANT_LAYERED]


def _grad(batch, U_dev, gin, probs):
    g = (B.fock_probs_backward(batch, U_dev, gin) if probs else B.fock_amplitudes_backward(batch, U_dev, gin))
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("m,occ", [
    (6, [1, 1, 1, 0, 0, 0]),
    (4, [2, 0, 1, 0]),
    (5, [0, 3, 0, 0, 0]),
    (7, [0, 0, 1, 0, 0, 0, 0]),
    (3, [0, 0, 0]),
    (9, [1, 0, 1, 0, 1, 0, 1, 0, 1]),
    (12, [1, 1, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0]),
    (20, [1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0]),
])
def test_backward_against_oracle(variant, m, occ):
    say("bwd", variant, m, occ)
    rng = np.random.default_rng(100 + m + sum(occ))
    Bn = 2
    U = W.haar_unitaries(rng, Bn, m).astype(np.complex64)
    n = sum(occ)
    plan = B.Plan(m, max(n, 1))
    batch = B.Batch(plan, np.tile(np.array(occ, np.int32), (Bn, 1)))
    N = fock_dim(m, n)
    gp = rng.uniform(0, 1, Bn * N).astype(np.float32)
    ga = (rng.standard_normal(Bn * N) + 1j * rng.standard_normal(Bn * N)).astype(np.complex64)
    Ud = to_dev_c64(U)
    for probs in (True, False):
        op = B.OP_PROBS_BACKWARD if probs else B.OP_AMPLITUDES_BACKWARD
        batch.set_config(op, variant)
        gin = torch.from_numpy(gp if probs else ga).to(DEV)
        G = _grad(batch, Ud, gin, probs)
        for b in range(Bn):
            sl = slice(b * N, (b + 1) * N)
            if n == 0:
                assert np.abs(G[b]).max() == 0
                continue
            ref = O.probs_grad(widen(U[b]), occ, gp[sl].astype(np.float64)) if probs else \
                O.amplitude_grad(widen(U[b]), occ, ga[sl].astype(np.complex128))
            e = rel_err(G[b], ref)
            assert e <= G_RTOL, (probs, b, e)
            # columns without input photons get exactly zero
            for i in range(m):
                if occ[i] == 0:
                    assert np.abs(G[b][:, i]).max() == 0


@pytest.mark.parametrize("variant", VARIANTS)
def test_total_probability_gradient_closed_form(variant):
    # L = sum_t p_t = 1 for unitary U, and dL/dU = 2 s_i U[:, i]
    wl = W.make("clements_m20_n5_b512", B=64)
    U = B.mesh_to_unitary(torch.from_numpy(wl.theta).to(DEV), torch.from_numpy(wl.x).to(DEV), wl.enc_scale)
    plan = B.Plan(wl.m, 5)
    batch = B.Batch(plan, wl.occ)
    batch.set_config(B.OP_PROBS_BACKWARD, variant)
    ones = torch.ones(batch.out_len, dtype=torch.float32, device=DEV)
    G = _grad(batch, U, ones, True)
    ref = 2.0 * U.cpu().numpy().astype(np.complex128) * wl.occ[:, None, :]
    assert rel_err(G, ref) < 1e-5


def test_c4_shape_gradient_against_oracle():
    """m=20, n=5, readout cross-entropy: G_U of sampled samples vs the oracle."""
    wl = W.make("clements_m20_n5_b512")
    say("clements_m20_n5_b512 gradient")
    theta = torch.from_numpy(wl.theta).to(DEV)
    x = torch.from_numpy(wl.x).to(DEV)
    U = B.mesh_to_unitary(theta, x, wl.enc_scale)
    plan = B.Plan(wl.m, 5)
    batch = B.Batch(plan, wl.occ)
    assert batch.get_config(B.OP_PROBS_BACKWARD)[0] == B.VARIANT_FUSED
    p = B.fock_probs(batch, U)
    torch.cuda.synchronize()
    N = fock_dim(20, 5)
    pn = p.cpu().numpy().reshape(wl.B, N)
    L, gp = O.readout_cross_entropy(pn, wl.readout_W, wl.readout_b, wl.labels)
    gp32 = torch.from_numpy(gp.astype(np.float32).ravel()).to(DEV)
    G = _grad(batch, U, gp32, True)
    U64 = U.cpu().numpy()
    for b in [0, 1, 255, 511]:
        ref = O.probs_grad(widen(U64[b]), wl.occ[b], gp[b].astype(np.float32).astype(np.float64))
        e = rel_err(G[b], ref)
        say("  sample", b, "rel err", e)
        assert e <= G_RTOL


def _oracle_loss(theta64, x64, wl, idx):
    Us = O.encoded_unitaries(theta64, x64[idx], wl.enc_scale)
    p = np.stack([O.probabilities(Us[i], wl.occ[b]) for i, b in enumerate(idx)])
    return O.readout_cross_entropy(p, wl.readout_W, wl.readout_b, wl.labels[idx])[0]


def test_full_chain_against_fp64_finite_differences():
    """theta -> U -> p -> readout CE on 8 samples of the m=20, n=5 workload:
    GPU gradient (mesh adjoint after SLOS adjoint) vs central differences
    (h = 1e-6) of the FP64 oracle loss on 16 seeded phases and 8 features."""
    wl = W.make("clements_m20_n5_b512")
    idx = np.arange(8)
    theta = torch.from_numpy(wl.theta).to(DEV)
    x = torch.from_numpy(wl.x[idx].copy()).to(DEV)
    U = B.mesh_to_unitary(theta, x, wl.enc_scale)
    plan = B.Plan(wl.m, 5)
    batch = B.Batch(plan, wl.occ[idx])
    p = B.fock_probs(batch, U)
    torch.cuda.synchronize()
    N = fock_dim(20, 5)
    pn = p.cpu().numpy().reshape(8, N).astype(np.float64)
    _, gp = O.readout_cross_entropy(pn, wl.readout_W, wl.readout_b, wl.labels[idx])
    gU = B.fock_probs_backward(batch, U, torch.from_numpy(gp.astype(np.float32).ravel()).to(DEV))
    gt, gx = B.mesh_to_unitary_backward(theta, x, wl.enc_scale, gU)
    torch.cuda.synchronize()
    gt = gt.cpu().numpy().astype(np.float64)
    gx = gx.cpu().numpy().astype(np.float64)
    th64 = wl.theta.astype(np.float64)
    x64 = wl.x.astype(np.float64)
    rng = np.random.default_rng(7)
    qs = rng.choice(th64.size, 16, replace=False)
    h = 1e-6
    fd = []
    for q in qs:
        e = np.zeros_like(th64)
        e[q] = h
        fd.append((_oracle_loss(th64 + e, x64, wl, idx) - _oracle_loss(th64 - e, x64, wl, idx)) / (2 * h))
    e_theta = rel_err(gt[qs], np.array(fd))
    say("  theta FD rel err", e_theta)
    assert e_theta <= G_RTOL
    fdx = []
    picks = [(0, 0), (1, 5), (3, 19), (7, 10), (2, 4), (5, 8), (6, 16), (4, 12)]
    for (b, k) in picks:
        e = np.zeros_like(x64)
        e[b, k] = h
        fdx.append((_oracle_loss(th64, x64 + e, wl, idx) - _oracle_loss(th64, x64 - e, wl, idx)) / (2 * h))
    e_x = rel_err(np.array([gx[b, k] for b, k in picks]), np.array(fdx))
    say("  x FD rel err", e_x)
    assert e_x <= G_RTOL


def test_large_state_m24_n8_gradients():
    """m=24, n=8 (layered, layers recomputed): closed form for sum p, and a
    sparse weighted loss whose exact gradient the oracle computes from the
    few outputs it touches."""
    wl = W.make("haar_m24_n8_b16")
    say("haar_m24_n8_b16 gradient")
    plan = B.Plan(wl.m, 8)
    batch = B.Batch(plan, wl.occ)
    U = to_dev_c64(wl.U)
    N = fock_dim(24, 8)
    G1 = _grad(batch, U, torch.ones(batch.out_len, dtype=torch.float32, device=DEV), True)
    ref1 = 2.0 * widen(wl.U) * wl.occ[:, None, :]
    assert rel_err(G1, ref1) < 1e-5
    rng = np.random.default_rng(3)
    w = np.zeros((16, N), np.float32)
    support = np.unique(rng.integers(0, N, 120))
    w[:, support] = rng.uniform(0, 1, support.size).astype(np.float32)
    G2 = _grad(batch, U, torch.from_numpy(w.ravel()).to(DEV), True)
    outs = np.stack([O.fock_unrank(24, 8, int(r)) for r in support])
    for b in [0, 9]:
        ref = O.probs_grad(widen(wl.U[b]), wl.occ[b], w[b, support].astype(np.float64), outputs=outs)
        e = rel_err(G2[b], ref)
        say("  sample", b, "sparse-loss rel err", e)
        assert e <= G_RTOL


def test_large_state_m24_n8_dense_loss_directional_fd():
    """m=24, n=8 on the workload's own loss, L = sum_b sum_t w_t p_bt with a
    dense w ~ U[0,1) over all 7,888,725 outputs (layered adjoint, layers
    recomputed): <G_U, V> against FP64 central differences (h = 1e-6) of the
    oracle loss, for the first and last sample and two seeded directions
    each.  Each direction V lives on one output mode's row j of U, so the
    outputs with t_j = 0 keep their probability at U +- hV and drop out of the
    difference exactly; the oracle evaluates the rest, a quarter of the basis,
    by Ryser permanents."""
    wl = W.make("haar_m24_n8_b16")
    say("haar_m24_n8_b16 dense-loss gradient")
    plan = B.Plan(wl.m, 8)
    batch = B.Batch(plan, wl.occ)
    U = to_dev_c64(wl.U)
    gp = torch.from_numpy(np.tile(wl.loss_w, wl.B)).to(DEV)
    G = _grad(batch, U, gp, True)
    del gp
    basis = O.fock_basis(24, 8)  # the basis order of the outputs
    say("  basis enumerated")
    w64 = wl.loss_w.astype(np.float64)
    rng = np.random.default_rng(55)
    h = 1e-6
    got, fd = [], []
    for b in (0, wl.B - 1):
        U64 = widen(wl.U[b])
        for _ in range(2):
            j = int(rng.integers(0, 24))
            V = np.zeros((24, 24), np.complex128)
            V[j, :] = rng.standard_normal(24) + 1j * rng.standard_normal(24)
            sel = basis[:, j] >= 1
            outs, ws = basis[sel], w64[sel]
            Lp = O.weighted_sum(O.probabilities(U64 + h * V, wl.occ[b], outs)[None, :], ws)[0]
            Lm = O.weighted_sum(O.probabilities(U64 - h * V, wl.occ[b], outs)[None, :], ws)[0]
            fd.append((Lp - Lm) / (2 * h))
            got.append(float(np.real(np.sum(np.conj(G[b]) * V))))
            say("  sample", b, "row", j, "gpu", got[-1], "fd", fd[-1])
    e = rel_err(np.array(got), np.array(fd))
    say("  directional rel err", e)
    assert e <= G_RTOL


def test_backward_deterministic_and_variants_agree():
    wl = W.make("clements_m20_n5_b512", B=24)
    U = B.mesh_to_unitary(torch.from_numpy(wl.theta).to(DEV), torch.from_numpy(wl.x).to(DEV), wl.enc_scale)
    plan = B.Plan(wl.m, 5)
    batch = B.Batch(plan, wl.occ)
    rng = np.random.default_rng(9)
    gp = torch.from_numpy(rng.uniform(0, 1, batch.out_len).astype(np.float32)).to(DEV)
    batch.set_config(B.OP_PROBS_BACKWARD, B.VARIANT_FUSED)
    g1 = _grad(batch, U, gp, True)
    g2 = _grad(batch, U, gp, True)
    assert np.array_equal(g1, g2)
    batch.set_config(B.OP_PROBS_BACKWARD, B.VARIANT_LAYERED)
    g3 = _grad(batch, U, gp, True)
    assert rel_err(g3, g1) < 1e-5


@pytest.mark.parametrize("block", [256, 512, 768, 1024])
def test_fused_adjoint_every_workgroup_size(block):
    """Every fused adjoint shape the autotuner may pick (256/512/768/1024
    threads, with their own per-thread state counts) against the oracle."""
    rng = np.random.default_rng(4242 + block)
    m, n, Bn = 12, 4, 6
    U = W.haar_unitaries(rng, Bn, m).astype(np.complex64)
    occ = np.zeros((Bn, m), dtype=np.int32)
    for b in range(Bn):
        for i in rng.choice(m, size=n, replace=True):
            occ[b, i] += 1
    say("fused adjoint block", block)
    plan = B.Plan(m, n)
    batch = B.Batch(plan, occ)
    batch.set_config(B.OP_PROBS_BACKWARD, B.VARIANT_FUSED, block)
    assert batch.get_config(B.OP_PROBS_BACKWARD) == (B.VARIANT_FUSED, block)
    Ud = to_dev_c64(U)
    gp = rng.random(batch.out_len).astype(np.float32)
    G = B.fock_probs_backward(batch, Ud, torch.from_numpy(gp).to(DEV))
    torch.cuda.synchronize()
    G = G.cpu().numpy()
    for b in range(Bn):
        sl = slice(batch.offsets[b], batch.offsets[b + 1])
        ref = O.probs_grad(widen(U[b]), occ[b], gp[sl].astype(np.float64))
        assert rel_err(G[b], ref) <= G_RTOL, (block, b, rel_err(G[b], ref))


@pytest.mark.parametrize("block", [256, 512, 768, 1024])
def test_fused_adjoint_mixed_photon_numbers(block):
    """One batch with n_b from 0 to 5 photons at m = 10: the smallest layers
    kept in LDS are sized for the largest n, and a sample with fewer photons
    keeps fewer of them (at this size the spare LDS can hold all of d_0..d_3,
    286 states, in which case the n = 5 samples recompute no lower layer)."""
    rng = np.random.default_rng(777 + block)
    m = 10
    ns = [5, 4, 3, 2, 1, 0, 5, 3, 2]
    occ = np.zeros((len(ns), m), dtype=np.int32)
    for b, n in enumerate(ns):
        for i in rng.choice(m, size=n, replace=True):
            occ[b, i] += 1
    U = W.haar_unitaries(rng, len(ns), m).astype(np.complex64)
    say("fused adjoint, mixed photon numbers, block", block)
    plan = B.Plan(m, 5)
    batch = B.Batch(plan, occ)
    batch.set_config(B.OP_PROBS_BACKWARD, B.VARIANT_FUSED, block)
    gp = rng.random(batch.out_len).astype(np.float32)
    G = B.fock_probs_backward(batch, to_dev_c64(U), torch.from_numpy(gp).to(DEV))
    torch.cuda.synchronize()
    G = G.cpu().numpy()
    for b, n in enumerate(ns):
        if n == 0:
            assert np.abs(G[b]).max() == 0
            continue
        sl = slice(batch.offsets[b], batch.offsets[b + 1])
        ref = O.probs_grad(widen(U[b]), occ[b], gp[sl].astype(np.float64))
        assert rel_err(G[b], ref) <= G_RTOL, (block, b, n, rel_err(G[b], ref))


@pytest.mark.parametrize("m,n,block", [(20, 5, 512), (20, 5, 768), (20, 5, 1024), (16, 5, 1024),
                                         (24, 4, 512), (32, 3, 256), (32, 3, 512)])
def test_fused_adjoint_full_slots_and_wide_columns(m, n, block):
    """The fused adjoint where layer n-1 fills most owned slots (18 per thread
    at 512 threads for m=20, n=5) and for the 24- and 32-mode instances,
    with bunched inputs, against the oracle: every chunk, the per-wave slot
    skipping and the table-free narrow pull run over full ranges."""
    rng = np.random.default_rng(7000 + 97 * m + n + block)
    Bn = 3
    U = W.haar_unitaries(rng, Bn, m).astype(np.complex64)
    occ = np.zeros((Bn, m), dtype=np.int32)
    for b in range(Bn):
        for i in rng.choice(m, size=n, replace=True):
            occ[b, i] += 1
    say("fused adjoint m", m, "n", n, "block", block)
    batch = B.Batch(B.Plan(m, n), occ)
    batch.set_config(B.OP_PROBS_BACKWARD, B.VARIANT_FUSED, block)
    assert batch.get_config(B.OP_PROBS_BACKWARD) == (B.VARIANT_FUSED, block)
    gp = rng.random(batch.out_len).astype(np.float32)
    G = B.fock_probs_backward(batch, to_dev_c64(U), torch.from_numpy(gp).to(DEV))
    torch.cuda.synchronize()
    G = G.cpu().numpy()
    for b in range(Bn):
        sl = slice(batch.offsets[b], batch.offsets[b + 1])
        ref = O.probs_grad(widen(U[b]), occ[b], gp[sl].astype(np.float64))
        assert rel_err(G[b], ref) <= G_RTOL, (m, n, block, b, rel_err(G[b], ref))


def test_autograd_resolves_lazy_conjugate_gradients():
    # L = Re(sum conj(a) w) hands the amplitude adjoint a lazily conjugated
    # gradient view; the wrapper must pass its values, not its raw memory
    from paper_2602_11092_amd.autograd import fock_amplitudes
    rng = np.random.default_rng(17)
    m, B_ = 5, 6
    U64 = W.haar_unitaries(rng, B_, m)
    occ = np.zeros((B_, m), dtype=np.int32)
    occ[:, :3] = 1
    batch = B.Batch(B.Plan(m, 3), occ)
    U = to_dev_c64(U64).requires_grad_(True)
    a = fock_amplitudes(U, batch)
    w = torch.from_numpy((rng.standard_normal(batch.out_len) + 1j * rng.standard_normal(batch.out_len))
                         .astype(np.complex64)).to(DEV)
    (a.conj() * w).real.sum().backward()
    direct = B.fock_amplitudes_backward(batch, U.detach(), w)
    torch.cuda.synchronize()
    assert torch.allclose(U.grad, direct, rtol=1e-6, atol=1e-7)
    with pytest.raises(ValueError):
        B.fock_amplitudes_backward(batch, U.detach(), w.conj())  # a lazy view is refused
