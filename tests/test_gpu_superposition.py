"""GPU parity of amplitude-encoded (superposition) inputs: sum_c x_c U|s_c>
per group and its adjoint (dL/dU per group, dL/dx per component), against
the FP64 oracle on the GPU's own complex64 inputs.

Tolerance: with sum |x_c|^2 = 1 per group the output sums at most a few
components' amplitudes, each within 1e-5 of the oracle's: 2e-5 absolute;
gradients to the relative bar 1e-4."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import oracle as O
from paper_2602_11092_amd import _binding as B
from paper_2602_11092_amd.autograd import fock_superposition_amplitudes
from tests.gpu_util import DEV, G_RTOL, rel_err, say, to_dev_c64, widen

pytestmark = pytest.mark.gpu

S_TOL = 2e-5
VARIANTS = [B.VARIANT_FUSED, B.VARIANT_LAYERED]


def _groups(seed, m, G, n_choices, k_max):
    """G groups of 1..k_max distinct n-photon components, random weights of unit norm."""
    rng = np.random.default_rng(seed)
    occ, off, xs = [], [0], []
    for g in range(G):
        n = int(rng.choice(n_choices))
        basis = O.fock_basis(m, n)
        k = int(rng.integers(1, min(k_max, len(basis)) + 1))
        pick = rng.choice(len(basis), size=k, replace=False)
        x = rng.standard_normal(k) + 1j * rng.standard_normal(k)
        x /= np.linalg.norm(x)
        occ += [basis[i] for i in pick]
        xs += list(x)
        off.append(off[-1] + k)
    U = W.haar_unitaries(rng, G, m).astype(np.complex64)
    return np.array(occ, dtype=np.int32), np.array(off), np.array(xs, dtype=np.complex64), U


def _setup(occ, off, variant):
    batch = B.Batch(B.Plan(occ.shape[1], int(occ.sum(1).max())), occ)
    batch.set_config(B.OP_AMPLITUDES, variant, 0)
    batch.set_config(B.OP_AMPLITUDES_BACKWARD, variant, 0)
    return batch, B.Superposition(batch, off)


@pytest.mark.parametrize("variant", VARIANTS)
def test_superposition_forward(variant):
    m = 5
    occ, off, x, U = _groups(1, m, 12, [1, 2, 3, 4], 6)
    batch, sup = _setup(occ, off, variant)
    say("superposition forward m5 variant", variant)
    out = B.fock_superposition_amplitudes(sup, to_dev_c64(U), torch.from_numpy(x).to(DEV))
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    for g in range(sup.G):
        c0, c1 = off[g], off[g + 1]
        ref = O.superposition_amplitudes(widen(U[g]), occ[c0:c1], x[c0:c1].astype(np.complex128))
        o0, o1 = sup.out_offsets[g], sup.out_offsets[g + 1]
        assert o1 - o0 == ref.size
        assert np.abs(out[o0:o1] - ref).max() <= S_TOL, g


def test_reversed_hong_ou_mandel():
    bs = (np.array([[1, 1j], [1j, 1]]) / np.sqrt(2)).astype(np.complex64)[None]
    occ = np.array([[2, 0], [0, 2]], dtype=np.int32)
    x = np.array([1, 1], dtype=np.complex64) / np.sqrt(2)
    for variant in VARIANTS:
        batch, sup = _setup(occ, [0, 2], variant)
        out = B.fock_superposition_amplitudes(sup, to_dev_c64(bs), torch.from_numpy(x.astype(np.complex64)).to(DEV))
        assert np.abs(out.cpu().numpy() - [0, 1j, 0]).max() <= 1e-6


@pytest.mark.parametrize("variant", VARIANTS)
def test_superposition_backward(variant):
    m = 5
    occ, off, x, U = _groups(2, m, 8, [2, 3], 5)
    batch, sup = _setup(occ, off, variant)
    rng = np.random.default_rng(3)
    G = (rng.standard_normal(sup.out_len) + 1j * rng.standard_normal(sup.out_len)).astype(np.complex64)
    say("superposition backward variant", variant)
    gU, gx = B.fock_superposition_amplitudes_backward(sup, to_dev_c64(U), torch.from_numpy(x).to(DEV),
                                                      torch.from_numpy(G).to(DEV))
    torch.cuda.synchronize()
    gU, gx = gU.cpu().numpy(), gx.cpu().numpy()
    for g in range(sup.G):
        c0, c1 = off[g], off[g + 1]
        o0, o1 = sup.out_offsets[g], sup.out_offsets[g + 1]
        Gg = G[o0:o1].astype(np.complex128)
        Ug = widen(U[g])
        ref_U = sum(O.amplitude_grad(Ug, occ[c], np.conj(np.complex128(x[c])) * Gg) for c in range(c0, c1))
        assert rel_err(gU[g], ref_U) <= G_RTOL, g
        for c in range(c0, c1):
            ref_x = np.vdot(O.amplitudes(Ug, occ[c]), Gg)
            assert abs(gx[c] - ref_x) <= G_RTOL * max(1.0, abs(ref_x)), (g, c)


def test_superposition_autograd_and_edge_cases():
    m = 4
    occ, off, x, U = _groups(4, m, 3, [2], 4)
    batch, sup = _setup(occ, off, B.VARIANT_FUSED)
    Ut = to_dev_c64(U).requires_grad_(True)
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    out = fock_superposition_amplitudes(Ut, xt, sup)
    w = torch.randn(out.shape[0], dtype=torch.complex64, device=DEV)
    (out.conj() * w).real.sum().backward()
    gU, gx = B.fock_superposition_amplitudes_backward(sup, Ut.detach(), xt.detach(), w)
    assert torch.allclose(Ut.grad, gU) and torch.allclose(xt.grad, gx)
    with pytest.raises(B.SlosError):  # offsets must end at the batch size
        B.Superposition(batch, [0, 1])
    # a single component with weight 1 is the plain amplitude vector
    b1 = B.Batch(B.Plan(m, 2), occ[:1])
    s1 = B.Superposition(b1, [0, 1])
    a = B.fock_superposition_amplitudes(s1, to_dev_c64(U[:1]), torch.ones(1, dtype=torch.complex64, device=DEV))
    ref = B.fock_amplitudes(b1, to_dev_c64(U[:1]))
    assert torch.equal(a, ref)
    # offsets out of order, or past the batch, are rejected before any is used
    with pytest.raises(B.SlosError):
        B.Superposition(batch, [0, 5, 3] if batch.B == 3 else [0, batch.B + 2, batch.B])
    with pytest.raises(B.SlosError):
        B.Superposition(batch, [0, 0, batch.B])  # an empty group
    # a group mixing photon numbers is rejected
    bad = B.Batch(B.Plan(m, 3), np.array([[1, 1, 0, 0], [1, 1, 1, 0]], dtype=np.int32))
    with pytest.raises(B.SlosError):
        B.Superposition(bad, [0, 2])


# ------------------------------------------------- one shared interferometer

@pytest.mark.parametrize("m,n,G", [(4, 2, 5), (6, 3, 64), (8, 4, 33)])
def test_shared_superposition_against_oracle(m, n, G):
    rng = np.random.default_rng(50 + m)
    U = W.haar_unitaries(rng, 1, m).astype(np.complex64)[0]
    s = B.SharedSuperposition(B.Plan(m, n), n)
    N = s.N
    assert N == O.fock_dim(m, n)
    X = ((rng.standard_normal((G, N)) + 1j * rng.standard_normal((G, N))) / np.sqrt(2 * N)).astype(np.complex64)
    Ud = to_dev_c64(U)
    Xd = torch.from_numpy(X).to(DEV)
    say("shared superposition m", m, "n", n, "G", G)
    out = B.fock_shared_superposition_amplitudes(s, Ud, Xd).cpu().numpy()
    basis = O.fock_basis(m, n)
    # Uhat's rows from the oracle: A[c] = a(U, basis_c)
    A = np.stack([O.amplitudes(widen(U), basis[c]) for c in range(N)])
    ref = X.astype(np.complex128) @ A
    assert np.abs(out - ref).max() <= S_TOL
    Gd = ((rng.standard_normal((G, N)) + 1j * rng.standard_normal((G, N)))).astype(np.complex64)
    gU, gX = B.fock_shared_superposition_amplitudes_backward(s, Ud, Xd, torch.from_numpy(Gd).to(DEV))
    torch.cuda.synchronize()
    gU, gX = gU.cpu().numpy(), gX.cpu().numpy()
    G64 = Gd.astype(np.complex128)
    assert rel_err(gX, G64 @ A.conj().T) <= G_RTOL
    gA = X.astype(np.complex128).conj().T @ G64  # dL/dA[c][t]
    ref_U = sum(O.amplitude_grad(widen(U), basis[c], gA[c]) for c in range(N))
    assert rel_err(gU, ref_U) <= G_RTOL


def test_shared_superposition_is_unitary_and_trains():
    # Uhat is unitary on the n-photon space: orthonormal inputs stay orthonormal
    m, n = 5, 3
    rng = np.random.default_rng(61)
    s = B.SharedSuperposition(B.Plan(m, n), n)
    N = s.N
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    X = torch.from_numpy(Q[:8].astype(np.complex64)).to(DEV)
    U = to_dev_c64(W.haar_unitaries(rng, 1, m)[0]).requires_grad_(True)
    from paper_2602_11092_amd.autograd import fock_shared_superposition_amplitudes
    out = fock_shared_superposition_amplitudes(U, X, s)
    gram = (out @ out.conj().T).detach().cpu().numpy()
    assert np.abs(gram - np.eye(8)).max() <= 1e-5
    out.abs().pow(2)[:, 0].sum().backward()
    assert U.grad is not None and torch.isfinite(U.grad.abs()).all()


def test_amplitude_encoded_layer_trains_against_oracle():
    from paper_2602_11092_amd import AmplitudeEncodedLayer
    m, n = 5, 2
    layer = AmplitudeEncodedLayer(m, n, measurement="probs").to(DEV)
    N = layer.state_size
    rng = np.random.default_rng(70)
    X = rng.standard_normal((6, N)) + 1j * rng.standard_normal((6, N))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Xd = torch.from_numpy(X.astype(np.complex64)).to(DEV)
    w = torch.from_numpy(rng.standard_normal((6, N)).astype(np.float32)).to(DEV)
    p = layer(Xd)
    (p * w).sum().backward()
    torch.cuda.synchronize()
    th = layer.theta.detach().cpu().numpy().astype(np.float64)
    U = O.mesh_unitary(th, m)
    basis = O.fock_basis(m, n)
    A = np.stack([O.amplitudes(U, basis[c]) for c in range(N)])
    X64 = Xd.cpu().numpy().astype(np.complex128)
    out = X64 @ A
    assert np.abs(p.detach().cpu().numpy() - np.abs(out) ** 2).max() <= 1e-5
    assert np.abs(p.detach().cpu().numpy().sum(1) - 1).max() <= 1e-5  # normalised inputs stay normalised
    # chain: dL/dout = 2 w out, dL/dA = X^H (2 w out), then the amplitude and mesh gradients
    gout = 2 * w.cpu().numpy().astype(np.float64) * out
    gA = X64.conj().T @ gout
    GU = sum(O.amplitude_grad(U, basis[c], gA[c]) for c in range(N))
    rt, _ = O.mesh_grad(th, None, 0.0, GU)
    assert rel_err(layer.theta.grad.cpu().numpy(), rt) <= G_RTOL
