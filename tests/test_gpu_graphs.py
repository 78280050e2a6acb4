"""HIP-graph capture of the extension entry points: each call is captured
once with preallocated outputs and workspaces, replayed several times with
eager work and synchronisations in between, and every replay must equal the
eager result bit for bit (the calls issue no memsets and allocate nothing)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import oracle as O
from paper_2602_11092_amd import _binding as B
from tests.gpu_util import DEV, say, to_dev_c64

pytestmark = pytest.mark.gpu


def _replays_match(fn, outs, reps=3):
    fn()
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    for rep in range(reps):
        for o in outs:
            o.zero_()
        torch.randn(1 << 16, device=DEV).sum().item()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), rep


@pytest.mark.parametrize("variant", [B.VARIANT_FUSED, B.VARIANT_LAYERED])
def test_graph_measurements(variant):
    rng = np.random.default_rng(12)
    m, Bn = 8, 16
    U = to_dev_c64(W.haar_unitaries(rng, Bn, m))
    occ = np.zeros((Bn, m), dtype=np.int32)
    occ[:, :4] = 1
    batch = B.Batch(B.Plan(m, 4, threshold=True), occ)
    for op in (B.OP_MODE_EXPECTATIONS, B.OP_THRESHOLD_PROBS, B.OP_SAMPLE, B.OP_PROBS_BACKWARD,
               B.OP_MODE_EXPECTATIONS_BACKWARD, B.OP_THRESHOLD_PROBS_BACKWARD):
        batch.set_config(op, variant, 0)
    e = torch.empty((Bn, m), dtype=torch.float32, device=DEV)
    P = torch.empty(batch.threshold_len, dtype=torch.float32, device=DEV)
    u = torch.from_numpy(rng.random((Bn, 128)).astype(np.float32)).to(DEV)
    shots = torch.empty((Bn, 128), dtype=torch.int32, device=DEV)
    we = torch.randn(Bn, m, device=DEV)
    wP = torch.randn(batch.threshold_len, device=DEV)
    gU1, gU2 = torch.empty_like(U), torch.empty_like(U)
    ws = {op: batch.workspace(op, DEV) for op in (B.OP_MODE_EXPECTATIONS, B.OP_THRESHOLD_PROBS, B.OP_SAMPLE,
                                                  B.OP_MODE_EXPECTATIONS_BACKWARD,
                                                  B.OP_THRESHOLD_PROBS_BACKWARD)}
    say("graph measurements variant", variant)

    def fn():
        B.fock_mode_expectations(batch, U, out=e, ws=ws[B.OP_MODE_EXPECTATIONS])
        B.fock_threshold_probs(batch, U, out=P, ws=ws[B.OP_THRESHOLD_PROBS])
        B.fock_sample(batch, U, u, out=shots, ws=ws[B.OP_SAMPLE])
        B.fock_mode_expectations_backward(batch, U, we, out=gU1, ws=ws[B.OP_MODE_EXPECTATIONS_BACKWARD])
        B.fock_threshold_probs_backward(batch, U, wP, out=gU2, ws=ws[B.OP_THRESHOLD_PROBS_BACKWARD])

    _replays_match(fn, [e, P, shots, gU1, gU2])


def test_graph_superposition_and_fidelity():
    rng = np.random.default_rng(13)
    m, n, G = 5, 3, 8
    basis = O.fock_basis(m, n)
    occ = np.tile(basis[:4], (G, 1)).astype(np.int32)
    batch = B.Batch(B.Plan(m, n), occ)
    sup = B.Superposition(batch, np.arange(G + 1) * 4)
    U = to_dev_c64(W.haar_unitaries(rng, G, m))
    x = torch.randn(G * 4, dtype=torch.complex64, device=DEV)
    out = torch.empty(sup.out_len, dtype=torch.complex64, device=DEV)
    gout = torch.randn(sup.out_len, dtype=torch.complex64, device=DEV)
    gU = torch.empty_like(U)
    gx = torch.empty_like(x)
    K = torch.empty((G, G), dtype=torch.float32, device=DEV)
    wf, wb = sup.workspace(False, DEV), sup.workspace(True, DEV)
    Kocc = np.array([1, 1, 0, 1, 0], dtype=np.int32)

    def fn():
        B.fock_superposition_amplitudes(sup, U, x, out=out, ws=wf)
        a, b = B.fock_superposition_amplitudes_backward(sup, U, x, gout, ws=wb)
        gU.copy_(a)
        gx.copy_(b)
        B.fock_fidelity_kernel(Kocc, U, out=K)

    _replays_match(fn, [out, gU, gx, K])


def test_graph_shared_superposition_and_probabilities():
    """The shared-interferometer calls (forward, adjoint with inputs and with
    G = 0, where dL/dA is cleared by a fill kernel) and the probabilities
    of their amplitudes with the adjoint of p = |a|^2."""
    rng = np.random.default_rng(14)
    m, n, G = 5, 2, 12
    ss = B.SharedSuperposition(B.Plan(m, n), n)
    N = ss.N
    U = to_dev_c64(W.haar_unitaries(rng, 1, m)[0])
    X = torch.randn(G, N, dtype=torch.complex64, device=DEV)
    gout = torch.randn(G, N, dtype=torch.complex64, device=DEV)
    out = torch.empty(G, N, dtype=torch.complex64, device=DEV)
    gU, gX, gU0 = torch.empty_like(U), torch.empty_like(X), torch.empty_like(U)
    X0 = torch.empty(0, N, dtype=torch.complex64, device=DEV)
    g0 = torch.empty(0, N, dtype=torch.complex64, device=DEV)
    p = torch.empty(G, N, dtype=torch.float32, device=DEV)
    wp = torch.rand(G, N, device=DEV)
    ga = torch.empty_like(X)
    say("graph shared superposition")

    def fn():
        B.fock_shared_superposition_amplitudes(ss, U, X, out=out)
        a, b = B.fock_shared_superposition_amplitudes_backward(ss, U, X, gout)
        gU.copy_(a)
        gX.copy_(b)
        c, _ = B.fock_shared_superposition_amplitudes_backward(ss, U, X0, g0, need_grad_x=False)
        gU0.copy_(c)
        B.fock_probs_from_amplitudes(out, out=p)
        B.fock_probs_from_amplitudes_backward(out, wp, out=ga)

    _replays_match(fn, [out, gU, gX, gU0, p, ga])
    assert torch.count_nonzero(gU0).item() == 0  # no inputs: zero gradient
