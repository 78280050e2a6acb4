"""The allocation-free mesh adjoint (static device scratch, no workspace
argument) against the workspace entry point: two calls in a row, the second
with a smaller input, bit for bit; and the host-side size limit."""
import math

import numpy as np
import pytest
import torch

from paper_2602_11092_amd import _binding as B
from tests.gpu_util import DEV, say

pytestmark = pytest.mark.gpu


def _inputs(rng, m, Bn):
    theta = torch.from_numpy(rng.uniform(0, 2 * math.pi, m * (m - 1)).astype(np.float32)).to(DEV)
    x = torch.from_numpy(rng.standard_normal((Bn, m)).astype(np.float32)).to(DEV)
    gU = torch.from_numpy((rng.standard_normal((Bn, m, m)) + 1j * rng.standard_normal((Bn, m, m)))
                          .astype(np.complex64)).to(DEV)
    return theta, x, gU


def test_mesh_adjoint_noalloc_matches_workspace_call():
    rng = np.random.default_rng(2026)
    cases = [(20, 512), (12, 37)]  # the second call is smaller
    inputs = [_inputs(rng, m, Bn) for m, Bn in cases]
    outs = []
    for (m, Bn), (theta, x, gU) in zip(cases, inputs):
        say("noalloc mesh adjoint m", m, "B", Bn)
        gt = torch.full((m * (m - 1),), float("nan"), device=DEV)
        gx = torch.full((Bn, m), float("nan"), device=DEV)
        B.mesh_to_unitary_backward_noalloc(theta, x, math.pi, gU, gt, gx)
        outs.append((gt, gx))
    torch.cuda.synchronize()
    for (m, Bn), (theta, x, gU), (gt, gx) in zip(cases, inputs, outs):
        ws = torch.empty(B.WorkspaceCache._round(B.mesh_workspace(m, Bn, DEV).numel()), dtype=torch.uint8,
                         device=DEV)
        rt, rx = B.mesh_to_unitary_backward(theta, x, math.pi, gU, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(gt, rt), (m, Bn)
        assert torch.equal(gx, rx), (m, Bn)
    # no features: grad_x must be absent, B = 1
    theta, _, gU = _inputs(rng, 6, 1)
    gt = torch.empty(30, device=DEV)
    B.mesh_to_unitary_backward_noalloc(theta, None, 0.0, gU, gt)
    rt, _ = B.mesh_to_unitary_backward(theta, None, 0.0, gU)
    torch.cuda.synchronize()
    assert torch.equal(gt, rt)


def test_mesh_adjoint_noalloc_rejects_sizes_beyond_its_scratch():
    m, Bn = 32, 1100  # 2048 complex per sample at m = 32: more than 16 MiB
    theta = torch.zeros(m * (m - 1), device=DEV)
    x = torch.zeros(Bn, m, device=DEV)
    gU = torch.zeros(Bn, m, m, dtype=torch.complex64, device=DEV)
    gt = torch.empty_like(theta)
    with pytest.raises(B.SlosError) as e:
        B.mesh_to_unitary_backward_noalloc(theta, x, math.pi, gU, gt)
    assert e.value.code == B.SLOS_EUNSUPPORTED
