"""torch.autograd.Function wrappers around the library's forward and
adjoint kernels (the hand-written backward of Sec. II-A-3's differentiable
simulation).  Gradients use PyTorch's convention dL/dRe + i dL/dIm, which is
also the library's."""
from __future__ import annotations

import math
from typing import Optional

import torch

from . import _binding as B


def _dense(t: torch.Tensor, dtype) -> torch.Tensor:
    """Plain contiguous memory of t's values (autograd may hand over lazy
    conjugate or negative views, whose memory holds other values)."""
    return t.resolve_conj().resolve_neg().to(dtype).contiguous()


class FockProbs(torch.autograd.Function):
    """U [B, m, m] complex64 -> probabilities float32 [out_len]."""

    @staticmethod
    def forward(ctx, U: torch.Tensor, batch: B.Batch):
        U = _dense(U, torch.complex64)
        ctx.batch = batch
        ctx.save_for_backward(U)
        return B.fock_probs(batch, U)

    @staticmethod
    def backward(ctx, grad_p):
        (U,) = ctx.saved_tensors
        gU = B.fock_probs_backward(ctx.batch, U, _dense(grad_p, torch.float32))
        return gU, None


class FockAmplitudes(torch.autograd.Function):
    """U [B, m, m] complex64 -> amplitudes complex64 [out_len]."""

    @staticmethod
    def forward(ctx, U: torch.Tensor, batch: B.Batch):
        U = _dense(U, torch.complex64)
        ctx.batch = batch
        ctx.save_for_backward(U)
        return B.fock_amplitudes(batch, U)

    @staticmethod
    def backward(ctx, grad_a):
        (U,) = ctx.saved_tensors
        gU = B.fock_amplitudes_backward(ctx.batch, U, _dense(grad_a, torch.complex64))
        return gU, None


class FockModeExpectations(torch.autograd.Function):
    """U [B, m, m] complex64 -> per-mode photon-number expectations float32 [B, m]."""

    @staticmethod
    def forward(ctx, U: torch.Tensor, batch: B.Batch, detector="pnr"):
        U = _dense(U, torch.complex64)
        ctx.batch = batch
        ctx.detector = detector
        ctx.save_for_backward(U)
        return B.fock_mode_expectations(batch, U, detector=detector)

    @staticmethod
    def backward(ctx, grad_e):
        (U,) = ctx.saved_tensors
        gU = B.fock_mode_expectations_backward(ctx.batch, U, _dense(grad_e, torch.float32), detector=ctx.detector)
        return gU, None, None


class FockThresholdProbs(torch.autograd.Function):
    """U [B, m, m] complex64 -> threshold-detector click probabilities float32 [threshold_len]."""

    @staticmethod
    def forward(ctx, U: torch.Tensor, batch: B.Batch):
        U = _dense(U, torch.complex64)
        ctx.batch = batch
        ctx.save_for_backward(U)
        return B.fock_threshold_probs(batch, U)

    @staticmethod
    def backward(ctx, grad_P):
        (U,) = ctx.saved_tensors
        gU = B.fock_threshold_probs_backward(ctx.batch, U, _dense(grad_P, torch.float32))
        return gU, None


class FockSuperposition(torch.autograd.Function):
    """U [G, m, m] and component weights x [C] (complex64) -> sum_c x_c U|s_c>
    per group, complex64 [out_len]."""

    @staticmethod
    def forward(ctx, U: torch.Tensor, x: torch.Tensor, sup: B.Superposition):
        U = _dense(U, torch.complex64)
        x = _dense(x, torch.complex64)
        ctx.sup = sup
        ctx.save_for_backward(U, x)
        return B.fock_superposition_amplitudes(sup, U, x)

    @staticmethod
    def backward(ctx, grad_out):
        U, x = ctx.saved_tensors
        gU, gx = B.fock_superposition_amplitudes_backward(ctx.sup, U, x, _dense(grad_out, torch.complex64),
                                                          need_grad_x=ctx.needs_input_grad[1])
        return gU, gx, None


class FockSharedSuperposition(torch.autograd.Function):
    """U [m, m] and dense inputs X [G, N] (complex64) -> U's action on each input, [G, N]."""

    @staticmethod
    def forward(ctx, U: torch.Tensor, X: torch.Tensor, s: B.SharedSuperposition):
        U = _dense(U, torch.complex64)
        X = _dense(X, torch.complex64)
        ctx.s = s
        ctx.save_for_backward(U, X)
        return B.fock_shared_superposition_amplitudes(s, U, X)

    @staticmethod
    def backward(ctx, grad_out):
        U, X = ctx.saved_tensors
        gU, gX = B.fock_shared_superposition_amplitudes_backward(ctx.s, U, X, _dense(grad_out, torch.complex64),
                                                                 need_grad_x=ctx.needs_input_grad[1])
        return gU, gX, None


class ProbsFromAmplitudes(torch.autograd.Function):
    """a (complex64, any shape) -> |a|^2 (float32), computed by the library."""

    @staticmethod
    def forward(ctx, a: torch.Tensor):
        a = _dense(a, torch.complex64)
        ctx.save_for_backward(a)
        return B.fock_probs_from_amplitudes(a)

    @staticmethod
    def backward(ctx, grad_p):
        (a,) = ctx.saved_tensors
        return B.fock_probs_from_amplitudes_backward(a, _dense(grad_p, torch.float32))


class MeshToUnitary(torch.autograd.Function):
    """theta [m(m-1)] float32 and features x [B, m] float32 (or None) ->
    U [B, m, m] complex64."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, x: Optional[torch.Tensor], enc_scale: float, m: int):
        theta = theta.contiguous()
        xx = x.contiguous() if x is not None else None
        ctx.enc_scale = enc_scale
        ctx.has_x = x is not None
        ctx.save_for_backward(theta, xx) if xx is not None else ctx.save_for_backward(theta)
        return B.mesh_to_unitary(theta, xx, enc_scale, m=m)

    @staticmethod
    def backward(ctx, gU):
        if ctx.has_x:
            theta, x = ctx.saved_tensors
        else:
            (theta,) = ctx.saved_tensors
            x = None
        need_gx = ctx.has_x and ctx.needs_input_grad[1]
        gt, gx = B.mesh_to_unitary_backward(theta, x, ctx.enc_scale, _dense(gU, torch.complex64), need_grad_x=need_gx)
        return gt, gx, None, None


def fock_probs(U: torch.Tensor, batch: B.Batch) -> torch.Tensor:
    return FockProbs.apply(U, batch)


def fock_amplitudes(U: torch.Tensor, batch: B.Batch) -> torch.Tensor:
    return FockAmplitudes.apply(U, batch)


def fock_mode_expectations(U: torch.Tensor, batch: B.Batch, detector="pnr") -> torch.Tensor:
    return FockModeExpectations.apply(U, batch, detector)


def fock_threshold_probs(U: torch.Tensor, batch: B.Batch) -> torch.Tensor:
    return FockThresholdProbs.apply(U, batch)


def fock_superposition_amplitudes(U: torch.Tensor, x: torch.Tensor, sup: B.Superposition) -> torch.Tensor:
    return FockSuperposition.apply(U, x, sup)


def fock_shared_superposition_amplitudes(U: torch.Tensor, X: torch.Tensor, s: B.SharedSuperposition) -> torch.Tensor:
    return FockSharedSuperposition.apply(U, X, s)


def probs_from_amplitudes(a: torch.Tensor) -> torch.Tensor:
    return ProbsFromAmplitudes.apply(a)


def mesh_to_unitary(theta: torch.Tensor, x: Optional[torch.Tensor], enc_scale: float = math.pi,
                    m: Optional[int] = None) -> torch.Tensor:
    if m is None:
        m = x.shape[1]
    return MeshToUnitary.apply(theta, x, enc_scale, m)
