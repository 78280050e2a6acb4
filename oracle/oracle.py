"""FP64 CPU oracle for linear-optical strong simulation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  It shares no code
with the GPU library (its own basis enumeration, its own mesh, its own
permanents) and it never calls it.

Contents, each following the passage it cites (arXiv 2602.11092):

* Fock basis of n photons in m modes, dimension C(m+n-1, n)
  (Sec. II-A-1).  Order convention: lexicographic order of the sorted list of
  occupied modes, so |n,0,...,0> comes first and |0,...,0,n> last (the paper
  does not fix an order).
* Output amplitudes as normalised permanents of sub-matrices of U
  (Sec. II-A-1), by Ryser's formula in C (``ryser.c``), complex128.
* Gradients of a real loss with respect to U through those permanents
  (Sec. II-A-3 trains U(theta) by gradient descent), via minor permanents.
* The parametrised interferometer U(theta) of phase shifters and beam
  splitters (Sec. II-A-3), laid out as a rectangular (Clements) mesh of
  Mach-Zehnder interferometers, with the data-encoding layer
  U(x, theta) = W2(theta2) S(x) W1(theta1) of Sec. II-C-1, and its gradient
  by the product rule, in float64 NumPy.
* Per-mode photon-number expectations <n_j> = sum_t t_j p_t over a set of
  output states (the measurement strategy of Sec. II-B), by that definition.
* Per-mode click probabilities of threshold detectors, P(t_j > 0) =
  sum_t [t_j > 0] p_t (the threshold-detection expectation values of
  Sec. II-B and Fig. 3), by that definition.
* Threshold-detector click probabilities P(c) = sum of p_t over the states
  t whose occupied modes are exactly c (the detector model of Sec. II-B),
  patterns ordered by click count, then lexicographically.
* Shot sampling from the output distribution by inverse transform (the
  shot-based readout of hardware, Sec. II-D): with a uniform u in [0, 1),
  the first state t whose cumulative probability (in basis order,
  normalised over the output states) exceeds u.
* Amplitude-encoded inputs (Sec. II-C-2): a superposition sum_c x_c |s_c>
  of n-photon Fock states maps to sum_c x_c U|s_c> (linearity of U's
  action), over the whole n-photon basis.
* The fidelity kernel k(x1, x2) = |<phi(x1)|phi(x2)>|^2 with
  |phi(x)> = U(x)|s> (the kernel-methods reproduction of Sec. III-A), as the
  inner product of the two full amplitude vectors.
* FP64 replicas of the two losses used by the benchmark workloads.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ryser.c")
_LIB = os.path.join(_HERE, "libryser_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ryser.c into a shared library next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
            "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        c_dp = ctypes.c_void_p
        lib.oracle_permanent.restype = None  # returns double complex: wrapped below
        lib.oracle_amplitudes.restype = ctypes.c_int
        lib.oracle_amplitudes.argtypes = [ctypes.c_int, c_dp, c_dp, ctypes.c_int64, c_dp, c_dp]
        lib.oracle_amplitude_grad.restype = ctypes.c_int
        lib.oracle_amplitude_grad.argtypes = [ctypes.c_int, c_dp, c_dp, ctypes.c_int64, c_dp, c_dp, c_dp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------------------
# Fock basis (Sec. II-A-1)
# ---------------------------------------------------------------------------

def fock_dim(m: int, n: int) -> int:
    """Number of n-photon states in m modes, C(m+n-1, n)."""
    return math.comb(m + n - 1, n)


def fock_basis(m: int, n: int) -> np.ndarray:
    """All n-photon occupation vectors over m modes, shape [C(m+n-1,n), m].

    Enumerated as the sorted mode lists (multisets of size n drawn from
    0..m-1) in lexicographic order, which is the order in which
    itertools.combinations_with_replacement yields them."""
    rows = []
    for modes in itertools.combinations_with_replacement(range(m), n):
        occ = [0] * m
        for j in modes:
            occ[j] += 1
        rows.append(occ)
    if n == 0:
        rows = [[0] * m]
    out = np.asarray(rows, dtype=np.int32).reshape(-1, m)
    assert out.shape[0] == fock_dim(m, n)
    return out


def _count_from(m: int, first: int, k: int) -> int:
    """Number of sorted mode lists of length k whose entries are >= first."""
    if k == 0:
        return 1
    return math.comb((m - first) + k - 1, k)


def fock_unrank(m: int, n: int, rank: int) -> np.ndarray:
    """Occupation vector of the state at position `rank` of fock_basis(m, n),
    found by counting how many lists start with each candidate mode."""
    if not 0 <= rank < fock_dim(m, n):
        raise ValueError("rank out of range")
    occ = np.zeros(m, dtype=np.int32)
    lo = 0
    for pos in range(n):
        remaining = n - pos - 1
        j = lo
        while True:
            block = _count_from(m, j, remaining)
            if rank < block:
                break
            rank -= block
            j += 1
        occ[j] += 1
        lo = j
    return occ


def fock_rank(m: int, n: int, occ: Sequence[int]) -> int:
    """Inverse of fock_unrank."""
    modes = [j for j in range(m) for _ in range(int(occ[j]))]
    assert len(modes) == n
    rank = 0
    lo = 0
    for pos, j in enumerate(modes):
        remaining = n - pos - 1
        for c in range(lo, j):
            rank += _count_from(m, c, remaining)
        lo = j
    return rank


# ---------------------------------------------------------------------------
# Permanents and amplitudes (Sec. II-A-1)
# ---------------------------------------------------------------------------

def permanent(A: np.ndarray) -> complex:
    """Permanent of a square complex matrix (Ryser, complex128)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    if n == 0:
        return 1.0 + 0j
    # Reuse the amplitude routine: with s = t = one photon per mode 0..n-1 and
    # U = A the amplitude equals Perm(A) (all factorials are 1).
    occ = np.ones(n, dtype=np.int32)
    out = np.zeros(1, dtype=np.complex128)
    rc = _load().oracle_amplitudes(n, _ptr(occ), _ptr(A), 1, _ptr(occ), _ptr(out))
    assert rc == 0
    return complex(out[0])


def amplitudes(U: np.ndarray, s: Sequence[int], outputs: Optional[np.ndarray] = None) -> np.ndarray:
    """a_t = Perm(U[R(t), C(s)]) / sqrt(prod s! prod t!) for every t in
    `outputs` (default: the whole basis, in fock_basis order)."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    m = U.shape[0]
    s = np.ascontiguousarray(s, dtype=np.int32)
    n = int(s.sum())
    if outputs is None:
        outputs = fock_basis(m, n)
    outputs = np.ascontiguousarray(outputs, dtype=np.int32).reshape(-1, m)
    out = np.zeros(outputs.shape[0], dtype=np.complex128)
    if n == 0:
        out[:] = 1.0
        return out
    rc = _load().oracle_amplitudes(m, _ptr(s), _ptr(U), outputs.shape[0], _ptr(outputs), _ptr(out))
    if rc != 0:
        raise ValueError("output state with a different photon number than the input")
    return out


def probabilities(U: np.ndarray, s: Sequence[int], outputs: Optional[np.ndarray] = None) -> np.ndarray:
    """p_t = |a_t|^2 (no renormalisation)."""
    return np.abs(amplitudes(U, s, outputs)) ** 2


def mode_expectations(U: np.ndarray, s: Sequence[int], outputs: Optional[np.ndarray] = None) -> np.ndarray:
    """<n_j> = sum_t t_j p_t over `outputs` (default: the whole basis), the
    per-mode photon-number expectation of Sec. II-B, no renormalisation."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    m = U.shape[0]
    n = int(np.sum(s))
    if outputs is None:
        outputs = fock_basis(m, n)
    outputs = np.asarray(outputs, dtype=np.float64).reshape(-1, m)
    if n == 0:
        return np.zeros(m)
    return probabilities(U, s, outputs.astype(np.int32)) @ outputs


def mode_click_probabilities(U: np.ndarray, s: Sequence[int], outputs: Optional[np.ndarray] = None) -> np.ndarray:
    """P(t_j > 0) = sum_t [t_j > 0] p_t over `outputs` (default: the whole basis)."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    m = U.shape[0]
    n = int(np.sum(s))
    if outputs is None:
        outputs = fock_basis(m, n)
    outputs = np.asarray(outputs, dtype=np.int32).reshape(-1, m)
    if n == 0:
        return np.zeros(m)
    return probabilities(U, s, outputs) @ (outputs > 0).astype(np.float64)


def superposition_amplitudes(U: np.ndarray, states: Sequence[Sequence[int]], x: Sequence[complex]) -> np.ndarray:
    """sum_c x_c a(U, s_c) over the n-photon basis; every s_c has n photons."""
    states = [np.asarray(st, dtype=np.int32) for st in states]
    n = int(states[0].sum())
    if any(int(st.sum()) != n for st in states):
        raise ValueError("components must have the same photon number")
    out = np.zeros(fock_dim(np.asarray(U).shape[0], n), dtype=np.complex128)
    for st, xc in zip(states, x):
        out += complex(xc) * amplitudes(U, st)
    return out


def click_patterns(m: int, n: int) -> list:
    """Click patterns of n photons over m modes: the non-empty sets of at most
    n modes, by size, then in lexicographic order (n = 0: the empty pattern)."""
    if n == 0:
        return [()]
    return [c for k in range(1, min(n, m) + 1) for c in itertools.combinations(range(m), k)]


def threshold_probs(U: np.ndarray, s: Sequence[int]) -> np.ndarray:
    """P(c) = sum_{t : {j : t_j > 0} = c} p_t for every click pattern c."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    m = U.shape[0]
    n = int(np.sum(s))
    basis = fock_basis(m, n)
    p = probabilities(U, s, basis)
    index = {c: i for i, c in enumerate(click_patterns(m, n))}
    out = np.zeros(len(index))
    for t, pt in zip(basis, p):
        out[index[tuple(int(j) for j in np.nonzero(t)[0])]] += pt
    return out


def sample_shots(U: np.ndarray, s: Sequence[int], u: np.ndarray, outputs: Optional[np.ndarray] = None) -> np.ndarray:
    """Output-state indices (into `outputs`, default the whole basis) drawn
    from p / sum(p) by inverse transform of the uniforms u in [0, 1)."""
    p = probabilities(U, s, outputs)
    cdf = np.cumsum(p)
    idx = np.searchsorted(cdf, np.asarray(u, dtype=np.float64) * cdf[-1], side="right")
    return np.minimum(idx, p.size - 1).astype(np.int64)


def fidelity(U1: np.ndarray, U2: np.ndarray, s: Sequence[int]) -> float:
    """|sum_t conj(a_t(U1)) a_t(U2)|^2 over the whole n-photon basis."""
    a1 = amplitudes(U1, s)
    a2 = amplitudes(U2, s)
    return float(abs(np.vdot(a1, a2)) ** 2)


def amplitude_grad(U: np.ndarray, s: Sequence[int], G_a: np.ndarray,
                   outputs: Optional[np.ndarray] = None) -> np.ndarray:
    """G_U = sum_t G_a[t] conj(d a_t / dU) for a real loss, in the convention
    G = dL/dRe + i dL/dIm (the one PyTorch uses)."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    m = U.shape[0]
    s = np.ascontiguousarray(s, dtype=np.int32)
    n = int(s.sum())
    if outputs is None:
        outputs = fock_basis(m, n)
    outputs = np.ascontiguousarray(outputs, dtype=np.int32).reshape(-1, m)
    G_a = np.ascontiguousarray(G_a, dtype=np.complex128)
    assert G_a.shape[0] == outputs.shape[0]
    GU = np.zeros((m, m), dtype=np.complex128)
    rc = _load().oracle_amplitude_grad(m, _ptr(s), _ptr(U), outputs.shape[0], _ptr(outputs),
                                       _ptr(G_a), _ptr(GU))
    if rc != 0:
        raise ValueError("bad input to amplitude_grad")
    return GU


def probs_grad(U: np.ndarray, s: Sequence[int], grad_p: np.ndarray,
               outputs: Optional[np.ndarray] = None) -> np.ndarray:
    """G_U for a real loss L(p) given dL/dp_t.  With p_t = |a_t|^2 the
    amplitude gradient is G_a[t] = 2 (dL/dp_t) a_t."""
    a = amplitudes(U, s, outputs)
    return amplitude_grad(U, s, 2.0 * np.asarray(grad_p, dtype=np.float64) * a, outputs)


# ---------------------------------------------------------------------------
# Mesh of phase shifters and beam splitters (Sec. II-A-3, Sec. II-C-1)
# ---------------------------------------------------------------------------

def beam_splitter() -> np.ndarray:
    """Balanced beam splitter (1/sqrt 2) [[1, i], [i, 1]]."""
    return np.array([[1.0, 1.0j], [1.0j, 1.0]], dtype=np.complex128) / math.sqrt(2.0)


def phase_shifter(alpha: float) -> np.ndarray:
    """Phase alpha on the upper mode of a pair."""
    return np.array([[np.exp(1j * alpha), 0.0], [0.0, 1.0]], dtype=np.complex128)


def mzi(theta: float, phi: float) -> np.ndarray:
    """Mach-Zehnder interferometer BS . PS(theta) . BS . PS(phi) (light meets
    PS(phi) first)."""
    return beam_splitter() @ phase_shifter(theta) @ beam_splitter() @ phase_shifter(phi)


def clements_layout(m: int):
    """Rectangular mesh: column c = 0..m-1 holds MZIs on mode pairs (k, k+1)
    with k = c mod 2, c mod 2 + 2, ... <= m-2.  Returns the list of
    (column, k) in parameter order (column-major, top-down)."""
    return [(c, k) for c in range(m) for k in range(c % 2, m - 1, 2)]


def _embed(m: int, k: int, T: np.ndarray) -> np.ndarray:
    E = np.eye(m, dtype=np.complex128)
    E[k:k + 2, k:k + 2] = T
    return E


def _embed_zero(m: int, k: int, D: np.ndarray) -> np.ndarray:
    """2x2 block D on modes (k, k+1) of an otherwise zero m x m matrix (the
    derivative of an embedded MZI)."""
    E = np.zeros((m, m), dtype=np.complex128)
    E[k:k + 2, k:k + 2] = D
    return E


def mesh_split(m: int) -> int:
    """Number of leading mesh columns that form W1 (the rest form W2)."""
    return m // 2


def mesh_factors(theta: np.ndarray, m: int):
    """W1 (columns < m//2) and W2 (the other columns) of the rectangular mesh
    with phases theta = (theta_q, phi_q) per MZI in layout order.  Each factor
    is the ordered product of its MZIs, the first MZI rightmost."""
    theta = np.asarray(theta, dtype=np.float64)
    layout = clements_layout(m)
    assert theta.shape == (2 * len(layout),)
    W1 = np.eye(m, dtype=np.complex128)
    W2 = np.eye(m, dtype=np.complex128)
    split = mesh_split(m)
    for q, (c, k) in enumerate(layout):
        E = _embed(m, k, mzi(theta[2 * q], theta[2 * q + 1]))
        if c < split:
            W1 = E @ W1
        else:
            W2 = E @ W2
    return W1, W2


def mesh_unitary(theta: np.ndarray, m: int) -> np.ndarray:
    """The whole mesh, W2 . W1 (no data encoding)."""
    W1, W2 = mesh_factors(theta, m)
    return W2 @ W1


def encoded_unitaries(theta: np.ndarray, x: np.ndarray, scale: float) -> np.ndarray:
    """U_b = W2 . diag(exp(i scale x_b)) . W1 for each row x_b of x
    (angle encoding between two trainable interferometers, Sec. II-C-1)."""
    x = np.asarray(x, dtype=np.float64)
    B, m = x.shape
    W1, W2 = mesh_factors(theta, m)
    S = np.exp(1j * scale * x)                      # [B, m]
    return np.einsum("jk,bk,ki->bji", W2, S, W1)


def _mzi_derivatives(theta: float, phi: float):
    """d/dtheta and d/dphi of mzi(theta, phi), by the product rule."""
    BS = beam_splitter()
    dPS_t = np.array([[1j * np.exp(1j * theta), 0.0], [0.0, 0.0]], dtype=np.complex128)
    dPS_p = np.array([[1j * np.exp(1j * phi), 0.0], [0.0, 0.0]], dtype=np.complex128)
    d_theta = BS @ dPS_t @ BS @ phase_shifter(phi)
    d_phi = BS @ phase_shifter(theta) @ BS @ dPS_p
    return d_theta, d_phi


def mesh_grad(theta: np.ndarray, x: Optional[np.ndarray], scale: float, G_U: np.ndarray):
    """Gradient of a real loss through U(x, theta) given G_U = dL/dRe U + i dL/dIm U
    (shape [B, m, m], or [m, m] when x is None).

    dL/dv = Re sum conj(G_U) * dU/dv for every real parameter v.  dU/dv is
    formed explicitly: for an MZI phase inside W1,
    dU_b/dv = W2 S_b (... dT_q/dv ...) with the other factors of W1 in place;
    likewise inside W2; for a feature, dU_b/dx_bk = W2 (i scale S_bk e_k e_k^T) W1.
    Returns (grad_theta [P], grad_x [B, m] or None)."""
    theta = np.asarray(theta, dtype=np.float64)
    G_U = np.asarray(G_U, dtype=np.complex128)
    if x is None:
        m = G_U.shape[-1]
        xx = np.zeros((1, m))
        G = G_U.reshape(1, m, m)
        scale_eff = 0.0
    else:
        xx = np.asarray(x, dtype=np.float64)
        G = G_U
        m = xx.shape[1]
        scale_eff = scale
    B = xx.shape[0]
    layout = clements_layout(m)
    split = mesh_split(m)
    T = [_embed(m, k, mzi(theta[2 * q], theta[2 * q + 1])) for q, (c, k) in enumerate(layout)]
    idx1 = [q for q, (c, k) in enumerate(layout) if c < split]
    idx2 = [q for q, (c, k) in enumerate(layout) if c >= split]
    W1, W2 = mesh_factors(theta, m)
    S = np.exp(1j * scale_eff * xx)                 # [B, m]

    def ordered_product(indices):
        P = np.eye(m, dtype=np.complex128)
        for q in indices:
            P = T[q] @ P
        return P

    grad_theta = np.zeros_like(theta)
    for group, is_first in ((idx1, True), (idx2, False)):
        for pos, q in enumerate(group):
            c, k = layout[q]
            after = ordered_product(group[pos + 1:])
            before = ordered_product(group[:pos])
            for v, dT in enumerate(_mzi_derivatives(theta[2 * q], theta[2 * q + 1])):
                dW = after @ _embed_zero(m, k, dT) @ before
                if is_first:
                    dU = np.einsum("jk,bk,ki->bji", W2, S, dW)
                else:
                    dU = np.einsum("jk,bk,ki->bji", dW, S, W1)
                grad_theta[2 * q + v] = np.real(np.sum(np.conj(G) * dU))
    grad_x = None
    if x is not None:
        grad_x = np.zeros_like(xx)
        for kk in range(m):
            # dU_b / dx_bk = W2[:, k] (i scale S_bk) W1[k, :]
            dU = np.einsum("j,b,i->bji", W2[:, kk], 1j * scale * S[:, kk], W1[kk, :])
            grad_x[:, kk] = np.real(np.sum(np.conj(G) * dU, axis=(1, 2)))
    return grad_theta, grad_x


# ---------------------------------------------------------------------------
# Loss replicas used by the benchmark workloads (float64)
# ---------------------------------------------------------------------------

def readout_cross_entropy(p: np.ndarray, W: np.ndarray, bias: np.ndarray, labels: np.ndarray):
    """Mean cross-entropy of logits = p W^T + bias.  Returns (L, dL/dp)."""
    p = np.asarray(p, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    logits = p @ W.T + np.asarray(bias, dtype=np.float64)
    z = logits - logits.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z).sum(axis=1, keepdims=True))
    logp = z - lse
    B = p.shape[0]
    L = -np.mean(logp[np.arange(B), labels])
    soft = np.exp(logp)
    soft[np.arange(B), labels] -= 1.0
    dlogits = soft / B
    return L, dlogits @ W


def weighted_sum(p: np.ndarray, w: np.ndarray):
    """L = sum_b sum_t w_t p_bt.  Returns (L, dL/dp)."""
    p = np.asarray(p, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    return float((p * w[None, :]).sum()), np.broadcast_to(w, p.shape).copy()
