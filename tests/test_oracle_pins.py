"""Pins of the FP64 oracle against results fixed by the mathematics and the
paper, not by the oracle itself (CPU only).

Each test checks one part of the oracle against an independent definition:
brute-force permutation sums, expansion of products of creation operators,
closed forms, invariants and finite differences.  A plausible mistake (a
dropped factorial, a transposed U, a wrong sign in Ryser's formula, a wrong
MZI phase order) makes at least one of them fail.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _haar(rng, m):
    Z = _rand_c(rng, m, m) / math.sqrt(2)
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    return Q * (d / np.abs(d))[None, :]


def _perm_bruteforce(A):
    n = A.shape[0]
    return sum(np.prod([A[r, p[r]] for r in range(n)]) for p in itertools.permutations(range(n)))


# ---------------------------------------------------------------- permanents

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_ryser_matches_permutation_sum(n):
    rng = np.random.default_rng(10 + n)
    for _ in range(3):
        A = _rand_c(rng, n, n)
        assert abs(O.permanent(A) - _perm_bruteforce(A)) < 1e-11 * max(1.0, abs(_perm_bruteforce(A)))


def test_permanent_identities():
    rng = np.random.default_rng(1)
    for n in range(1, 9):
        assert abs(O.permanent(np.ones((n, n))) - math.factorial(n)) < 1e-9 * math.factorial(n)
        d = _rand_c(rng, n)
        assert abs(O.permanent(np.diag(d)) - np.prod(d)) < 1e-12 * max(1, abs(np.prod(d)))
        A = _rand_c(rng, n, n)
        assert abs(O.permanent(A) - O.permanent(A.T)) < 1e-10 * max(1, abs(O.permanent(A)))
        # multilinear in each row
        c = 0.3 - 1.7j
        B = A.copy()
        B[0] *= c
        assert abs(O.permanent(B) - c * O.permanent(A)) < 1e-10 * max(1, abs(O.permanent(B)))


# ---------------------------------------------------------------- basis

@pytest.mark.parametrize("m,n", [(1, 3), (2, 2), (3, 3), (4, 2), (5, 3), (6, 3), (3, 0)])
def test_basis_count_order_and_rank(m, n):
    basis = O.fock_basis(m, n)
    assert basis.shape == (math.comb(m + n - 1, n), m)
    assert (basis.sum(axis=1) == n).all()
    # brute force: every occupation vector with sum n, once
    every = [v for v in itertools.product(range(n + 1), repeat=m) if sum(v) == n]
    assert sorted(map(tuple, basis)) == sorted(every)
    # order: sorted mode lists ascending lexicographically
    lists = [tuple(j for j in range(m) for _ in range(int(t[j]))) for t in basis]
    assert lists == sorted(lists)
    if n > 0:
        assert tuple(basis[0]) == (n,) + (0,) * (m - 1)
        assert tuple(basis[-1]) == (0,) * (m - 1) + (n,)
    for r in range(basis.shape[0]):
        assert (O.fock_unrank(m, n, r) == basis[r]).all()
        assert O.fock_rank(m, n, basis[r]) == r


# ---------------------------------------------------------------- amplitudes

def _amplitudes_by_creation_operators(U, s):
    """Independent definition: the output state is prod_k (sum_j U[j, i_k] a_j^+)|0>.
    Expand the product of linear forms as a polynomial in the a_j^+; the
    coefficient c_t of prod_j (a_j^+)^{t_j} maps to amplitude
    c_t sqrt(prod t!) / sqrt(prod s!), since (a^+)^t |0> = sqrt(t!) |t> and the
    input is prod_i (a_i^+)^{s_i}/sqrt(s_i!) |0>."""
    m = U.shape[0]
    poly = {tuple([0] * m): 1.0 + 0j}
    for i in range(m):
        for _ in range(int(s[i])):
            new = {}
            for mono, c in poly.items():
                for j in range(m):
                    t = list(mono)
                    t[j] += 1
                    new[tuple(t)] = new.get(tuple(t), 0) + c * U[j, i]
            poly = new
    sfact = np.prod([math.factorial(int(v)) for v in s])
    return {t: c * math.sqrt(np.prod([math.factorial(v) for v in t]) / sfact) for t, c in poly.items()}


@pytest.mark.parametrize("m,s", [((2), (1, 1)), (3, (1, 1, 1)), (4, (2, 0, 1, 0)), (4, (0, 3, 0, 0)),
                                 (5, (1, 0, 1, 0, 1)), (3, (2, 2, 0))])
def test_amplitudes_match_creation_operator_expansion(m, s):
    rng = np.random.default_rng(m * 7 + sum(s))
    U = _rand_c(rng, m, m)  # any matrix: the map is defined for non-unitary U too
    ref = _amplitudes_by_creation_operators(U, s)
    basis = O.fock_basis(m, sum(s))
    a = O.amplitudes(U, s)
    for k, t in enumerate(basis):
        assert abs(a[k] - ref[tuple(int(v) for v in t)]) < 1e-11 * max(1, abs(a[k]))


def test_hong_ou_mandel_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "hom_50_50.txt")) if l.strip() and l[0] != "#"]
    p = O.probabilities(O.beam_splitter(), [1, 1])
    basis = O.fock_basis(2, 2)
    for t0, t1, prob in rows:
        k = [tuple(b) for b in basis].index((int(t0), int(t1)))
        assert abs(p[k] - float(prob)) < 1e-15


def test_identity_and_permutation_unitaries():
    rng = np.random.default_rng(3)
    m = 5
    s = np.array([2, 0, 1, 1, 0], np.int32)
    basis = O.fock_basis(m, 4)
    for perm in [list(range(m)), list(rng.permutation(m))]:
        P = np.zeros((m, m))
        for i, j in enumerate(perm):
            P[j, i] = 1.0  # photon in mode i leaves in mode perm[i]
        p = O.probabilities(P, s)
        t = np.zeros(m, np.int32)
        for i in range(m):
            t[perm[i]] += s[i]
        k = [tuple(b) for b in basis].index(tuple(t))
        assert abs(p[k] - 1.0) < 1e-14
        assert abs(p.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("m,s", [(4, (1, 1, 0, 0)), (6, (1, 1, 1, 0, 0, 0)), (5, (3, 0, 0, 1, 0)),
                                 (7, (1, 0, 2, 0, 1, 0, 1)), (8, (1, 1, 1, 1, 0, 0, 0, 0))])
def test_probabilities_sum_to_one(m, s):
    U = _haar(np.random.default_rng(m), m)
    assert abs(O.probabilities(U, s).sum() - 1.0) < 1e-12


def test_single_photon_fixes_index_convention():
    rng = np.random.default_rng(4)
    m = 4
    U = _haar(rng, m)
    assert np.abs(U - U.T).max() > 0.1
    for i in range(m):
        s = np.zeros(m, np.int32)
        s[i] = 1
        p = O.probabilities(U, s)  # basis for n=1: |1000>, |0100>, ... i.e. mode j at rank j
        assert np.allclose(p, np.abs(U[:, i]) ** 2, atol=1e-15)


def test_all_photons_in_one_mode_closed_form():
    rng = np.random.default_rng(5)
    m, n, i = 4, 4, 2
    U = _haar(rng, m)
    s = np.zeros(m, np.int32)
    s[i] = n
    basis = O.fock_basis(m, n)
    a = O.amplitudes(U, s)
    for k, t in enumerate(basis):
        ref = math.sqrt(math.factorial(n) / np.prod([math.factorial(int(v)) for v in t])) \
            * np.prod([U[j, i] ** int(t[j]) for j in range(m)])
        assert abs(a[k] - ref) < 1e-13


def test_time_reversal():
    rng = np.random.default_rng(6)
    m = 4
    U = _haar(rng, m)
    basis = O.fock_basis(m, 3)
    for s in basis[::3]:
        p_fwd = O.probabilities(U, s)
        for k, t in enumerate(basis[::4]):
            p_rev = O.probabilities(U.T, t, outputs=s[None, :])[0]
            assert abs(O.probabilities(U, s, outputs=t[None, :])[0] - p_rev) < 1e-14


def test_fourier_suppression_law_golden():
    ms = [int(l) for l in open(os.path.join(GOLDEN, "fourier_suppression.txt")) if l.strip() and l[0] != "#"]
    for m in ms:
        F = np.exp(2j * np.pi * np.outer(np.arange(m), np.arange(m)) / m) / math.sqrt(m)
        s = np.ones(m, np.int32)
        p = O.probabilities(F, s)
        basis = O.fock_basis(m, m)
        kept = 0
        for k, t in enumerate(basis):
            if (np.arange(m) @ t) % m != 0:
                assert p[k] < 1e-24
            elif p[k] > 1e-6:
                kept += 1
        assert kept > 0
        assert abs(p.sum() - 1) < 1e-12


def test_mean_photon_number_marginals():
    rng = np.random.default_rng(7)
    m = 6
    U = _haar(rng, m)
    s = np.array([1, 2, 0, 1, 0, 0], np.int32)
    p = O.probabilities(U, s)
    basis = O.fock_basis(m, 4)
    lhs = p @ basis
    rhs = (np.abs(U) ** 2) @ s
    assert np.allclose(lhs, rhs, atol=1e-13)


def test_phase_invariance_of_probabilities():
    rng = np.random.default_rng(8)
    m = 5
    U = _haar(rng, m)
    s = np.array([1, 1, 0, 1, 0], np.int32)
    D1 = np.diag(np.exp(1j * rng.uniform(0, 6, m)))
    D2 = np.diag(np.exp(1j * rng.uniform(0, 6, m)))
    assert np.allclose(O.probabilities(U, s), O.probabilities(D1 @ U @ D2, s), atol=1e-14)


# ---------------------------------------------------------------- gradients

def test_gradient_of_total_probability_closed_form():
    rng = np.random.default_rng(9)
    m = 5
    U = _haar(rng, m)
    s = np.array([1, 0, 2, 1, 0], np.int32)
    N = O.fock_dim(m, 4)
    G = O.probs_grad(U, s, np.ones(N))
    ref = 2.0 * U * s[None, :]   # d(sum_t p_t)/dU = 2 s_i U[:, i] for unitary U
    assert np.abs(G - ref).max() < 1e-12


@pytest.mark.parametrize("m,s", [(3, (1, 1, 1)), (4, (2, 0, 1, 0)), (5, (1, 0, 1, 0, 1))])
def test_gradient_matches_central_differences(m, s):
    rng = np.random.default_rng(20 + m)
    U = _rand_c(rng, m, m) * 0.6
    s = np.array(s, np.int32)
    N = O.fock_dim(m, int(s.sum()))
    w = rng.uniform(0, 1, N)
    L = lambda V: float(w @ O.probabilities(V, s))
    G = O.probs_grad(U, s, w)
    h = 1e-6
    for j in range(m):
        for i in range(m):
            E = np.zeros((m, m))
            E[j, i] = 1
            d_re = (L(U + h * E) - L(U - h * E)) / (2 * h)
            d_im = (L(U + 1j * h * E) - L(U - 1j * h * E)) / (2 * h)
            assert abs(G[j, i] - (d_re + 1j * d_im)) < 1e-7 * max(1, abs(G[j, i]))


def test_amplitude_gradient_matches_central_differences():
    rng = np.random.default_rng(31)
    m = 4
    U = _rand_c(rng, m, m) * 0.7
    s = np.array([1, 1, 0, 1], np.int32)
    N = O.fock_dim(m, 3)
    C = _rand_c(rng, N)
    L = lambda V: float(np.real(np.sum(np.conj(C) * O.amplitudes(V, s))))
    G = O.amplitude_grad(U, s, C)
    h = 1e-6
    for j in range(m):
        for i in range(m):
            E = np.zeros((m, m))
            E[j, i] = 1
            d_re = (L(U + h * E) - L(U - h * E)) / (2 * h)
            d_im = (L(U + 1j * h * E) - L(U - 1j * h * E)) / (2 * h)
            assert abs(G[j, i] - (d_re + 1j * d_im)) < 1e-7 * max(1, abs(G[j, i]))


# ---------------------------------------------------------------- mesh

def test_mzi_limits():
    swap = O.mzi(0.0, 0.7)
    assert abs(swap[0, 0]) < 1e-15 and abs(swap[1, 1]) < 1e-15
    assert abs(abs(swap[0, 1]) - 1) < 1e-15 and abs(abs(swap[1, 0]) - 1) < 1e-15
    bar = O.mzi(np.pi, 0.3)
    assert abs(bar[0, 1]) < 1e-15 and abs(bar[1, 0]) < 1e-15
    half = O.mzi(np.pi / 2, 1.1)
    assert np.allclose(np.abs(half) ** 2, 0.5, atol=1e-15)
    # phi is applied first, on the upper input mode: it only rephases column 0
    assert np.allclose(O.mzi(0.4, 0.9)[:, 1], O.mzi(0.4, 0.0)[:, 1], atol=1e-15)


@pytest.mark.parametrize("m,count,first", [(12, 66, 33), (20, 190, 95), (5, 10, 4), (2, 1, 1)])
def test_clements_layout_counts(m, count, first):
    layout = O.clements_layout(m)
    assert len(layout) == count == m * (m - 1) // 2
    assert sum(1 for c, k in layout if c < O.mesh_split(m)) == first
    # MZIs of one column act on disjoint pairs
    for c in range(m):
        ks = [k for cc, k in layout if cc == c]
        assert all(b - a >= 2 for a, b in zip(ks, ks[1:]))


def test_mesh_unitary_and_bar_state():
    rng = np.random.default_rng(11)
    m = 7
    theta = rng.uniform(0, 2 * np.pi, m * (m - 1))
    U = O.mesh_unitary(theta, m)
    assert np.abs(U.conj().T @ U - np.eye(m)).max() < 1e-13
    bar = np.zeros(m * (m - 1))
    bar[0::2] = np.pi
    Ub = O.mesh_unitary(bar, m)
    assert np.abs(np.abs(Ub) - np.eye(m)).max() < 1e-13
    s = np.array([1, 0, 1, 1, 0, 0, 1], np.int32)
    p = O.probabilities(Ub, s)
    k = O.fock_rank(m, 4, s)
    assert abs(p[k] - 1) < 1e-13


def test_mesh_layout_first_column_acts_first():
    # One MZI swapping modes (0,1) in column 0 and a bar everywhere else:
    # input mode 0 must leave in mode 1.  A reversed product order or a
    # transposed embedding would change this.
    m = 4
    layout = O.clements_layout(m)
    th = np.zeros(m * (m - 1))
    th[0::2] = np.pi
    th[0] = 0.0      # first MZI (column 0, modes 0-1) becomes a swap
    qq = [q for q, (c, k) in enumerate(layout) if (c, k) == (1, 1)][0]
    th[2 * qq] = 0.0  # column 1 MZI on modes (1,2) swaps as well
    U = O.mesh_unitary(th, m)
    # photon: 0 -> 1 (column 0) -> 2 (column 1)
    assert abs(abs(U[2, 0]) - 1) < 1e-14


def test_mesh_gradient_matches_central_differences():
    rng = np.random.default_rng(12)
    m, B = 5, 3
    theta = rng.uniform(0, 2 * np.pi, m * (m - 1))
    x = rng.standard_normal((B, m))
    C = _rand_c(rng, B, m, m)
    scale = np.pi
    L = lambda th, xx: float(np.real(np.sum(np.conj(C) * O.encoded_unitaries(th, xx, scale))))
    gt, gx = O.mesh_grad(theta, x, scale, C)
    h = 1e-6
    for q in range(theta.size):
        e = np.zeros_like(theta)
        e[q] = h
        fd = (L(theta + e, x) - L(theta - e, x)) / (2 * h)
        assert abs(gt[q] - fd) < 1e-7 * max(1, abs(fd))
    for b in range(B):
        for k in range(m):
            e = np.zeros_like(x)
            e[b, k] = h
            fd = (L(theta, x + e) - L(theta, x - e)) / (2 * h)
            assert abs(gx[b, k] - fd) < 1e-7 * max(1, abs(fd))
    # no-encoding variant
    C1 = C[0]
    L1 = lambda th: float(np.real(np.sum(np.conj(C1) * O.mesh_unitary(th, m))))
    gt1, gx1 = O.mesh_grad(theta, None, 0.0, C1)
    assert gx1 is None
    for q in range(0, theta.size, 3):
        e = np.zeros_like(theta)
        e[q] = h
        assert abs(gt1[q] - (L1(theta + e) - L1(theta - e)) / (2 * h)) < 1e-7


def test_angle_encoding_spectrum_is_bounded_by_photon_number():
    # Sec. II-C-1: with the data on one phase shifter between two trainable
    # interferometers, every output probability is a trigonometric
    # polynomial of degree <= n in the encoded phase.
    rng = np.random.default_rng(13)
    m = 4
    theta = rng.uniform(0, 2 * np.pi, m * (m - 1))
    for s in ([1, 1, 0, 0], [1, 1, 1, 0], [2, 1, 0, 1]):
        n = sum(s)
        K = 4 * n + 4
        xs = np.zeros((K, m))
        xs[:, 1] = 2 * np.pi * np.arange(K) / K
        xs[:, 0] = 0.37
        P = np.stack([O.probabilities(U, s) for U in O.encoded_unitaries(theta, xs, 1.0)])  # [K, N]
        spec = np.fft.fft(P, axis=0) / K
        freqs = np.abs(np.fft.fftfreq(K, 1.0 / K))
        assert np.abs(spec[freqs > n]).max() < 1e-12
        assert np.abs(spec[freqs == n]).max() > 1e-6  # the top frequency is reached


# ---------------------------------------------------------------- loss replicas

def test_readout_cross_entropy_gradient():
    rng = np.random.default_rng(14)
    B, N, C = 4, 9, 3
    p = rng.uniform(0, 1, (B, N))
    W = rng.standard_normal((C, N))
    bias = rng.standard_normal(C)
    labels = rng.integers(0, C, B)
    L, g = O.readout_cross_entropy(p, W, bias, labels)
    h = 1e-6
    for b in range(B):
        for t in range(N):
            e = np.zeros_like(p)
            e[b, t] = h
            fd = (O.readout_cross_entropy(p + e, W, bias, labels)[0]
                  - O.readout_cross_entropy(p - e, W, bias, labels)[0]) / (2 * h)
            assert abs(g[b, t] - fd) < 1e-8
    # against the textbook value for uniform logits
    L0, _ = O.readout_cross_entropy(np.zeros((2, N)), np.zeros((C, N)), np.zeros(C), np.array([0, 1]))
    assert abs(L0 - math.log(C)) < 1e-14


def test_weighted_sum_loss():
    # hand-expanded: 0.5*2 + 0.25*4 + 0.1*2 + 0.15*4 = 2.8; dL/dp_bt = w_t
    p = np.array([[0.5, 0.25], [0.1, 0.15]])
    L, g = O.weighted_sum(p, np.array([2.0, 4.0]))
    assert abs(L - 2.8) < 1e-15
    assert np.array_equal(g, np.array([[2.0, 4.0], [2.0, 4.0]]))
    # w = 1 on unitaries: each sample's probabilities sum to 1, so L = B
    rng = np.random.default_rng(31)
    s = [1, 0, 2, 0]
    P = np.stack([O.probabilities(_haar(rng, 4), s) for _ in range(3)])
    L1, _ = O.weighted_sum(P, np.ones(P.shape[1]))
    assert abs(L1 - 3.0) < 1e-12
    # a weight on a single output picks that output's probability out
    w = np.zeros(P.shape[1])
    w[7] = 1.0
    assert abs(O.weighted_sum(P, w)[0] - P[:, 7].sum()) < 1e-15


def test_mode_expectations_closed_form():
    # full space: <n_j> = sum_i s_i |U_ji|^2 (each photon leaves input mode i
    # towards j with probability |U_ji|^2), including bunched inputs
    rng = np.random.default_rng(17)
    for m, s in [(4, [1, 0, 2, 0]), (5, [1, 1, 1, 0, 0]), (6, [0, 3, 0, 0, 1, 0])]:
        U = _haar(rng, m)
        e = O.mode_expectations(U, s)
        want = np.array([sum(s[i] * abs(U[j, i]) ** 2 for i in range(m)) for j in range(m)])
        assert np.abs(e - want).max() < 1e-13
        assert abs(e.sum() - sum(s)) < 1e-12
    assert np.all(O.mode_expectations(_haar(rng, 3), [0, 0, 0]) == 0)


def test_mode_expectations_unbunched_two_photons_by_hand():
    # two photons in modes 0 and 1 of 3, outputs restricted to t_j <= 1:
    # p(a, b) = |U_a0 U_b1 + U_a1 U_b0|^2 for output modes a < b
    rng = np.random.default_rng(18)
    U = _haar(rng, 3)
    outs = np.array([[1, 1, 0], [1, 0, 1], [0, 1, 1]], dtype=np.int32)
    e = O.mode_expectations(U, [1, 1, 0], outputs=outs)
    pair = {}
    for a, b in [(0, 1), (0, 2), (1, 2)]:
        pair[(a, b)] = abs(U[a, 0] * U[b, 1] + U[a, 1] * U[b, 0]) ** 2
    want = [pair[(0, 1)] + pair[(0, 2)], pair[(0, 1)] + pair[(1, 2)], pair[(0, 2)] + pair[(1, 2)]]
    assert np.abs(e - want).max() < 1e-14


def _perm_brute(A):
    n = A.shape[0]
    return sum(np.prod([A[i, p[i]] for i in range(n)]) for p in itertools.permutations(range(n)))


def test_fidelity_permanent_identity_and_invariants():
    # <phi1|phi2> = Perm(U1[:,C]^H U2[:,C]) / prod s!, C the input modes with
    # multiplicity (Cauchy-Binet over the output basis), by brute-force permanents
    rng = np.random.default_rng(19)
    for m, s in [(3, [1, 1, 0]), (4, [2, 0, 1, 0]), (5, [1, 0, 1, 1, 0]), (4, [0, 3, 0, 1])]:
        U1, U2 = _haar(rng, m), _haar(rng, m)
        C = [i for i in range(m) for _ in range(s[i])]
        M = U1[:, C].conj().T @ U2[:, C]
        f = abs(_perm_brute(M) / np.prod([math.factorial(v) for v in s])) ** 2
        F = O.fidelity(U1, U2, s)
        assert abs(F - f) < 1e-13
        assert 0.0 <= F <= 1.0 + 1e-13
        assert abs(F - O.fidelity(U2, U1, s)) < 1e-13           # symmetric
        assert abs(O.fidelity(U1, U1, s) - 1.0) < 1e-12         # a state with itself
        V = _haar(rng, m)
        assert abs(O.fidelity(V @ U1, V @ U2, s) - F) < 1e-12   # common output unitary
    # one photon in mode i: |(U1^H U2)_ii|^2
    U1, U2 = _haar(rng, 4), _haar(rng, 4)
    assert abs(O.fidelity(U1, U2, [0, 0, 1, 0]) - abs((U1.conj().T @ U2)[2, 2]) ** 2) < 1e-14


def test_threshold_probs_closed_forms():
    rng = np.random.default_rng(21)
    m = 4
    U = _haar(rng, m)
    pats = O.click_patterns(m, 2)
    assert len(pats) == 4 + 6 and pats[:4] == [(0,), (1,), (2,), (3,)] and pats[4] == (0, 1)
    # one photon in mode 1: P({j}) = |U_j1|^2
    P1 = O.threshold_probs(U, [0, 1, 0, 0])
    assert np.abs(P1 - np.abs(U[:, 1]) ** 2).max() < 1e-14
    # two photons in mode 2: P({j}) = |U_j2|^4, P({j,k}) = 2 |U_j2 U_k2|^2
    P2 = O.threshold_probs(U, [0, 0, 2, 0])
    u = U[:, 2]
    want = [abs(u[j]) ** 4 for j in range(m)] + [2 * abs(u[j] * u[k]) ** 2 for j, k in pats[4:]]
    assert np.abs(P2 - want).max() < 1e-14
    assert abs(O.threshold_probs(U, [1, 1, 1, 0]).sum() - 1) < 1e-12
    # Hong-Ou-Mandel: |1,1> through a 50:50 splitter never clicks both detectors
    bs = np.array([[1, 1j], [1j, 1]]) / np.sqrt(2)
    assert np.abs(O.threshold_probs(bs, [1, 1]) - [0.5, 0.5, 0.0]).max() < 1e-15
    assert np.all(O.threshold_probs(U, [0, 0, 0, 0]) == [1.0])


def test_sample_shots_pins():
    rng = np.random.default_rng(23)
    # identity: the output is the input state with certainty
    s = [0, 2, 1, 0]
    r = O.fock_rank(4, 3, s)
    assert np.all(O.sample_shots(np.eye(4), s, rng.random(100)) == r)
    # Hong-Ou-Mandel: p = (1/2, 0, 1/2) over |2,0>, |1,1>, |0,2>
    bs = np.array([[1, 1j], [1j, 1]]) / np.sqrt(2)
    u = np.array([0.0, 0.25, 0.4999, 0.5001, 0.75, 0.999999])
    assert list(O.sample_shots(bs, [1, 1], u)) == [0, 0, 0, 2, 2, 2]
    # empirical frequencies follow p (chi-square, 6 sigma for its degrees of freedom)
    U = _haar(rng, 4)
    s = [1, 1, 0, 0]
    p = O.probabilities(U, s)
    S = 40000
    counts = np.bincount(O.sample_shots(U, s, rng.random(S)), minlength=p.size)
    keep = p * S > 5
    chi2 = (((counts - p * S) ** 2) / (p * S))[keep].sum()
    dof = int(keep.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_superposition_amplitudes_pins():
    rng = np.random.default_rng(29)
    # (|2,0> + |0,2>)/sqrt2 through a 50:50 splitter is i|1,1> (reversed Hong-Ou-Mandel)
    bs = np.array([[1, 1j], [1j, 1]]) / np.sqrt(2)
    out = O.superposition_amplitudes(bs, [[2, 0], [0, 2]], [1 / np.sqrt(2), 1 / np.sqrt(2)])
    assert np.abs(out - [0, 1j, 0]).max() < 1e-15
    # the identity places the weights at the components' basis positions
    m, n = 4, 3
    comps = [[1, 1, 1, 0], [0, 0, 2, 1], [3, 0, 0, 0]]
    x = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    want = np.zeros(O.fock_dim(m, n), dtype=complex)
    for c, xc in zip(comps, x):
        want[O.fock_rank(m, n, c)] = xc
    assert np.abs(O.superposition_amplitudes(np.eye(m), comps, x) - want).max() < 1e-15
    # U acts unitarily on the n-photon space: the norm is kept
    U = _haar(rng, m)
    x /= np.linalg.norm(x)
    assert abs(np.linalg.norm(O.superposition_amplitudes(U, comps, x)) - 1) < 1e-12


def test_mode_click_probabilities_closed_forms():
    rng = np.random.default_rng(33)
    U = _haar(rng, 4)
    # one photon: a click is the photon, P = |U_ji|^2
    assert np.abs(O.mode_click_probabilities(U, [0, 0, 1, 0]) - np.abs(U[:, 2]) ** 2).max() < 1e-14
    # two photons from mode 1: P(click j) = |U_j1|^2 (2 - |U_j1|^2)
    q = np.abs(U[:, 1]) ** 2
    assert np.abs(O.mode_click_probabilities(U, [0, 2, 0, 0]) - q * (2 - q)).max() < 1e-14
    # Hong-Ou-Mandel: the photons leave together, each detector clicks half the time
    bs = np.array([[1, 1j], [1j, 1]]) / np.sqrt(2)
    assert np.abs(O.mode_click_probabilities(bs, [1, 1]) - [0.5, 0.5]).max() < 1e-15
    # clicks never exceed photons: sum_j P(click j) <= n, and <= the PNR expectations mode by mode
    s = [1, 1, 1, 0]
    c, e = O.mode_click_probabilities(U, s), O.mode_expectations(U, s)
    assert c.sum() <= 3 + 1e-12 and np.all(c <= e + 1e-14)
