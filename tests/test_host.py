"""Host-side checks of the GPU library (CPU only): the shared library loads
and exports every symbol include/slos.h declares, the basis order and the
transition tables agree with an independent enumeration, and argument errors
come back as status codes before any device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_11092_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "slos.h")).read()
    return sorted(set(re.findall(r"SLOS_API\s+[\w\s\*]+?\b(\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared_symbols()
    assert len(names) >= 20
    lib = B.lib()
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for each of them
    assert sorted(B.SIGNATURES) == names


@pytest.mark.parametrize("m,n", [(1, 1), (2, 3), (6, 3), (16, 6), (20, 5), (24, 8), (32, 16)])
def test_fock_dim(m, n):
    assert B.slos_fock_dim(m, n) == math.comb(m + n - 1, n)


def test_fock_dim_invalid():
    assert B.slos_fock_dim(0, 2) == -1
    assert B.slos_fock_dim(3, -1) == -1


@pytest.mark.parametrize("m,n", [(3, 3), (5, 2), (6, 3), (4, 5)])
def test_rank_unrank_match_oracle_order(m, n):
    basis = O.fock_basis(m, n)
    for r, t in enumerate(basis):
        assert (B.slos_fock_unrank(m, n, r) == t).all()
        assert B.slos_fock_rank(m, n, t) == r


def test_rank_unrank_large_sample():
    m, n = 24, 8
    rng = np.random.default_rng(0)
    for r in rng.integers(0, math.comb(m + n - 1, n), 200):
        occ = B.slos_fock_unrank(m, n, int(r))
        assert occ.sum() == n
        assert B.slos_fock_rank(m, n, occ) == r
        assert (occ == O.fock_unrank(m, n, int(r))).all()


@pytest.mark.parametrize("m,k", [(1, 3), (2, 2), (3, 3), (5, 3), (6, 4), (4, 1)])
def test_transition_tables_against_enumeration(m, k):
    pred, succ, nrm, minoff = B.slos_transition_tables(m, k)
    layer = O.fock_basis(m, k)
    prev = O.fock_basis(m, k - 1)
    for r, t in enumerate(layer):
        modes = [j for j in range(m) for _ in range(int(t[j]))]
        seen = set()
        for p in range(k):
            e = int(pred[p, r])
            if p > 0 and modes[p] == modes[p - 1]:
                assert e == -1
                continue
            j = e & 31
            assert j == modes[p]
            tm = t.copy()
            tm[j] -= 1
            assert (e >> 5) == O.fock_rank(m, k - 1, tm)
            seen.add(j)
        assert seen == {j for j in range(m) if t[j] > 0}
        assert abs(nrm[r] - math.sqrt(np.prod([math.factorial(int(v)) for v in t]))) <= 1e-6 * nrm[r]
    for r, t in enumerate(prev):
        for j in range(m):
            tp = t.copy()
            tp[j] += 1
            assert succ[j, r] == O.fock_rank(m, k, tp)
    for c in range(m + 1):
        first = next((r for r, t in enumerate(layer) if min(j for j in range(m) if t[j] > 0) >= c), len(layer))
        assert minoff[c] == first


@pytest.mark.parametrize("m,k", [(2, 2), (5, 3), (8, 4), (12, 5), (20, 5), (24, 3)])
def test_successor_below_the_smallest_mode_is_a_shift(m, k):
    # the fused adjoint forms rank(t' + e_j) for a mode j below the smallest
    # occupied mode of t' as t' + minoff_k(j+1) - N_{k-1} (the states of layer
    # k whose smallest mode j holds one photon end that mode's block, in the
    # order of t'); checked against the successor table and, for small
    # spaces, against the oracle's ranking
    _, succ, _, minoff = B.slos_transition_tables(m, k)
    _, _, _, minoff_p = B.slos_transition_tables(m, k - 1, want_succ=False)
    Nkm1 = math.comb(m + k - 2, k - 1)
    for j in range(m):
        t = np.arange(minoff_p[j + 1], Nkm1)
        assert np.array_equal(succ[j, t], t + minoff[j + 1] - Nkm1)
        if m <= 8:
            for r in t:
                tp = O.fock_unrank(m, k - 1, int(r)).copy()
                tp[j] += 1
                assert O.fock_rank(m, k, tp) == r + minoff[j + 1] - Nkm1


def test_transition_table_edge_counts():
    # every (k-1)-photon state has m successors, so layer k has m * N_{k-1} edges
    for m, k in [(5, 3), (7, 4), (20, 3)]:
        pred, _, _, _ = B.slos_transition_tables(m, k, want_succ=False)
        assert int((pred >= 0).sum()) == m * math.comb(m + k - 2, k - 1)


def test_argument_errors_without_device():
    L = B.lib()
    h = ctypes.c_void_p()
    assert L.slos_plan_create(0, 3, 0, ctypes.byref(h)) == B.SLOS_EINVAL
    assert L.slos_plan_create(33, 3, 0, ctypes.byref(h)) == B.SLOS_EINVAL
    assert L.slos_plan_create(6, 0, 0, ctypes.byref(h)) == B.SLOS_EINVAL
    assert L.slos_plan_create(6, 17, 0, ctypes.byref(h)) == B.SLOS_EINVAL
    assert L.slos_plan_create(6, 3, 16, ctypes.byref(h)) == B.SLOS_EINVAL
    assert L.slos_plan_create(6, 3, 0, None) == B.SLOS_EINVAL
    assert b"m must be" in L.slos_last_error() or len(L.slos_last_error()) > 0
    occ = np.zeros(6, np.int32)
    assert L.slos_fock_unrank(6, 3, 56, occ.ctypes.data_as(ctypes.c_void_p)) == B.SLOS_EINVAL
    assert L.slos_fock_unrank(6, 3, -1, occ.ctypes.data_as(ctypes.c_void_p)) == B.SLOS_EINVAL
    assert L.slos_fock_unrank(6, 3, 0, None) == B.SLOS_EINVAL
    bad = np.array([1, 1, 0, 0, 0, -1], np.int32)
    assert L.slos_fock_rank(6, 1, bad.ctypes.data_as(ctypes.c_void_p)) == -1
    assert L.slos_transition_tables(6, 0, None, None, None, None) == B.SLOS_EINVAL
    assert L.slos_transition_tables(40, 2, None, None, None, None) == B.SLOS_EINVAL
    # compute calls with a NULL batch / bad sizes return before touching the device
    assert L.fock_probs(None, None, None, None, 0, None) == B.SLOS_EINVAL
    assert L.fock_amplitudes(None, None, None, None, 0, None) == B.SLOS_EINVAL
    assert L.fock_probs_backward(None, None, None, None, None, 0, None) == B.SLOS_EINVAL
    assert L.fock_amplitudes_backward(None, None, None, None, None, 0, None) == B.SLOS_EINVAL
    assert L.slos_batch_create(None, 1, None, ctypes.byref(h)) == B.SLOS_EINVAL
    n = ctypes.c_size_t()
    assert L.mesh_workspace_bytes(1, 4, ctypes.byref(n)) == B.SLOS_EINVAL
    assert L.mesh_workspace_bytes(20, 512, ctypes.byref(n)) == B.SLOS_OK and n.value > 0
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    assert L.mesh_to_unitary(40, 1, fake, None, 1.0, fake, fake, 1 << 20, None) == B.SLOS_EINVAL
    assert L.mesh_to_unitary(6, 3, fake, None, 1.0, fake, fake, 1 << 20, None) == B.SLOS_EINVAL  # x NULL needs B = 1
    assert L.mesh_to_unitary(6, 1, fake, fake, 1.0, fake, fake, 8, None) == B.SLOS_EWORKSPACE
    assert L.mesh_to_unitary(6, 1, fake, fake, 1.0, fake, None, 1 << 20, None) == B.SLOS_EWORKSPACE
    assert L.mesh_to_unitary_backward(6, 1, fake, None, 1.0, fake, fake, fake, fake, 1 << 20, None) == B.SLOS_EINVAL
    assert L.mesh_to_unitary_backward(6, 0, fake, fake, 1.0, fake, fake, None, fake, 1 << 20, None) == B.SLOS_EINVAL


def test_plan_without_device_fails_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a device is present")
    except Exception:
        pass
    h = ctypes.c_void_p()
    assert B.lib().slos_plan_create(6, 3, 0, ctypes.byref(h)) == B.SLOS_EHIP
    assert not h.value


def _unbunched_basis(m, k):
    # the Fock basis order restricted to states with every t_j <= 1
    return [t for t in O.fock_basis(m, k) if int(np.max(t, initial=0)) <= 1]


def _dual_rail_basis(m, k):
    # the Fock basis order restricted to states with at most one photon per pair (2g, 2g+1)
    return [t for t in O.fock_basis(m, k) if int(np.max(t.reshape(-1, 2).sum(1), initial=0)) <= 1]


@pytest.mark.parametrize("m,n", [(1, 1), (4, 2), (6, 3), (8, 8), (24, 8), (32, 5)])
def test_unbunched_dim(m, n):
    assert B.slos_unbunched_dim(m, n) == math.comb(m, n)
    assert B.slos_unbunched_dim(3, 4) == 0  # more photons than modes
    assert B.slos_unbunched_dim(0, 1) == -1


@pytest.mark.parametrize("space,m,k", [("unbunched", 4, 1), ("unbunched", 5, 2), ("unbunched", 6, 3),
                                        ("unbunched", 7, 4), ("unbunched", 5, 5), ("dual_rail", 4, 1),
                                        ("dual_rail", 4, 2), ("dual_rail", 6, 2), ("dual_rail", 8, 3),
                                        ("dual_rail", 10, 5)])
def test_restricted_transition_tables_against_enumeration(space, m, k):
    dual = space == "dual_rail"
    pred, succ, nrm, minoff = B.slos_transition_tables(m, k, unbunched=not dual, dual_rail=dual)
    basis = _dual_rail_basis if dual else _unbunched_basis
    layer = basis(m, k)
    prev = basis(m, k - 1)
    assert pred.shape == (k, len(layer))
    assert len(layer) == (math.comb(m // 2, k) * 2 ** k if dual else math.comb(m, k))
    rank = {tuple(int(v) for v in t): r for r, t in enumerate(layer)}
    rank_prev = {tuple(int(v) for v in t): r for r, t in enumerate(prev)}
    for r, t in enumerate(layer):
        modes = [j for j in range(m) if t[j] > 0]
        for p in range(k):
            # one entry per occupied mode: no bunching, so none is empty
            e = int(pred[p, r])
            assert e >= 0
            j = e & 31
            assert j == modes[p]
            tm = t.copy()
            tm[j] -= 1
            assert (e >> 5) == rank_prev[tuple(int(v) for v in tm)]
        assert nrm[r] == 1.0
    for r, t in enumerate(prev):
        for j in range(m):
            tp = t.copy()
            tp[j] += 1
            want = rank.get(tuple(int(v) for v in tp), -1)
            assert succ[j, r] == want, (t, j)
    for c in range(m + 1):
        first = next((r for r, t in enumerate(layer) if min(j for j in range(m) if t[j] > 0) >= c), len(layer))
        assert minoff[c] == first


@pytest.mark.parametrize("q", [1, 2, 3, 5])
def test_dual_rail_logical_order(q):
    # with one photon per pair, state index = the qubit string read big-endian
    m = 2 * q
    assert B.slos_space_dim(m, q, B.PLAN_DUAL_RAIL) == 2 ** q
    layer = _dual_rail_basis(m, q)
    for idx, t in enumerate(layer):
        bits = [int(t[2 * g + 1]) for g in range(q)]
        assert int("".join(map(str, bits)), 2) == idx
    # and the library's tables agree on the size
    pred, _, _, _ = B.slos_transition_tables(m, q, want_succ=False, dual_rail=True)
    assert pred.shape == (q, 2 ** q)


def test_space_dim_flags():
    assert B.slos_space_dim(6, 3) == math.comb(8, 3)
    assert B.slos_space_dim(6, 3, B.PLAN_UNBUNCHED) == 20
    assert B.slos_space_dim(6, 3, B.PLAN_DUAL_RAIL) == 8
    assert B.slos_space_dim(6, 4, B.PLAN_DUAL_RAIL) == 0
    assert B.slos_space_dim(5, 2, B.PLAN_DUAL_RAIL) == -1  # odd m
    assert B.slos_space_dim(6, 2, B.PLAN_UNBUNCHED | B.PLAN_DUAL_RAIL) == -1
    assert B.slos_space_dim(6, 2, 16) == -1
    assert B.slos_space_dim(6, 2, B.PLAN_THRESHOLD) == math.comb(7, 2)


def test_unbunched_argument_errors_without_device():
    # argument checks come before any device call
    L = B.lib()
    h = ctypes.c_void_p()
    assert L.slos_plan_create(3, 4, B.PLAN_UNBUNCHED, ctypes.byref(h)) == B.SLOS_EINVAL  # n_max > m
    assert L.slos_plan_create(3, 2, 16, ctypes.byref(h)) == B.SLOS_EINVAL  # unknown flag
    assert L.slos_plan_create(5, 2, B.PLAN_DUAL_RAIL, ctypes.byref(h)) == B.SLOS_EINVAL  # odd m
    assert L.slos_plan_create(6, 4, B.PLAN_DUAL_RAIL, ctypes.byref(h)) == B.SLOS_EINVAL  # n_max > m/2
    assert L.slos_plan_create(6, 2, B.PLAN_DUAL_RAIL | B.PLAN_UNBUNCHED, ctypes.byref(h)) == B.SLOS_EINVAL
    with pytest.raises(B.SlosError):
        B.slos_transition_tables(3, 4, unbunched=True)


def test_quantum_layer_computation_space_arguments():
    from paper_2602_11092_amd import QuantumLayer
    assert QuantumLayer(6, [1, 1, 1, 0, 0, 0], computation_space="unbunched").output_size == 20
    assert QuantumLayer(6, [1, 1, 1, 0, 0, 0]).output_size == 56
    with pytest.raises(ValueError):
        QuantumLayer(3, [2, 1, 1], computation_space="unbunched")
    assert QuantumLayer(6, [1, 0, 1, 0, 1, 0], computation_space="dual_rail").output_size == 8
    with pytest.raises(ValueError):
        QuantumLayer(5, [1, 0, 1, 0, 0], computation_space="dual_rail")
    with pytest.raises(ValueError):
        QuantumLayer(3, [1, 1, 0], computation_space="dual")
    assert QuantumLayer(6, [1, 1, 1, 0, 0, 0], measurement="mode_expectations").output_size == 6


@pytest.mark.parametrize("m,n", [(4, 0), (4, 1), (4, 2), (5, 3), (3, 5), (20, 5), (24, 8)])
def test_threshold_dim(m, n):
    want = 1 if n == 0 else sum(math.comb(m, k) for k in range(1, min(n, m) + 1))
    assert B.slos_threshold_dim(m, n) == want
    assert B.slos_threshold_dim(0, 2) == -1


def test_threshold_layer_output_size():
    from paper_2602_11092_amd import QuantumLayer
    assert QuantumLayer(4, [1, 1, 0, 0], measurement="threshold_probs").output_size == 4 + 6


@pytest.mark.parametrize("flags,m,n", [(0, 5, 3), (B.PLAN_UNBUNCHED, 6, 3), (B.PLAN_DUAL_RAIL, 8, 3),
                                       (B.PLAN_DUAL_RAIL, 6, 3), (B.PLAN_UNBUNCHED, 4, 4)])
def test_space_rank_unrank_match_enumeration(flags, m, n):
    basis = O.fock_basis(m, n)
    if flags == B.PLAN_UNBUNCHED:
        basis = [t for t in basis if t.max() <= 1]
    elif flags == B.PLAN_DUAL_RAIL:
        basis = [t for t in basis if t.reshape(-1, 2).sum(1).max() <= 1]
    assert B.slos_space_dim(m, n, flags) == len(basis)
    for r, t in enumerate(basis):
        assert np.array_equal(B.slos_space_unrank(m, n, flags, r), t)
        assert B.slos_space_rank(m, n, flags, t) == r
    if flags:  # a state outside the space has no rank
        out = np.zeros(m, dtype=np.int32)
        out[0] = 2
        out[1] = n - 2
        assert B.slos_space_rank(m, n, flags, out) == -1
    with pytest.raises(B.SlosError):
        B.slos_space_unrank(m, n, flags, len(basis))


@pytest.mark.parametrize("m,n", [(4, 0), (4, 2), (5, 3), (3, 5)])
def test_threshold_pattern_order(m, n):
    pats = O.click_patterns(m, n)
    assert B.slos_threshold_dim(m, n) == len(pats)
    for q, c in enumerate(pats):
        want = np.zeros(m, dtype=np.int32)
        want[list(c)] = 1
        assert np.array_equal(B.slos_threshold_pattern(m, n, q), want)
    with pytest.raises(B.SlosError):
        B.slos_threshold_pattern(m, n, len(pats))


def test_workspace_cache_retires_instead_of_freeing():
    """A workspace handed to a call may be captured in a HIP graph: the cache
    never frees one while it lives, grows geometrically, and keeps separate
    buffers per key (op and stream)."""
    c = B.WorkspaceCache()
    a = c.get(("op", 1), 1000, "cpu")
    assert a.numel() == 1024 and a.dtype.itemsize == 1
    assert c.get(("op", 1), 700, "cpu") is a          # fits: the same buffer
    b = c.get(("op", 1), 5000, "cpu")                   # grows: a is retired, not dropped
    assert b is not a and b.numel() == 8192
    assert c.retired() == 1 and any(r is a for r in c._retired)
    assert c.get(("op", 1), 1000, "cpu") is b          # smaller again: keeps the larger one
    other = c.get(("op", 2), 1000, "cpu")               # another stream: its own buffer
    assert other is not b
    assert c.get(("op", 1), 0, "cpu") is b
    assert B.WorkspaceCache._round(1) == 256 and B.WorkspaceCache._round(257) == 512


def test_autotune_gate_comparison_and_cache_files(tmp_path):
    """Host logic of the autotuner: the gate's comparison rejects a
    perturbed output, a non-finite one and a shape mismatch; the cache file
    round-trips entries and survives a missing or corrupt file."""
    from paper_2602_11092_amd import autotune as T
    ref = np.linspace(0, 1, 50).astype(np.float32)
    assert T.agrees(B.OP_PROBS, ref.copy(), ref)
    assert not T.agrees(B.OP_PROBS, ref + 2e-6, ref)
    bad = ref.copy()
    bad[3] = np.nan
    assert not T.agrees(B.OP_PROBS, bad, ref)
    assert not T.agrees(B.OP_PROBS, ref[:-1], ref)
    g = np.ones((2, 3, 3), np.complex64)
    assert T.agrees(B.OP_PROBS_BACKWARD, g * (1 + 5e-6), g)
    assert not T.agrees(B.OP_PROBS_BACKWARD, g * (1 + 5e-5), g)
    shots = np.arange(100, dtype=np.int32).reshape(2, 50)
    near = shots.copy()
    near[0, 0] += 1  # one shot of 100 on the other side of a boundary
    assert T.agrees(B.OP_SAMPLE, near, shots)
    near[1, :5] += 1
    assert not T.agrees(B.OP_SAMPLE, near, shots)
    path = str(tmp_path / "sub" / "tune.json")
    assert T._load_cache(path) == {}
    T._store_cache(path, "k1", 1, {"variant": 3, "block": 1024, "tile": 4, "us": 50.0})
    T._store_cache(path, "k1", 3, {"variant": 1, "block": 768, "tile": 0, "us": 200.0})
    assert T._load_cache(path)["k1"]["1"]["tile"] == 4 and T._load_cache(path)["k1"]["3"]["block"] == 768
    open(path, "w").write("{ not json")
    assert T._load_cache(path) == {}
