"""GPU tests of the autotuner: it times only configurations the library
accepts, keeps the fastest, and the tuned batch still matches the FP64
oracle (probabilities and gradients)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import oracle as O
from paper_2602_11092_amd import _binding as B
from paper_2602_11092_amd.autotune import autotune
from tests.gpu_util import DEV, G_RTOL, P_TOL, rel_err, say, to_dev_c64, widen

pytestmark = pytest.mark.gpu


def _mixed_batch(seed=7, B_=24, m=8):
    rng = np.random.default_rng(seed)
    U = W.haar_unitaries(rng, B_, m).astype(np.complex64)
    occ = np.zeros((B_, m), dtype=np.int32)
    for b in range(B_):
        n = int(rng.integers(1, 5))
        for i in rng.choice(m, size=n, replace=True):
            occ[b, i] += 1
    return U, occ


@pytest.mark.parametrize("case", ["mixed_m8", "haar_m6_n3_b64"])
def test_autotune_choice_and_parity(case):
    if case == "mixed_m8":
        U64, occ = _mixed_batch()
        m, n_max = 8, int(occ.sum(1).max())
    else:
        wl = W.make("haar_m6_n3_b64")
        U64, occ, m, n_max = wl.U.astype(np.complex64), wl.occ, wl.m, 3
    say("autotune", case)
    plan = B.Plan(m, n_max)
    batch = B.Batch(plan, occ)
    Ud = to_dev_c64(U64)
    rep = autotune(batch, Ud, ops=(B.OP_PROBS, B.OP_PROBS_BACKWARD), warmup=1, iters=2)
    for op in (B.OP_PROBS, B.OP_PROBS_BACKWARD):
        r = rep[op]
        assert r["timings"], op
        assert (r["variant"], r["block"], r["tile"]) in [(v, b, t) for v, b, t, _ in r["timings"]]
        assert r["us"] == min(us for _, _, _, us in r["timings"])
        assert not r["rejected"], r["rejected"]  # every supported configuration agrees with the reference
        assert batch.get_config(op) == (r["variant"], r["block"])
        say(op, [(v, b, t, round(us, 1)) for v, b, t, us in r["timings"]])
    # the tuned batch still matches the oracle
    p = B.fock_probs(batch, Ud)
    rng = np.random.default_rng(3)
    gp = rng.random(batch.out_len).astype(np.float32)
    gU = B.fock_probs_backward(batch, Ud, torch.from_numpy(gp).to(DEV))
    torch.cuda.synchronize()
    p, gU = p.cpu().numpy(), gU.cpu().numpy()
    for b in range(batch.B):
        o0, o1 = batch.offsets[b], batch.offsets[b + 1]
        ref = O.probabilities(widen(U64[b]), occ[b])
        assert np.abs(p[o0:o1] - ref).max() <= P_TOL
        if occ[b].sum() > 0:
            g_ref = O.probs_grad(widen(U64[b]), occ[b], gp[o0:o1].astype(np.float64))
            assert rel_err(gU[b], g_ref) <= G_RTOL, (b, rel_err(gU[b], g_ref))


def test_autotune_skips_unsupported_candidates():
    # the fused adjoint at 768 threads is built for at most 20 modes; with 22
    # modes only the supported candidates appear in the timings
    U64, occ = _mixed_batch(seed=11, B_=8, m=22)
    plan = B.Plan(22, int(occ.sum(1).max()))
    batch = B.Batch(plan, occ)
    rep = autotune(batch, to_dev_c64(U64), ops=(B.OP_PROBS_BACKWARD,), warmup=1, iters=1)
    blocks = [(v, b) for v, b, _, _ in rep[B.OP_PROBS_BACKWARD]["timings"]]
    assert (B.VARIANT_FUSED, 768) not in blocks
    assert (B.VARIANT_LAYERED, 256) in blocks
    with pytest.raises(B.SlosError):
        batch.set_config(B.OP_PROBS_BACKWARD, B.VARIANT_FUSED, 768)


def test_autotune_measurement_ops():
    # the expectation, threshold and sampling ops are tuned on their own entry points
    U64, occ = _mixed_batch(seed=21, B_=16, m=8)
    batch = B.Batch(B.Plan(8, int(occ.sum(1).max()), threshold=True), occ)
    Ud = to_dev_c64(U64)
    ops = (B.OP_MODE_EXPECTATIONS, B.OP_THRESHOLD_PROBS, B.OP_SAMPLE, B.OP_MODE_EXPECTATIONS_BACKWARD,
           B.OP_THRESHOLD_PROBS_BACKWARD)
    rep = autotune(batch, Ud, ops=ops, warmup=1, iters=1)
    for op in ops:
        assert rep[op]["timings"] and batch.get_config(op) == (rep[op]["variant"], rep[op]["block"])
    e = B.fock_mode_expectations(batch, Ud).cpu().numpy()
    for b in range(batch.B):
        assert np.abs(e[b] - O.mode_expectations(widen(U64[b]), occ[b])).max() <= 2e-5


def test_autotune_cache_round_trip(tmp_path):
    """The choice is stored under the batch's key and reused without timing;
    a stored choice the batch no longer accepts is tuned again."""
    import json
    U64, occ = _mixed_batch(seed=11, B_=10, m=6)
    batch = B.Batch(B.Plan(6, int(occ.sum(1).max())), occ)
    Ud = to_dev_c64(U64)
    path = str(tmp_path / "tune.json")
    rep1 = autotune(batch, Ud, ops=(B.OP_PROBS, B.OP_PROBS_BACKWARD), warmup=1, iters=1, cache=path)
    data = json.load(open(path))
    from paper_2602_11092_amd.autotune import cache_key
    key = cache_key(batch, Ud.device)
    assert key in data and set(data[key]) == {str(B.OP_PROBS), str(B.OP_PROBS_BACKWARD)}
    fresh = B.Batch(batch.plan, occ)
    rep2 = autotune(fresh, Ud, ops=(B.OP_PROBS, B.OP_PROBS_BACKWARD), warmup=1, iters=1, cache=path)
    for op in (B.OP_PROBS, B.OP_PROBS_BACKWARD):
        assert rep2[op]["cached"] and not rep2[op]["timings"]
        assert fresh.get_config_ex(op) == (rep1[op]["variant"], rep1[op]["block"], rep1[op]["tile"])
    # a stored configuration this batch rejects (768 threads is an adjoint size only) is tuned again
    data[key][str(B.OP_PROBS)] = {"variant": B.VARIANT_FUSED, "block": 768, "tile": 0, "us": 1.0}
    json.dump(data, open(path, "w"))
    rep3 = autotune(B.Batch(batch.plan, occ), Ud, ops=(B.OP_PROBS,), warmup=1, iters=1, cache=path)
    assert not rep3[B.OP_PROBS]["cached"] and rep3[B.OP_PROBS]["timings"]
