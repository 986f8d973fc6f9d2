"""Autotuner: candidates accepted by the library, cache round trip, and (GPU)
a tuned plan gives the same product as the default one."""
import json

import numpy as np
import pytest

from paper_2603_21444_amd import binding
from paper_2603_21444_amd import autotune


def test_every_candidate_is_accepted_by_the_library():
    p = binding.Plan()
    for b, cands in autotune.CANDIDATES.items():
        for lanes, sub in cands:
            for s in autotune.SYM_SUB_CANDIDATES:
                t = binding.default_tuning()
                t.lanes[b], t.sub[b], t.sym_sub[b] = lanes, sub, s
                p.set_tuning(t)  # raises SpgError when rejected
    for sub in autotune.HEAVY_SUB_CANDIDATES:
        t = binding.default_tuning()
        t.sub[autotune.HEAVY_BIN] = t.sym_sub[autotune.HEAVY_BIN] = sub
        p.set_tuning(t)


def test_every_edge_candidate_is_accepted_and_capacity_enforced():
    p = binding.Plan()
    for b in range(1, autotune.LAST_TUNED_EDGE_BIN + 1):
        for f in autotune.EDGE_FRACTIONS:
            t = binding.default_tuning()
            t.bin_edge[b] = autotune.edge_for(b, f)
            p.set_tuning(t)
        t = binding.default_tuning()
        t.bin_edge[b] = autotune.BIN_EDGES[b] + 1  # beyond the bin's tables
        with pytest.raises(binding.SpgError):
            p.set_tuning(t)
        t.bin_edge[b] = -1
        with pytest.raises(binding.SpgError):
            p.set_tuning(t)


def test_library_rejects_bad_symbolic_sub():
    p = binding.Plan()
    for bad in (0, 3, 128):
        t = binding.default_tuning()
        t.sym_sub[4] = bad
        with pytest.raises(binding.SpgError):
            p.set_tuning(t)


def test_candidates_cover_the_default():
    # the library caps lanes-per-entry at lanes-per-row
    t = binding.default_tuning()
    for b, cands in autotune.CANDIDATES.items():
        assert (t.lanes[b], min(t.sub[b], t.lanes[b])) in cands, b
        assert t.sym_sub[b] in autotune.SYM_SUB_CANDIDATES, b
    assert t.sub[autotune.HEAVY_BIN] in autotune.HEAVY_SUB_CANDIDATES
    assert t.sym_sub[autotune.HEAVY_BIN] in autotune.HEAVY_SUB_CANDIDATES


def test_json_round_trip():
    t = binding.default_tuning()
    t.lanes[5], t.sub[5], t.sym_sub[5] = 32, 8, 16
    t.heavy_slots = 7
    t.bin_edge[6] = autotune.edge_for(6, 0.75)
    d = json.loads(json.dumps(autotune._to_json(t)))
    u = autotune._from_json(d)
    assert list(u.bin_edge) == list(t.bin_edge)
    assert list(u.lanes) == list(t.lanes)
    assert list(u.sub) == list(t.sub)
    assert list(u.sym_sub) == list(t.sym_sub)
    assert u.heavy_slots == 7 and u.max_window == t.max_window


def test_cache_key_separates_workloads():
    class M:
        def __init__(self, shape):
            self.shape = shape
    a, b = [M((100, 50))], [M((50, 70))]
    k1 = autotune._key(a, b, "float32", [0, 10, 1000] + [0] * 13)
    k2 = autotune._key(a, b, "float64", [0, 10, 1000] + [0] * 13)
    k3 = autotune._key(a, b, "float32", [0, 10, 3000] + [0] * 13)
    k4 = autotune._key(a, b, "float32", [0, 11, 1100] + [0] * 13)
    assert len({k1, k2, k3}) == 3
    assert k1 == k4  # same rounded histogram


@pytest.mark.gpu
def test_tuned_plan_matches_default(tmp_path):
    import torch
    from paper_2603_21444_amd import synth
    import oracle
    from helpers import assert_same_csr
    A = synth.varnnz_csr(3000, 4000, 1, 60, 41, np.float64, "u01", stream=0)
    B = synth.varnnz_csr(4000, 5000, 1, 60, 41, np.float64, "u01", stream=1)
    dA, dB = binding.to_device(A), binding.to_device(B)
    t = autotune.tune([dA], [dB], reps=1, cache_path=str(tmp_path / "t.json"), share=0.0)
    assert (tmp_path / "t.json").exists()
    t2 = autotune.tune([dA], [dB], reps=1, cache_path=str(tmp_path / "t.json"))
    assert list(t2.lanes) == list(t.lanes) and list(t2.sub) == list(t.sub)
    assert list(t2.sym_sub) == list(t.sym_sub)
    plan = binding.Plan(tuning=t)
    rp, nnz = plan.symbolic([dA], [dB])
    col, vals = plan.numeric([dA], [dB], rp, nnz)
    torch.cuda.synchronize()
    got = binding.DeviceCSR((3000, 5000), rp, col, vals).to_host()
    ref, S = oracle.spgemm(A, B, with_abs=True)
    assert_same_csr(got, ref, S, np.float64, what="tuned plan")


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_every_candidate_gives_the_oracle_product(dtype):
    """Every bin under each of its candidates (and the extreme lanes-per-entry
    settings 1 and 64, in both passes) gives the oracle's product on rows
    spanning all LDS bins."""
    import torch
    from paper_2603_21444_amd import synth
    import oracle
    from helpers import assert_same_csr
    A = synth.varnnz_csr(3000, 4000, 0, 200, 9, dtype, "normal", stream=0)
    B = synth.varnnz_csr(4000, 30000, 0, 64, 9, dtype, "normal", stream=1)
    dA, dB = binding.to_device(A), binding.to_device(B)
    ref, S = oracle.spgemm(A.with_data(A.data.astype(np.float64)),
                           B.with_data(B.data.astype(np.float64)), with_abs=True)
    settings = []
    for i in range(4):
        t = binding.default_tuning()
        for b, cands in autotune.CANDIDATES.items():
            t.lanes[b], t.sub[b] = cands[i % len(cands)]
            t.sym_sub[b] = autotune.SYM_SUB_CANDIDATES[i % len(autotune.SYM_SUB_CANDIDATES)]
        settings.append((f"candidate {i}", t))
    for sub, ssub in ((1, 64), (64, 1)):
        t = binding.default_tuning()
        for b in range(1, autotune.HEAVY_BIN + 1):  # the heavy rows' too
            t.sub[b], t.sym_sub[b] = sub, ssub
        settings.append((f"sub {sub} sym_sub {ssub}", t))
    for sub in autotune.HEAVY_SUB_CANDIDATES:
        t = binding.default_tuning()
        t.sub[autotune.HEAVY_BIN] = t.sym_sub[autotune.HEAVY_BIN] = sub
        settings.append((f"heavy rows: sub {sub}", t))
    for f in autotune.EDGE_FRACTIONS[1:] + (0.3,):
        t = binding.default_tuning()
        for b in range(1, 12):
            t.bin_edge[b] = autotune.edge_for(b, f)
        settings.append((f"bin edges at {f} of capacity", t))
    t = binding.default_tuning()
    for b in range(1, 12):  # decreasing raw edges: made non-decreasing by the library
        t.bin_edge[b] = min(autotune.BIN_EDGES[b], 300 - 20 * b)
    settings.append(("non-monotone edges", t))
    for what, t in settings:
        plan = binding.Plan(tuning=t)
        rp, nnz = plan.symbolic([dA], [dB])
        col, vals = plan.numeric([dA], [dB], rp, nnz)
        torch.cuda.synchronize()
        got = binding.DeviceCSR(A.shape[:1] + B.shape[1:], rp, col, vals).to_host()
        assert_same_csr(got, ref, S, dtype, what=what)
