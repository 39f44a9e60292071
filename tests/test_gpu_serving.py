"""Serving engine: every result matches the oracle, a request's result is the
same alone and inside a mixed stream, admission by HBM footprint, errors."""
import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_15332_amd as pkg
    from paper_2411_15332_amd import serving
    return pkg, serving


def _gates(P, r):
    return P.gate_array(synth.qnn_ansatz(r.n, r.layers))


def _drain(eng, count, timeout_us=30_000_000):
    got = {}
    while len(got) < count:
        res = eng.poll(wait_us=200_000)
        assert res or eng.stats()["in_flight"] or eng.stats()["queued"], "engine stalled"
        got.update(res)
    return got


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c128", 1e-12)])
def test_mixed_stream_matches_oracle_and_solo(P, dtype, tol):
    pkg, serving = P
    reqs = synth.poisson_requests(40, 1e9, seed=7, n_range=(8, 16), layer_range=(2, 5))
    with serving.ServingEngine(dtype, max_batch=16, n_streams=4) as eng:
        for r in reqs:
            eng.submit(r.rid, r.n, _gates(pkg, r), r.params, 0)
        mixed = _drain(eng, len(reqs))
        st = eng.stats()
    assert st["completed"] == len(reqs) and st["groups"] < len(reqs)
    for r in reqs:
        ref = O.loss_z(r.n, synth.qnn_ansatz(r.n, r.layers), r.params)
        assert abs(mixed[r.rid] - ref) <= tol, (r.n, r.layers)
    # alone: one request per engine, one request per group
    for r in reqs[:12]:
        with serving.ServingEngine(dtype, max_batch=1, n_streams=1) as eng:
            eng.submit(r.rid, r.n, _gates(pkg, r), r.params, 0)
            solo = _drain(eng, 1)
        assert solo[r.rid] == mixed[r.rid]


def test_admission_by_hbm_footprint(P):
    pkg, serving = P
    n = 18                               # 2 MiB per complex64 state
    reqs = synth.poisson_requests(12, 1e9, seed=3, n_range=(n, n), layer_range=(2, 2))
    budget = 3 * (1 << n) * 8            # room for three states at a time
    with serving.ServingEngine("c64", max_batch=8, n_streams=4, hbm_budget_bytes=budget) as eng:
        for r in reqs:
            eng.submit(r.rid, r.n, _gates(pkg, r), r.params, 0)
        got = {}
        peak = 0
        while len(got) < len(reqs):
            got.update(eng.poll(wait_us=100_000))
            st = eng.stats()
            peak = max(peak, st["state_bytes"])
            assert st["state_bytes"] <= budget
        assert st["largest_group"] <= 3
    for r in reqs[:3]:
        ref = O.loss_z(n, synth.qnn_ansatz(n, 2), r.params)
        assert abs(got[r.rid] - ref) <= 1e-5


def test_submit_validation(P):
    pkg, serving = P
    with serving.ServingEngine("c64") as eng:
        with pytest.raises(pkg.SVError):
            eng.submit(1, 4, [synth.Gate("X", 5)])
        with pytest.raises(pkg.SVError):
            eng.submit(2, 4, [synth.Gate("RY", 0, -1, 0.0, 3)], np.zeros(2))
        with pytest.raises(pkg.SVError) as e:
            eng.submit(3, 31, [synth.Gate("X", 0)])
        assert e.value.status == -4
        assert eng.poll() == []
