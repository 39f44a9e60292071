"""Serving engine: every result matches the oracle, a request's result is the
same alone and inside a mixed stream, admission by HBM footprint, errors."""
import time

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
    import time
    got = {}
    t0 = time.perf_counter()
    while len(got) < count:
        res = eng.poll(wait_us=200_000)
        assert res or eng.stats()["in_flight"] or eng.stats()["queued"], "engine stalled"
        got.update(res)
        assert (time.perf_counter() - t0) * 1e6 < timeout_us, f"engine did not drain: {len(got)}/{count}"
    return got


@pytest.mark.parametrize("stepped", [False, True])
@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c128", 1e-12)])
def test_mixed_stream_matches_oracle_and_solo(P, dtype, tol, stepped):
    pkg, serving = P
    reqs = synth.poisson_requests(40, 1e9, seed=7, n_range=(8, 16), layer_range=(2, 5))
    with serving.ServingEngine(dtype, max_batch=16, n_streams=4, stepped=stepped) as eng:
        for r in reqs:
            eng.submit(r.rid, r.n, _gates(pkg, r), r.params, 0)
        mixed = _drain(eng, len(reqs))
        st = eng.stats()
    assert st["completed"] == len(reqs) and st["groups"] < len(reqs)
    for r in reqs:
        ref = O.loss_z(r.n, synth.qnn_ansatz(r.n, r.layers), r.params)
        assert abs(mixed[r.rid] - ref) <= tol, (r.n, r.layers)
    # alone: one request per engine, one request per group or step
    for r in reqs[:12]:
        with serving.ServingEngine(dtype, max_batch=1, n_streams=1, stepped=stepped) as eng:
            eng.submit(r.rid, r.n, _gates(pkg, r), r.params, 0)
            solo = _drain(eng, 1)
        assert solo[r.rid] == mixed[r.rid]


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c128", 1e-12)])
def test_stepped_requests_join_while_others_run(P, dtype, tol):
    """Requests of different n and depth submitted while earlier ones are
    still on the GPU join at the next step: all results match the oracle and
    equal each request's result alone, and steps held several requests."""
    pkg, serving = P
    reqs = synth.poisson_requests(24, 1e9, seed=21, n_range=(13, 19), layer_range=(2, 9))
    with serving.ServingEngine(dtype, max_batch=8, n_streams=2, stepped=True, max_active=16) as eng:
        got = {}
        for i, r in enumerate(reqs):
            eng.submit(r.rid, r.n, _gates(pkg, r), r.params, 0)
            if i % 4 == 3:
                got.update(eng.poll(wait_us=0))   # launch steps between arrivals
        st0 = eng.stats()
        got.update(_drain(eng, len(reqs) - len(got)))
        st = eng.stats()
    assert st["completed"] == len(reqs) and st["largest_group"] > 1 and st0["in_flight"] > 0
    for r in reqs:
        ref = O.loss_z(r.n, synth.qnn_ansatz(r.n, r.layers), r.params)
        assert abs(got[r.rid] - ref) <= tol, (r.n, r.layers)
    for r in reqs[:4]:
        with serving.ServingEngine(dtype, max_batch=1, n_streams=1, stepped=True, max_active=1) as eng:
            eng.submit(r.rid, r.n, _gates(pkg, r), r.params, 0)
            assert _drain(eng, 1)[r.rid] == got[r.rid]


@pytest.mark.parametrize("stepped", [False, True])
def test_admission_by_hbm_footprint(P, stepped):
    pkg, serving = P
    n = 18                               # 2 MiB per complex64 state
    reqs = synth.poisson_requests(12, 1e9, seed=3, n_range=(n, n), layer_range=(2, 2))
    budget = 3 * (1 << n) * 8            # room for three states at a time
    with serving.ServingEngine("c64", max_batch=8, n_streams=4, hbm_budget_bytes=budget,
                               stepped=stepped) as eng:
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


def test_stepped_state_buffers_across_sizes(P):
    """The stepped engine keeps finished requests' state buffers for the
    next requests of the same size; a request of another size that needs new
    memory beyond the budget first returns them to the pool. Six n = 17
    requests, then three n = 18 ones under a budget of three n = 18 states,
    then n = 17 again: every result against the oracle, the live state bytes
    within the budget throughout."""
    pkg, serving = P
    budget = 3 * (1 << 18) * 8
    rounds = [synth.poisson_requests(6, 1e9, seed=5, n_range=(17, 17), layer_range=(2, 2)),
              synth.poisson_requests(3, 1e9, seed=6, n_range=(18, 18), layer_range=(2, 2)),
              synth.poisson_requests(4, 1e9, seed=7, n_range=(17, 17), layer_range=(2, 2))]
    got = {}
    with serving.ServingEngine("c64", max_batch=8, n_streams=2, hbm_budget_bytes=budget, stepped=True) as eng:
        for k, reqs in enumerate(rounds):
            for r in reqs:
                eng.submit(1000 * k + r.rid, r.n, _gates(pkg, r), r.params, 0)
            want = sum(len(x) for x in rounds[:k + 1])
            t0 = time.time()
            while len(got) < want:
                assert time.time() - t0 < 60, "requests did not finish"
                got.update(eng.poll(wait_us=100_000))
                assert eng.stats()["state_bytes"] <= budget
    for k, reqs in enumerate(rounds):
        for r in reqs:
            ref = O.loss_z(r.n, synth.qnn_ansatz(r.n, 2), r.params)
            assert abs(got[1000 * k + r.rid] - ref) <= 1e-5


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
    # a state that could never fit the HBM budget is refused at submission,
    # and small states behind a waiting larger one still run
    with serving.ServingEngine("c64", hbm_budget_bytes=(1 << 16) * 8) as eng:
        with pytest.raises(pkg.SVError) as e:
            eng.submit(4, 17, [synth.Gate("X", 0)])
        assert e.value.status == -2
        assert eng.poll() == []


@pytest.mark.parametrize("stepped", [False, True])
def test_registered_circuits(P, stepped):
    """Requests submitted by registered circuit handle give the results of
    the same requests submitted with their gate lists."""
    pkg, serving = P
    reqs = synth.poisson_requests(16, 1e9, seed=5, n_range=(10, 15), layer_range=(2, 4))
    with serving.ServingEngine("c64", max_batch=8, n_streams=2, stepped=stepped) as eng:
        cid = {}
        for r in reqs:
            k = (r.n, r.layers)
            if k not in cid:
                cid[k] = eng.register(r.n, _gates(pkg, r), len(r.params), 0)
            eng.submit_registered(r.rid, cid[k], r.params)
        by_handle = _drain(eng, len(reqs))
        with pytest.raises(pkg.SVError):
            eng.submit_registered(999, len(cid) + 5, reqs[0].params)
        with pytest.raises(pkg.SVError):
            eng.submit_registered(998, cid[(reqs[0].n, reqs[0].layers)], reqs[0].params[:-1])
    with serving.ServingEngine("c64", max_batch=8, n_streams=2, stepped=stepped) as eng:
        for r in reqs:
            eng.submit(r.rid, r.n, _gates(pkg, r), r.params, 0)
        by_gates = _drain(eng, len(reqs))
    assert by_handle == by_gates
