"""Capacity: n = 33 complex128 and n = 34 complex64 (128 GiB each) in place on
one GPU, with the capacity gate mix (an H layer generated on demand, then 200
seeded layers of mostly diagonal / permutation gates with 10% dense RX/RY).

At these sizes the oracle cannot hold the state, so parity is checked on
  - sampled amplitudes the oracle computes one index at a time: the same mix
    with the dense gates left out (every gate monomial), full depth;
  - properties that hold at any size: the FP64 norm, and the mirror circuit
    (the 200 layers, then their inverse) returning H^n|0> = 2^(-n/2)
    everywhere, checked on every amplitude;
and at n = 26 (1 GiB) on every sampled amplitude against the full-state oracle
for the full mix at reduced depth, with the same tile shape as the large runs.
"""
import gc
import math

import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

# Per-amplitude tolerances against the FP64 oracle, plus two scale-aware ones
# (the absolute bound alone is loose when amplitudes are ~2^(-n/2)): the
# relative max error 2^(n/2) max|delta| and the normwise error
# ||delta||_2 / ||psi||_2. The complex64 norm bound holds because the FP32
# phases are rounded with error diffusion: T / TDG rounded to nearest would
# each shrink the norm of the half they touch by 3.4e-8.
TOL = {"c128": dict(amp=1e-12, rel=1e-11, normwise=1e-11, norm=1e-12),
       "c64": dict(amp=1e-5, rel=1e-4, normwise=1e-4, norm=1e-5)}
CASES = [(33, "c128"), (34, "c64")]


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_15332_amd as pkg
    return pkg


def _release():
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _full_uniform_error(sv, n):
    """max |a_i - 2^(-n/2)| and sqrt(sum |a_i - 2^(-n/2)|^2) over the whole
    state, chunked so the temporaries stay small."""
    import torch
    t = sv.tensor[0]
    c = 2.0 ** (-0.5 * n)
    mx, ss = 0.0, 0.0
    step = 1 << 27
    for lo in range(0, t.numel(), step):
        d = (t[lo:lo + step].to(torch.complex128) - c).abs()
        mx = max(mx, float(d.max()))
        ss += float((d * d).sum())
    return mx, math.sqrt(ss)


@pytest.mark.parametrize("n,dt", CASES)
def test_capacity_monomial_mix_sampled_vs_oracle(P, n, dt):
    """Full depth, no dense gates: 4096 seeded amplitudes vs the oracle's
    one-index walk; FP64 norm."""
    gates = synth.capacity_circuit(n, 200, 0, p_dense=0.0)
    idx = np.random.default_rng(11).integers(0, 1 << n, 4096, dtype=np.int64)
    idx[:2] = (0, (1 << n) - 1)
    want = O.monomial_amplitudes(n, gates[n:], idx)
    print(f"capacity monomial n={n} {dt}: {len(gates)} gates", flush=True)
    sv = P.StateVector(n, dt)
    try:
        sv.apply(P.gate_array(gates))
        st = sv.plan_stats()
        got = sv.amplitudes(idx)
        nrm = sv.norm()[0]
    finally:
        sv.close()
        del sv
        _release()
    # the H layer and the 1-qubit gates after it: a generated product state
    assert st["generated_product"] >= n
    err = np.abs(got - want)
    print(f"  passes={st['passes']} max|d|={err.max():.3e} "
          f"scaled={err.max() * 2 ** (n / 2):.3e} |norm-1|={abs(nrm - 1):.3e}", flush=True)
    assert err.max() <= TOL[dt]["amp"]
    assert err.max() * 2 ** (n / 2) <= TOL[dt]["rel"]
    assert abs(nrm - 1.0) <= TOL[dt]["norm"]


@pytest.mark.parametrize("n,dt", CASES)
def test_capacity_mirror_full_state(P, n, dt):
    """Full mix (10% dense), full depth: norm after the circuit; then the
    inverse of the 200 layers returns every amplitude to 2^(-n/2)."""
    gates = synth.capacity_circuit(n, 200, 0)
    body = gates[n:]
    inv = synth.inverse_circuit(body)
    print(f"capacity mirror n={n} {dt}: {len(gates)} + {len(inv)} gates", flush=True)
    sv = P.StateVector(n, dt)
    try:
        sv.apply(P.gate_array(gates))
        st = sv.plan_stats()
        nrm = sv.norm()[0]
        sv.apply(P.gate_array(inv))
        nrm2 = sv.norm()[0]
        idx = np.random.default_rng(12).integers(0, 1 << n, 4096, dtype=np.int64)
        samp = sv.amplitudes(idx)
        mx, l2 = _full_uniform_error(sv, n)
    finally:
        sv.close()
        del sv
        _release()
    print(f"  passes={st['passes']} |norm-1|={abs(nrm - 1):.3e} after mirror {abs(nrm2 - 1):.3e} "
          f"max|d|={mx:.3e} normwise={l2:.3e}", flush=True)
    assert st["generated_product"] >= n   # the H layer and the 1-qubit gates after it
    assert abs(nrm - 1.0) <= TOL[dt]["norm"]
    assert abs(nrm2 - 1.0) <= TOL[dt]["norm"]
    assert np.max(np.abs(samp - 2.0 ** (-0.5 * n))) <= TOL[dt]["amp"]
    assert mx <= TOL[dt]["amp"]
    assert l2 <= TOL[dt]["normwise"]


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_capacity_mix_vs_state_oracle_n26(P, dt):
    """The full mix (dense gates included) at n = 26, 12 layers, against the
    full-state oracle on 8192 sampled amplitudes plus the norm."""
    n = 26
    gates = synth.capacity_circuit(n, 12, 5)
    psi = O.simulate(n, gates)
    idx = np.random.default_rng(13).integers(0, 1 << n, 8192, dtype=np.int64)
    want = psi[idx]
    want_norm = O.norm2(psi)
    del psi
    sv = P.StateVector(n, dt)
    try:
        sv.apply(P.gate_array(gates))
        st = sv.plan_stats()
        got = sv.amplitudes(idx)
        nrm = sv.norm()[0]
    finally:
        sv.close()
        del sv
        _release()
    assert st["generated_product"] >= n
    err = np.abs(got - want)
    print(f"capacity n=26 {dt}: max|d|={err.max():.3e}", flush=True)
    assert err.max() <= TOL[dt]["amp"]
    assert abs(nrm - want_norm) <= TOL[dt]["norm"]
