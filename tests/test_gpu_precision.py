"""Precision report: complex64 and complex128 QNN batches against the FP64
oracle. Each case asserts the parity bounds and prints one line with the
measured errors (run with -s to see them):
  max |d amp| over the batch's states, max |d <Z_0>| and max |d norm|,
with <Z_0> and the norm reduced in FP64 on the GPU for both precisions."""
import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_15332_amd as pkg
    return pkg


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,L", [(10, 8), (14, 8), (18, 4)])
def test_qnn_batch_error_vs_oracle(P, dtype, n, L):
    B = 4
    gates = synth.qnn_ansatz(n, L)
    params = synth.qnn_params(n, L, B, 500 + n)
    with P.StateVector(n, dtype, batch=B) as sv:
        sv.set_basis(0)
        sv.apply(P.gate_array(gates), params)
        got = sv.numpy().astype(np.complex128)
        z = sv.expect_z(0)
        nrm = sv.norm()
    d_amp = d_z = d_norm = 0.0
    for b in range(B):
        ref = O.simulate(n, gates, params[b])
        d_amp = max(d_amp, float(np.max(np.abs(got[b] - ref))))
        d_z = max(d_z, abs(z[b] - O.expect_z(ref, 0)))
        d_norm = max(d_norm, abs(nrm[b] - 1.0))
    print(f"precision {dtype} n={n} L={L} B={B}: max|d amp| {d_amp:.2e}  max|d <Z0>| {d_z:.2e}  "
          f"max|d norm| {d_norm:.2e}", flush=True)
    assert d_amp <= TOL[dtype] and d_z <= TOL[dtype] and d_norm <= TOL[dtype]
