"""The allocation-free readout sv_expect_z_noalloc against sv_expect_z and
sv_norm (the same FP64 fixed-order reduction, but with partial sums in a
file-scope device array and the result left in device memory): two calls in a
row on one GPU, the second on a smaller input, so that whatever the first left
in the shared array must not leak into the second."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_15332_amd as pkg
    return pkg


def _readouts(P, n, dtype, batch, layers, seed):
    """States of the QNN ansatz for `batch` seeded parameter sets; the
    handle-based readouts (<Z_0>, <Z_{n-1}>, norm) and the no-allocation ones
    for the same states."""
    import torch
    gates = synth.qnn_ansatz(n, layers)
    params = synth.qnn_params(n, layers, batch, seed)
    with P.StateVector(n, dtype, batch) as sv:
        sv.apply(gates, params)
        want = [sv.expect_z(0), sv.expect_z(n - 1), sv.norm()]
        got = []
        for q in (0, n - 1, -1):
            out = torch.full((batch,), float("nan"), dtype=torch.float64, device=sv.tensor.device)
            P.sv.expect_z_noalloc(sv.tensor, n, q, out, stream=sv.stream)
            sv.stream.synchronize()
            got.append(out.cpu().numpy())
    return want, got


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_readout_matches_handle_readout(P, dtype):
    # a larger input (1,024 partial sums per state), then a smaller one (one
    # partial sum per state, fewer states) on the same shared scratch
    for n, batch, layers, seed in ((22, 5, 2, 11), (12, 2, 3, 12)):
        want, got = _readouts(P, n, dtype, batch, layers, seed)
        for w, g in zip(want, got):
            err = float(np.max(np.abs(w - g)))
            print(f"noalloc {dtype} n={n} batch={batch}: max|d| = {err:.3e}", flush=True)
            assert np.all(np.isfinite(g))
            assert err <= TOL[dtype]


def test_noalloc_rejects_oversized_batch(P):
    import torch
    n, batch = 22, 65   # 65 * 1024 partial sums > 65,536
    state = torch.zeros((batch, 1 << n), dtype=torch.complex64, device="cuda")
    out = torch.full((batch,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SVError) as e:
        P.sv.expect_z_noalloc(state, n, 0, out)
    assert e.value.status == P.sv.SV_EINVAL and "scratch" in P.last_error()
    assert torch.all(out == 7.0)
