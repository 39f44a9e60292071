"""Adjoint backward (sv_adjoint_expect_z / QNNFunction) against the oracle's
parameter-shift rule (exact for exp(-i t P / 2)) and central differences."""
import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu
TOL_PS = {"c128": 1e-10, "c64": 1e-4}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2411_15332_amd as pkg
    return pkg


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,L,B", [(3, 2, 3), (6, 2, 2), (12, 2, 2), (14, 1, 2)])
def test_adjoint_matches_parameter_shift(P, n, L, B, dtype):
    gates = synth.qnn_ansatz(n, L)
    params = synth.qnn_params(n, L, B, 100 + n)
    with P.StateVector(n, dtype, batch=B) as sv:
        f, g = sv.adjoint_expect_z(gates, params, qubit=0)
    which = list(range(params.shape[1])) if n <= 6 else list(range(0, params.shape[1], 7))
    for b in range(B):
        assert abs(f[b] - O.loss_z(n, gates, params[b])) <= TOL_PS[dtype]
        ps = O.grad_param_shift(n, gates, params[b], which)
        assert np.max(np.abs(g[b, which] - ps)) <= TOL_PS[dtype]
        if b == 0 and dtype == "c128":
            fd = O.grad_fd(n, gates, params[b], which[:6])
            assert np.max(np.abs(g[b, which[:6]] - fd)) <= 1e-7


def test_adjoint_general_circuit(P):
    """Rotations on every axis between non-parametric gates of every kind,
    gradient on a qubit other than 0."""
    n = 11
    rng = np.random.default_rng(3)
    base = synth.random_circuit(n, 3, 9)
    gates, k = [], 0
    for g in base:
        gates.append(g)
        if g.name in ("RX", "RY", "RZ"):
            gates[-1] = g._replace(param=k)
            k += 1
    params = rng.uniform(-3, 3, size=(2, k))
    with P.StateVector(n, "c128", batch=2) as sv:
        f, g = sv.adjoint_expect_z(gates, params, qubit=4)
        final = sv.numpy()
    for b in range(2):
        ref = O.simulate(n, gates, params[b])
        assert np.max(np.abs(final[b] - ref)) <= 1e-12
        assert abs(f[b] - O.expect_z(ref, 4)) <= 1e-12
        ps = O.grad_param_shift(n, gates, params[b], list(range(k)), qubit=4)
        assert np.max(np.abs(g[b] - ps)) <= 1e-10


def _rotation_layers(n, layers, seed):
    """Layers of RX / RY / RZ (random axis) on every qubit, each with its own
    parameter, separated by CNOT chains; returns (gates, number of parameters)."""
    rng = np.random.default_rng(seed)
    gates, k = [], 0
    for layer in range(layers):
        for q in range(n):
            gates.append(synth.Gate(("RX", "RY", "RZ")[int(rng.integers(3))], q, -1, 0.0, k))
            k += 1
        for q in range(layer % 2, n - 1, 2):
            gates.append(synth.Gate("CNOT", q, q + 1))
    return gates, k


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_high_qubit_terms(P, dtype):
    """X and Y generators on qubits >= 12, whose partners lie outside a
    2^12-amplitude chunk (the fused high-qubit inner products), next to Z terms
    and low-qubit terms of the same runs; gradient on a high qubit."""
    n = 16
    gates, k = _rotation_layers(n, 3, 11)
    params = np.random.default_rng(12).uniform(-3, 3, size=(2, k))
    high_xy = [g.param for g in gates if g.param >= 0 and g.q0 >= 12 and g.name != "RZ"]
    assert len(high_xy) >= 6
    which = high_xy + [g.param for g in gates if g.param >= 0 and g.q0 < 12][::9]
    with P.StateVector(n, dtype, batch=2) as sv:
        f, g = sv.adjoint_expect_z(gates, params, qubit=13)
    for b in range(2):
        assert abs(f[b] - O.loss_z(n, gates, params[b], qubit=13)) <= TOL_PS[dtype]
        ps = O.grad_param_shift(n, gates, params[b], which, qubit=13)
        assert np.max(np.abs(g[b, which] - ps)) <= TOL_PS[dtype]


@pytest.mark.parametrize("n,dt", [(16, "c128"), (20, "c128"), (20, "c64")])
def test_adjoint_z_terms_on_every_bit_class(P, n, dt):
    """Z generators (RZ) on thread bits (q < 10), on register-slot bits of
    the sub-chunk kernel (q = 10, 11) and on sub-chunk base bits (q >= 12):
    at n = 20 a block walks 8 sub-chunks, so q = 12..14 take the signed sums
    over the block's sub-chunks and q >= 15 a sign uniform over the block;
    X / Y generators on every low qubit in the runs before them (thread and
    slot bits of the 12-term kernel). Every sampled RZ gradient, and the X / Y
    ones on slot bits, against parameter shift."""
    gates, k = [], 0
    for layer in range(3):
        for q in range(n):
            gates.append(synth.Gate(("RY", "RX")[(q + layer) % 2], q, -1, 0.0, k))
            k += 1
        for q in range(n):
            gates.append(synth.Gate("RZ", q, -1, 0.0, k))
            k += 1
        for q in range(layer % 2, n - 1, 2):
            gates.append(synth.Gate("CNOT", q, q + 1))
    params = np.random.default_rng(31).uniform(-3, 3, size=(2, k))
    rz = [g for g in gates if g.name == "RZ"]
    zq = (3, 10, 11, 12, 13, 15) if n == 16 else (3, 10, 11, 12, 14, 15, 19)
    which = [g.param for g in rz if g.q0 in zq]
    which += [g.param for g in gates if g.name in ("RX", "RY") and g.q0 in (9, 10, 11)][:4]
    assert {g.q0 for g in rz if g.param in which} >= {10, 12, 15}
    tol = (1e-12, 1e-10) if dt == "c128" else (1e-5, 1e-4)
    with P.StateVector(n, dt, batch=2) as sv:
        f, g = sv.adjoint_expect_z(gates, params, qubit=2)
    for b in range(2):
        assert abs(f[b] - O.loss_z(n, gates, params[b], qubit=2)) <= tol[0]
        ps = O.grad_param_shift(n, gates, params[b], which, qubit=2)
        assert np.max(np.abs(g[b, which] - ps)) <= tol[1]


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_adjoint_z_terms_across_diagonal_gates(P, dt):
    """Z-generator gradients taken after undoing only diagonal gates (an RZ
    run's own undo, fixed CZ / S / T) join an earlier run's read of the
    states; a non-diagonal gate to undo first (H, CNOT) sends them out at the
    point they belong to. Every gradient against parameter shift."""
    n = 14
    gates, k = [], 0
    for q in range(n):
        gates.append(synth.Gate("RY", q, -1, 0.0, k)); k += 1
    gates.append(synth.Gate("H", 3))
    for q in range(n):
        gates.append(synth.Gate("RZ", q, -1, 0.0, k)); k += 1
    gates += [synth.Gate("CZ", 0, 1), synth.Gate("S", 2), synth.Gate("T", 12)]
    for q in range(7):
        gates.append(synth.Gate("RZ", q, -1, 0.0, k)); k += 1
    gates.append(synth.Gate("CNOT", 1, 2))
    for q in range(n):
        gates.append(synth.Gate("RX", q, -1, 0.0, k)); k += 1
    params = np.random.default_rng(41).uniform(-3, 3, size=(2, k))
    tol = (1e-12, 1e-10) if dt == "c128" else (1e-5, 1e-4)
    with P.StateVector(n, dt, batch=2) as sv:
        f, g = sv.adjoint_expect_z(gates, params, qubit=4)
    for b in range(2):
        assert abs(f[b] - O.loss_z(n, gates, params[b], qubit=4)) <= tol[0]
        ps = O.grad_param_shift(n, gates, params[b], list(range(k)), qubit=4)
        assert np.max(np.abs(g[b] - ps)) <= tol[1]


def test_adjoint_more_than_eight_high_qubits(P):
    """A run with X / Y generators on 9 qubits >= 12 takes two fused launches
    (8 qubits, then 1); every high-qubit gradient against parameter shift."""
    n = 21
    gates = [synth.Gate("RY", q, -1, 0.0, q) for q in range(n)]
    gates += [synth.Gate("CNOT", q, q + 1) for q in range(n - 1)]
    gates += [synth.Gate("RX" if q % 2 else "RY", q, -1, 0.0, n + q) for q in range(n)]
    params = np.random.default_rng(21).uniform(-3, 3, size=(1, 2 * n))
    which = [n + q for q in range(12, n)] + [q for q in (12, 16, 20)] + [n + 3]
    with P.StateVector(n, "c128", batch=1) as sv:
        f, g = sv.adjoint_expect_z(gates, params, qubit=20)
    assert abs(f[0] - O.loss_z(n, gates, params[0], qubit=20)) <= 1e-10
    ps = O.grad_param_shift(n, gates, params[0], which, qubit=20)
    assert np.max(np.abs(g[0, which] - ps)) <= 1e-10


def test_adjoint_rejects_nonrotation_parameters(P):
    gates = [synth.Gate("P", 0, -1, 0.0, 0)]
    with P.StateVector(4, "c128") as sv:
        with pytest.raises(P.SVError) as e:
            sv.adjoint_expect_z(gates, np.zeros((1, 1)), qubit=0)
        assert e.value.status == -4


def test_qnn_autograd_function(P):
    import torch
    n, L, B = 8, 3, 4
    params = synth.qnn_params(n, L, B, 5)
    x = torch.tensor(params[:, :n], requires_grad=True)
    theta = torch.tensor(params[:, n:], requires_grad=True)
    w = torch.tensor([0.5, -1.0, 2.0, 0.25], dtype=torch.float64)
    f = P.qnn_expect(theta, x, n, L, "c128")
    (f * w).sum().backward()
    gates = synth.qnn_ansatz(n, L)
    for b in range(B):
        assert abs(f[b].item() - O.loss_z(n, gates, params[b])) <= 1e-12
        ps = O.grad_param_shift(n, gates, params[b], list(range(params.shape[1])))
        got = np.concatenate([x.grad[b].numpy(), theta.grad[b].numpy()])
        assert np.max(np.abs(got - w[b].item() * ps)) <= 1e-10
    # the cached state handle serves later calls: without gradients, then
    # with gradients again, on other parameters
    params2 = synth.qnn_params(n, L, B, 6)
    with torch.no_grad():
        f2 = P.qnn_expect(torch.tensor(params2[:, n:]), torch.tensor(params2[:, :n]), n, L, "c128")
    x2 = torch.tensor(params2[:, :n], requires_grad=True)
    t2 = torch.tensor(params2[:, n:], requires_grad=True)
    f3 = P.qnn_expect(t2, x2, n, L, "c128")
    f3.sum().backward()
    for b in range(B):
        ref = O.loss_z(n, gates, params2[b])
        assert abs(f2[b].item() - ref) <= 1e-12 and abs(f3[b].item() - ref) <= 1e-12
    ps = O.grad_param_shift(n, gates, params2[1], list(range(params2.shape[1])))
    got = np.concatenate([x2.grad[1].numpy(), t2.grad[1].numpy()])
    assert np.max(np.abs(got - ps)) <= 1e-10
    P.release_cache()


C4 = dict(n=20, L=10, B=256, seed=0)


@pytest.fixture(scope="module")
def c4_reference():
    """Oracle gradients of the differentiation workload for parameter sets 0
    and 1: 32 seeded angles each by parameter shift, the first 8 of them by
    central differences (h = 1e-6), and the loss."""
    n, L, B = C4["n"], C4["L"], C4["B"]
    gates = synth.qnn_ansatz(n, L)
    params = synth.qnn_params(n, L, B, C4["seed"])
    rng = np.random.default_rng(4)
    ref = {}
    for b in (0, 1):
        which = sorted(rng.choice(np.arange(n + 2 * n * L), size=32, replace=False).tolist())
        ps = O.grad_param_shift(n, gates, params[b], which)
        fd = O.grad_fd(n, gates, params[b], which[:8], h=1e-6)
        ref[b] = (which, ps, fd, O.loss_z(n, gates, params[b]))
    return gates, params, ref


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_differentiation_config_n20(P, c4_reference, dtype):
    """The differentiation workload as the benchmark runs it: n = 20, 10
    layers, 400 rotation angles plus 20 encoding angles, 256 parameter sets in
    one call; sets 0 and 1 against the oracle's parameter shift (32 angles
    each) and central differences (8 angles each)."""
    gates, params, ref = c4_reference
    n, B = C4["n"], C4["B"]
    with P.StateVector(n, dtype, batch=B) as sv:
        f, g = sv.adjoint_expect_z(gates, params, qubit=0)
    assert g.shape == (B, params.shape[1]) and np.all(np.isfinite(g))
    tol_fd = 1e-7 if dtype == "c128" else 1e-4
    for b, (which, ps, fd, loss) in ref.items():
        assert abs(f[b] - loss) <= TOL_PS[dtype]
        assert np.max(np.abs(g[b, which] - ps)) <= TOL_PS[dtype]
        assert np.max(np.abs(g[b, which[:8]] - fd)) <= tol_fd
