"""Pins of the CPU FP64 oracle against what the paper and the mathematics fix.

None of these checks re-uses the oracle's own arithmetic: each compares it with
an independent route (paper-printed values, Kronecker-product operators formed
with numpy, scipy's matrix exponential, closed forms, invariants).
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import gates as G
from oracle import oracle as O
from oracle import ref_kron as K
from oracle import rh as RH

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Pauli matrices: X and Y as printed in Sec. III-A1, Z textbook.
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


# ---------------------------------------------------------------- gate table

ANGLES = [0.0, 0.3, 1.7, math.pi, 4.9, -2.2]


@pytest.mark.parametrize("name", [n for n in synth.GATE_NAMES
                                  if n != "MARK" and n not in synth.MATRIX_GATES])
def test_gate_unitary(name):
    for a in ANGLES:
        m = (G.angles_matrix(name, [a, 0.3 * a + 0.1, -0.7 * a, 0.2][:G.MULTI_ANGLE[name]])
             if name in G.MULTI_ANGLE else G.matrix(name, a))
        assert np.allclose(m.conj().T @ m, np.eye(m.shape[0]), atol=1e-15)


def test_paper_pauli_x_y():
    assert np.array_equal(G.matrix("X"), PX)
    assert np.array_equal(G.matrix("Y"), PY)


def test_paper_yx_dax_example():
    rows = _golden_lines("paper_yx_dax.txt")
    yx = np.kron(G.matrix("Y"), G.matrix("X")).reshape(-1)
    nz = np.flatnonzero(yx)
    assert list(nz) == [int(r[0]) for r in rows]
    for r in rows:
        assert yx[int(r[0])] == complex(float(r[1]), float(r[2]))
    # memory figures of the example: 4 entries of 24 B vs 16 elements of 16 B
    assert len(nz) * 24 == 96 and yx.size * 16 == 256


@pytest.mark.parametrize("name,pauli", [("RX", PX), ("RY", PY), ("RZ", PZ)])
def test_rotations_are_exponentials(name, pauli):
    for a in ANGLES:
        ref = scipy.linalg.expm(-0.5j * a * pauli)
        assert np.allclose(G.matrix(name, a), ref, atol=1e-14)


def test_gate_identities():
    m = G.matrix
    assert np.allclose(m("S") @ m("S"), m("Z"))
    assert np.allclose(m("T") @ m("T"), m("S"))
    assert np.allclose(m("SDG"), m("S").conj().T)
    assert np.allclose(m("TDG"), m("T").conj().T)
    assert np.allclose(m("P", math.pi / 2), m("S"))
    assert np.allclose(m("P", math.pi / 4), m("T"))
    assert np.allclose(m("H") @ m("X") @ m("H"), m("Z"))
    assert np.allclose(m("H") * math.sqrt(2), [[1, 1], [1, -1]])
    assert np.allclose(m("CPHASE", math.pi), m("CZ"))
    ih = np.kron(np.eye(2), m("H"))          # H on the low local bit = the target
    assert np.allclose(ih @ m("CZ") @ ih, m("CNOT"))
    rng = np.random.default_rng(1)
    A = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    B = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    assert np.allclose(m("SWAP") @ np.kron(A, B) @ m("SWAP"), np.kron(B, A))
    # CNOT with the first operand as control: |10> -> |11>
    e10 = np.zeros(4)
    e10[2] = 1
    assert np.allclose(m("CNOT") @ e10, [0, 0, 0, 1])


# ------------------------------------------------- two independent embeddings

@pytest.mark.parametrize("n", [2, 3, 4])
def test_2q_embeddings_agree(n):
    rng = np.random.default_rng(n)
    g = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    for q0 in range(n):
        for q1 in range(n):
            if q0 != q1:
                assert np.allclose(K.embed_2q_kron(n, q0, q1, g), K.embed_2q_def(n, q0, q1, g))


def test_1q_embedding_is_paper_kron_order():
    # paper qubit k = 1 is the leftmost factor = most significant bit = q = n-1
    n = 3
    U = K.embed_1q(n, n - 1, G.matrix("X"))
    assert np.array_equal(U @ np.eye(8)[:, 0], np.eye(8)[:, 4])


# ----------------------------------------- per-gate oracle vs brute-force MTP

def _all_single_gates(n, rng):
    out = []
    for name in synth.GATE_NAMES:
        if name in synth.MATRIX_GATES or name in synth.MULTI_ANGLE:
            continue   # pinned separately (test_matrix_gates_*, test_multi_angle_gates_vs_kron)
        ar = G.arity(name)
        ang = float(rng.uniform(0, 2 * math.pi))
        if ar == 1:
            out += [synth.Gate(name, q, -1, ang) for q in range(n)]
        elif ar == 2 and n >= 2:
            out += [synth.Gate(name, a, b, ang) for a in range(n) for b in range(n) if a != b]
        elif ar == 3 and n >= 3:
            out += [synth.Gate(name, a, b, 0.0, -1, 0, c) for a in range(n) for b in range(n)
                    for c in range(n) if len({a, b, c}) == 3]
        elif ar == 0:
            out += [synth.Gate(name, -1, -1, 0.0, -1, int(j)) for j in
                    sorted(set([0, (1 << n) - 1, int(rng.integers(1 << n))]))]
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_every_gate_every_position_vs_kron(n):
    rng = np.random.default_rng(100 + n)
    for g in _all_single_gates(n, rng):
        psi0 = synth.random_state(n, int(rng.integers(1 << 30)))
        ref = K.mtp_operator(n, g) @ psi0
        got = O.simulate(n, [g], psi0=psi0)
        assert np.max(np.abs(got - ref)) < 1e-14, g


@pytest.mark.parametrize("n,depth,seed", [(5, 10, 0), (8, 4, 1), (10, 2, 2)])
def test_random_circuit_vs_kron(n, depth, seed):
    gates = synth.random_circuit(n, depth, seed)
    ref = K.simulate_kron(n, gates)
    got = O.simulate(n, gates)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_capacity_mix_vs_kron():
    gates = synth.capacity_circuit(7, 6, 3)
    assert np.max(np.abs(O.simulate(7, gates) - K.simulate_kron(7, gates))) < 1e-12


def test_qnn_ansatz_vs_kron():
    n, L = 5, 3
    gates = synth.qnn_ansatz(n, L)
    p = synth.qnn_params(n, L, 1, 7)[0]
    assert np.max(np.abs(O.simulate(n, gates, p) - K.simulate_kron(n, gates, p))) < 1e-12


# -------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 4, 9, 13])
def test_hadamard_layer_on_basis_states(n):
    hl = [synth.Gate("H", q) for q in range(n)]
    psi = O.simulate(n, hl)
    assert np.max(np.abs(psi - 2.0 ** (-n / 2))) < 1e-15
    j = (0x2D5B & ((1 << n) - 1)) | 1
    psi = O.simulate(n, hl, psi0=O.basis_state(n, j))
    r = np.arange(1 << n)
    par = np.array([bin(x & j).count("1") & 1 for x in r])
    assert np.max(np.abs(psi - 2.0 ** (-n / 2) * (1 - 2 * par))) < 1e-15


@pytest.mark.parametrize("n", [2, 5, 12])
def test_ghz(n):
    gates = [synth.Gate("H", 0)] + [synth.Gate("CNOT", q, q + 1) for q in range(n - 1)]
    psi = O.simulate(n, gates)
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - ref)) < 1e-15


def test_norm_and_mirror():
    n = 11
    gates = synth.random_circuit(n, 12, 5)
    psi = O.simulate(n, gates)
    assert abs(O.norm2(psi) - 1.0) < 1e-13
    back = O.apply(psi, n, synth.inverse_circuit(gates))
    assert np.max(np.abs(back - O.basis_state(n))) < 1e-13


def test_readouts():
    n = 6
    for j in (0, 5, 63, 42):
        psi = O.basis_state(n, j)
        for q in range(n):
            assert O.expect_z(psi, q) == 1 - 2 * ((j >> q) & 1)
    for a in ANGLES:
        for name in ("RY", "RX"):
            psi = O.simulate(1, [synth.Gate(name, 0, -1, a)])
            assert abs(O.expect_z(psi, 0) - math.cos(a)) < 1e-15
        psi = O.simulate(1, [synth.Gate("RY", 0, -1, 0.7), synth.Gate("RZ", 0, -1, a)])
        assert abs(O.expect_z(psi, 0) - math.cos(0.7)) < 1e-15
    psi = synth.random_state(9, 3)
    assert abs(O.norm2(psi) - 1.0) < 1e-14
    assert abs(O.inner(psi, psi) - 1.0) < 1e-14
    phi = synth.random_state(9, 4)
    assert abs(O.inner(psi, phi) - np.vdot(psi, phi)) < 1e-14


# ----------------------------------------------------------- RH and Alg. 1

def test_paper_sign_example():
    (row,) = [r for r in _golden_lines("paper_rh_signs.txt") if r[0] == "sign"]
    kv = dict(x.split("=") for x in row[1:4])
    assert RH.compute_sign(int(kv["r"]), int(kv["c"]), int(kv["n"])) == int(row[4])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_quadrant_sign_matches_kronecker_hadamard(n):
    Hn = K.kron_all([G.matrix("H")] * n) * math.sqrt(1 << n)
    for r in range(1 << n):
        for c in range(1 << n):
            assert RH.compute_sign(r, c, n) == round(Hn[r, c].real)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_rh_mvm_methods_vs_kron_and_oracle(n):
    S = synth.random_state(n, 50 + n)
    ref = K.kron_all([G.matrix("H")] * n) @ S
    via_oracle = O.simulate(n, [synth.Gate("H", q) for q in range(n)], psi0=S)
    assert np.max(np.abs(via_oracle - ref)) < 1e-14
    outs = [RH.rh_mvm_logarithm(S)[0], RH.rh_mvm_quarter(S)[0]]
    if n <= 5:
        outs.append(RH.rh_mvm_non_optimized(S)[0])
    if n >= 2:
        outs.append(RH.rh_mvm_block(S, 2 if n > 2 else 1)[0])
    for o in outs:
        assert np.max(np.abs(o - ref)) < 1e-13


def test_sign_counts_table2_and_n5_examples():
    rows = _golden_lines("paper_rh_signs.txt")
    S = synth.random_state(5, 0)
    for r in rows:
        kv = dict(x.split("=") for x in r[1:] if "=" in x)
        if r[0] == "quarter":
            _, cnt = RH.rh_mvm_quarter(S)
            assert cnt == int(kv["rows"]) * int(kv["per_row"])
        elif r[0] == "block":
            b = int(kv["b"])
            _, cnt = RH.rh_mvm_block(S, b)
            assert cnt == 16 * int(kv["per_row"])
        elif r[0] == "logarithm":
            _, cnt = RH.rh_mvm_logarithm(S)
            assert cnt == 16 * (int(kv["per_row"]) - 1)   # index 0 is not computed
    for n in range(2, 8):
        S = synth.random_state(n, n)
        assert RH.rh_mvm_logarithm(S)[1] == RH.sign_count_formula("logarithm", n)
        assert RH.rh_mvm_quarter(S)[1] == RH.sign_count_formula("quarter", n)
        for b in (1, 2):
            if (1 << (n - 1)) % b == 0:
                assert RH.rh_mvm_block(S, b)[1] == RH.sign_count_formula("block", n, b)
    S = synth.random_state(4, 1)
    assert RH.rh_mvm_non_optimized(S)[1] == RH.sign_count_formula("non-optimized", 4)


def test_theorem3_optimal_block():
    for n in (3, 5, 7, 9):
        f = {b: (1 << (n - 1)) // b + b - 1 for b in [1 << i for i in range(n)]}
        best = min(f.values())
        b_opt = math.sqrt(1 << (n - 1))
        # the optimum over powers of two sits at the power(s) of two next to sqrt(2^(n-1))
        assert any(f[b] == best and b / 2 <= b_opt <= 2 * b for b in f)


# ---------------------------------------------------------------- Grover

@pytest.mark.parametrize("n", [3, 4, 6, 9, 12])
def test_grover_closed_form(n):
    m = synth.grover_marked(n, n)
    k = synth.grover_iterations(n)
    psi = O.simulate(n, synth.grover_circuit(n, m))
    a, b, p = O.grover_closed_form(n, k)
    sgn = (-1) ** k
    assert abs(psi[m] - sgn * a) < 1e-12
    others = np.delete(psi, m)
    assert np.max(np.abs(others - sgn * b)) < 1e-12
    assert abs(abs(psi[m]) ** 2 - p) < 1e-12


def test_grover_golden_n20():
    rows = {r[0]: float(r[1]) for r in _golden_lines("grover_n20.txt")}
    a, b, p = O.grover_closed_form(20, 804)
    assert rows["marked"] == a and rows["unmarked"] == b and rows["p_success"] == p
    assert synth.grover_iterations(20) == int(rows["iterations"])


# ------------------------------------------------------------- gradients

def test_gradients_single_qubit_closed_form():
    # f(t) = <Z> of RY(t)|0> = cos t, so df/dt = -sin t
    g = [synth.Gate("RY", 0, -1, 0.0, 0)]
    for t in ANGLES:
        p = np.array([t])
        assert abs(O.grad_param_shift(1, g, p, [0])[0] + math.sin(t)) < 1e-15
        assert abs(O.grad_fd(1, g, p, [0])[0] + math.sin(t)) < 1e-9


def test_gradients_ps_fd_kron_agree():
    n, L = 4, 2
    gates = synth.qnn_ansatz(n, L)
    p = synth.qnn_params(n, L, 1, 11)[0]
    which = list(range(len(p)))
    ps = O.grad_param_shift(n, gates, p, which)
    fd = O.grad_fd(n, gates, p, which)
    assert np.max(np.abs(ps - fd)) < 1e-8
    # third route: d psi / dt with the gate's matrix replaced by -i/2 P U(t),
    # every operator formed by brute-force Kronecker products
    Zn = K.embed_1q(n, 0, PZ)
    psi = K.simulate_kron(n, gates, p)
    for k, par in enumerate(which):
        dpsi = np.zeros(1 << n, dtype=complex)
        dpsi[0] = 1.0
        for g in gates:
            U = K.mtp_operator(n, g, p)
            if g.param == par:
                Pm = K.embed_1q(n, g.q0, G.generator(g.name))
                U = -0.5j * Pm @ U
            dpsi = U @ dpsi
        d = 2 * np.real(np.vdot(psi, Zn @ dpsi))
        assert abs(d - ps[k]) < 1e-12


# ------------------------------------------------ one-at-a-time monomial amplitudes

_MONO_1Q = ("X", "Y", "Z", "S", "SDG", "T", "TDG", "RZ", "P", "I")
_MONO_2Q = ("CNOT", "CZ", "SWAP", "CPHASE")


def _random_monomial_circuit(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        if rng.random() < 0.6:
            name = _MONO_1Q[int(rng.integers(len(_MONO_1Q)))]
            out.append(synth.Gate(name, int(rng.integers(n)), -1, float(rng.uniform(0, 2 * math.pi))))
        else:
            q0, q1 = (int(x) for x in rng.choice(n, 2, replace=False))
            name = _MONO_2Q[int(rng.integers(len(_MONO_2Q)))]
            out.append(synth.Gate(name, q0, q1, float(rng.uniform(0, 2 * math.pi))))
    return out


@pytest.mark.parametrize("n,seed", [(6, 0), (8, 1), (9, 2)])
def test_monomial_amplitudes_vs_kronecker(n, seed):
    """Every amplitude of a random monomial circuit, walked one index at a
    time, equals the Kronecker-operator product applied to H^n|0> and to a
    basis state."""
    gates = _random_monomial_circuit(n, 60, seed)
    U = K.circuit_operator(n, gates)
    idx = np.arange(1 << n)
    uni = np.full(1 << n, 2.0 ** (-0.5 * n), dtype=complex)
    assert np.max(np.abs(O.monomial_amplitudes(n, gates, idx) - U @ uni)) < 1e-14
    j = 37 % (1 << n)
    e = np.zeros(1 << n, dtype=complex)
    e[j] = 1.0
    assert np.max(np.abs(O.monomial_amplitudes(n, gates, idx, initial=j) - U @ e)) < 1e-14


def test_monomial_amplitudes_capacity_mix_vs_state_oracle():
    """The capacity mix without dense gates at n = 12, after its H layer:
    sampled one-index amplitudes equal the full-state oracle's."""
    n = 12
    g = synth.capacity_circuit(n, 30, 3, p_dense=0.0)
    assert all(x.name == "H" for x in g[:n])
    psi = O.simulate(n, g)
    idx = np.random.default_rng(0).integers(0, 1 << n, 500)
    assert np.max(np.abs(O.monomial_amplitudes(n, g[n:], idx) - psi[idx])) < 1e-14


def test_monomial_amplitudes_closed_forms():
    n = 11
    allx = [synth.Gate("X", q) for q in range(n)]
    # X on every qubit maps |0> to |2^n - 1>.
    a = O.monomial_amplitudes(n, allx, [0, (1 << n) - 1, 5], initial=0)
    assert np.array_equal(a, np.array([0, 1, 0], dtype=complex))
    # A CNOT chain is the classical map b_{q+1} ^= b_q (ascending q) on basis states.
    chain = [synth.Gate("CNOT", q, q + 1) for q in range(n - 1)]
    j = 0b10110011101
    x = j
    for q in range(n - 1):
        x ^= ((x >> q) & 1) << (q + 1)
    assert O.monomial_amplitudes(n, chain, [x], initial=j)[0] == 1
    # Z on qubit 0 of the uniform state: sign (-1)^{b_0}.
    z = O.monomial_amplitudes(3, [synth.Gate("Z", 0)], range(8))
    assert np.allclose(z, 2 ** -1.5 * np.array([1, -1] * 4))
    with pytest.raises(ValueError):
        O.monomial_amplitudes(3, [synth.Gate("H", 0)], [0])


# ------------------------------------------------ matrix gates (U1, U2)

def test_matrix_gates_reproduce_named_gates():
    """A U1 / U2 carrying a named gate's matrix acts as that gate."""
    n = 5
    rng = np.random.default_rng(7)
    psi0 = synth.random_state(n, 3)
    cases = [("RX", 1.3), ("H", 0.0), ("T", 0.0), ("RZ", 2.2)]
    for name, ang in cases:
        params = synth.matrix_params(G.matrix(name, ang))
        for q in range(n):
            a = O.simulate(n, [synth.Gate(name, q, -1, ang)], psi0=psi0)
            b = O.simulate(n, [synth.Gate("U1", q, -1, 0.0, 0)], params, psi0=psi0)
            assert np.max(np.abs(a - b)) < 1e-15
    for name, ang in [("CNOT", 0.0), ("SWAP", 0.0), ("CPHASE", 0.7)]:
        params = synth.matrix_params(G.matrix(name, ang))
        for q0, q1 in [(0, 3), (4, 1), (2, 3)]:
            a = O.simulate(n, [synth.Gate(name, q0, q1, ang)], psi0=psi0)
            b = O.simulate(n, [synth.Gate("U2", q0, q1, 0.0, 0)], params, psi0=psi0)
            assert np.max(np.abs(a - b)) < 1e-15
    # U2 = A (x) B acts as A on its first operand and B on its second
    A, B = synth.random_unitary(2, rng), synth.random_unitary(2, rng)
    p = np.concatenate([synth.matrix_params(np.kron(A, B)), synth.matrix_params(A),
                        synth.matrix_params(B)])
    a = O.simulate(n, [synth.Gate("U2", 3, 1, 0.0, 0)], p, psi0=psi0)
    b = O.simulate(n, [synth.Gate("U1", 3, -1, 0.0, 32), synth.Gate("U1", 1, -1, 0.0, 40)], p,
                   psi0=psi0)
    assert np.max(np.abs(a - b)) < 1e-14


@pytest.mark.parametrize("n", [3, 6])
def test_matrix_gates_vs_kronecker(n):
    """Random U1 on every qubit and random U2 on every ordered pair against the
    Kronecker-product operators (element-wise 2-qubit embedding)."""
    rng = np.random.default_rng(n)
    gates, params = [], []
    for q in range(n):
        gates.append(synth.Gate("U1", q, -1, 0.0, len(params)))
        params += synth.matrix_params(synth.random_unitary(2, rng)).tolist()
    for a in range(n):
        for b in range(n):
            if a != b:
                gates.append(synth.Gate("U2", a, b, 0.0, len(params)))
                params += synth.matrix_params(synth.random_unitary(4, rng)).tolist()
    params = np.array(params)
    psi0 = synth.random_state(n, 5)
    U = np.eye(1 << n, dtype=complex)
    for g in gates:
        m = G.params_matrix(g.name, params, g.param)
        E = K.embed_1q(n, g.q0, m) if g.name == "U1" else K.embed_2q_def(n, g.q0, g.q1, m)
        U = E @ U
    want = U @ psi0
    got = O.simulate(n, gates, params, psi0=psi0)
    assert np.max(np.abs(got - want)) < 1e-13


# ------------------------------------------ Table 1 additions (CY ... CSWAP)

def _bits(i, q):
    return (i >> q) & 1


def _expected_basis_image(g, i):
    """(index, phase) of gate g applied to |i>, from the gates' bit logic."""
    a, b, c = g.q0, g.q1, g.q2
    if g.name == "CCX":
        return (i ^ (1 << c)) if _bits(i, a) and _bits(i, b) else i, 1
    if g.name == "CSWAP":
        if _bits(i, a) and _bits(i, b) != _bits(i, c):
            return i ^ (1 << b) ^ (1 << c), 1
        return i, 1
    if g.name == "DCX":   # |x y> -> |y, x xor y> on (q0, q1)
        x, y = _bits(i, a), _bits(i, b)
        j = i & ~((1 << a) | (1 << b))
        return j | (y << a) | ((x ^ y) << b), 1
    if g.name == "CY":    # Y on q1 when q0 = 1: |0> -> i|1>, |1> -> -i|0>
        if not _bits(i, a):
            return i, 1
        return i ^ (1 << b), (1j if not _bits(i, b) else -1j)
    if g.name == "ISWAP":  # |01>, |10> exchanged with a factor i
        if _bits(i, a) != _bits(i, b):
            return i ^ (1 << a) ^ (1 << b), 1j
        return i, 1
    raise ValueError(g.name)


@pytest.mark.parametrize("name", ["CY", "ISWAP", "DCX", "CCX", "CSWAP"])
def test_table1_monomials_by_bit_logic(name):
    """Each basis state goes to one basis state times a phase, as the gate's
    definition in words says; checked on every basis state of n = 4 for every
    operand placement."""
    n = 4
    ar = G.arity(name)
    placements = ([(a, b, -1) for a in range(n) for b in range(n) if a != b] if ar == 2 else
                  [(a, b, c) for a in range(n) for b in range(n) for c in range(n) if len({a, b, c}) == 3])
    for a, b, c in placements:
        g = synth.Gate(name, a, b, 0.0, -1, 0, c)
        for i in range(1 << n):
            psi = np.zeros(1 << n, dtype=complex)
            psi[i] = 1.0
            out = O.simulate(n, [g], psi0=psi)
            j, ph = _expected_basis_image(g, i)
            ref = np.zeros(1 << n, dtype=complex)
            ref[j] = ph
            assert np.array_equal(out, ref), (g, i)


def test_table1_monomials_one_nonzero_per_row():
    """Table 1 lists CY, iSWAP, DCX, CCX and CSWAP with one non-zero per row."""
    for name in ("CY", "ISWAP", "DCX", "CCX", "CSWAP"):
        m = G.matrix(name)
        assert all(np.count_nonzero(r) == 1 for r in m), name


@pytest.mark.parametrize("theta", [0.0, 0.3, -1.7, 2.9, math.pi])
def test_table1_diagonals_are_exponentials(theta):
    """CRZ = exp(-i t/2 |1><1| (x) Z), RZZ = exp(-i t/2 Z (x) Z) and
    CU1 = exp(i t |11><11|), with scipy's matrix exponential."""
    P1 = np.diag([0, 1]).astype(complex)
    crz = scipy.linalg.expm(-0.5j * theta * np.kron(P1, PZ))
    rzz = scipy.linalg.expm(-0.5j * theta * np.kron(PZ, PZ))
    cu1 = scipy.linalg.expm(1j * theta * np.kron(P1, P1))
    assert np.allclose(G.matrix("CRZ", theta), crz, atol=1e-14)
    assert np.allclose(G.matrix("RZZ", theta), rzz, atol=1e-14)
    assert np.allclose(G.matrix("CU1", theta), cu1, atol=1e-14)


def test_table1_identities():
    I2 = np.eye(2, dtype=complex)
    H = np.array([[1, 1], [1, -1]], dtype=complex) / math.sqrt(2)
    S = np.diag([1, 1j])
    cnot = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
    # CY = (I (x) S) CNOT (I (x) S^dagger)
    assert np.allclose(G.matrix("CY"), np.kron(I2, S) @ cnot @ np.kron(I2, S.conj().T), atol=1e-15)
    # iSWAP^2 = Z (x) Z
    sw = G.matrix("ISWAP")
    assert np.allclose(sw @ sw, np.kron(PZ, PZ), atol=1e-15)
    # DCX = CNOT(q1 -> q0) CNOT(q0 -> q1), and DCX^3 = I (a 3-cycle)
    cnot10 = np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], dtype=complex)
    d = G.matrix("DCX")
    assert np.allclose(d, cnot10 @ cnot, atol=0)
    assert np.allclose(d @ d @ d, np.eye(4), atol=0)
    # CCX = (I (x) I (x) H) CCZ (I (x) I (x) H)
    ccz = np.diag([1, 1, 1, 1, 1, 1, 1, -1]).astype(complex)
    hh = np.kron(np.kron(I2, I2), H)
    assert np.allclose(G.matrix("CCX"), hh @ ccz @ hh, atol=1e-15)
    # CSWAP(c; a, b) = CCX(c, b -> a) CCX(c, a -> b) CCX(c, b -> a), built
    # from the element-wise embedding of CCX on 3 qubits
    def ccx_on(c, x, t):
        return K.mtp_operator(3, synth.Gate("CCX", c, x, 0.0, -1, 0, t))
    fred = ccx_on(2, 0, 1) @ ccx_on(2, 1, 0) @ ccx_on(2, 0, 1)
    assert np.allclose(K.mtp_operator(3, synth.Gate("CSWAP", 2, 1, 0.0, -1, 0, 0)), fred, atol=0)


@pytest.mark.parametrize("n", [3, 4, 5])
def test_3q_embedding_vs_definition(n):
    """The Kronecker embedding of a 3-qubit gate against the element-wise
    definition U[r, c] = G[l(r), l(c)] when r and c agree off the 3 qubits."""
    rng = np.random.default_rng(n)
    g = synth.random_unitary(8, rng)
    N = 1 << n
    for a, b, c in [(0, 1, 2), (n - 1, 0, 1), (1, n - 1, 0)]:
        U = K.embed_3q_kron(n, a, b, c, g)
        r = np.arange(N)[:, None]
        col = np.arange(N)[None, :]
        mask = (1 << a) | (1 << b) | (1 << c)
        same = (r & ~mask) == (col & ~mask)
        lr = (((r >> a) & 1) << 2) | (((r >> b) & 1) << 1) | ((r >> c) & 1)
        lc = (((col >> a) & 1) << 2) | (((col >> b) & 1) << 1) | ((col >> c) & 1)
        ref = np.where(same, g[lr, lc], 0.0)
        assert np.allclose(U, ref, atol=1e-15)


# ------------------------------------------------ remaining Table 1 gates (f2)

def _ry(t):
    return scipy.linalg.expm(-0.5j * t * PY)


def test_table1_sparsity_of_two_qubit_gates():
    """Table 1: RXX, RYY, RZX and ECR are 50% zeros (two non-zeros per row);
    CH, CSX, CU and CU3 are 62.5% zeros."""
    rng = np.random.default_rng(1)
    for name in ("RXX", "RYY", "RZX", "ECR", "CH", "CSX", "CU", "CU3"):
        if name in G.MULTI_ANGLE:
            m = G.angles_matrix(name, rng.uniform(0.2, 1.2, G.MULTI_ANGLE[name]))
        else:
            m = G.matrix(name, 0.7)
        zeros = np.count_nonzero(np.abs(m) < 1e-15) / m.size
        assert zeros == (0.5 if name in ("RXX", "RYY", "RZX", "ECR") else 0.625), name


@pytest.mark.parametrize("theta", [0.0, 0.4, -2.2, math.pi])
def test_two_qubit_rotations_are_exponentials(theta):
    for name, a, b in (("RXX", PX, PX), ("RYY", PY, PY), ("RZX", PZ, PX)):
        ref = scipy.linalg.expm(-0.5j * theta * np.kron(a, b))
        assert np.allclose(G.matrix(name, theta), ref, atol=1e-14), name


def test_sx_r_u_definitions():
    H = np.array([[1, 1], [1, -1]], dtype=complex) / math.sqrt(2)
    S = np.diag([1, 1j])
    sx = G.matrix("SX")
    assert np.allclose(sx @ sx, PX, atol=1e-15)
    assert np.allclose(sx, H @ S @ H, atol=1e-15)
    assert np.allclose(G.matrix("SXDG"), sx.conj().T, atol=0)
    rng = np.random.default_rng(2)
    for _ in range(5):
        t, p, l = rng.uniform(-3, 3, 3)
        ref_r = scipy.linalg.expm(-0.5j * t * (math.cos(p) * PX + math.sin(p) * PY))
        assert np.allclose(G.angles_matrix("R", [t, p]), ref_r, atol=1e-14)
        # U(t, p, l) = e^{i(p+l)/2} RZ(p) RY(t) RZ(l)
        rz = lambda a: scipy.linalg.expm(-0.5j * a * PZ)
        ref_u = np.exp(0.5j * (p + l)) * rz(p) @ _ry(t) @ rz(l)
        assert np.allclose(G.angles_matrix("U", [t, p, l]), ref_u, atol=1e-14)
        # textbook special cases
        assert np.allclose(G.angles_matrix("U", [t, -math.pi / 2, math.pi / 2]),
                           scipy.linalg.expm(-0.5j * t * PX), atol=1e-14)
        assert np.allclose(G.angles_matrix("R", [t, math.pi / 2]), _ry(t), atol=1e-14)


def test_controlled_and_echoed_gates():
    I2 = np.eye(2, dtype=complex)
    P0, P1 = np.diag([1, 0]).astype(complex), np.diag([0, 1]).astype(complex)
    H = (PX + PZ) / math.sqrt(2)
    # ECR = (X (x) I - Y (x) X) / sqrt 2 = RZX(-pi/4) (X (x) I) RZX(pi/4)
    ecr = (np.kron(PX, I2) - np.kron(PY, PX)) / math.sqrt(2)
    rzx = lambda t: scipy.linalg.expm(-0.5j * t * np.kron(PZ, PX))
    assert np.allclose(G.matrix("ECR"), ecr, atol=1e-15)
    assert np.allclose(G.matrix("ECR"), rzx(-math.pi / 4) @ np.kron(PX, I2) @ rzx(math.pi / 4), atol=1e-14)
    # controlled gates: |0><0| (x) I + |1><1| (x) V
    ctrl = lambda v: np.kron(P0, I2) + np.kron(P1, v)
    assert np.allclose(G.matrix("CH"), ctrl(H), atol=1e-15)
    csx = G.matrix("CSX")
    assert np.allclose(csx @ csx, ctrl(PX), atol=1e-15)
    rng = np.random.default_rng(3)
    t, p, l, g = rng.uniform(-3, 3, 4)
    u = G.angles_matrix("U", [t, p, l])
    assert np.allclose(G.angles_matrix("CU3", [t, p, l]), ctrl(u), atol=0)
    assert np.allclose(G.angles_matrix("CU", [t, p, l, g]), ctrl(np.exp(1j * g) * u), atol=1e-15)


@pytest.mark.parametrize("n", [2, 4])
def test_multi_angle_gates_vs_kron(n):
    """R, U, CU3, CU (angles from the parameter vector) through the C oracle
    against the Kronecker operator, at every operand placement."""
    rng = np.random.default_rng(40 + n)
    for name, k in synth.MULTI_ANGLE.items():
        params = rng.uniform(-math.pi, math.pi, k + 2)
        if G.arity(name) == 1:
            gs = [synth.Gate(name, q, -1, 0.0, 1) for q in range(n)]
        else:
            gs = [synth.Gate(name, a, b, 0.0, 2) for a in range(n) for b in range(n) if a != b]
        for g in gs:
            psi0 = synth.random_state(n, int(rng.integers(1 << 30)))
            ref = K.mtp_operator(n, g, params) @ psi0
            got = O.simulate(n, [g], params, psi0=psi0)
            assert np.max(np.abs(got - ref)) < 1e-14, g
