"""Host planner checks on the CPU (no GPU): the C ABI library loads and exports
every declared symbol, argument validation, and the pass plans — executed by a
slow numpy emulation of the documented op semantics — reproduce the oracle."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import synth
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
P = pytest.importorskip("paper_2411_15332_amd")
from plan_emulator import OP_EXCH, run_plan  # noqa: E402


def _declared_symbols():
    names = []
    for h in ("sv.h", "sv_debug.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        names += re.findall(r"^\S[^\n(]*?\b(sv_[a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(P.sv.LIB_PATH)
    names = _declared_symbols()
    assert "sv_alloc" in names and "sv_apply_circuit" in names and "sv_debug_plan" in names
    for name in names:
        assert hasattr(L, name), name


def test_gate_record_layout():
    assert P.sv.GATE_DTYPE.itemsize == 32
    kinds = P.GATE_KIND
    assert set(kinds) == set(synth.GATE_NAMES)
    src = open(os.path.join(ROOT, "include", "sv.h")).read()
    for name, code in kinds.items():
        assert re.search(rf"SV_GATE_{name} = {code}\b", src), name


@pytest.mark.parametrize("bad", [
    [synth.Gate("X", 12)],
    [synth.Gate("CNOT", 3, 3)],
    [synth.Gate("CZ", 0, -1)],
    [synth.Gate("MARK", -1, -1, 0.0, -1, 1 << 12)],
    [synth.Gate("RY", 0, -1, 0.0, 5)],
    [synth.Gate("H", 0, -1, 0.0, 0)],
    [synth.Gate("CCX", 0, 1, 0.0, -1, 0, 1)],       # target equals a control
    [synth.Gate("CCX", 0, 1, 0.0, -1, 0, 12)],      # target out of range
    [synth.Gate("CSWAP", 2, 2, 0.0, -1, 0, 3)],
    [synth.Gate("CY", 4, 4)],
    [synth.Gate("CRZ", 0, 1, 0.0, 3)],              # parameter not supplied
    [synth.Gate("DCX", 0, 1, 0.0, 0)],              # takes no parameter
])
def test_validation_rejects(bad):
    with pytest.raises(P.SVError) as e:
        P.debug_plan(12, bad)
    assert e.value.status == -1
    assert P.last_error()


# The emulation runs in FP64 with the plan's constants, which a complex64 plan
# holds in FP32 (as the kernel receives them): its tolerance is the complex64
# parity bound.
EMU_TOL = {"c128": 1e-12, "c64": 1e-5}


def _emulate(n, gates, dtype="c128", psi0=None, basis=0, **kw):
    plan = P.debug_plan(n, gates, dtype=dtype, basis=basis if psi0 is None else None, **kw)
    psi = O.basis_state(n, basis) if psi0 is None else psi0.copy()
    return run_plan(plan, psi, n), plan


CASES = [(10, 3, 0), (11, 4, 1), (12, 4, 2), (13, 3, 3), (14, 2, 4)]


@pytest.mark.parametrize("n,depth,seed", CASES)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_plan_emulation_random_circuits(n, depth, seed, dtype):
    gates = synth.random_circuit(n, depth, seed)
    ref = O.simulate(n, gates)
    got, plan = _emulate(n, gates, dtype)
    assert np.max(np.abs(got - ref)) < EMU_TOL[dtype]
    if not plan["small"]:
        assert plan["gates"] == len([g for g in gates if g.name != "I"])


@pytest.mark.parametrize("opts", [dict(fuse=False), dict(min_low=3), dict(min_low=7),
                                  dict(max_dense=1), dict(gen_h=False)])
def test_plan_options(opts):
    n = 12
    gates = synth.capacity_circuit(n, 3, 5)
    ref = O.simulate(n, gates)
    got, plan = _emulate(n, gates, **opts)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("n", [11, 14, 15])
def test_every_gate_kind_every_position(n):
    gates, params = synth.all_kinds_circuit(n, n)
    psi0 = synth.random_state(n, 9)
    ref = O.simulate(n, gates, params, psi0=psi0)
    for dt in ("c128", "c64"):
        got, _ = _emulate(n, gates, dt, psi0=psi0, params=params)
        assert np.max(np.abs(got - ref)) < EMU_TOL[dt]


@pytest.mark.parametrize("j", [0, 5, 1023])
def test_generation_prologue(j):
    n = 12
    # Hadamards on distinct qubits up to the first other gate: generated as
    # the RH layer
    gates = [synth.Gate("H", q) for q in (3, 0, 7, 11, 5)] + [synth.Gate("CNOT", 3, 4)] + \
        synth.random_circuit(n, 2, 1)
    ref = O.simulate(n, gates, psi0=O.basis_state(n, j))
    got, plan = _emulate(n, gates, basis=j)
    assert plan["generated_h"] == 5 and plan["generated_product"] == 0
    assert np.max(np.abs(got - ref)) < 1e-12
    # followed by more 1-qubit gates: the whole 1-qubit prefix becomes a
    # generated product state
    gates = [synth.Gate("H", q) for q in (3, 0, 7, 11, 5)] + synth.random_circuit(n, 2, 1)
    lead = 5 + next(i for i, g in enumerate(gates[5:]) if g.name in ("CNOT", "CZ", "SWAP", "CPHASE"))
    ref = O.simulate(n, gates, psi0=O.basis_state(n, j))
    got, plan = _emulate(n, gates, basis=j)
    assert plan["generated_h"] == 0 and plan["generated_product"] == lead
    assert np.max(np.abs(got - ref)) < 1e-12
    only_h = [synth.Gate("H", q) for q in range(n)]
    got, plan = _emulate(n, only_h, basis=j)
    assert plan["generated_h"] == n and len(plan["passes"]) == 1
    ref = O.simulate(n, only_h, psi0=O.basis_state(n, j))
    assert np.max(np.abs(got - ref)) < 1e-15


def test_grover_plan():
    n = 12
    m = synth.grover_marked(n, 1)
    gates = synth.grover_circuit(n, m, iterations=3)
    ref = O.simulate(n, gates)
    got, _ = _emulate(n, gates)
    assert np.max(np.abs(got - ref)) < 1e-12


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_small_path_plans(n):
    gates = synth.random_circuit(n, 6, n)
    ref = O.simulate(n, gates)
    got, plan = _emulate(n, gates)
    assert plan["small"]
    assert np.max(np.abs(got - ref)) < 1e-12


def test_large_plan_statistics():
    gates = synth.random_circuit(28, 100, 0)
    plan = P.debug_plan(28, gates)
    npass = len(plan["passes"])
    assert plan["gates"] == len(gates)
    # the first pass generates the product state left by the leading layer of
    # 1-qubit gates: it writes and reads nothing
    gen = int(plan["passes"][0]["flags"]) & 8 != 0
    assert gen and plan["generated_product"] == 28
    assert plan["hbm_bytes"] == npass * 2 * (1 << 28) * 16 - (1 << 28) * 16
    # every gate of a pass lies on its tile qubits or is diagonal
    assert 30 < npass < 200
    assert plan["k"] == plan["R"] + plan["w"] and plan["w"] >= 8


def test_relabel_only_pass_orders_loads_before_stores():
    # X/Y on tile qubits held by thread bits are applied by relabelling the
    # store addresses; with no LDS exchange in the pass, the kernel needs a
    # barrier between the tile's loads and its permuted stores.
    n = 16
    # (a general input state: from a known basis state the two gates would be
    # folded into a generated product state)
    gates = [synth.Gate("X", 11), synth.Gate("Y", 10)]
    plan = P.debug_plan(n, gates, basis=None)
    assert plan["relabels"] >= 1 and plan["exchanges"] == 0
    assert all(int(p["flags"]) & 2 for p in plan["passes"] if int(p["store_layout"]) != 0)
    plain = P.debug_plan(n, [synth.Gate("Z", 11)], basis=None)
    assert not any(int(p["flags"]) & 2 for p in plain["passes"])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,seed", [(13, 0), (14, 1)])
def test_diagonal_heavy_mix(n, seed, dtype):
    """Runs of phases on every kind of position (register, thread and
    tile-base bits), with X and Y relabels in between, so that merged uniform
    diagonals with single and AND terms, half- and quarter-slot diagonals and
    register relabels all occur; results against the oracle."""
    rng = np.random.default_rng(seed)
    one = ("Z", "S", "SDG", "T", "TDG", "P", "RZ", "X", "Y", "H")
    two = ("CZ", "CPHASE", "CNOT")
    gates = [synth.Gate("H", q) for q in range(n)]
    for _ in range(6):
        for q in range(n):
            name = one[int(rng.integers(len(one)))]
            gates.append(synth.Gate(name, q, -1, float(rng.uniform(0, 2 * math.pi))))
        for _ in range(n):
            q0, q1 = (int(x) for x in rng.choice(n, 2, replace=False))
            name = two[int(rng.integers(len(two)))]
            gates.append(synth.Gate(name, q0, q1, float(rng.uniform(0, 2 * math.pi))))
    ref = O.simulate(n, gates)
    got, plan = _emulate(n, gates, dtype)
    assert np.max(np.abs(got - ref)) < EMU_TOL[dtype]
    codes = set(int(c) for c in plan["ops"]["code"])
    assert {3, 16, 17, 18} <= codes, codes          # UDN, D1H, D2Q, D1HU
    assert plan["relabels"] > 0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,depth,seed,kind", [(16, 14, 3, "random"), (17, 10, 4, "random"),
                                              (16, 12, 6, "capacity")])
def test_remapped_plans(n, depth, seed, kind, dtype):
    """Multi-pass plans whose stores permute the tile's bits (qubit
    remapping), including the passes that put qubits back, against the
    oracle; remapping never costs passes here and does move qubits."""
    gates = (synth.random_circuit(n, depth, seed) if kind == "random"
             else synth.capacity_circuit(n, depth, seed))
    ref = O.simulate(n, gates)
    got, plan = _emulate(n, gates, dtype)
    assert np.max(np.abs(got - ref)) < EMU_TOL[dtype]
    fixed = P.debug_plan(n, gates, dtype=dtype, remap=False)
    assert len(plan["passes"]) <= len(fixed["passes"])
    lay = plan["layouts"]
    moved = 0
    for p in plan["passes"]:
        L0 = lay[int(p["layout_begin"])]
        Ls = lay[int(p["layout_begin"]) + int(p["store_layout"])]
        moved += int(sorted(L0["thr_goff"][:8].tolist()) != sorted(Ls["thr_goff"][:8].tolist())
                     or sorted(L0["reg_goff"][:plan["R"]].tolist()) != sorted(Ls["reg_goff"][:plan["R"]].tolist()))
    assert moved > 0


@pytest.mark.parametrize("n", [3, 6, 9])
def test_small_path_every_kind(n):
    gates, params = synth.all_kinds_circuit(n, 40 + n)
    ref = O.simulate(n, gates, params)
    for dt in ("c128", "c64"):
        got, plan = _emulate(n, gates, dt, params=params)
        assert plan["small"]
        assert np.max(np.abs(got - ref)) < EMU_TOL[dt]


def test_matrix_gate_validation():
    g1 = [synth.Gate("U1", 0, -1, 0.0, 2)]
    with pytest.raises(P.SVError):
        P.debug_plan(12, g1, params=np.zeros(9))      # 2 + 8 > 9 reals
    P.debug_plan(12, g1, params=np.zeros(10))
    with pytest.raises(P.SVError):
        P.debug_plan(12, [synth.Gate("U2", 0, 1, 0.0, -1)])   # matrix must come from params
    with pytest.raises(P.SVError):
        P.debug_plan(12, [synth.Gate("U2", 3, 3, 0.0, 0)], params=np.zeros(32))


@pytest.mark.parametrize("n", [5, 12, 14, 16])
def test_table1_gates_lowered_and_ccx(n):
    gates, params = synth.table1_circuit(n, 70 + n)
    psi0 = synth.random_state(n, 3)
    ref = O.simulate(n, gates, params, psi0=psi0)
    for dt in ("c128", "c64"):
        got, plan = _emulate(n, gates, dt, psi0=psi0, params=params)
        assert np.max(np.abs(got - ref)) < EMU_TOL[dt]
        if not plan["small"]:
            codes = {int(o["code"]) for o in plan["ops"]}
            assert 23 in codes   # CCX applied as a monomial op, not decomposed


def test_ccx_control_placements():
    """CCX with controls on every combination of register, thread and
    tile-base bits: targets among the tile qubits, controls drawn from the
    low (thread) bits, the others and the high (tile-base) bits."""
    n = 15
    rng = np.random.default_rng(5)
    gates = [synth.Gate("H", q) for q in range(n)]
    for t in (6, 7, 8, 9):
        for c0, c1 in ((0, 1), (2, 13), (14, 12), (7 if t != 7 else 8, 3), (10, 11)):
            if t in (c0, c1):
                continue
            gates.append(synth.Gate("RX", t, -1, float(rng.uniform(0, 6))))
            gates.append(synth.Gate("CCX", c0, c1, 0.0, -1, 0, t))
            gates.append(synth.Gate("RZ", c0, -1, float(rng.uniform(0, 6))))
    psi0 = synth.random_state(n, 4)
    ref = O.simulate(n, gates, psi0=psi0)
    for dt in ("c128", "c64"):
        got, plan = _emulate(n, gates, dt, psi0=psi0)
        assert np.max(np.abs(got - ref)) < EMU_TOL[dt]
        ccx = [o for o in plan["ops"] if int(o["code"]) == 23]
        kinds = {(int(o["b"]) != 0, int(o["sa"]) != 0xFF, int(o["sb"]) != 0xFF) for o in ccx}
        assert len(kinds) >= 2, kinds


@pytest.mark.parametrize("n,seed", [(13, 0), (15, 1)])
def test_automatic_low_qubits(n, seed):
    """min_low = 0: the planner picks 6 or 4 contiguous low qubits by its
    cost estimate; the plan it picks is as correct as either."""
    gates = synth.random_circuit(n, 8, seed)
    ref = O.simulate(n, gates)
    for dt in ("c128", "c64"):
        got, plan = _emulate(n, gates, dt, min_low=0)
        assert plan["min_low"] in (4, 6)
        fixed = [len(P.debug_plan(n, gates, dtype=dt, min_low=c)["passes"]) for c in (6, 4)]
        assert len(plan["passes"]) == fixed[0 if plan["min_low"] == 6 else 1]
        assert np.max(np.abs(got - ref)) < EMU_TOL[dt]


@pytest.mark.parametrize("n,dtype", [(16, "c128"), (20, "c64"), (28, "c128")])
def test_pass_layout_ranges(n, dtype):
    """Each pass's [layout_begin, layout_begin + n_layouts) holds every layout
    its exchanges and its store use, and the ranges tile the layout array (the
    kernel warms exactly that range)."""
    gates = synth.random_circuit(n, 6, 7)
    d = P.debug_plan(n, gates, dtype=dtype, min_low=0)
    passes, ops = d["passes"], d["ops"]
    assert len(passes) > 0
    nxt = 0
    for p in passes:
        lb, nl = int(p["layout_begin"]), int(p["n_layouts"])
        assert lb == nxt and nl >= 1
        nxt = lb + nl
        used = [int(p["store_layout"])]
        for o in ops[int(p["op_begin"]):int(p["op_end"])]:
            if int(o["code"]) == OP_EXCH:
                used += [int(o["a"]), int(o["b"])]
        assert max(used) < nl
    assert nxt == len(d["layouts"])


def _monomial_heavy(n, layers, seed):
    """Layers dominated by permutation gates (X, Y, SWAP, CNOT, CCX) with
    diagonals (RZ, T, CZ, CPHASE), an occasional dense RX / H and MARK on
    seeded indices: most of them act on qubits outside a pass's tile."""
    rng = np.random.default_rng(seed)
    gates = [synth.Gate("H", q) for q in range(n)]
    for _ in range(layers):
        for q in range(n):
            r = rng.random()
            if r < 0.3:
                gates.append(synth.Gate("X", q))
            elif r < 0.45:
                gates.append(synth.Gate("Y", q))
            elif r < 0.6:
                gates.append(synth.Gate("RZ", q, -1, float(rng.uniform(0, 6))))
            elif r < 0.7:
                gates.append(synth.Gate("T", q))
            elif r < 0.76:
                gates.append(synth.Gate(("RX", "H")[int(rng.integers(2))], q, -1, float(rng.uniform(0, 6))))
        perm = rng.permutation(n)
        for i in range(n // 2):
            a, b = int(perm[2 * i]), int(perm[2 * i + 1])
            kind = ("SWAP", "SWAP", "CNOT", "CZ", "CPHASE")[int(rng.integers(5))]
            gates.append(synth.Gate(kind, a, b, float(rng.uniform(0, 6))))
        if rng.random() < 0.5:
            c0, c1, t = (int(x) for x in rng.choice(n, 3, replace=False))
            gates.append(synth.Gate("CCX", c0, c1, 0.0, -1, 0, t))
        gates.append(synth.Gate("MARK", -1, -1, 0.0, -1, int(rng.integers(1 << n))))
    return gates


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,seed,min_low", [(16, 1, 4), (17, 2, 6), (18, 3, 0)])
def test_monomials_off_the_tile(n, seed, min_low, dtype):
    """X / Y on qubits outside a pass's tile flip bits of the global address
    translation, SWAPs with a qubit outside the tile exchange the qubits'
    physical bits; diagonals, CNOT / CCX controls and MARK then read the tile
    base through both. The emulated plans reproduce the oracle, move no data
    for those gates (fewer passes than without remapping, where every SWAP
    takes tile slots), and end in canonical order."""
    gates = _monomial_heavy(n, 12, seed)
    ref = O.simulate(n, gates)
    got, plan = _emulate(n, gates, dtype, min_low=min_low)
    assert np.max(np.abs(got - ref)) < EMU_TOL[dtype]
    assert plan["relabels"] > 0
    fixed = P.debug_plan(n, gates, dtype=dtype, remap=False, min_low=min_low or 6)
    assert len(plan["passes"]) < len(fixed["passes"])


@pytest.mark.parametrize("args,what", [
    ((0, 20, 2, 1, 0, 4096, 0), "NULL"),            # state NULL
    ((4096, 20, 2, 1, 0, 0, 0), "NULL"),            # out NULL
    ((4096, 20, 3, 1, 0, 4096, 0), "dtype"),
    ((4096, 35, 2, 1, 0, 4096, 0), "n_qubits"),
    ((4096, 20, 2, 0, 0, 4096, 0), "batch"),
    ((4096, 20, 2, 1, 20, 4096, 0), "qubit"),
    ((4096, 20, 2, 1, -2, 4096, 0), "qubit"),
    ((4100, 20, 2, 1, 0, 4096, 0), "misaligned"),
    ((4096, 22, 1, 65, 0, 4096, 0), "scratch"),     # 65 * 1024 partial sums
    ((4096, 10, 1, 65536, 0, 4096, 0), "batch"),
])
def test_noalloc_readout_rejects_before_any_launch(args, what):
    """Argument errors of the allocation-free readout are found on the host
    before any HIP call (the pointers here are never dereferenced)."""
    L = P.lib()
    st = L.sv_expect_z_noalloc(*[ctypes.c_void_p(a) if i in (0, 5, 6) else a for i, a in enumerate(args)])
    assert st == P.sv.SV_EINVAL
    assert what in P.last_error()


@pytest.mark.parametrize("n,dtype,basis", [(13, "c128", 0), (15, "c128", 12345), (14, "c64", 77),
                                           (16, "c64", 0)])
@pytest.mark.parametrize("lead", ["none", "h", "one_qubit"])
def test_recorded_basis_state_is_generated_by_the_first_pass(n, dtype, basis, lead):
    """sv_alloc / sv_set_basis only record the basis state; the plan's first
    pass then generates it: the basis state itself (a 2-qubit gate first), a
    Hadamard layer on it, or the product state of a leading run of 1-qubit
    gates. Whatever the buffer held before must not leak into the result."""
    gates = synth.random_circuit(n, 3, n + basis)
    gates = [g for g in gates if g.q1 >= 0] + gates   # a 2-qubit gate first
    if lead == "h":
        gates = [synth.Gate("H", q) for q in range(0, n, 3)] + gates
    elif lead == "one_qubit":
        gates = synth.random_circuit(n, 1, 7)[:n] + gates
    ref = O.simulate(n, gates, psi0=O.basis_state(n, basis))
    plan = P.debug_plan(n, gates, dtype=dtype, basis=basis, basis_in_memory=False)
    want = {"none": 1, "h": 1, "one_qubit": 8}[lead]
    assert not plan["small"] and int(plan["passes"][0]["flags"]) & 9 == want
    assert (plan["generated_h"] > 0) == (lead == "h")
    assert (plan["generated_product"] > 0) == (lead == "one_qubit")
    garbage = np.random.default_rng(5).standard_normal(1 << n) * (1 + 1j)
    got = run_plan(plan, garbage, n)
    assert np.max(np.abs(got - ref)) < EMU_TOL[dtype]
