"""Seeded synthetic circuit generators.

This module only draws random numbers and lists gates by name. It holds none of
the simulation arithmetic (no gate matrices, no amplitude updates), so both the
CPU oracle and the GPU path can consume its output without sharing any of the
method's code.

A gate is a ``Gate`` record:
  name   gate kind, one of GATE_NAMES
  q0     first qubit (target of a 1-qubit gate; control of CNOT; first operand
         of a 2-qubit gate = the high bit of the gate-local 2-bit index)
  q1     second qubit, -1 for 1-qubit and n-qubit gates
  angle  rotation / phase angle in radians (RX, RY, RZ, P, CPHASE)
  param  -1, or an index into a per-circuit parameter vector that replaces
         ``angle`` (used by the QNN ansatz)
  index  basis index for MARK (sign flip of one basis state), else 0
  q2     third qubit of a 3-qubit gate (CCX: q0, q1 controls, q2 target;
         CSWAP: q0 control, q1 and q2 exchanged), -1 otherwise

Qubit q is bit q of the amplitude index (qubit 0 is the least significant bit).
"""
from __future__ import annotations

import math
from typing import List, NamedTuple, Optional, Sequence

import numpy as np


class Gate(NamedTuple):
    name: str
    q0: int
    q1: int = -1
    angle: float = 0.0
    param: int = -1
    index: int = 0
    q2: int = -1      # third qubit of CCX / CSWAP


ONE_QUBIT = ("I", "X", "Y", "Z", "H", "S", "SDG", "T", "TDG", "RX", "RY", "RZ", "P", "U1",
             "SX", "SXDG", "R", "U")
# Table 1 two-qubit gates beyond the config mix: controlled Y, iSWAP, double
# CNOT, controlled RZ, ZZ rotation and controlled phase (CU1 = CPHASE).
TABLE1_2Q = ("CY", "ISWAP", "DCX", "CRZ", "RZZ", "CU1", "RXX", "RYY", "RZX", "ECR", "CH", "CSX",
             "CU3", "CU")
# Gates whose several angles come from the parameter vector at `param`.
MULTI_ANGLE = {"R": 2, "U": 3, "CU3": 3, "CU": 4}
TWO_QUBIT = ("CNOT", "CZ", "SWAP", "CPHASE", "U2") + TABLE1_2Q
THREE_QUBIT = ("CCX", "CSWAP")
# U1 / U2: a general 2x2 / 4x4 matrix taken from the parameter vector at
# `param` (8 / 32 reals: row-major (re, im) pairs), see matrix_params().
MATRIX_GATES = ("U1", "U2")
N_QUBIT = ("MARK",)
GATE_NAMES = ONE_QUBIT + TWO_QUBIT + THREE_QUBIT + N_QUBIT
ANGLED = ("RX", "RY", "RZ", "P", "CPHASE")

# Gate pools of the seeded random workloads.
RANDOM_1Q_POOL = ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ")
RANDOM_2Q_POOL = ("CNOT", "CZ", "SWAP", "CPHASE")
CAPACITY_DENSE_POOL = ("RX", "RY")
CAPACITY_SPARSE_POOL = ("RZ", "S", "T", "X")
CAPACITY_2Q_POOL = ("CZ", "CPHASE", "CNOT")


def _layer_pairs(rng: np.random.Generator, n: int, pool: Sequence[str],
                 p_pair: float) -> List[Gate]:
    """Shuffle the qubits, pair them up (perm[2i], perm[2i+1]) and give each
    pair a gate drawn uniformly from ``pool`` with probability ``p_pair``."""
    perm = rng.permutation(n)
    out = []
    for i in range(n // 2):
        a, b = int(perm[2 * i]), int(perm[2 * i + 1])
        if rng.random() < p_pair:
            name = pool[int(rng.integers(len(pool)))]
            ang = float(rng.uniform(0.0, 2.0 * math.pi)) if name == "CPHASE" else 0.0
            out.append(Gate(name, a, b, ang))
    return out


def random_circuit(n: int, depth: int, seed: int) -> List[Gate]:
    """Random circuit of the plain-method workloads (n=12 depth 20; n=28 depth 100).

    Per layer: for q = 0..n-1 a gate drawn uniformly from RANDOM_1Q_POOL
    (angles U[0, 2pi)), then the qubits are shuffled and paired, and each pair
    gets a gate from RANDOM_2Q_POOL with probability 0.5 (CPHASE angle U[0, 2pi)).
    RNG: numpy PCG64 seeded with ``seed``; draw order as written here.
    """
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    for _ in range(depth):
        for q in range(n):
            name = RANDOM_1Q_POOL[int(rng.integers(len(RANDOM_1Q_POOL)))]
            ang = float(rng.uniform(0.0, 2.0 * math.pi)) if name in ANGLED else 0.0
            gates.append(Gate(name, q, -1, ang))
        if n >= 2:
            gates.extend(_layer_pairs(rng, n, RANDOM_2Q_POOL, 0.5))
    return gates


def capacity_circuit(n: int, layers: int, seed: int, p_dense: float = 0.1) -> List[Gate]:
    """Capacity workload: an H layer on every qubit, then ``layers`` layers in
    which each qubit gets, with probability p_dense (0.1), a dense gate from
    CAPACITY_DENSE_POOL and otherwise a gate from CAPACITY_SPARSE_POOL, followed
    by random disjoint pairs (probability 0.5) from CAPACITY_2Q_POOL.
    p_dense = 0 gives the same draw sequence with only sparse gates."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = [Gate("H", q) for q in range(n)]
    for _ in range(layers):
        for q in range(n):
            if rng.random() < p_dense:
                name = CAPACITY_DENSE_POOL[int(rng.integers(len(CAPACITY_DENSE_POOL)))]
            else:
                name = CAPACITY_SPARSE_POOL[int(rng.integers(len(CAPACITY_SPARSE_POOL)))]
            ang = float(rng.uniform(0.0, 2.0 * math.pi)) if name in ANGLED else 0.0
            gates.append(Gate(name, q, -1, ang))
        if n >= 2:
            gates.extend(_layer_pairs(rng, n, CAPACITY_2Q_POOL, 0.5))
    return gates


def matrix_params(m: np.ndarray) -> np.ndarray:
    """A 2x2 or 4x4 complex matrix as the reals a U1 / U2 gate reads from the
    parameter vector: row-major (re, im) pairs."""
    m = np.asarray(m, dtype=np.complex128)
    out = np.empty(2 * m.size)
    out[0::2] = m.real.ravel()
    out[1::2] = m.imag.ravel()
    return out


def random_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """A random dim x dim unitary (QR of a complex Gaussian matrix with the
    phases of R's diagonal divided out)."""
    z = rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def grover_iterations(n: int) -> int:
    """Iteration count floor(pi/4 * sqrt(2^n)) (804 for n = 20)."""
    return int(math.floor(math.pi / 4.0 * math.sqrt(2.0 ** n)))


def grover_marked(n: int, seed: int) -> int:
    """Seeded marked index, uniform in [0, 2^n)."""
    rng = np.random.default_rng(seed)
    return int(rng.integers(0, 1 << n))


def grover_circuit(n: int, marked: int, iterations: Optional[int] = None) -> List[Gate]:
    """Grover search as a gate list: an H layer, then per iteration the phase
    oracle MARK(marked), an H layer, MARK(0) (the zero-state reflection
    I - 2|0><0|) and an H layer. Each iteration therefore equals -D*O with the
    diffusion D = 2|s><s| - I, i.e. a global factor (-1)^iterations."""
    k = grover_iterations(n) if iterations is None else iterations
    gates: List[Gate] = [Gate("H", q) for q in range(n)]
    for _ in range(k):
        gates.append(Gate("MARK", -1, -1, 0.0, -1, marked))
        gates.extend(Gate("H", q) for q in range(n))
        gates.append(Gate("MARK", -1, -1, 0.0, -1, 0))
        gates.extend(Gate("H", q) for q in range(n))
    return gates


def qnn_ansatz(n: int, layers: int) -> List[Gate]:
    """Hardware-efficient ansatz of the QNN workloads, with parameter references.

    Parameter vector layout: params[0:n] = the input encoding x (RY(x_q) on every
    qubit), params[n + (2*l + 0)*n + q] = RY angle of layer l on qubit q,
    params[n + (2*l + 1)*n + q] = RZ angle. Each layer ends with the CNOT ring
    CNOT(q, (q+1) mod n) for q = 0..n-1 in that order. Output: <Z_0>.
    """
    gates: List[Gate] = [Gate("RY", q, -1, 0.0, q) for q in range(n)]
    for l in range(layers):
        gates.extend(Gate("RY", q, -1, 0.0, n + (2 * l + 0) * n + q) for q in range(n))
        gates.extend(Gate("RZ", q, -1, 0.0, n + (2 * l + 1) * n + q) for q in range(n))
        if n >= 2:
            gates.extend(Gate("CNOT", q, (q + 1) % n) for q in range(n))
    return gates


def qnn_n_params(n: int, layers: int) -> int:
    return n + 2 * n * layers


def qnn_params(n: int, layers: int, batch: int, seed: int) -> np.ndarray:
    """[batch, n + 2nL] float64: x ~ U[-pi, pi]^n then theta ~ N(0, 1)^(2nL)."""
    rng = np.random.default_rng(seed)
    out = np.empty((batch, qnn_n_params(n, layers)), dtype=np.float64)
    for b in range(batch):
        out[b, :n] = rng.uniform(-math.pi, math.pi, size=n)
        out[b, n:] = rng.standard_normal(2 * n * layers)
    return out


class QNNRequest(NamedTuple):
    rid: int
    arrival_s: float      # offset from stream start, seconds
    n: int
    layers: int
    params: np.ndarray    # [n + 2nL] float64


def poisson_requests(count: int, rate_hz: float, seed: int,
                     n_range=(8, 20), layer_range=(4, 16)) -> List[QNNRequest]:
    """Poisson stream of QNN requests: exponential inter-arrival times at
    ``rate_hz``, n ~ U{n_range}, L ~ U{layer_range} (inclusive),
    x ~ U[-pi, pi]^n, theta ~ N(0, 1)^(2nL)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate_hz)) if rate_hz > 0 else 0.0
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        layers = int(rng.integers(layer_range[0], layer_range[1] + 1))
        p = np.empty(qnn_n_params(n, layers))
        p[:n] = rng.uniform(-math.pi, math.pi, size=n)
        p[n:] = rng.standard_normal(2 * n * layers)
        out.append(QNNRequest(rid, t, n, layers, p))
    return out


def random_state(n: int, seed: int) -> np.ndarray:
    """Seeded normalised complex128 state (Gaussian real and imaginary parts)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def all_kinds_circuit(n: int, seed: int):
    """Every gate kind on every qubit (2- and 3-qubit kinds with random
    partners, MARK with a random index), shuffled. U1 / U2 take random unitaries from the
    returned parameter vector. Returns (gates, params)."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    params: List[float] = []
    for name in GATE_NAMES:
        for q in range(n):
            ang = float(rng.uniform(0.0, 2.0 * math.pi))
            if name in MATRIX_GATES:
                off = len(params)
                params.extend(matrix_params(random_unitary(2 if name == "U1" else 4, rng)).tolist())
                if name == "U2":
                    if n < 2:
                        continue
                    gates.append(Gate(name, q, int((q + 1 + rng.integers(n - 1)) % n), 0.0, off))
                else:
                    gates.append(Gate(name, q, -1, 0.0, off))
            elif name in MULTI_ANGLE:
                if name in TWO_QUBIT and n < 2:
                    continue
                off = len(params)
                params.extend(rng.uniform(-math.pi, math.pi, MULTI_ANGLE[name]).tolist())
                q1 = int((q + 1 + rng.integers(n - 1)) % n) if name in TWO_QUBIT else -1
                gates.append(Gate(name, q, q1, 0.0, off))
            elif name in TWO_QUBIT:
                if n < 2:
                    continue
                gates.append(Gate(name, q, int((q + 1 + rng.integers(n - 1)) % n), ang))
            elif name in THREE_QUBIT:
                if n < 3:
                    continue
                others = [int(x) for x in rng.permutation([x for x in range(n) if x != q])[:2]]
                gates.append(Gate(name, q, others[0], 0.0, -1, 0, others[1]))
            elif name == "MARK":
                gates.append(Gate(name, -1, -1, 0.0, -1, int(rng.integers(0, 1 << n))))
            else:
                gates.append(Gate(name, q, -1, ang))
    order = rng.permutation(len(gates))
    return [gates[i] for i in order], np.array(params, dtype=np.float64)


def table1_circuit(n: int, seed: int, layers: int = 4):
    """The Table 1 gates beyond the config mix (SX, SXDG, R, U and the
    2- and 3-qubit ones of TABLE1_2Q and THREE_QUBIT), three of each per layer
    at random distinct operands, between layers of RY on every qubit. The
    angled ones read their angles from the returned parameter vector.
    Returns (gates, params)."""
    rng = np.random.default_rng(seed)
    gates: List[Gate] = []
    params: List[float] = []
    for _ in range(layers):
        for q in range(n):
            gates.append(Gate("RY", q, -1, float(rng.uniform(0, 2 * math.pi))))
        for name in ("SX", "SXDG", "R", "U") + TABLE1_2Q + THREE_QUBIT:
            for _ in range(3):
                qs = [int(x) for x in rng.permutation(n)[:3]]
                q1 = qs[1] if name in TWO_QUBIT else -1
                if name in MULTI_ANGLE:
                    params.extend(rng.uniform(-math.pi, math.pi, MULTI_ANGLE[name]).tolist())
                    gates.append(Gate(name, qs[0], q1, 0.0, len(params) - MULTI_ANGLE[name]))
                elif name in ("CRZ", "RZZ", "CU1", "RXX", "RYY", "RZX"):
                    params.append(float(rng.uniform(-math.pi, math.pi)))
                    gates.append(Gate(name, qs[0], q1, 0.0, len(params) - 1))
                elif name in ("SX", "SXDG"):
                    gates.append(Gate(name, qs[0]))
                elif name in THREE_QUBIT:
                    gates.append(Gate(name, qs[0], qs[1], 0.0, -1, 0, qs[2]))
                else:
                    gates.append(Gate(name, qs[0], qs[1]))
    return gates, np.array(params, dtype=np.float64)


def amplitude_gate_updates(n: int, gates: Sequence[Gate]) -> int:
    """Work measure: every gate counts 2^n amplitude updates per state."""
    return len(gates) * (1 << n)


_SELF_INVERSE = ("I", "X", "Y", "Z", "H", "CNOT", "CZ", "SWAP", "MARK")
_INVERSE_NAME = {"S": "SDG", "SDG": "S", "T": "TDG", "TDG": "T"}


def inverse_circuit(gates: Sequence[Gate]) -> List[Gate]:
    """Gate list of the inverse circuit: reversed order, each gate replaced by
    its inverse (named inverse, or the same rotation with the angle negated).
    Parameter references are not supported (resolve them first)."""
    out = []
    for g in reversed(gates):
        if g.param >= 0:
            raise ValueError("resolve parameter references before inverting")
        if g.name in _SELF_INVERSE:
            out.append(g)
        elif g.name in _INVERSE_NAME:
            out.append(g._replace(name=_INVERSE_NAME[g.name]))
        else:  # RX, RY, RZ, P, CPHASE
            out.append(g._replace(angle=-g.angle))
    return out


def resolve_params(gates: Sequence[Gate], params) -> List[Gate]:
    """Replace parameter references by the referenced angle values."""
    return [g._replace(angle=float(params[g.param]), param=-1) if g.param >= 0 else g
            for g in gates]
