"""Gate matrices of the CPU FP64 oracle — TEST INFRASTRUCTURE ONLY.

Textbook definitions in complex128. The paper prints X and Y (Sec. III-A1, the
Y (x) X example) and the Hadamard's 1/sqrt(N) magnitude (Sec. III-B1, the RH
structure); the rest follow the standard definitions (rotations are
exp(-i theta P / 2), P in {X, Y, Z}).

A 2-qubit matrix acts on the local index (b_q0 << 1) | b_q1: the first operand
is the high bit, e.g. CNOT(q0 = control, q1 = target).

Parity pins (tests/test_oracle_pins.py): unitarity, the paper's X, Y and Y (x) X,
rotations against scipy's matrix exponential of the Pauli matrices, and the
algebraic identities S^2 = Z, T^2 = S, CPHASE(pi) = CZ, CNOT = (I (x) H) CZ (I (x) H).
"""
from __future__ import annotations

import cmath
import math

import numpy as np

SQRT1_2 = 1.0 / math.sqrt(2.0)

_FIXED_1Q = {
    "I": [[1, 0], [0, 1]],
    "X": [[0, 1], [1, 0]],
    "Y": [[0, -1j], [1j, 0]],
    "Z": [[1, 0], [0, -1]],
    "H": [[SQRT1_2, SQRT1_2], [SQRT1_2, -SQRT1_2]],
    "S": [[1, 0], [0, 1j]],
    "SDG": [[1, 0], [0, -1j]],
    "T": [[1, 0], [0, cmath.exp(1j * math.pi / 4)]],
    "TDG": [[1, 0], [0, cmath.exp(-1j * math.pi / 4)]],
}

_FIXED_2Q = {
    "CNOT": [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
    "CZ": [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, -1]],
    "SWAP": [[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
}


def matrix(name: str, angle: float = 0.0) -> np.ndarray:
    """The gate's 2x2 or 4x4 complex128 matrix (MARK has none: it is n-qubit;
    U1 / U2 take theirs from the parameters, see params_matrix)."""
    if name in _FIXED_1Q:
        return np.array(_FIXED_1Q[name], dtype=np.complex128)
    if name in _FIXED_2Q:
        return np.array(_FIXED_2Q[name], dtype=np.complex128)
    c, s = math.cos(angle / 2.0), math.sin(angle / 2.0)
    if name == "RX":
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if name == "RY":
        return np.array([[c, -s], [s, c]], dtype=np.complex128)
    if name == "RZ":
        return np.array([[cmath.exp(-0.5j * angle), 0], [0, cmath.exp(0.5j * angle)]],
                        dtype=np.complex128)
    if name == "P":
        return np.array([[1, 0], [0, cmath.exp(1j * angle)]], dtype=np.complex128)
    if name == "CPHASE":
        return np.diag([1, 1, 1, cmath.exp(1j * angle)]).astype(np.complex128)
    raise ValueError(f"no matrix for gate {name!r}")


def arity(name: str) -> int:
    """1 or 2 for matrix gates, 0 for the n-qubit MARK."""
    if name == "MARK":
        return 0
    return 2 if name in _FIXED_2Q or name in ("CPHASE", "U2") else 1


def params_matrix(name: str, params, offset: int) -> np.ndarray:
    """The matrix of a U1 (2x2) or U2 (4x4) gate: row-major (re, im) pairs
    of reals read from the parameter vector starting at `offset`."""
    size = 2 if name == "U1" else 4
    v = np.asarray(params, dtype=np.float64)[offset: offset + 2 * size * size]
    if v.size != 2 * size * size:
        raise ValueError(f"{name} needs {2 * size * size} reals from parameter {offset}")
    return (v[0::2] + 1j * v[1::2]).reshape(size, size)


def generator(name: str) -> np.ndarray:
    """Pauli P with gate = exp(-i angle P / 2) for the parametric rotations."""
    return {"RX": np.array(_FIXED_1Q["X"], dtype=np.complex128),
            "RY": np.array(_FIXED_1Q["Y"], dtype=np.complex128),
            "RZ": np.array(_FIXED_1Q["Z"], dtype=np.complex128)}[name]
