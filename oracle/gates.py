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
The Table 1 additions (CY, ISWAP, DCX, CRZ, RZZ, CU1, CCX, CSWAP) are pinned by
the bit logic of the permutations, matrix exponentials of their generators,
and textbook identities (CY = (I (x) S) CNOT (I (x) S^dagger), ISWAP^2 = Z (x) Z,
DCX^3 = I, CCX = (I (x) I (x) H) CCZ (I (x) I (x) H), CSWAP from three CCX).
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
    # square root of X and its inverse
    "SX": [[0.5 + 0.5j, 0.5 - 0.5j], [0.5 - 0.5j, 0.5 + 0.5j]],
    "SXDG": [[0.5 - 0.5j, 0.5 + 0.5j], [0.5 + 0.5j, 0.5 - 0.5j]],
    "S": [[1, 0], [0, 1j]],
    "SDG": [[1, 0], [0, -1j]],
    "T": [[1, 0], [0, cmath.exp(1j * math.pi / 4)]],
    "TDG": [[1, 0], [0, cmath.exp(-1j * math.pi / 4)]],
}

_FIXED_2Q = {
    "CNOT": [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
    "CZ": [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, -1]],
    "SWAP": [[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
    # controlled Y (q0 = control)
    "CY": [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, -1j], [0, 0, 1j, 0]],
    # SWAP with a factor i on the two exchanged states
    "ISWAP": [[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]],
    # double CNOT: |x y> -> |y, x xor y> (CNOT q0 -> q1, then CNOT q1 -> q0)
    "DCX": [[1, 0, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1], [0, 1, 0, 0]],
    # echoed cross-resonance: (X (x) I - Y (x) X) / sqrt 2
    "ECR": [[0, 0, SQRT1_2, 1j * SQRT1_2], [0, 0, 1j * SQRT1_2, SQRT1_2],
            [SQRT1_2, -1j * SQRT1_2, 0, 0], [-1j * SQRT1_2, SQRT1_2, 0, 0]],
    # controlled H and controlled SX (q0 = control)
    "CH": [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, SQRT1_2, SQRT1_2], [0, 0, SQRT1_2, -SQRT1_2]],
    "CSX": [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0.5 + 0.5j, 0.5 - 0.5j], [0, 0, 0.5 - 0.5j, 0.5 + 0.5j]],
}

# 3-qubit monomial gates (Table 1): local index (b_q0 << 2) | (b_q1 << 1) | b_q2.
# CCX (Toffoli): q0, q1 controls, q2 target. CSWAP (Fredkin): q0 control,
# q1 and q2 exchanged.
def _perm8(a: int, b: int) -> np.ndarray:
    m = np.eye(8, dtype=np.complex128)
    m[[a, b]] = m[[b, a]]
    return m


_FIXED_3Q = {
    "CCX": _perm8(6, 7),
    "CSWAP": _perm8(5, 6),
}


def matrix(name: str, angle: float = 0.0) -> np.ndarray:
    """The gate's 2x2 or 4x4 complex128 matrix (MARK has none: it is n-qubit;
    U1 / U2 take theirs from the parameters, see params_matrix)."""
    if name in _FIXED_1Q:
        return np.array(_FIXED_1Q[name], dtype=np.complex128)
    if name in _FIXED_2Q:
        return np.array(_FIXED_2Q[name], dtype=np.complex128)
    if name in _FIXED_3Q:
        return _FIXED_3Q[name].copy()
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
    if name in ("CPHASE", "CU1"):
        return np.diag([1, 1, 1, cmath.exp(1j * angle)]).astype(np.complex128)
    if name == "CRZ":   # controlled RZ (q0 = control)
        return np.diag([1, 1, cmath.exp(-0.5j * angle), cmath.exp(0.5j * angle)]).astype(np.complex128)
    if name == "RZZ":   # exp(-i angle Z (x) Z / 2)
        m, p = cmath.exp(-0.5j * angle), cmath.exp(0.5j * angle)
        return np.diag([m, p, p, m]).astype(np.complex128)
    if name == "RXX":   # exp(-i angle X (x) X / 2)
        return np.array([[c, 0, 0, -1j * s], [0, c, -1j * s, 0], [0, -1j * s, c, 0],
                         [-1j * s, 0, 0, c]], dtype=np.complex128)
    if name == "RYY":   # exp(-i angle Y (x) Y / 2)
        return np.array([[c, 0, 0, 1j * s], [0, c, -1j * s, 0], [0, -1j * s, c, 0],
                         [1j * s, 0, 0, c]], dtype=np.complex128)
    if name == "RZX":   # exp(-i angle Z (x) X / 2): Z on q0, X on q1
        return np.array([[c, -1j * s, 0, 0], [-1j * s, c, 0, 0], [0, 0, c, 1j * s],
                         [0, 0, 1j * s, c]], dtype=np.complex128)
    raise ValueError(f"no matrix for gate {name!r}")


# Gates with several angles, read from the parameter vector at `param`:
# R(theta, phi), U(theta, phi, lambda), CU3(theta, phi, lambda),
# CU(theta, phi, lambda, gamma).
MULTI_ANGLE = {"R": 2, "U": 3, "CU3": 3, "CU": 4}


def _u3(theta: float, phi: float, lam: float) -> np.ndarray:
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    return np.array([[c, -cmath.exp(1j * lam) * s],
                     [cmath.exp(1j * phi) * s, cmath.exp(1j * (phi + lam)) * c]], dtype=np.complex128)


def _controlled(u: np.ndarray) -> np.ndarray:
    m = np.eye(4, dtype=np.complex128)
    m[2:, 2:] = u
    return m


def angles_matrix(name: str, angles) -> np.ndarray:
    """Matrix of a several-angle gate (MULTI_ANGLE) from its angles.
    R(t, p) = exp(-i t (cos p X + sin p Y) / 2); U(t, p, l) =
    [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]];
    CU3 = controlled U; CU(t, p, l, g) = controlled e^{ig} U(t, p, l)."""
    a = [float(x) for x in angles]
    if name == "R":
        t, ph = a
        c, s = math.cos(t / 2.0), math.sin(t / 2.0)
        return np.array([[c, -1j * cmath.exp(-1j * ph) * s], [-1j * cmath.exp(1j * ph) * s, c]],
                        dtype=np.complex128)
    if name == "U":
        return _u3(*a)
    if name == "CU3":
        return _controlled(_u3(*a))
    if name == "CU":
        return _controlled(cmath.exp(1j * a[3]) * _u3(*a[:3]))
    raise ValueError(f"{name!r} is not a several-angle gate")


TWO_QUBIT_ANGLED = ("CPHASE", "CU1", "CRZ", "RZZ", "RXX", "RYY", "RZX", "CU3", "CU")


def arity(name: str) -> int:
    """1, 2 or 3 for matrix gates, 0 for the n-qubit MARK."""
    if name == "MARK":
        return 0
    if name in _FIXED_3Q:
        return 3
    return 2 if name in _FIXED_2Q or name in TWO_QUBIT_ANGLED or name == "U2" else 1


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
