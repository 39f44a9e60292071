"""CPU FP64 oracle driver — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this module. The product path never calls it.

It computes the plain definition of full-state simulation (paper Sec. II-A: each
gate is U = I^(k-1) (x) G (x) I^(n-k) applied as U|phi>), one dense gate at a
time in double-precision complex, through ``liboracle.so`` (plain C, built with
gcc from ``liboracle.c``). Readouts follow Sec. II-A too: probabilities are
|alpha|^2, the norm is sum |alpha|^2 = 1, and <Z_q> = sum |alpha_i|^2 (1 - 2 b_q(i)).

Gradients (no counterpart in the paper; used to pin the adjoint backward):
parameter shift, exact for gates exp(-i theta P / 2):
    df/dtheta = (f(theta + pi/2) - f(theta - pi/2)) / 2,
and central finite differences (f(theta + h) - f(theta - h)) / (2h).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

from . import gates as G

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "liboracle.c")

_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fcx-limited-range",
                               "-shared", "-fPIC", SRC_PATH, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.or_apply_1q.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
        L.or_apply_2q.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        L.or_apply_mark.argtypes = [P, ctypes.c_int, ctypes.c_uint64]
        L.or_run.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P]
        L.or_run.restype = ctypes.c_int64
        L.or_norm2.argtypes = [P, ctypes.c_int]
        L.or_norm2.restype = ctypes.c_double
        L.or_expect_z.argtypes = [P, ctypes.c_int, ctypes.c_int]
        L.or_expect_z.restype = ctypes.c_double
        L.or_inner.argtypes = [P, P, ctypes.c_int, P, P]
        L.or_max_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def set_threads(k: int) -> None:
    lib().or_set_threads(int(k))


def max_threads() -> int:
    return int(lib().or_max_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def basis_state(n: int, j: int = 0) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[j] = 1.0
    return psi


def _angle(g, params) -> float:
    if g.param >= 0:
        if params is None:
            raise ValueError("gate references a parameter but no params were given")
        return float(params[g.param])
    return float(g.angle)


def gate_matrix(g, params: Optional[np.ndarray] = None) -> np.ndarray:
    """The 2x2, 4x4 or 8x8 matrix of one gate record (angles and matrices that
    the gate reads from the parameter vector taken from ``params``)."""
    if g.name in ("U1", "U2"):
        if params is None or g.param < 0:
            raise ValueError(f"{g.name} reads its matrix from the parameters")
        return G.params_matrix(g.name, params, g.param)
    if g.name in G.MULTI_ANGLE:
        k = G.MULTI_ANGLE[g.name]
        if params is None or g.param < 0 or g.param + k > len(params):
            raise ValueError(f"{g.name} reads {k} angles from the parameters")
        return G.angles_matrix(g.name, np.asarray(params, dtype=np.float64)[g.param: g.param + k])
    return G.matrix(g.name, _angle(g, params))


def encode(gates: Sequence, params: Optional[np.ndarray] = None):
    """Gate list -> flat arrays (kind, q0, q1, q2, mats[64], idx) for or_run."""
    ng = len(gates)
    kind = np.zeros(ng, dtype=np.int32)
    q0 = np.zeros(ng, dtype=np.int32)
    q1 = np.zeros(ng, dtype=np.int32)
    q2 = np.full(ng, -1, dtype=np.int32)
    mats = np.zeros((ng, 64), dtype=np.complex128)
    idx = np.zeros(ng, dtype=np.uint64)
    for k, g in enumerate(gates):
        a = G.arity(g.name)
        if a == 0:
            kind[k] = 3
            idx[k] = g.index
            continue
        m = gate_matrix(g, params)
        kind[k] = 4 if a == 3 else a
        q0[k] = g.q0
        q1[k] = g.q1
        if a == 3:
            q2[k] = g.q2
        mats[k, : m.size] = m.reshape(-1)
    return kind, q0, q1, q2, mats, idx


def apply(psi: np.ndarray, n: int, gates: Sequence, params: Optional[np.ndarray] = None) -> np.ndarray:
    """Apply ``gates`` to ``psi`` in place (complex128, length 2^n)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == (1 << n)
    if not gates:
        return psi
    kind, q0, q1, q2, mats, idx = encode(gates, params)
    r = lib().or_run(_ptr(psi), n, len(gates), _ptr(kind), _ptr(q0), _ptr(q1), _ptr(q2), _ptr(mats),
                     _ptr(idx))
    if r < 0:
        raise ValueError(f"oracle rejected gate #{-r - 1}: {gates[-r - 1]}")
    return psi


def simulate(n: int, gates: Sequence, params: Optional[np.ndarray] = None,
             psi0: Optional[np.ndarray] = None) -> np.ndarray:
    """Final state of ``gates`` applied to ``psi0`` (default |0...0>)."""
    psi = basis_state(n) if psi0 is None else np.array(psi0, dtype=np.complex128, copy=True)
    return apply(psi, n, gates, params)


def norm2(psi: np.ndarray) -> float:
    n = int(psi.size).bit_length() - 1
    return float(lib().or_norm2(_ptr(np.ascontiguousarray(psi)), n))


def expect_z(psi: np.ndarray, q: int) -> float:
    n = int(psi.size).bit_length() - 1
    return float(lib().or_expect_z(_ptr(np.ascontiguousarray(psi)), n, q))


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    n = int(a.size).bit_length() - 1
    re = ctypes.c_double()
    im = ctypes.c_double()
    lib().or_inner(_ptr(np.ascontiguousarray(a)), _ptr(np.ascontiguousarray(b)), n,
                   ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def loss_z(n: int, gates: Sequence, params: np.ndarray, qubit: int = 0) -> float:
    """f(params) = <Z_qubit> of the circuit applied to |0...0>."""
    return expect_z(simulate(n, gates, params), qubit)


def grad_param_shift(n: int, gates: Sequence, params: np.ndarray, which: Sequence[int],
                     qubit: int = 0) -> np.ndarray:
    """d<Z_qubit>/d params[p] for p in ``which`` by the parameter-shift rule.

    Every gate that references params[p] must be RX/RY/RZ (exp(-i t P/2)), and
    each parameter may be used by one gate only (the rule then is exact)."""
    out = np.empty(len(which))
    for k, p in enumerate(which):
        users = [g for g in gates if g.param == p]
        if len(users) != 1 or users[0].name not in ("RX", "RY", "RZ"):
            raise ValueError(f"parameter {p} is not used by exactly one rotation")
        pp = np.array(params, dtype=np.float64, copy=True)
        pp[p] = params[p] + math.pi / 2
        fp = loss_z(n, gates, pp, qubit)
        pp[p] = params[p] - math.pi / 2
        fm = loss_z(n, gates, pp, qubit)
        out[k] = 0.5 * (fp - fm)
    return out


def grad_fd(n: int, gates: Sequence, params: np.ndarray, which: Sequence[int],
            qubit: int = 0, h: float = 1e-6) -> np.ndarray:
    """Central finite differences (f(p + h) - f(p - h)) / (2h)."""
    out = np.empty(len(which))
    for k, p in enumerate(which):
        pp = np.array(params, dtype=np.float64, copy=True)
        pp[p] = params[p] + h
        fp = loss_z(n, gates, pp, qubit)
        pp[p] = params[p] - h
        fm = loss_z(n, gates, pp, qubit)
        out[k] = (fp - fm) / (2.0 * h)
    return out


def _row_nonzero(mat: np.ndarray):
    """For a matrix with exactly one non-zero per row: (column, value) per row."""
    cols = np.empty(mat.shape[0], dtype=np.int64)
    vals = np.empty(mat.shape[0], dtype=np.complex128)
    for r in range(mat.shape[0]):
        nz = np.flatnonzero(mat[r])
        if len(nz) != 1:
            raise ValueError("gate is not monomial (one non-zero per row)")
        cols[r] = nz[0]
        vals[r] = mat[r, nz[0]]
    return cols, vals


def monomial_amplitudes(n: int, gates: Sequence, indices: Sequence[int], initial="uniform",
                        params: Optional[np.ndarray] = None) -> np.ndarray:
    """Selected amplitudes <i|U_m ... U_1|psi_in> of a circuit of monomial gates
    (one non-zero per row: diagonal, permutation or permutation-with-phase,
    the gates the paper's DAX form stores as one value and one index per row,
    Sec. III-A), computed one index at a time without the state.

    For a monomial U, (U psi)[i] = U[i, c(i)] psi[c(i)] with c(i) the column of
    row i's non-zero, so the amplitude is the product of the visited entries
    times psi_in at the index reached after walking the gates from last to
    first. The embedded U = I..(x) G (x)..I has U[i, c] = G[r(i), r(c)] where i
    and c agree off the gate's qubits (r = the local row, (b_q0 << 1) | b_q1,
    or (b_q0 << 2) | (b_q1 << 1) | b_q2 for a 3-qubit gate).
    initial: "uniform" (psi_in = 2^(-n/2) everywhere, i.e. H^n|0>) or a basis
    index j (psi_in = |j>). Returns complex128 [len(indices)]."""
    idx = np.array(indices, dtype=np.int64).copy()
    amp = np.ones(len(idx), dtype=np.complex128)
    for g in reversed(list(gates)):
        if g.name == "MARK":
            amp = np.where(idx == np.int64(g.index), -amp, amp)
            continue
        mat = gate_matrix(g, params)
        cols, vals = _row_nonzero(mat)
        if G.arity(g.name) == 1:
            r = (idx >> g.q0) & 1
            c = cols[r]
            idx = (idx & ~np.int64(1 << g.q0)) | (c << g.q0)
        elif G.arity(g.name) == 3:
            qs = (g.q0, g.q1, g.q2)
            r = (((idx >> qs[0]) & 1) << 2) | (((idx >> qs[1]) & 1) << 1) | ((idx >> qs[2]) & 1)
            c = cols[r]
            idx = idx & ~np.int64(sum(1 << q for q in qs))
            for sh, q in zip((2, 1, 0), qs):
                idx = idx | (((c >> sh) & 1) << q)
        else:
            r = (((idx >> g.q0) & 1) << 1) | ((idx >> g.q1) & 1)
            c = cols[r]
            idx = (idx & ~np.int64((1 << g.q0) | (1 << g.q1))) | ((c >> 1) << g.q0) | ((c & 1) << g.q1)
        amp = amp * vals[r]
    if isinstance(initial, str):
        if initial != "uniform":
            raise ValueError("initial must be 'uniform' or a basis index")
        return amp * (2.0 ** (-0.5 * n))
    return np.where(idx == np.int64(initial), amp, 0.0 + 0.0j)


def grover_closed_form(n: int, k: int):
    """Textbook Grover amplitudes after k iterations of D*O from H^n|0>, with
    D = 2|s><s| - I: (marked, unmarked, success probability), where
    theta = arcsin(2^(-n/2)), marked = sin((2k+1) theta) and every unmarked
    amplitude = cos((2k+1) theta) / sqrt(N - 1)."""
    N = float(1 << n)
    theta = math.asin(1.0 / math.sqrt(N))
    a = math.sin((2 * k + 1) * theta)
    b = math.cos((2 * k + 1) * theta) / math.sqrt(N - 1.0)
    return a, b, a * a
