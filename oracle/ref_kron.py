"""Brute-force matrix-tensor-product (MTP) simulation — TEST INFRASTRUCTURE ONLY.

This is the paper's 'Matrix' method (Sec. II-A): for each gate the full
2^n x 2^n operation matrix U = I^(k-1) (x) G (x) I^(n-k) is formed with
Kronecker products and multiplied into the state (MVM). It is O(4^n) per gate,
so it is used only for n <= 10, to pin the per-gate oracle.

Ordering: the paper's qubit k (1-based) is the k-th Kronecker factor from the
left, i.e. the most significant index bit; this code's qubit q is bit q, so
paper qubit k is q = n - k and a 1-qubit gate on q is
I^(n-1-q) (x) G (x) I^q.

Two independent embeddings of a 2-qubit gate are provided: a Kronecker product
conjugated by a bit-permutation matrix, and the element-wise definition
U[r, c] = G[l(r), l(c)] when r and c agree outside {q0, q1}.
"""
from __future__ import annotations

from functools import reduce
from typing import Optional, Sequence

import numpy as np

from . import gates as G

I2 = np.eye(2, dtype=np.complex128)


def kron_all(factors):
    return reduce(np.kron, factors)


def embed_1q(n: int, q: int, g: np.ndarray) -> np.ndarray:
    """I^(n-1-q) (x) G (x) I^q."""
    return kron_all([I2] * (n - 1 - q) + [g] + [I2] * q)


def bit_permutation_matrix(n: int, dest: Sequence[int]) -> np.ndarray:
    """Permutation matrix Pm with Pm[sigma(i), i] = 1, where sigma moves bit b of
    i to bit dest[b]."""
    N = 1 << n
    Pm = np.zeros((N, N), dtype=np.complex128)
    for i in range(N):
        j = 0
        for b in range(n):
            if (i >> b) & 1:
                j |= 1 << dest[b]
        Pm[j, i] = 1.0
    return Pm


def embed_2q_kron(n: int, q0: int, q1: int, g: np.ndarray) -> np.ndarray:
    """G (x) I^(n-2) acts on bits (n-1, n-2) as (high, low); relabel those bits to
    (q0, q1) and the remaining bits, in order, to the remaining positions."""
    K = kron_all([g] + [I2] * (n - 2)) if n > 2 else g.copy()
    rest = [b for b in range(n) if b not in (q0, q1)]
    dest = [0] * n
    for src, d in zip(range(n - 2), rest):
        dest[src] = d
    dest[n - 1] = q0
    dest[n - 2] = q1
    Pm = bit_permutation_matrix(n, dest)
    return Pm @ K @ Pm.T


def embed_3q_kron(n: int, q0: int, q1: int, q2: int, g: np.ndarray) -> np.ndarray:
    """G (x) I^(n-3) acts on bits (n-1, n-2, n-3) as (high, mid, low); relabel
    those bits to (q0, q1, q2) and the remaining bits, in order, to the rest."""
    K = kron_all([g] + [I2] * (n - 3)) if n > 3 else g.copy()
    rest = [b for b in range(n) if b not in (q0, q1, q2)]
    dest = [0] * n
    for src, d in zip(range(n - 3), rest):
        dest[src] = d
    dest[n - 1], dest[n - 2], dest[n - 3] = q0, q1, q2
    Pm = bit_permutation_matrix(n, dest)
    return Pm @ K @ Pm.T


def embed_2q_def(n: int, q0: int, q1: int, g: np.ndarray) -> np.ndarray:
    """Element-wise definition of the embedded 2-qubit operator."""
    N = 1 << n
    r = np.arange(N)[:, None]
    c = np.arange(N)[None, :]
    mask = (1 << q0) | (1 << q1)
    same = ((r & ~mask) == (c & ~mask))
    lr = (((r >> q0) & 1) << 1) | ((r >> q1) & 1)
    lc = (((c >> q0) & 1) << 1) | ((c >> q1) & 1)
    U = np.where(same, g[lr, lc], 0.0).astype(np.complex128)
    return U


def mtp_operator(n: int, gate, params: Optional[np.ndarray] = None) -> np.ndarray:
    """The full 2^n x 2^n operation matrix of one gate."""
    if gate.name == "MARK":
        d = np.ones(1 << n, dtype=np.complex128)
        d[gate.index] = -1.0
        return np.diag(d)
    if gate.name in ("U1", "U2"):
        g = G.params_matrix(gate.name, params, gate.param)
    elif gate.name in G.MULTI_ANGLE:
        k = G.MULTI_ANGLE[gate.name]
        g = G.angles_matrix(gate.name, params[gate.param: gate.param + k])
    else:
        ang = float(params[gate.param]) if gate.param >= 0 else gate.angle
        g = G.matrix(gate.name, ang)
    if G.arity(gate.name) == 1:
        return embed_1q(n, gate.q0, g)
    if G.arity(gate.name) == 3:
        return embed_3q_kron(n, gate.q0, gate.q1, gate.q2, g)
    return embed_2q_kron(n, gate.q0, gate.q1, g)


def simulate_kron(n: int, gates: Sequence, params: Optional[np.ndarray] = None,
                  psi0: Optional[np.ndarray] = None) -> np.ndarray:
    """psi <- U_g psi for every gate, each U_g formed in full (n <= 10)."""
    if n > 10:
        raise ValueError("brute-force MTP is limited to n <= 10")
    psi = np.zeros(1 << n, dtype=np.complex128)
    if psi0 is None:
        psi[0] = 1.0
    else:
        psi[:] = psi0
    for g in gates:
        psi = mtp_operator(n, g, params) @ psi
    return psi


def circuit_operator(n: int, gates: Sequence, params: Optional[np.ndarray] = None) -> np.ndarray:
    """The product U_m ... U_1 of a whole circuit (n <= 8)."""
    U = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        U = mtp_operator(n, g, params) @ U
    return U
