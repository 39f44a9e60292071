"""DAX and DAS compressed operators, their MTP and MVM (host ablation).

The paper's whole-operator formats (Sec. III-A), written from their
description, for the host ablations of the paper (Matrix vs DAX vs DAS,
Figs. 6-7). The GPU path applies each gate in its own gate-local form and
never builds a whole-operator structure.

- DAX (Sec. III-A1): every non-zero element is an entry of (real part,
  imaginary part, index), the index being the element's position in the
  row-major flattened matrix (r * n_cols + c). 24 bytes per entry.
- DAS (Sec. III-A1): an entry holds the value and a 64-bit word whose low 63
  bits count the zeros in front of the element within its row (since the
  previous non-zero of the row, or the row start) and whose flag bit marks
  the last non-zero of the row. 24 bytes per entry.
- Matrix: the dense 2^n x 2^n complex128 operator (16 bytes per element).

MTP (Sec. III-A2): the number of non-zeros of A (x) B is nnz(A) nnz(B); each
value is the product of one entry of A and one of B; the DAX position is the
binary concatenation of the row indices and of the column indices
(row = r_A * rows_B + r_B, col = c_A * cols_B + c_B). For DAS, entries of a
result row pair each entry of A's row with each entry of B's row (A outer, B
inner) and the distance before an entry follows the three cases of the
paper's distance equation; the positions are then the end-to-end sums of the
distances. MVM (Sec. III-A2): S_next[r] += M[r][c] * S[c] over the non-zeros.

Every row of the operators handled here has at least one non-zero (they are
products of invertible gate matrices), which a DAS row needs for its flag.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

ENTRY_BYTES = 24    # real, imaginary (FP64) and a 64-bit index or distance word
DENSE_BYTES = 16    # one complex128 element of the 'Matrix' structure


@dataclass
class DAX:
    rows: int
    cols: int
    val: np.ndarray    # complex128 [nnz]
    idx: np.ndarray    # int64 [nnz]: r * cols + c

    @property
    def nnz(self) -> int:
        return int(self.val.size)

    def nbytes(self) -> int:
        return ENTRY_BYTES * self.nnz


@dataclass
class DAS:
    rows: int
    cols: int
    val: np.ndarray    # complex128 [nnz], row by row, columns ascending
    dis: np.ndarray    # int64 [nnz]: zeros in front of the element within its row
    last: np.ndarray   # bool [nnz]: the last non-zero of its row

    @property
    def nnz(self) -> int:
        return int(self.val.size)

    def nbytes(self) -> int:
        return ENTRY_BYTES * self.nnz


# ------------------------------------------------------------------ encoders

def dax_encode(mat: np.ndarray) -> DAX:
    """Non-zero elements of a matrix with their flattened row-major index."""
    m = np.asarray(mat, dtype=np.complex128)
    flat = m.reshape(-1)
    idx = np.flatnonzero(flat).astype(np.int64)
    return DAX(m.shape[0], m.shape[1], flat[idx].copy(), idx)


def das_encode(mat: np.ndarray) -> DAS:
    """Row by row: each non-zero with the zeros in front of it in its row and
    a flag on the row's last non-zero."""
    m = np.asarray(mat, dtype=np.complex128)
    vals, dis, last = [], [], []
    for r in range(m.shape[0]):
        cols = np.flatnonzero(m[r])
        if cols.size == 0:
            raise ValueError("a DAS row needs a non-zero element")
        prev = -1
        for k, c in enumerate(cols):
            vals.append(m[r, c])
            dis.append(c - prev - 1)
            last.append(k == cols.size - 1)
            prev = c
    return DAS(m.shape[0], m.shape[1], np.array(vals, dtype=np.complex128),
               np.array(dis, dtype=np.int64), np.array(last, dtype=bool))


# ------------------------------------------------------- positions, decoding

def dax_positions(d: DAX):
    """(row, col) of every DAX entry: the index split by the column count."""
    return d.idx // d.cols, d.idx % d.cols


def das_positions(d: DAS):
    """(row, col) of every DAS entry: rows advance after each flagged entry;
    within a row the column is the end-to-end sum of (distance + 1), minus 1."""
    row = np.concatenate([[0], np.cumsum(d.last)[:-1]]).astype(np.int64)
    step = d.dis + 1
    csum = np.cumsum(step)
    # subtract the running sum at the start of each entry's row
    row_start = np.concatenate([[True], d.last[:-1]])
    base = np.where(row_start, csum - step, 0)
    base = np.maximum.accumulate(base)
    col = csum - base - 1
    return row, col


def to_dense(d) -> np.ndarray:
    r, c = dax_positions(d) if isinstance(d, DAX) else das_positions(d)
    m = np.zeros((d.rows, d.cols), dtype=np.complex128)
    m[r, c] = d.val
    return m


# ---------------------------------------------------------------------- MTP

def matrix_mtp(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """The 'Matrix' method: the dense Kronecker product."""
    return np.kron(a, b)


def dax_mtp(a: DAX, b: DAX) -> DAX:
    """A (x) B in DAX: every pair of entries, value a * b, row and column the
    concatenations (r_a r_b), (c_a c_b); entries kept in row-major order."""
    ra, ca = dax_positions(a)
    rb, cb = dax_positions(b)
    rows = (ra[:, None] * b.rows + rb[None, :]).reshape(-1)
    cols = (ca[:, None] * b.cols + cb[None, :]).reshape(-1)
    val = (a.val[:, None] * b.val[None, :]).reshape(-1)
    idx = rows * (a.cols * b.cols) + cols
    order = np.argsort(idx, kind="stable")
    return DAX(a.rows * b.rows, a.cols * b.cols, val[order], idx[order])


def _das_rows(d: DAS):
    """Row of each entry and its rank within the row (0 = first non-zero)."""
    row = np.concatenate([[0], np.cumsum(d.last)[:-1]]).astype(np.int64)
    first = np.concatenate([[True], d.last[:-1]])
    start = np.flatnonzero(first)
    rank = np.arange(d.nnz) - start[row]
    return row, rank


def das_mtp(a: DAS, b: DAS) -> DAS:
    """A (x) B in DAS. Result row (r_a, r_b) holds, for each entry A_i of row
    r_a in order and each entry B_j of row r_b in order, the value A_i B_j;
    the zeros in front of it within that row are
        A_i.dis * cols_B + B_j.dis               if A_i, B_j both first in their rows,
        A_i.dis * cols_B + B_j.dis + B_last_dis  if B_j is first, A_i is not,
        B_j.dis                                  otherwise,
    with B_last_dis the zeros behind the last non-zero of row r_b; the entry is
    the last of its row when A_i and B_j both are."""
    ra, ia = _das_rows(a)
    rb, jb = _das_rows(b)
    # zeros behind the last non-zero of each B row: cols - 1 - its column
    _, cb = das_positions(b)
    b_tail = np.zeros(b.rows, dtype=np.int64)
    b_tail[rb[b.last]] = b.cols - 1 - cb[b.last]
    A_first = (ia == 0)[:, None]
    B_first = (jb == 0)[None, :]
    dis = np.where(A_first & B_first, a.dis[:, None] * b.cols + b.dis[None, :],
                   np.where(B_first, a.dis[:, None] * b.cols + b.dis[None, :] + b_tail[rb][None, :],
                            np.broadcast_to(b.dis[None, :], (a.nnz, b.nnz))))
    last = a.last[:, None] & b.last[None, :]
    val = a.val[:, None] * b.val[None, :]
    # order: result row (r_a, r_b), then A_i, then B_j
    rrow = ra[:, None] * b.rows + rb[None, :]
    keys = (np.broadcast_to(jb[None, :], rrow.shape).reshape(-1),
            np.broadcast_to(ia[:, None], rrow.shape).reshape(-1), rrow.reshape(-1))
    order = np.lexsort(keys)
    return DAS(a.rows * b.rows, a.cols * b.cols, val.reshape(-1)[order], dis.reshape(-1)[order],
               last.reshape(-1)[order])


def mtp_chain(kind: str, gate: np.ndarray, m: int):
    """The MTP of m identical gates, G (x) G (x) ... (x) G, in one structure:
    'matrix' (dense), 'dax' or 'das'."""
    if kind == "matrix":
        out = np.asarray(gate, dtype=np.complex128)
        for _ in range(m - 1):
            out = matrix_mtp(out, gate)
        return out
    enc, mtp = (dax_encode, dax_mtp) if kind == "dax" else (das_encode, das_mtp)
    g = enc(gate)
    out = g
    for _ in range(m - 1):
        out = mtp(out, g)
    return out


# ---------------------------------------------------------------------- MVM

def matrix_mvm(m: np.ndarray, s: np.ndarray) -> np.ndarray:
    return m @ s


def dax_mvm(d: DAX, s: np.ndarray) -> np.ndarray:
    """S_next[r] += M[r][c] * S[c] for every DAX entry (index parsed into r, c)."""
    r, c = dax_positions(d)
    out = np.zeros(d.rows, dtype=np.complex128)
    np.add.at(out, r, d.val * s[c])
    return out


def das_mvm(d: DAS, s: np.ndarray) -> np.ndarray:
    """The same product with positions decoded from the distances."""
    r, c = das_positions(d)
    out = np.zeros(d.rows, dtype=np.complex128)
    np.add.at(out, r, d.val * s[c])
    return out


# ---------------------------------------------------- Table 1 / Theorem 1

def zero_ratio(mat: np.ndarray) -> float:
    m = np.asarray(mat)
    return 1.0 - np.count_nonzero(m) / m.size


def memory_improvement(n_qubits: int, nnz: int) -> float:
    """Bytes of the dense 2^n x 2^n operator over bytes of its DAX (or DAS)."""
    return DENSE_BYTES * float(4 ** n_qubits) / (ENTRY_BYTES * nnz)
