"""RH (regularity-oriented Hadamard) routines of the paper — TEST INFRASTRUCTURE ONLY.

Sec. III-B: H^(x)n is stored as the single magnitude 1/sqrt(N) (N = 2^n) and the
sign of each element is derived from its (row, column) index on demand. These
functions follow the paper's procedures step by step, in pure Python, for small
n only; they are an independent route to H^(x)n |psi> used to pin the oracle and
the GPU path's Hadamard handling.

- ``compute_sign``: the quadrant recursion of Sec. III-B2 (Fig. 3): split the
  matrix into four quadrants, only the lower-right one carries a minus sign,
  descend into the quadrant holding (r, c) until 1x1, and multiply the signs.
- ``rh_mvm_non_optimized``: prescale S by 1/sqrt(N), then one signed dot
  product per row, every sign computed (Table 2: 2^n * 2^n signs).
- ``rh_mvm_quarter``: Method 1, signs of the upper-left quarter only.
- ``rh_mvm_block``: Method 2 with block size b (Theorem 3's optimum is
  b = sqrt(2^(n-1))).
- ``rh_mvm_logarithm``: Method 3 (the sign rule behind Algorithm 1): in a
  quarter row only the signs at the n - 1 powers of two are computed; the
  sign at any other c is the product of the signs at the powers of two that
  make up c, so the row's whole sign table is built by doubling over those
  bits. The quarter then yields both halves of the result, since
  H^n = [[H', H'], [H', -H']] with H' = H^(n-1).

Reading of a garbled step: in Algorithm 1 the exponent p of the doubling rule is
undefined in the printed text; it is read so that a sign is the product of the
sign at the highest power of two not above c and the sign at the remainder,
which is the product over c's bits used here.

Each function also returns the number of compute_sign calls it made, so the
counts of Table 2 (and the n = 5 examples of Methods 1-3) can be checked.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np


def compute_sign(r: int, c: int, n: int) -> int:
    """Sign of H^(x)n[r][c] by quadrant recursion (rows/cols of size 2^n)."""
    sign = 1
    size = 1 << n
    while size > 1:
        half = size >> 1
        lower = r >= half
        right = c >= half
        if lower and right:
            sign = -sign
        if lower:
            r -= half
        if right:
            c -= half
        size = half
    return sign


def rh_mvm_non_optimized(S: np.ndarray) -> Tuple[np.ndarray, int]:
    N = S.size
    n = N.bit_length() - 1
    Sp = S * (1.0 / math.sqrt(N))
    out = np.zeros(N, dtype=np.complex128)
    count = 0
    for r in range(N):
        acc = 0j
        for c in range(N):
            acc += compute_sign(r, c, n) * Sp[c]
            count += 1
        out[r] = acc
    return out, count


def _quarter_updates(out, Sp, r, c, s, h):
    out[r] += s * Sp[c]
    out[r] += s * Sp[c + h]
    out[r + h] += s * Sp[c]
    out[r + h] += -s * Sp[c + h]


def rh_mvm_quarter(S: np.ndarray) -> Tuple[np.ndarray, int]:
    N = S.size
    n = N.bit_length() - 1
    if n == 0:
        return S.astype(np.complex128).copy(), 0
    h = N // 2
    Sp = S * (1.0 / math.sqrt(N))
    out = np.zeros(N, dtype=np.complex128)
    count = 0
    for r in range(h):
        for c in range(h):
            s = compute_sign(r, c, n)
            count += 1
            _quarter_updates(out, Sp, r, c, s, h)
    return out, count


def rh_mvm_block(S: np.ndarray, b: int) -> Tuple[np.ndarray, int]:
    N = S.size
    n = N.bit_length() - 1
    if n == 0:
        return S.astype(np.complex128).copy(), 0
    h = N // 2
    if b < 1 or h % b != 0 or not (b & (b - 1)) == 0:
        raise ValueError("block size must be a power of two dividing 2^(n-1)")
    Sp = S * (1.0 / math.sqrt(N))
    out = np.zeros(N, dtype=np.complex128)
    count = 0
    for r in range(h):
        first = [0] * b
        for c in range(b):
            first[c] = compute_sign(r, c, n)
            count += 1
        for blk in range(h // b):
            lead = first[0] if blk == 0 else compute_sign(r, blk * b, n)
            if blk > 0:
                count += 1
            for c in range(b):
                s = first[c] if blk == 0 else lead * first[c]
                _quarter_updates(out, Sp, r, blk * b + c, s, h)
    return out, count


def rh_mvm_logarithm(S: np.ndarray) -> Tuple[np.ndarray, int]:
    """Method 3 (logarithm-based signs) of Sec. III-B2: n - 1 computed signs
    per quarter row, the rest by products over the bits of the column."""
    N = S.size
    n = N.bit_length() - 1
    if n == 0:
        return S.astype(np.complex128).copy(), 0
    h = N // 2
    Sp = S * (1.0 / math.sqrt(N))          # the RH magnitude, applied once
    left, right = Sp[:h], Sp[h:]
    top = np.empty(h, dtype=np.complex128)
    bottom = np.empty(h, dtype=np.complex128)
    count = 0
    for r in range(h):
        table = np.ones(1)                 # signs of columns 0 .. 2^k - 1 of row r
        for k in range(n - 1):
            s = compute_sign(r, 1 << k, n)
            count += 1
            table = np.concatenate([table, s * table])
        top[r] = table @ (left + right)    # [H' H'] row r
        bottom[r] = table @ (left - right)  # [H' -H'] row r
    return np.concatenate([top, bottom]), count


def sign_count_formula(method: str, n: int, b: int = 1) -> int:
    """Table 2: number of sign computations of each method."""
    if method == "non-optimized":
        return (1 << n) * (1 << n)
    if method == "quarter":
        return (1 << (n - 1)) * (1 << (n - 1))
    if method == "block":
        return (1 << (n - 1)) * ((1 << (n - 1)) // b + b - 1)
    if method == "logarithm":
        return (1 << (n - 1)) * (n - 1)
    raise ValueError(method)
