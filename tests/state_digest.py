"""Whole-state digests for parity checks of states too large to store.

TEST INFRASTRUCTURE. A digest of a state psi (complex, length 2^n) is, for
each block of 2^16 consecutive amplitudes, the two weighted sums
    S1_b = sum_i w1(i) psi_i,   S2_b = sum_i w2(i) psi_i,
with real weights in [-1/2, 1/2) from integer hashes of the index i
(multiplicative hashing modulo 2^32, exact in integer arithmetic). Every
amplitude enters one block with two unrelated weights, so any amplitude that
differs by more than the tolerance, a sign error or two amplitudes exchanged
changes a block sum. The same function digests the oracle's state (stored by
tests/golden/make_golden.py) and the device state read back in a test.
"""
from __future__ import annotations

import numpy as np

BLOCK_BITS = 16
_M1, _A1 = np.uint64(0x9E3779B1), np.uint64(0)
_M2, _A2 = np.uint64(0x85EBCA77), np.uint64(0x165667B1)
_MASK = np.uint64(0xFFFFFFFF)


def weights(lo: int, hi: int):
    i = np.arange(lo, hi, dtype=np.uint64)
    w1 = ((i * _M1 + _A1) & _MASK).astype(np.float64) * 2.0 ** -32 - 0.5
    w2 = ((i * _M2 + _A2) & _MASK).astype(np.float64) * 2.0 ** -32 - 0.5
    return w1, w2


def digest(psi: np.ndarray, chunk_bits: int = 22) -> np.ndarray:
    """[blocks, 2] complex128: the sums S1_b and S2_b of every block."""
    N = psi.size
    bb = min(BLOCK_BITS, int(N).bit_length() - 1)
    nb = N >> bb
    out = np.empty((nb, 2), dtype=np.complex128)
    step = max(1 << chunk_bits, 1 << bb)
    for lo in range(0, N, step):
        hi = min(N, lo + step)
        w1, w2 = weights(lo, hi)
        x = np.asarray(psi[lo:hi], dtype=np.complex128).reshape(-1, 1 << bb)
        b0 = lo >> bb
        out[b0: b0 + x.shape[0], 0] = (x * w1.reshape(x.shape)).sum(axis=1)
        out[b0: b0 + x.shape[0], 1] = (x * w2.reshape(x.shape)).sum(axis=1)
    return out
