"""Pins of the DAX / DAS structures (host ablation infrastructure) against the
paper's worked example, Theorem 1, Table 1 and dense Kronecker products."""
import math

import numpy as np
import pytest

from ablation import compressed as C
from oracle import gates as G

PX = G.matrix("X")
PY = G.matrix("Y")


def test_paper_yx_dax_example():
    """Sec. III-A1: Y (x) X has its non-zeros at indices 3, 6, 9, 12; the DAX
    needs 4 * 24 B = 96 B against 16 * 16 B = 256 B (2.7x)."""
    d = C.dax_mtp(C.dax_encode(PY), C.dax_encode(PX))
    assert d.idx.tolist() == [3, 6, 9, 12]
    assert np.array_equal(d.val, np.array([-1j, -1j, 1j, 1j]))
    assert d.nbytes() == 96 and C.DENSE_BYTES * 16 == 256
    assert round(256 / 96, 1) == 2.7
    assert np.array_equal(C.to_dense(d), np.kron(PY, PX))


def test_paper_das_example():
    """Sec. III-A2: in Y's first row, -i has one zero in front and none behind
    and is the row's last non-zero. Y (x) X in DAS: one entry per row with
    3, 2, 1, 0 zeros in front."""
    y = C.das_encode(PY)
    assert y.dis.tolist() == [1, 0] and y.last.tolist() == [True, True]
    d = C.das_mtp(y, C.das_encode(PX))
    assert d.dis.tolist() == [3, 2, 1, 0] and d.last.all()
    assert np.array_equal(d.val, np.array([-1j, -1j, 1j, 1j]))
    assert np.array_equal(C.to_dense(d), np.kron(PY, PX))


def _random_sparse(rows, cols, density, rng):
    m = np.where(rng.random((rows, cols)) < density,
                 rng.normal(size=(rows, cols)) + 1j * rng.normal(size=(rows, cols)), 0)
    for r in range(rows):   # every row keeps a non-zero (DAS rows need one)
        if not m[r].any():
            m[r, rng.integers(cols)] = 1.0 + 0.5j
    return m


@pytest.mark.parametrize("seed", range(6))
def test_mtp_and_mvm_match_dense(seed):
    """Both structures' MTP equals the dense Kronecker product (rows with 1..n
    non-zeros exercise all three DAS distance cases) and their MVM equals the
    dense product."""
    rng = np.random.default_rng(seed)
    shapes = [(2, 2), (4, 4), (2, 4), (8, 8), (4, 2)]
    a = _random_sparse(*shapes[seed % 5], 0.5, rng)
    b = _random_sparse(*shapes[(seed + 2) % 5], 0.4, rng)
    ref = np.kron(a, b)
    for enc, mtp, mvm in ((C.dax_encode, C.dax_mtp, C.dax_mvm), (C.das_encode, C.das_mtp, C.das_mvm)):
        d = mtp(enc(a), enc(b))
        assert d.nnz == np.count_nonzero(a) * np.count_nonzero(b)
        assert np.array_equal(C.to_dense(d), ref)
        s = rng.normal(size=ref.shape[1]) + 1j * rng.normal(size=ref.shape[1])
        assert np.allclose(mvm(d, s), ref @ s, atol=1e-12)


def test_theorem1_zero_ratio():
    """R(A (x) B) = R(A) + (1 - R(A)) R(B)."""
    rng = np.random.default_rng(9)
    for _ in range(5):
        a = _random_sparse(4, 4, rng.uniform(0.2, 0.8), rng)
        b = _random_sparse(8, 8, rng.uniform(0.2, 0.8), rng)
        d = C.dax_mtp(C.dax_encode(a), C.dax_encode(b))
        r = 1.0 - d.nnz / (32 * 32)
        ra, rb = C.zero_ratio(a), C.zero_ratio(b)
        assert math.isclose(r, ra + (1 - ra) * rb, abs_tol=1e-12)


# Table 1 categories: (gate, arity, sparsity(n), memory improvement(n)) for the
# MTP of n / arity identical gates.
TABLE1 = [
    ("X", 1, lambda n: 1 - 2.0 ** -n, lambda n: 2 / 3 * 2.0 ** n),
    ("CNOT", 2, lambda n: 1 - 2.0 ** -n, lambda n: 2 / 3 * 2.0 ** n),
    ("RXX", 2, lambda n: 1 - 2.0 ** (-n / 2), lambda n: 2 / 3 * 2.0 ** (n / 2)),
    ("CH", 2, lambda n: 1 - (3 / 8) ** (n / 2), lambda n: 2 / 3 * (8 / 3) ** (n / 2)),
    ("CCX", 3, lambda n: 1 - 2.0 ** -n, lambda n: 2 / 3 * 2.0 ** n),
]


@pytest.mark.parametrize("name,k,spars,mem", TABLE1)
@pytest.mark.parametrize("kind", ["dax", "das"])
def test_table1_sparsity_and_memory(name, k, spars, mem, kind):
    g = G.matrix(name, 0.9)
    for m in (1, 2, 3, 4):
        n = k * m
        if n > 12:
            continue
        d = C.mtp_chain(kind, g, m)
        assert math.isclose(1 - d.nnz / 4.0 ** n, spars(n), rel_tol=1e-12)
        assert math.isclose(C.memory_improvement(n, d.nnz), mem(n), rel_tol=1e-12)


def test_hadamard_gains_nothing():
    """Table 1: the Hadamard is dense, so DAX and DAS store more than the
    dense operator (24 B against 16 B per element)."""
    d = C.mtp_chain("dax", G.matrix("H"), 6)
    assert d.nnz == 4 ** 6
    assert C.memory_improvement(6, d.nnz) == pytest.approx(2 / 3)
