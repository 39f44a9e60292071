"""Host ablations of the paper's formats (CPU, FP64): Matrix vs DAX vs DAS for
the MTP of m identical gates and the MVM with a state (the shape of Figs. 6-7),
and the RH sign methods against the dense Hadamard product (the shape of
Fig. 8 and the sign counts of Table 2). Not a test: run
    python tests/f3_ablation.py [--quick]
It prints markdown tables of seconds (best of a few runs) and counts."""
import argparse
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), ".."))

from ablation import compressed as C  # noqa: E402
from oracle import gates as G  # noqa: E402
from oracle import rh as RH  # noqa: E402

GATES = [("H", 1), ("X", 1), ("Y", 1), ("SWAP", 2), ("CNOT", 2), ("CCX", 3)]
MATRIX_MAX_N = 12    # 4^12 x 16 B = 256 MiB dense operator
COMPRESSED_MAX_NNZ = 1 << 24


def best_of(fn, reps):
    best, out = float("inf"), None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        best = min(best, time.perf_counter() - t0)
    return best, out


def fmt(t):
    return "—" if t is None else (f"{t * 1e3:.2f} ms" if t < 1 else f"{t:.2f} s")


def mtp_mvm_table(ns):
    rng = np.random.default_rng(0)
    print("| gate | n | Matrix MTP | DAX MTP | DAS MTP | Matrix MVM | DAX MVM | DAS MVM | nnz |")
    print("|---|---|---|---|---|---|---|---|---|")
    for name, k in GATES:
        g = G.matrix(name)
        nnz1 = np.count_nonzero(g)
        for n in ns:
            if n % k:
                continue
            m = n // k
            nnz = nnz1 ** m
            s = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
            reps = 3 if n <= 12 else 1
            row = {}
            if n <= MATRIX_MAX_N:
                row["mm"], M = best_of(lambda: C.mtp_chain("matrix", g, m), reps)
                row["mv"], _ = best_of(lambda: C.matrix_mvm(M, s), reps)
                del M
            if nnz <= COMPRESSED_MAX_NNZ:
                row["dm"], D = best_of(lambda: C.mtp_chain("dax", g, m), reps)
                row["dv"], _ = best_of(lambda: C.dax_mvm(D, s), reps)
                del D
                row["sm"], S = best_of(lambda: C.mtp_chain("das", g, m), reps)
                row["sv"], _ = best_of(lambda: C.das_mvm(S, s), reps)
                del S
            print(f"| {name} | {n} | {fmt(row.get('mm'))} | {fmt(row.get('dm'))} | {fmt(row.get('sm'))} | "
                  f"{fmt(row.get('mv'))} | {fmt(row.get('dv'))} | {fmt(row.get('sv'))} | {nnz} |", flush=True)


def rh_table(ns):
    rng = np.random.default_rng(1)
    print()
    print("| n | Matrix (dense H^n S) | RH non-optimized | RH quarter | RH block (b = sqrt(2^(n-1))) | RH logarithm | signs: non-opt / quarter / block / log |")
    print("|---|---|---|---|---|---|---|")
    for n in ns:
        S = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        Hn = np.array([[1.0]])
        for _ in range(n):
            Hn = np.kron(Hn, G.matrix("H").real)
        tm, _ = best_of(lambda: Hn @ S, 3)
        b = max(1, int(round((2 ** (n - 1)) ** 0.5)))
        b = 1 << (b.bit_length() - 1)   # a power of two dividing the half size
        tn, (_, cn) = best_of(lambda: RH.rh_mvm_non_optimized(S), 1)
        tq, (_, cq) = best_of(lambda: RH.rh_mvm_quarter(S), 1)
        tb, (_, cb) = best_of(lambda: RH.rh_mvm_block(S, b), 1)
        tl, (_, cl) = best_of(lambda: RH.rh_mvm_logarithm(S), 1)
        print(f"| {n} | {fmt(tm)} | {fmt(tn)} | {fmt(tq)} | {fmt(tb)} | {fmt(tl)} | {cn} / {cq} / {cb} / {cl} |",
              flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="small sizes only")
    a = ap.parse_args()
    mtp_mvm_table([6, 12] if a.quick else [6, 12, 18, 24])
    rh_table([4, 6] if a.quick else [4, 6, 8, 10])


if __name__ == "__main__":
    main()
