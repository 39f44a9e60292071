"""Writes the stored expected values of tests/golden that are not printed in
the paper. It calls only the oracle (and the seeded generators and the digest
helper of tests/, neither of which holds simulation arithmetic).

    python tests/golden/make_golden.py            # grover_n20.txt
    python tests/golden/make_golden.py random28   # random_n28_d100_s0.npz (minutes)
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def grover():
    n, k = 20, 804
    a, b, p = O.grover_closed_form(n, k)
    with open(os.path.join(HERE, "grover_n20.txt"), "w") as f:
        f.write("# Grover search at n = 20 after k = floor(pi/4 sqrt(2^20)) = 804 iterations\n")
        f.write("# of D*O from H^n|0>, D = 2|s><s| - I (textbook closed form, FP64):\n")
        f.write("# marked = sin((2k+1) theta), unmarked = cos((2k+1) theta)/sqrt(N-1),\n")
        f.write("# theta = asin(2^(-n/2)). Written by make_golden.py from oracle/ only.\n")
        f.write(f"iterations {k}\n")
        f.write(f"marked {a!r}\n")
        f.write(f"unmarked {b!r}\n")
        f.write(f"p_success {p!r}\n")


RANDOM28 = dict(n=28, depth=100, seed=0, sample_seed=2028, samples=16384)


def random28():
    """The plain method at scale: the seeded n = 28, depth-100 random circuit
    from |0...0>, simulated gate by gate by the oracle (Sec. II-A). Stores
    16,384 seeded sampled amplitudes, the whole-state digest (every amplitude
    enters one of 4,096 block sums), the norm and <Z_q> of every qubit."""
    from state_digest import digest
    c = RANDOM28
    n = c["n"]
    gates = synth.random_circuit(n, c["depth"], c["seed"])
    t0 = time.time()
    psi = O.simulate(n, gates)
    print(f"oracle: {len(gates)} gates on 2^{n} amplitudes in {time.time() - t0:.1f} s", flush=True)
    idx = np.random.default_rng(c["sample_seed"]).integers(0, 1 << n, size=c["samples"])
    np.savez(os.path.join(HERE, "random_n28_d100_s0.npz"),
             n=n, depth=c["depth"], seed=c["seed"], gates=len(gates),
             idx=idx.astype(np.int64), amp=psi[idx], digest=digest(psi),
             norm=O.norm2(psi), z=np.array([O.expect_z(psi, q) for q in range(n)]))


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "random28":
        random28()
    else:
        grover()
