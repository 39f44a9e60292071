"""Writes the stored expected values of tests/golden that are not printed in
the paper. It calls only the oracle (the textbook Grover closed form)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
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


if __name__ == "__main__":
    main()
