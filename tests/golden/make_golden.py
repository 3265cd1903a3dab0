"""Writes the stored expected values under tests/golden/ from the oracle only.

psi_coefficients.txt: the monomial coefficients Gamma_d (leading first) of
psi_d, the degree-d polynomial interpolating f_d(t) = max(0, t)^(10 d) at the
d + 1 Chebyshev points of the second kind (Sec. 5, eq. def:fN, eq. chebfun-f),
for d = 1 .. 15, as the oracle computes them.

Run from the repository root: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import arrabit as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    lines = ["# Gamma_d of psi_d (Sec. 5, eq. def:fN, eq. chebfun-f), leading coefficient first.",
             "# Written by tests/golden/make_golden.py from the oracle (oracle/arrabit.py).",
             "# d gamma_1 ... gamma_{d+1}"]
    for d in range(1, 16):
        g = O.interpolant_coefficients(d)
        lines.append(" ".join([str(d)] + [repr(float(x)) for x in g]))
    with open(os.path.join(HERE, "psi_coefficients.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
