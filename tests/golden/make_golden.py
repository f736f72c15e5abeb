"""Writes tests/golden/plain_oracle_sample.txt: oracle solutions (hex floats)
of sampled columns of the plain workload (N=256, sigma=0.1, 256 right-hand
sides uniform[-1, 1), seed 1).  Calls only the oracle and the seeded input
generator.  Run: python tests/golden/make_golden.py"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1807_07382_amd import inputs  # noqa: E402

COLUMNS = (0, 1, 63, 64, 127, 200, 255)
ROWS = (0, 1, 2, 127, 253, 254, 255)


def main():
    w = inputs.plain()
    dg = oracle.assemble_d4(w["n"], w["sigma"])
    X = oracle.solve(dg, w["F"])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plain_oracle_sample.txt")
    with open(out, "w") as fh:
        fh.write("# oracle x[row, col] for the plain workload (N=256, sigma=0.1, seed 1);\n")
        fh.write("# written by tests/golden/make_golden.py from oracle/ only\n")
        fh.write("# row col x(hex)\n")
        for j in COLUMNS:
            for i in ROWS:
                fh.write(f"{i} {j} {float(X[i, j]).hex()}\n")


if __name__ == "__main__":
    main()
