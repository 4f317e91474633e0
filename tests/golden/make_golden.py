"""Regenerates the oracle-written golden files (calls only oracle/ and workloads/)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import gbs, dense  # noqa: E402


def main():
    r, U = W.workload_problem("gbs_n4_d6_chi16")
    al, be, ga = gbs.coefficients(r, U)
    lines = []
    for D in (3, 4, 5, 6):
        H = dense.php_quadrature(al, be, ga, D)
        ev, _ = dense.ground_states(H, 1)
        lines.append(f"{D} {ev[0]:.11f}")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
