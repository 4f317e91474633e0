"""Writes tests/golden/cfg1_oracle.txt: the FP64 oracle's two-site DMRG on the
16-mode workload (Haar U from seed 1, r ~ U[0.5, 1.0], cutoff 12, chi 64, the
seeded random-normal initial MPS, Lanczos tolerance 1e-10, 4 sweeps): the
energy and largest discarded weight after each sweep and the photon-number
marginals of all modes at the end.  Calls only oracle/ and workloads/."""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import gbs, operators, mpo as omp, dmrg as odmrg, mps as omps  # noqa: E402

NAME = "gbs_n16_d12_chi64"
SWEEPS = 4
TOL = 1e-10
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg1_oracle.txt")


def main():
    w = W.WORKLOADS[NAME]
    r, U = W.workload_problem(NAME)
    al, be, ga = gbs.coefficients(r, U)
    ops = [operators.local_operators(w.D_raw, al[s, s], be[s, s], ga[s, s]) for s in range(w.N)]
    Ws = omp.cores(al, be, ga, ops)
    m0 = W.random_mps(w.N, w.d, w.chi, w.mps_seed)
    t0 = time.time()

    def cb(st):
        print(f"sweep {st['sweep']}: E = {st['energy']:.15e}, max disc {st['max_discarded']:.3e}, "
              f"matvecs {st['matvecs']}, unconverged {st['unconverged']}, {time.time() - t0:.0f} s", flush=True)

    mps, stats = odmrg.dmrg(m0, Ws, w.chi, SWEEPS, tol=TOL, krylov_max=32, max_iter=200, callback=cb)
    marg = omps.marginals(mps)
    with open(OUT, "w") as f:
        f.write(f"# FP64 oracle two-site DMRG, {NAME}: N={w.N} D={w.D_raw} chi={w.chi} seed={w.seed} "
                f"mps_seed={w.mps_seed} tol={TOL} sweeps={SWEEPS} (written by make_cfg1.py)\n")
        for st in stats:
            f.write(f"sweep {st['sweep']} {st['energy']:.17e} {st['max_discarded']:.17e} {st['matvecs']}\n")
        for j in range(w.N):
            f.write("marginal " + str(j) + " " + " ".join(f"{x:.17e}" for x in marg[j]) + "\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
