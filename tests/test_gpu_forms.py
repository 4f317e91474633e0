"""The arithmetic forms on the 16-mode workload (cutoff 12, chi = 64, r ~ U[0.5,
1.0], Haar U from seed 1) against the FP64 oracle's own DMRG run of the same
seeded state (tests/golden/cfg1_oracle.txt, written by
tests/golden/make_cfg1.py, which calls only oracle/ and workloads/):
  * plain FP64: four sweeps with the oracle's Lanczos tolerance;
  * FP32 (3M MFMA) and BF16x3 bulk sweeps followed by FP64 refinement.
At chi = 64 each two-site step discards about 2e-3 of the weight, and in the
first sweep from the random start ten of the oracle's local solves stop
unconverged at its 200-matvec cap.  Such results depend on each side's Krylov
details, so the two runs leave sweep 0 about 5e-5 apart and settle in nearby
truncated minima (this is the regime where DMRG parity is unpinned).  The
errors against the oracle are printed for every form.  The plain FP64 run is
gated at 1e-4 relative in energy and 1e-4 in the marginals, an order above
what was observed (1.6e-5, 2.0e-5) and far below the 1e-2 scale of the
sweep-to-sweep changes; the fast forms are gated more loosely."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "cfg1_oracle.txt")


def _golden():
    energies, disc, marg = [], [], []
    for line in open(GOLD):
        if line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "sweep":
            energies.append(float(f[2]))
            disc.append(float(f[3]))
        elif f[0] == "marginal":
            marg.append([float(x) for x in f[2:]])
    return np.array(energies), np.array(disc), np.array(marg)


@pytest.fixture(scope="module")
def runs():
    import paper_2410_18740_amd as P
    ctx = P.Context(0)
    w = W.WORKLOADS["gbs_n16_d12_chi64"]
    r, U = W.workload_problem("gbs_n16_d12_chi64")
    out = {}
    for name, sched in (("fp64", [0, 0, 0, 0]), ("fp32", [1, 1, 0, 0]), ("bf16x3", [2, 2, 0, 0])):
        mpo = P.MPO(ctx, r, U, w.D_raw, w.d)
        mps = P.MPS(ctx, W.random_mps(w.N, w.d, w.chi, w.mps_seed))
        es = []
        for prec in sched:
            # the oracle's settings: tolerance 1e-10, 32 Krylov vectors, up to 200 matvecs
            st = P.dmrg_sweep(ctx, mpo, mps, P.SweepOpts(chi_max=w.chi, tol=1e-6 if prec else 1e-10,
                                                          max_matvecs=200, krylov_max=32, precision=prec))
            es.append(st["energy"])
        out[name] = (es, P.marginals(ctx, mps, mpo))
        print(name, [f"{e:.12f}" for e in es], flush=True)
    yield out
    ctx.close()


def test_plain_fp64_follows_the_oracle_run(runs):
    E, _, M = _golden()
    es, m = runs["fp64"]
    dE = np.abs(np.array(es) - E)
    dM = np.abs(m - M).max()
    print("fp64 against the oracle: |dE| per sweep " + " ".join(f"{x:.2e}" for x in dE) +
          f", max |d marginal| {dM:.2e}")
    assert dE[-1] <= 1e-4 * abs(E[-1])
    assert dM <= 1e-4


@pytest.mark.parametrize("form", ["fp32", "bf16x3"])
def test_fast_form_then_refine_against_the_oracle(runs, form):
    E, _, M = _golden()
    ef, mf = runs[form]
    e64, m64 = runs["fp64"]
    dE = abs(ef[-1] - E[-1])
    dM = np.abs(mf - M).max()
    print(f"{form} + refine against the oracle: |dE| = {dE:.3e} (E = {E[-1]:.8f}), max |d marginal| = {dM:.3e}; "
          f"against the GPU FP64 run: |dE| = {abs(ef[-1] - e64[-1]):.3e}")
    assert np.isfinite(ef).all()
    assert dE <= 1e-3 * abs(E[-1])
    assert dM <= 1e-2
