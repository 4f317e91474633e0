"""The arithmetic forms on the 16-mode workload (cutoff 12, chi = 64, r ~ U[0.5,
1.0], Haar U from seed 1): FP32 (3M MFMA) and BF16x3 bulk sweeps followed by
FP64 refinement, against the plain FP64 run from the same seeded state.  The
oracle cannot sweep this size in test time; the FP64 path is pinned to it on
smaller workloads, and here the fast forms' energy and marginal differences
from it are reported, with a loose gate (a fast form may settle in a nearby
truncated minimum)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


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
            st = P.dmrg_sweep(ctx, mpo, mps, P.SweepOpts(chi_max=w.chi, tol=1e-6 if prec else 1e-9,
                                                          max_matvecs=40, krylov_max=24, precision=prec))
            es.append(st["energy"])
        out[name] = (es, P.marginals(ctx, mps, mpo))
        print(name, [f"{e:.10f}" for e in es], flush=True)
    yield out
    ctx.close()


@pytest.mark.parametrize("form", ["fp32", "bf16x3"])
def test_fast_form_then_refine_tracks_fp64(runs, form):
    e64, m64 = runs["fp64"]
    ef, mf = runs[form]
    dE = abs(ef[-1] - e64[-1])
    dM = np.abs(mf - m64).max()
    print(f"{form}: |dE| = {dE:.3e} (E = {e64[-1]:.8f}), max |d marginal| = {dM:.3e}")
    assert np.isfinite(ef).all()
    assert dE <= 1e-3 * max(1.0, abs(e64[-1]))
    assert dM <= 1e-2
