"""GPU tests of the precision schedule (tn_dmrg_solve: FP32 / BF16x3 bulk
sweeps, automatic switch, FP64 refinement), of checkpoint and resume
(tn_mps_checkpoint, tn_mps_import), of bitwise determinism, and of the
context's lifetime rules at the C ABI."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from oracle import dmrg as odmrg
from tests.gpu_helpers import problem, oracle_cores

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2410_18740_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def four_mode():
    w, r, U = problem("gbs_n4_d6_chi16")
    Ws = oracle_cores(r, U, 6)
    m0 = W.random_mps(4, 6, 16, w.mps_seed)
    ref, st = odmrg.dmrg(m0, Ws, 16, 8, tol=1e-12)
    return dict(w=w, r=r, U=U, m0=m0, E=st[-1]["energy"])


@pytest.mark.parametrize("bulk", [1, 2])
def test_solve_switches_to_fp64_refinement_and_reaches_the_oracle(ctx, four_mode, bulk):
    """tn_dmrg_solve on the 4-mode workload: fast bulk sweeps, the automatic
    switch once the bulk energy stagnates, FP64 refinement sweeps, and the
    result within 1e-10 of the oracle's FP64 DMRG energy.  A second run with
    the target set to the oracle energy + 1e-10 reaches it at a finite time."""
    import paper_2410_18740_amd as P
    opts = P.SweepOpts(chi_max=16, krylov_max=32, max_matvecs=200)
    kw = dict(max_sweeps=20, bulk_precision=bulk, max_refine=2, switch_tol=1e-6, conv_tol=1e-13,
              bulk_tol=1e-6, refine_tol=1e-12, lbo_bulk=0, lbo_refine=0)
    m = P.MPO(ctx, four_mode["r"], four_mode["U"], 6)
    mp = P.MPS(ctx, four_mode["m0"])
    res = P.dmrg_solve(ctx, m, mp, opts, target=-1.0, **kw)
    print(f"solve form {bulk}: sweeps {res['sweeps']}, refine {res['refine_sweeps']}, "
          f"|E - E_oracle| = {abs(res['energy'] - four_mode['E']):.3e}")
    assert 1 <= res["refine_sweeps"] <= 2
    assert res["sweeps"] > res["refine_sweeps"]
    assert res["reached"] == 0
    assert abs(res["energy"] - four_mode["E"]) < 1e-10
    assert mp.sweeps == res["sweeps"]
    mp2 = P.MPS(ctx, four_mode["m0"])
    res2 = P.dmrg_solve(ctx, m, mp2, opts, target=four_mode["E"] + 1e-10, **kw)
    print(f"  to target: sweeps {res2['sweeps']}, refine {res2['refine_sweeps']}, t_target {res2['t_target']:.3f} s")
    assert res2["reached"] == 1
    assert np.isfinite(res2["t_target"]) and 0 < res2["t_target"] <= res2["seconds"]
    assert res2["energy"] <= four_mode["E"] + 1e-10


def test_solve_without_refinement_stops_at_the_switch(ctx, four_mode):
    """max_refine = 0: the schedule stops when the bulk energy stagnates and
    runs no FP64 sweep."""
    import paper_2410_18740_amd as P
    m = P.MPO(ctx, four_mode["r"], four_mode["U"], 6)
    mp = P.MPS(ctx, four_mode["m0"])
    res = P.dmrg_solve(ctx, m, mp, P.SweepOpts(chi_max=16, max_matvecs=200), max_sweeps=20, bulk_precision=1,
                       max_refine=0, target=-1.0, switch_tol=1e-6, bulk_tol=1e-6, lbo_bulk=0)
    assert res["refine_sweeps"] == 0 and res["reached"] == 0
    assert res["sweeps"] < 20


def test_plain_fp64_solve_matches_the_oracle(ctx, four_mode):
    import paper_2410_18740_amd as P
    m = P.MPO(ctx, four_mode["r"], four_mode["U"], 6)
    mp = P.MPS(ctx, four_mode["m0"])
    res = P.dmrg_solve(ctx, m, mp, P.SweepOpts(chi_max=16, max_matvecs=200), max_sweeps=12, bulk_precision=0,
                       target=-1.0, conv_tol=1e-13, bulk_tol=1e-12, lbo_bulk=0)
    assert res["refine_sweeps"] == 0
    assert abs(res["energy"] - four_mode["E"]) < 1e-10


def _sweeps(ctx, m, mp, n, lbo):
    import paper_2410_18740_amd as P
    o = P.SweepOpts(chi_max=16, tol=1e-12, lbo=lbo)
    return [P.dmrg_sweep(ctx, m, mp, o)["energy"] for _ in range(n)]


@pytest.mark.parametrize("lbo", [0, 1])
def test_checkpoint_resume_continues_the_run(ctx, lbo):
    """A checkpoint after three sweeps (tensors, centre, sweep counter and the
    MPO's isometries) imported into a fresh MPS and MPO, and one more sweep on
    each: the resumed energy equals the continued one to 1e-12, the tensors
    agree, and the sweep counter carries over."""
    import paper_2410_18740_amd as P
    N, D, d = 5, 8, (5 if lbo else 8)
    r, U = W.make_problem(N, 8, (0.4, 0.6))
    m = P.MPO(ctx, r, U, D, d)
    mp = P.MPS(ctx, W.random_mps(N, d, 16, 3))
    _sweeps(ctx, m, mp, 3, lbo)
    buf = mp.checkpoint(m)
    assert int(buf[5]) == 3 and mp.sweeps == 3
    mp2, iso = P.MPS.from_checkpoint(ctx, buf)
    assert mp2.sweeps == 3 and iso.shape == (N, D, d)
    assert np.abs(iso - m.isometries()).max() == 0.0
    m2 = P.MPO(ctx, r, U, D, d, iso=iso)
    e_a = _sweeps(ctx, m, mp, 1, lbo)[0]
    e_b = _sweeps(ctx, m2, mp2, 1, lbo)[0]
    print(f"resume (lbo={lbo}): |dE| = {abs(e_a - e_b):.3e}")
    assert abs(e_a - e_b) < 1e-12
    ta, tb = mp.export(), mp2.export()
    assert max(np.abs(a - b).max() for a, b in zip(ta, tb)) < 1e-10
    assert mp2.sweeps == 4


def test_import_rejects_damaged_checkpoints(ctx):
    import paper_2410_18740_amd as P
    r, U = W.make_problem(4, 1, (0.5, 0.5))
    m = P.MPO(ctx, r, U, 4)
    mp = P.MPS(ctx, W.random_mps(4, 4, 8, 1))
    buf = mp.checkpoint(m)
    for i, v in ((0, 1.0), (1, 2.0), (2, 5.0), (4, 7.0), (6, 3.0)):
        bad = buf.copy()
        bad[i] = v
        with pytest.raises(P.TnError) as ei:
            P.MPS.from_checkpoint(ctx, bad)
        assert ei.value.code == -1
    with pytest.raises(P.TnError):
        P.MPS.from_checkpoint(ctx, buf[:-2])
    bad = buf.copy()
    bad[-1] = np.nan
    with pytest.raises(P.TnError):
        P.MPS.from_checkpoint(ctx, bad)
    # no MPO: no isometries
    mp3, iso = P.MPS.from_checkpoint(ctx, mp.checkpoint())
    assert iso is None and mp3.N == 4


@pytest.mark.parametrize("prec", [0, 1])
def test_identical_runs_are_bitwise_identical(ctx, prec):
    """The same inputs and options twice give bit-identical tensors and
    energies (no atomics or order-dependent reductions on the path)."""
    import paper_2410_18740_amd as P
    r, U = W.make_problem(6, 4, (0.5, 0.8))
    outs = []
    for _ in range(2):
        m = P.MPO(ctx, r, U, 8, 5)
        mp = P.MPS(ctx, W.random_mps(6, 5, 24, 5))
        o = P.SweepOpts(chi_max=24, tol=1e-10, precision=prec, lbo=1, max_matvecs=30)
        es = [P.dmrg_sweep(ctx, m, mp, o)["energy"] for _ in range(2)]
        outs.append((es, mp.export(), m.isometries()))
    assert outs[0][0] == outs[1][0]
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a.view(np.float64), b.view(np.float64))
    assert np.array_equal(outs[0][2].view(np.float64), outs[1][2].view(np.float64))


def test_handles_may_outlive_their_context_at_the_abi():
    """Raw C ABI: destroy the context first, then its MPO and MPS (the
    context's host object lives until the last handle is gone); a call on
    the closed context returns TN_ESTATE, and destroying a closed context
    again is a no-op."""
    import torch
    from paper_2410_18740_amd import _lib as L
    lib = L.lib()
    torch.cuda.init()
    ctx = C.c_void_p()
    assert lib.tn_ctx_create(0, None, None, C.byref(ctx)) == 0
    r, U = W.make_problem(3, 2, (0.4, 0.4))
    rr = np.ascontiguousarray(r)
    UU = np.ascontiguousarray(U).view(np.float64).copy()
    prob = L.tn_problem(3, 4, 4, L.dptr(rr), L.dptr(UU), None, 0.0)
    mpo = C.c_void_p()
    assert lib.tn_mpo_build(ctx, C.byref(prob), C.byref(mpo)) == 0
    t = W.random_mps(3, 4, 4, 2)
    flat = np.concatenate([x.reshape(-1) for x in t]).view(np.float64).copy()
    dims = np.array([1] + [x.shape[2] for x in t], dtype=np.int32)
    mps = C.c_void_p()
    assert lib.tn_mps_create(ctx, 3, 4, L.dptr(dims, C.c_int32), L.dptr(flat), C.byref(mps)) == 0
    e = C.c_double()
    assert lib.tn_energy(ctx, mpo, mps, C.byref(e), None) == 0
    lib.tn_ctx_destroy(ctx)
    assert lib.tn_energy(ctx, mpo, mps, C.byref(e), None) == L.TN_ESTATE
    iso = np.zeros(2 * 3 * 4 * 4)
    assert lib.tn_mpo_isometries(mpo, L.dptr(iso)) == L.TN_ESTATE
    lib.tn_ctx_destroy(ctx)
    lib.tn_mpo_destroy(mpo)
    lib.tn_mps_destroy(mps)          # the last reference: the context goes here


def test_profiling_counts_every_matvec_of_a_sweep(ctx, four_mode):
    """The matvec profiling (HIP events per launch, kept in a ring of slots that
    are read back when a slot comes round again or at read-out): after a sweep
    with profiling on, the read-out covers every matvec of the sweep, with
    finite non-negative phase times; stopping it resets the counters."""
    import paper_2410_18740_amd as P
    mpo = P.MPO(ctx, four_mode["r"], four_mode["U"], 6)
    mps = P.MPS(ctx, four_mode["m0"])
    ctx.profile(1)
    st = P.dmrg_sweep(ctx, mpo, mps, P.SweepOpts(chi_max=16, precision=P.FP32, tol=1e-10, max_matvecs=16))
    pr = ctx.profile(-1)
    ctx.profile(0)
    print(f"sweep matvecs {st['matvecs']}, profiled {pr['matvecs']}, GEMM ms {pr['ms_gemm_l'] + pr['ms_gemm_r']:.3f}")
    assert st["matvecs"] > 8  # more matvecs than ring slots: slots were reused
    assert pr["matvecs"] == st["matvecs"]
    assert pr["lanczos_iters"] == st["matvecs"]
    for k in ("ms_convert", "ms_gemm_l", "ms_ops", "ms_gemm_r", "ms_reduce"):
        assert np.isfinite(pr[k]) and pr[k] >= 0.0
    assert pr["ms_gemm_l"] > 0.0 and pr["ms_gemm_r"] > 0.0 and pr["flops_matvec"] > 0.0
    z = ctx.profile(-1)
    assert z["matvecs"] == 0 and z["ms_gemm_l"] == 0.0
