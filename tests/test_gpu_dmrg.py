"""End-to-end GPU DMRG parity with the oracle on the 4-mode workload
(r = 0.5, Haar U from seed 0, cutoff 6, chi 16, 6 sweeps, tolerance 1e-12),
plus exact diagonalisation, probabilities and marginals."""
import numpy as np
import pytest

import workloads as W
from oracle import gbs, dense, dmrg as odmrg, mps as omps
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
    ref, st = odmrg.dmrg(m0, Ws, 16, 6, tol=1e-12)
    al, be, ga = gbs.coefficients(r, U)
    H = dense.php_quadrature(al, be, ga, 6)
    ev, vec = dense.ground_states(H, 1)
    return dict(w=w, r=r, U=U, Ws=Ws, m0=m0, ref=ref, st=st, E_ed=ev[0], gs=vec[:, 0])


def _run(ctx, cfg, chi, sweeps, prec_schedule, tol=1e-12):
    import paper_2410_18740_amd as P
    m = P.MPO(ctx, cfg["r"], cfg["U"], 6)
    mp = P.MPS(ctx, cfg["m0"] if chi == 16 else W.random_mps(4, 6, chi, 1000))
    stats = []
    for sw in range(sweeps):
        prec = prec_schedule(sw)
        stats.append(P.dmrg_sweep(ctx, m, mp, P.SweepOpts(chi_max=chi, tol=tol if prec == 0 else 1e-7,
                                                          precision=prec)))
    return m, mp, stats


def test_dmrg_fp64_matches_oracle(ctx, four_mode):
    m, mp, stats = _run(ctx, four_mode, 16, 6, lambda s: 0)
    E = stats[-1]["energy"]
    print("GPU E", E, "oracle E", four_mode["st"][-1]["energy"], "ED", four_mode["E_ed"])
    assert abs(E - four_mode["st"][-1]["energy"]) < 1e-10
    assert E >= four_mode["E_ed"] - 1e-12
    assert stats[-1]["unconverged_steps"] == 0
    t = mp.export()
    P_gpu = omps.probabilities(t)
    P_ref = omps.probabilities(four_mode["ref"])
    print(f"fp64: |E - E_oracle| = {abs(E - four_mode['st'][-1]['energy']):.3e}, "
          f"max |dP(n)| = {np.abs(P_gpu - P_ref).max():.3e}")
    assert np.abs(P_gpu - P_ref).max() < 1e-8
    assert abs(stats[-1]["max_discarded"] - four_mode["st"][-1]["max_discarded"]) < 1e-10


def test_dmrg_full_rank_matches_ed(ctx, four_mode):
    m, mp, stats = _run(ctx, four_mode, 36, 3, lambda s: 0)
    P_gpu = omps.probabilities(mp.export())
    print(f"full rank: |E - E_ED| = {abs(stats[-1]['energy'] - four_mode['E_ed']):.3e}, "
          f"max |dP(n)| = {np.abs(P_gpu - np.abs(four_mode['gs']) ** 2).max():.3e}")
    assert abs(stats[-1]["energy"] - four_mode["E_ed"]) < 1e-10
    assert np.abs(P_gpu - np.abs(four_mode["gs"]) ** 2).max() < 1e-8


@pytest.mark.parametrize("prec", [1, 2])
def test_fast_form_then_fp64_refine(ctx, four_mode, prec):
    """Bulk sweeps in FP32 / BF16x3, then FP64 refinement sweeps reach the FP64
    result to 1e-10."""
    m, mp, stats = _run(ctx, four_mode, 16, 6, lambda s: prec if s < 3 else 0)
    print(f"form {prec} + FP64 refine: |E - E_oracle| = "
          f"{abs(stats[-1]['energy'] - four_mode['st'][-1]['energy']):.3e}")
    assert abs(stats[-1]["energy"] - four_mode["st"][-1]["energy"]) < 1e-10


def test_marginals_match_oracle(ctx, four_mode):
    import paper_2410_18740_amd as P
    m, mp, stats = _run(ctx, four_mode, 16, 6, lambda s: 0)
    marg = P.marginals(ctx, mp, m)
    ref = omps.marginals(mp.export())
    ref2 = omps.marginals(four_mode["ref"])
    print(f"marginals: max |d| = {np.abs(marg - ref).max():.3e} (same state), "
          f"{np.abs(marg - ref2).max():.3e} (oracle's DMRG state)")
    assert np.abs(marg - ref).max() < 1e-12
    assert np.abs(marg - ref2).max() < 1e-8


def test_energy_entry_point_matches_sweep(ctx, four_mode):
    import paper_2410_18740_amd as P
    m, mp, stats = _run(ctx, four_mode, 16, 2, lambda s: 0)
    e, n = P.energy(ctx, m, mp)
    assert abs(e - stats[-1]["energy"]) < 1e-13
    assert abs(n - 1.0) < 1e-12
    assert abs(e - odmrg.energy(mp.export(), four_mode["Ws"])) < 1e-12


def test_sampler_matches_oracle_stream(ctx, four_mode):
    import paper_2410_18740_amd as P
    from oracle import sampler
    m, mp, stats = _run(ctx, four_mode, 16, 4, lambda s: 0)
    t = mp.export()
    smp = P.sample(ctx, mp, m, 400, 2004).cpu().numpy()
    ref, tie = sampler.sample(t, 400, 2004, with_ties=True)
    bad, nties = sampler.stream_mismatches(smp, ref, tie)
    print(f"sampler: {bad} of 400 samples differ from the oracle's stream outside rounding ties "
          f"({nties} samples hold a tie)")
    assert bad == 0


def test_sweep_reports_truncation_flops(ctx):
    """The sweep's svd_flops is the sum over its 2(N-1) truncations of the
    dense stages' implementation flops for the shapes the sweep visits
    (6 modes, d 6, chi 48: Gram sizes 6 to 216, both eigensolver routes)."""
    import paper_2410_18740_amd as P
    N, d, chi = 6, 6, 48
    U = W.haar_unitary(N, np.random.default_rng(3))
    r = np.full(N, 0.5)
    mpo = P.MPO(ctx, r, U, d)
    mps = P.MPS(ctx, W.random_mps(N, d, chi, 7))
    st = P.dmrg_sweep(ctx, mpo, mps, P.SweepOpts(chi_max=chi, precision=P.FP64, tol=1e-8, max_matvecs=8))
    dims = W.bond_dims(N, d, chi)

    def flops(p, q, k):
        f = 8.0 * p * p * q + 8.0 * k * p * q
        if p > 32:
            f += 24.0 * (p - 1) * p * (2 * p - 1) / 6.0 + 8.0 * k * p * (p - 1)
        return f

    # the left-to-right half takes the Gram matrix on the left side (p = m),
    # the right-to-left half on the right side (p = n)
    want = 0.0
    for s in range(N - 1):
        m, n = dims[s] * d, d * dims[s + 2]
        k = max(1, min(chi, m, n))
        want += flops(m, n, k) + flops(n, m, k)
    print(f"svd_flops {st['svd_flops']:.6e} want {want:.6e}")
    assert abs(st["svd_flops"] - want) <= 1e-12 * want
    assert st["t_svd"] > 0.0
