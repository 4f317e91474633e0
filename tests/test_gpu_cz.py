"""GPU parity of the global-CZ (non-Gaussian) parent Hamiltonian (Sec. II.C.2)
with the oracle: MPO structure bit-exact, local operators, two-site matvec and
environment updates through the X^2 and XP + PX legs, <H> and sigma_H^2, DMRG
at full Schmidt rank against exact diagonalisation, and joint LBO sweeps."""
import numpy as np
import pytest

import workloads as W
from oracle import cz, mpo as ompo, dmrg as odmrg, operators
from tests.gpu_helpers import rand_env, to_dev, from_dev

pytestmark = pytest.mark.gpu

KAPPA = 0.3


@pytest.fixture(scope="module")
def ctx():
    import paper_2410_18740_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _case(N, D, seed, kappa=KAPPA, iso=None):
    r, U = W.make_problem(N, seed, (0.3, 0.7))
    al, be, ga, ops = cz.site_operators(r, U, D)
    if iso is not None:
        ops = [tuple(operators.project(o, W_) for o in o5) for o5, W_ in zip(ops, iso)]
    return r, U, cz.cores(al, be, ga, kappa, ops)


@pytest.mark.parametrize("N", [2, 3, 5, 8, 16])
def test_cz_structure_bit_exact(ctx, N):
    import paper_2410_18740_amd as P
    r, U = W.make_problem(N, 1, (0.3, 0.7))
    w, kinds = P.MPO(ctx, r, U, 4, kappa=KAPPA).structure()
    w_ref, kinds_ref = cz.structure(N)
    assert list(w) == list(w_ref)
    for s in range(N):
        assert np.array_equal(kinds[s], kinds_ref[s]), s


def test_cz_site_operators(ctx):
    import paper_2410_18740_amd as P
    r, U = W.make_problem(4, 2, (0.3, 0.7))
    m = P.MPO(ctx, r, U, 6, kappa=KAPPA)
    al, be, ga, ops = cz.site_operators(r, U, 6)
    for s in range(4):
        assert np.abs(m.site_ops(s) - np.stack(ops[s])).max() < 1e-12


@pytest.mark.parametrize("N,D,site,cl,cr", [(4, 4, 1, 4, 4), (6, 3, 2, 9, 9), (7, 3, 3, 20, 13)])
def test_cz_heff_and_envs(ctx, N, D, site, cl, cr):
    import paper_2410_18740_amd as P
    rng = np.random.default_rng(N + site)
    r, U, Ws = _case(N, D, N + 10)
    m = P.MPO(ctx, r, U, D, kappa=KAPPA)
    Le = rand_env(Ws[site].shape[0], cl, rng)
    Re = rand_env(Ws[site + 1].shape[1], cr, rng)
    th = rng.standard_normal((cl, D, D, cr)) + 1j * rng.standard_normal((cl, D, D, cr))
    ref = odmrg.heff_matvec(Le, Ws[site], Ws[site + 1], Re, th)
    for prec, tol in ((P.FP64, 1e-13), (P.FP32, 3e-6)):
        out = from_dev(P.heff_apply(ctx, m, site, to_dev(Le), to_dev(Re), to_dev(th), prec))
        err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
        print(f"cz heff N={N} site={site} prec={prec} err={err:.3e}")
        assert err < tol
    A = rng.standard_normal((cl, D, cr)) + 1j * rng.standard_normal((cl, D, cr))
    ref = odmrg.env_left_update(Le, A, Ws[site])
    out = from_dev(P.env_update(ctx, m, site, +1, to_dev(Le), to_dev(A), P.FP64))
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-13
    Rin = rand_env(Ws[site].shape[1], cr, rng)
    ref = odmrg.env_right_update(Rin, A, Ws[site])
    out = from_dev(P.env_update(ctx, m, site, -1, to_dev(Rin), to_dev(A), P.FP64))
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-13


def test_cz_energy_and_variance(ctx):
    import paper_2410_18740_amd as P
    N, D, chi = 6, 4, 10
    r, U, Ws = _case(N, D, 3)
    t = W.random_mps(N, D, chi, 4)
    m, mps = P.MPO(ctx, r, U, D, kappa=KAPPA), P.MPS(ctx, t)
    e, n2 = P.energy(ctx, m, mps)
    assert abs(e - odmrg.energy(t, Ws)) < 1e-10 * max(1.0, abs(e))
    e2, h2, var = P.energy_variance(ctx, m, mps)
    eo, h2o, varo = odmrg.energy_variance(t, Ws)
    print(f"cz <H> {e:.12f} / {eo:.12f}; <H^2> {h2:.10f} / {h2o:.10f}")
    assert abs(h2 - h2o) < 1e-10 * max(1.0, h2o) and abs(var - varo) < 1e-9 * max(1.0, h2o)


def test_cz_dmrg_full_rank_matches_exact_diagonalisation(ctx):
    """Three modes, cutoff 4, full Schmidt rank: FP64 DMRG reaches the lowest
    eigenvalue of the dense PHP; kappa = 0 and kappa = 0.3 differ."""
    import paper_2410_18740_amd as P
    N, D = 3, 4
    r, U = W.make_problem(N, 5, (0.3, 0.6))
    al, be, ga, _ = cz.site_operators(r, U, D)
    out = {}
    for kappa in (0.0, KAPPA):
        e0 = np.linalg.eigvalsh(cz.dense_php(al, be, ga, kappa, D))[0]
        m, mps = P.MPO(ctx, r, U, D, kappa=kappa), P.MPS(ctx, W.random_mps(N, D, 16, 6))
        opts = P.SweepOpts(chi_max=16, tol=1e-12, max_matvecs=400, precision=P.FP64)
        for _ in range(6):
            st = P.dmrg_sweep(ctx, m, mps, opts)
        out[kappa] = (st["energy"], e0)
        print(f"kappa {kappa}: DMRG {st['energy']:.12e}, ED {e0:.12e}")
        assert abs(st["energy"] - e0) < 1e-10
    assert abs(out[0.0][1] - out[KAPPA][1]) > 1e-4


def test_cz_joint_lbo_sweeps_consistent(ctx):
    """Joint LBO + DMRG sweeps with the CZ terms (D_raw 6 -> d 3): the energy the
    sweep reports equals the oracle's <H> of the exported state in the raw box
    (physical state W A, CZ cores with raw operators), and it decreases."""
    import paper_2410_18740_amd as P
    N, D, d, chi = 5, 6, 3, 9
    r, U, Wraw = _case(N, D, 9)
    m, mps = P.MPO(ctx, r, U, D, d, kappa=KAPPA), P.MPS(ctx, W.random_mps(N, d, chi, 21))
    opts = P.SweepOpts(chi_max=chi, tol=1e-10, max_matvecs=200, lbo=1, precision=P.FP64)
    es = [P.dmrg_sweep(ctx, m, mps, opts)["energy"] for _ in range(3)]
    t, iso = mps.export(), list(m.isometries())
    phys = [np.einsum("im,amb->aib", W_, A) for W_, A in zip(iso, t)]
    e_ref = odmrg.energy(phys, Wraw)
    print(f"cz LBO sweeps {es}, oracle {e_ref:.12f}")
    assert abs(es[-1] - e_ref) < 1e-9 * max(1.0, abs(e_ref))
    assert es[-1] <= es[0] + 1e-12
