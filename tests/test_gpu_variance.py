"""GPU parity of the energy variance sigma_H^2 = <(PHP)^2> - <PHP>^2 (Sec.
II.E.2) with the oracle's two-layer contraction, with and without a local
basis, plus its two limits: a DMRG state converged at full Schmidt rank is an
eigenstate (sigma_H ~ 0), and a truncated bond leaves sigma_H > 0."""
import numpy as np
import pytest

import workloads as W
from oracle import gbs, lbo, mpo as ompo, dmrg as odmrg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2410_18740_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _raw_cores(r, U, D):
    al, be, ga, raw = lbo.local_ops(r, U, D)
    return ompo.cores(al, be, ga, raw)


@pytest.mark.parametrize("N,D,chi,seed", [(6, 4, 8, 1), (7, 5, 20, 2), (9, 3, 27, 3)])
def test_variance_matches_oracle_fock_basis(ctx, N, D, chi, seed):
    """Random (non-canonical) MPS in the Fock basis; bonds span several GEMM
    tiles at chi = 20, 27 with ragged edges."""
    import paper_2410_18740_amd as P
    r, U = W.make_problem(N, seed, (0.3, 0.8))
    t = W.random_mps(N, D, chi, seed + 40)
    mpo, mps = P.MPO(ctx, r, U, D), P.MPS(ctx, t)
    e, h2, var = P.energy_variance(ctx, mpo, mps)
    eo, h2o, varo = odmrg.energy_variance(t, _raw_cores(r, U, D))
    print(f"N={N} D={D} chi={chi}: <H> {e:.12f} / {eo:.12f}, <H^2> {h2:.12f} / {h2o:.12f}, var {var:.6e}")
    assert abs(e - eo) < 1e-10 * max(1.0, abs(eo))
    assert abs(h2 - h2o) < 1e-10 * max(1.0, abs(h2o))
    assert abs(var - varo) < 1e-9 * max(1.0, abs(h2o))


def test_variance_with_local_basis_matches_oracle(ctx):
    """After joint LBO + DMRG sweeps (D_raw 6 -> d 3) the physical state is
    W A in the raw box; (PHP)^2 is taken there, which differs from the square
    of the projected operator."""
    import paper_2410_18740_amd as P
    N, D, d, chi = 5, 6, 3, 9
    r, U = W.make_problem(N, 9, (0.4, 0.7))
    mpo, mps = P.MPO(ctx, r, U, D, d), P.MPS(ctx, W.random_mps(N, d, chi, 21))
    opts = P.SweepOpts(chi_max=chi, tol=1e-10, max_matvecs=200, lbo=1)
    for _ in range(2):
        P.dmrg_sweep(ctx, mpo, mps, opts)
    t, iso = mps.export(), list(mpo.isometries())
    e, h2, var = P.energy_variance(ctx, mpo, mps)
    eo, h2o, varo = odmrg.energy_variance(t, _raw_cores(r, U, D), iso)
    # the square of the projected operator gives a smaller <H^2>
    al, be, ga, raw = lbo.local_ops(r, U, D)
    _, h2p, _ = odmrg.energy_variance(t, lbo.cores_in_basis(al, be, ga, raw, iso))
    print(f"<H> {e:.10f} / {eo:.10f}; <H^2> raw box {h2:.10f} / {h2o:.10f}, projected {h2p:.10f}")
    assert abs(e - eo) < 1e-10 and abs(h2 - h2o) < 1e-10 * max(1.0, h2o)
    assert h2o > h2p + 1e-6


def test_variance_limits(ctx):
    """Full Schmidt rank (chi = D^(N/2)) converged by DMRG: an eigenstate of PHP,
    sigma_H^2 ~ 0.  The same instance at chi = 4: sigma_H^2 clearly > 0."""
    import paper_2410_18740_amd as P
    N, D = 4, 4
    r, U = W.make_problem(N, 5, (0.4, 0.6))
    out = {}
    for chi in (16, 4):
        mpo, mps = P.MPO(ctx, r, U, D), P.MPS(ctx, W.random_mps(N, D, chi, 8))
        opts = P.SweepOpts(chi_max=chi, tol=1e-12, max_matvecs=400)
        for _ in range(6):
            P.dmrg_sweep(ctx, mpo, mps, opts)
        out[chi] = P.energy_variance(ctx, mpo, mps)
        print(f"chi {chi}: <H> {out[chi][0]:.10e}, sigma^2 {out[chi][2]:.3e}")
    assert abs(out[16][2]) < 1e-9
    assert out[4][2] > 1e-6
