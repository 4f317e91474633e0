"""Degenerate cases and error paths of the C ABI on the GPU: the vacuum
(r = 0, where PHP is the number operator and <H> = 0 is exact), the shortest
chain (N = 2, where one two-site step is an exact diagonalisation of PHP),
and rejected arguments (mismatched handles, empty or out-of-range sizes, a
state that is not canonical, an eigensolver size beyond the LDS limit)."""
import numpy as np
import pytest

import workloads as W
from oracle import gbs, dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2410_18740_amd as P
    c = P.Context(0)
    yield c
    c.close()


def test_vacuum_energy_is_zero(ctx):
    import paper_2410_18740_amd as P
    N, D = 5, 4
    r, U = W.make_problem(N, 3, (0.0, 0.0))
    m = P.MPO(ctx, r, U, D)
    mp = P.MPS(ctx, W.random_mps(N, D, 3, 9))
    for _ in range(2):
        st = P.dmrg_sweep(ctx, m, mp, P.SweepOpts(chi_max=3, tol=1e-12, max_matvecs=100))
    assert abs(st["energy"]) < 1e-12
    e, n2 = P.energy(ctx, m, mp)
    assert abs(e) < 1e-12


@pytest.mark.parametrize("D", [3, 6])
def test_two_mode_chain_is_exact(ctx, D):
    import paper_2410_18740_amd as P
    r, U = W.make_problem(2, 11, (0.4, 0.9))
    al, be, ga = gbs.coefficients(r, U)
    ev, _ = dense.ground_states(dense.php_quadrature(al, be, ga, D), 1)
    m = P.MPO(ctx, r, U, D)
    mp = P.MPS(ctx, W.random_mps(2, D, D, 5))
    st = P.dmrg_sweep(ctx, m, mp, P.SweepOpts(chi_max=D, tol=1e-12, max_matvecs=400))
    assert abs(st["energy"] - ev[0]) < 1e-10


def test_abi_rejects_bad_arguments(ctx):
    import torch
    import paper_2410_18740_amd as P
    r, U = W.make_problem(4, 0, (0.5, 0.5))
    m4 = P.MPO(ctx, r, U, 4)
    r5, U5 = W.make_problem(5, 0, (0.5, 0.5))
    m5 = P.MPO(ctx, r5, U5, 4)
    mp = P.MPS(ctx, W.random_mps(4, 4, 4, 1))
    ok = P.SweepOpts(chi_max=4, tol=1e-10)
    with pytest.raises(P.TnError):                      # MPO and MPS of different length
        P.dmrg_sweep(ctx, m5, mp, ok)
    for bad in (P.SweepOpts(chi_max=0), P.SweepOpts(tol=0.0), P.SweepOpts(krylov_max=1),
                P.SweepOpts(precision=7), P.SweepOpts(sigma_cut=1.0), P.SweepOpts(lbo_matvecs=-1)):
        with pytest.raises(P.TnError):
            P.dmrg_sweep(ctx, m4, mp, bad)
    with pytest.raises(P.TnError):                      # not canonical yet: no centre
        P.sample(ctx, mp, m4, 10, 1)
    P.dmrg_sweep(ctx, m4, mp, ok)                       # a valid sweep leaves the centre at site 0
    with pytest.raises(P.TnError):
        P.sample(ctx, mp, m4, 0, 1)
    with pytest.raises(P.TnError):
        P.marginals(ctx, mp, m4, 5)
    with pytest.raises(P.TnError):
        P.marginals(ctx, mp, m4, 0)
    assert P.sample(ctx, mp, m4, 3, 1).shape == (3, 4)
    x = torch.zeros((4, 4, 4, 4), dtype=torch.complex128, device="cuda")
    e = torch.zeros((4, 4, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.TnError):                      # window (3, 4) runs past the chain
        P.heff_apply(ctx, m4, 3, e, e, x)
    a = torch.zeros((3, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.TnError):
        P.cgemm(ctx, a[:0], a)                          # empty operand
    with pytest.raises(P.TnError):                      # eigensolver size beyond the LDS-staged limit
        P.truncate(ctx, torch.ones((3300, 4), dtype=torch.complex128, device="cuda"), 2)
    # the context stays usable after every error
    assert np.isfinite(P.dmrg_sweep(ctx, m4, mp, ok)["energy"])
