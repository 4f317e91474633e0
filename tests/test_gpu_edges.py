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


def test_failure_paths_are_reported_and_leave_handles_usable():
    """Error paths forced from the host: an allocator that refuses gives
    TN_ENOMEM and the context, MPO and MPS stay usable once it allows again;
    a matvec cap of 1 is reported as unconverged steps, never silently; a NaN
    in a host MPS tensor is refused when the MPS is created (TN_EINVAL)."""
    import paper_2410_18740_amd as P
    gate = {"open": True}
    ctx = P.Context(0, use_torch_allocator=True, alloc_gate=lambda nbytes: gate["open"])
    try:
        r, U = W.make_problem(6, 3, (0.4, 0.6))
        m = P.MPO(ctx, r, U, 6)
        mp = P.MPS(ctx, W.random_mps(6, 6, 8, 5))
        P.dmrg_sweep(ctx, m, mp, P.SweepOpts(chi_max=8, tol=1e-10))
        big = P.MPS(ctx, W.random_mps(6, 6, 36, 6))
        gate["open"] = False
        with pytest.raises(P.TnError) as ei:
            P.dmrg_sweep(ctx, m, big, P.SweepOpts(chi_max=36, tol=1e-10))
        assert ei.value.code == -2             # TN_ENOMEM
        gate["open"] = True
        e = P.dmrg_sweep(ctx, m, big, P.SweepOpts(chi_max=36, tol=1e-10))["energy"]
        assert np.isfinite(e)
        st = P.dmrg_sweep(ctx, m, mp, P.SweepOpts(chi_max=8, tol=1e-14, max_matvecs=1))
        assert st["unconverged_steps"] > 0
        t = W.random_mps(6, 6, 8, 7)
        t[2] = t[2].copy()
        t[2][0, 0, 0] = np.nan
        with pytest.raises(P.TnError) as ei:
            P.MPS(ctx, t)
        assert ei.value.code == -1             # TN_EINVAL
        assert np.isfinite(P.dmrg_sweep(ctx, m, mp, P.SweepOpts(chi_max=8, tol=1e-10))["energy"])
        # creation under a refusing allocator: TN_ENOMEM, nothing left half built
        gate["open"] = False
        for make in (lambda: P.MPO(ctx, r, U, 6), lambda: P.MPS(ctx, W.random_mps(6, 6, 8, 5)),
                     lambda: P.MLP(ctx, 8, 16, 3)):
            with pytest.raises(P.TnError) as ei:
                make()
            assert ei.value.code == -2
        gate["open"] = True
        assert np.isfinite(P.dmrg_sweep(ctx, P.MPO(ctx, r, U, 6), P.MPS(ctx, W.random_mps(6, 6, 8, 5)),
                                        P.SweepOpts(chi_max=8, tol=1e-10))["energy"])
    finally:
        ctx.close()


def test_checkpoint_export_and_reimport(ctx):
    """An MPS exported after sweeps and re-created from the host copy has the
    same FP64 <H>, and one further sweep from either reaches the same <H>."""
    import paper_2410_18740_amd as P
    r, U = W.make_problem(5, 8, (0.4, 0.6))
    m = P.MPO(ctx, r, U, 6)
    mp = P.MPS(ctx, W.random_mps(5, 6, 16, 3))
    o = P.SweepOpts(chi_max=16, tol=1e-12)
    for _ in range(3):
        P.dmrg_sweep(ctx, m, mp, o)
    copy = P.MPS(ctx, mp.export())
    copy.canonicalize()
    e0, _ = P.energy(ctx, m, mp)
    e1, _ = P.energy(ctx, m, copy)
    assert abs(e0 - e1) < 1e-12 * max(1.0, abs(e0))
    a = P.dmrg_sweep(ctx, m, mp, o)["energy"]
    b = P.dmrg_sweep(ctx, m, copy, o)["energy"]
    # the re-created copy is re-canonicalised (tensors move by rounding), so
    # the next sweep agrees to rounding of the converged energy
    assert abs(a - b) < 1e-12 * max(1.0, abs(a))


def test_non_finite_operators_give_enumeric_and_leave_the_mps_at_its_last_step(ctx):
    """A NaN met inside a sweep: a gate-parameterised basis with squeezing
    r = 800 on one site overflows its operators (cosh r), so the sweep's
    contractions turn non-finite.  The call returns TN_ENUMERIC, the MPS keeps
    the tensors of its last completed step (bit for bit, finite, canonical),
    and the same MPS sweeps normally again with a sound MPO."""
    import paper_2410_18740_amd as P
    r, U = W.make_problem(5, 2, (0.4, 0.6))
    good = P.MPO(ctx, r, U, 6)
    mp = P.MPS(ctx, W.random_mps(5, 6, 12, 3))
    opts = P.SweepOpts(chi_max=12, tol=1e-10)
    e0 = P.dmrg_sweep(ctx, good, mp, opts)["energy"]
    before = mp.export()
    bad = P.MPO(ctx, r, U, 6)
    params = np.zeros((5, 8))
    params[3, 2] = 800.0
    P.plbo_enable(ctx, bad, params)
    with pytest.raises(P.TnError) as ei:
        P.dmrg_sweep(ctx, bad, mp, opts)
    assert ei.value.code == -4                  # TN_ENUMERIC
    after = mp.export()
    for a, b in zip(before, after):
        assert np.all(np.isfinite(b))
        assert np.array_equal(a.view(np.float64), b.view(np.float64))
    for A in after[1:]:                         # right-canonical behind the centre at site 0
        M = A.reshape(A.shape[0], -1)
        assert np.abs(M @ M.conj().T - np.eye(A.shape[0])).max() < 1e-12
    e1 = P.dmrg_sweep(ctx, good, mp, opts)["energy"]
    assert np.isfinite(e1) and abs(e1 - e0) <= 1e-2 * abs(e0)
