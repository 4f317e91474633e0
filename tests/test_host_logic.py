"""Host-side logic of the library that issues no GPU work: the squeezed local
basis of the learned warm start against the oracle's construction."""
import numpy as np
import pytest

from oracle import mlp as omlp


@pytest.mark.parametrize("zeta,D,d", [(0.0, 8, 8), (0.3 + 0.2j, 12, 5), (0.9 * np.exp(2.5j), 24, 10),
                                      (1.4j, 40, 6), (0.2, 10, 10)])
def test_squeezed_basis_matches_oracle(zeta, D, d):
    import paper_2410_18740_amd as P
    got = P.squeezed_basis(zeta, D, d)
    ref = omlp.squeezed_basis(zeta, D, d)
    # the cut columns are far from orthogonal at large |zeta|: one or two
    # Gram-Schmidt passes differ by rounding amplified by that conditioning
    assert np.abs(got - ref).max() < 1e-9
    assert np.abs(got.conj().T @ got - np.eye(d)).max() < 1e-12


def test_squeezed_basis_rejects_bad_arguments():
    import paper_2410_18740_amd as P
    for args in [(0.1, 4, 5), (0.1, 0, 1), (np.nan, 4, 2), (30.0, 4, 2)]:
        with pytest.raises(P.TnError):
            P.squeezed_basis(*args)


@pytest.mark.parametrize("N", [5, 20])
def test_ws_features_match_oracle(N):
    import paper_2410_18740_amd as P
    import workloads as W
    r, U = W.make_problem(N, 31 + N, (0.3, 1.2))
    got = P.ws_features(r, U)
    ref = np.stack([omlp.features(r, U, j) for j in range(N)])
    assert got.shape == (N, omlp.IN_DIM)
    assert np.abs(got - ref).max() < 1e-6


def test_ws_targets_match_oracle():
    import paper_2410_18740_amd as P
    rng = np.random.default_rng(4)
    rhos = []
    for k in range(6):
        A = rng.standard_normal((10, 10)) + 1j * rng.standard_normal((10, 10))
        A *= np.exp(-0.4 * np.arange(10))[:, None]
        rho = A @ A.conj().T
        rhos.append(rho / np.trace(rho))
    zeta, nbar = 0.35 * np.exp(1.9j), 0.2
    Wb = omlp.squeezed_basis(zeta, 48, 30)
    lam = np.array([nbar ** k / (nbar + 1) ** (k + 1) for k in range(30)])
    rhos.append(((Wb * lam) @ Wb.conj().T)[:10, :10])
    rhos = np.array(rhos)
    got = P.ws_targets(rhos)
    ref = np.stack([omlp.targets_from_moments(*omlp.moments(r_)) for r_ in rhos])
    assert np.abs(got - ref).max() < 1e-6 * max(1.0, np.abs(ref).max())


def test_ws_initial_state_matches_oracle():
    import paper_2410_18740_amd as P
    y = np.array([[0.3, -0.1, 0.4], [0.0, 0.0, 0.0], [-0.5, 0.2, 1.1], [0.1, 0.6, 0.05]], dtype=np.float32)
    D, d, chi = 12, 5, 7
    iso, A = P.ws_initial_state(y, D, d, chi, seed=3, noise=0.0)
    iso_r, amps = omlp.initial_product_state(y.astype(np.float64), D, d)
    dims = [1, 5, 7, 5, 1]
    for s in range(4):
        assert A[s].shape == (dims[s], d, dims[s + 1])
        assert np.abs(iso[s] - iso_r[s]).max() < 1e-9
        assert np.abs(A[s][0, :, 0] - amps[s]).max() < 1e-7
        rest = A[s].copy()
        rest[0, :, 0] = 0
        assert np.abs(rest).max() == 0.0
    _, An = P.ws_initial_state(y, D, d, chi, seed=3, noise=1e-3)
    _, An2 = P.ws_initial_state(y, D, d, chi, seed=3, noise=1e-3)
    noise = np.concatenate([(a - b).reshape(-1) for a, b in zip(An, A)])
    assert all(np.array_equal(a, b) for a, b in zip(An, An2))
    assert abs(np.std(noise.real) - 1e-3) < 2e-4 and abs(np.mean(noise.real)) < 2e-4


def test_ws_gaussian_params_match_oracle():
    import paper_2410_18740_amd as P
    import workloads as W
    from oracle import gbs
    for N, seed, kind, rr in ((6, 3, "haar", (0.3, 1.2)), (20, 4, "brickwork", (0.1, 0.2))):
        r, U = W.make_problem(N, seed, rr, kind=kind)
        got = P.ws_gaussian_params(r, U)
        V = gbs.covariance(r, U)
        ref = np.stack([omlp.gaussian_params(V, j) for j in range(N)])
        assert np.abs(got - ref).max() < 1e-6


def test_cutoff_report_matches_oracle():
    import paper_2410_18740_amd as P
    import workloads as W
    from oracle import gbs, cutoff
    for N, seed, kind, rr, d in ((3, 4, "haar", (0.3, 0.6), 3), (12, 9, "haar", (0.5, 1.2), 6),
                                 (16, 5, "brickwork", (0.1, 0.2), 4)):
        r, U = W.make_problem(N, seed, rr, kind=kind)
        rep = P.cutoff_report(r, U, d, D_max=200, tol=1e-10)
        tails, eps, (lo, hi) = cutoff.eps_bounds(gbs.covariance(r, U), d)
        assert np.allclose(rep["eps_mode"], tails, rtol=1e-9, atol=1e-15)
        assert abs(rep["eps"] - eps) <= 1e-9 * eps + 1e-16 and abs(rep["eps_D_bounds"][1] - hi) <= 1e-9 * hi + 1e-15
        for j in range(N):
            zeta = complex(*omlp.gaussian_params(gbs.covariance(r, U), j)[:2])
            assert rep["D_eff"][j] == cutoff.effective_cutoff(zeta, d, 200, 1e-10), (N, seed, j)


def test_cutoff_report_rejects_bad_arguments():
    import paper_2410_18740_amd as P
    r, U = np.array([0.3, 0.4]), np.eye(2, dtype=complex)
    for kw in (dict(d=0), dict(d=5, D_max=4), dict(d=2, tol=0.0), dict(d=2, D_max=5000)):
        with pytest.raises(P.TnError):
            P.cutoff_report(r, U, **kw)
    with pytest.raises(P.TnError):
        P.cutoff_report(np.array([0.3, np.nan]), U, 2)


# ------------------------------------------------------------------ gate-parameterised basis (host part)
def _plbo_params(rng):
    return rng.uniform(-1, 1, 8) * [0.4, 0.4, 0.5, 3, 3, 0.3, 0.1, 0.1]


@pytest.mark.parametrize("d", [1, 4, 9])
def test_plbo_operators_match_oracle(d):
    """The library's closed form at d + 4 levels (eq. SymplecticBasisTransformation)
    against the oracle's product of gate exponentials in 200 levels."""
    import paper_2410_18740_amd as P
    from oracle import plbo
    rng = np.random.default_rng(10 + d)
    for _ in range(2):
        p = _plbo_params(rng)
        got = P.plbo_ops(d, p, 1.1, 0.8, 0.3)
        ref = plbo.transformed_ops(p, d, 1.1, 0.8, 0.3)
        for k in range(5):
            assert np.abs(got[k] - ref[k]).max() < 1e-11, (d, k)


def test_plbo_parameter_derivatives_match_oracle_differences():
    """Forward-mode derivatives of the operators, contracted with a random slot
    environment, against the oracle's five-point differences of the energy."""
    import paper_2410_18740_amd as P
    from oracle import plbo
    d, a, b, g = 6, 1.3, 0.7, 0.2
    rng = np.random.default_rng(21)
    p = _plbo_params(rng)
    G = rng.normal(size=(6, d, d)) + 1j * rng.normal(size=(6, d, d))
    _, dops = P.plbo_ops(d, p, a, b, g, derivatives=True)
    got = np.array([sum(np.real(np.sum(G[k + 1] * dops[j, k])) for k in range(5)) for j in range(8)])
    ref = plbo.param_gradient(G, p, d, a, b, g, L=160)
    assert np.abs(got - ref).max() < 1e-7 * max(1.0, np.abs(ref).max())


def test_plbo_fock_isometry_matches_oracle():
    """<n|U|m>, n < D: the library's banded Taylor exponentials against the
    oracle's dense expm; the columns are orthonormal when D holds the basis."""
    import paper_2410_18740_amd as P
    from oracle import plbo
    rng = np.random.default_rng(5)
    for d, D in ((1, 10), (5, 24)):
        p = _plbo_params(rng)
        W = P.plbo_fock_isometry(D, d, p)
        assert np.abs(W - plbo.fock_isometry(p, D, d)).max() < 1e-11
    W = P.plbo_fock_isometry(60, 5, p)
    assert np.abs(W.conj().T @ W - np.eye(5)).max() < 1e-9


def test_plbo_host_entry_points_reject_bad_arguments():
    import paper_2410_18740_amd as P
    with pytest.raises(P.TnError):
        P.plbo_ops(0, np.zeros(8), 1, 1, 0)
    with pytest.raises(P.TnError):
        P.plbo_ops(65, np.zeros(8), 1, 1, 0)
    bad = np.zeros(8)
    bad[3] = np.nan
    with pytest.raises(P.TnError):
        P.plbo_ops(4, bad, 1, 1, 0)
    with pytest.raises(P.TnError):
        P.plbo_fock_isometry(3, 4, np.zeros(8))
    with pytest.raises(P.TnError):
        P.plbo_fock_isometry(8, 4, np.zeros(8), levels=4)


def test_noise_decomposition_matches_oracle():
    """Uniform-loss split V_eta = Q + C: the library's pure squeezing and
    factor L against the oracle (C = L L^T, Q = covariance(r', U))."""
    import paper_2410_18740_amd as P
    import workloads as W
    from oracle import noisy
    for N, seed, eta in ((3, 1, 0.8), (8, 2, 0.4), (12, 3, 1.0)):
        r, U = W.make_problem(N, seed, (0.3, 1.2))
        rp, Lc = P.noise_uniform_loss(r, U, eta)
        rp_o, C, _ = noisy.decompose_uniform_loss(r, U, eta)
        assert np.abs(rp - rp_o).max() < 1e-14
        assert np.abs(Lc @ Lc.T - C).max() < 1e-13
    with pytest.raises(P.TnError):
        P.noise_uniform_loss(r, U, 0.0)


def _plbo_site_G(d=3, seed=12):
    """Slot environments of site 1 of a random 4-mode MPS (oracle)."""
    import workloads as W
    from oracle import plbo, gbs, mpo as ompo, dmrg as odmrg
    r, U = W.make_problem(4, seed, (0.4, 0.7))
    al, be, ga = gbs.coefficients(r, U)
    rng = np.random.default_rng(seed)
    dims = [1, d, 5, d, 1]
    t = [rng.normal(size=(dims[s], d, dims[s + 1])) + 1j * rng.normal(size=(dims[s], d, dims[s + 1])) for s in range(4)]
    ops = [plbo.transformed_ops(np.zeros(8), d, al[s, s], be[s, s], ga[s, s], L=40) for s in range(4)]
    Ws = ompo.cores(al, be, ga, [o[:3] for o in ops])
    Gf = plbo.core_environment(odmrg.left_envs(t, Ws)[1], t[1], odmrg.right_envs(t, Ws)[2])
    Gf /= np.sum(np.abs(t[1]) ** 2)
    G = plbo.slot_gradients(Gf, plbo.slot_coefficients(plbo.gaussian_core_maker(al, be, ga, 1), d))
    return G, al[1, 1], be[1, 1], ga[1, 1]


def test_plbo_lbfgs_reaches_the_oracle_minimum():
    """The library's L-BFGS on the site energy (exact derivatives, Armijo
    backtracking) reaches the minimum value of scipy's L-BFGS-B run by the
    oracle from the same start.  The parameters themselves are not unique
    (squeeze, rotation and shear compose to the same Gaussian unitary in
    many ways), so the check is the energy, and the oracle's energy at the
    library's parameters."""
    import paper_2410_18740_amd as P
    from oracle import plbo
    G, a, b, g = _plbo_site_G()
    d = G.shape[1]
    mask = [0, 0, 1, 1, 1, 1, 0, 0]
    p0 = np.array([0, 0, 0.05, 0.1, 0.05, 0.02, 0, 0])
    o = P.PlboOpts(steps=300, lr=0.05, optimizer=P.PLBO_LBFGS, mask=0b111100)
    p, E = P.plbo_minimize(G, p0, a, b, g, o)
    pr, Er = plbo.minimize_site(G, p0, d, a, b, g, mask, L=40)
    E0 = plbo.site_energy(G, plbo.transformed_ops(p0, d, a, b, g, L=40))
    assert E < E0
    assert abs(E - Er) < 1e-8 * max(1.0, abs(Er)), (E, Er)
    assert np.all(p[[0, 1, 6, 7]] == 0.0)
    # three free parameters (r, phi, theta): the optimum is then unique up to
    # r -> -r with phi -> phi + pi, and the oracle evaluates the library's point
    o3 = P.PlboOpts(steps=300, lr=0.05, optimizer=P.PLBO_LBFGS, mask=0b11100)
    p3, E3 = P.plbo_minimize(G, p0, a, b, g, o3)
    _, Er3 = plbo.minimize_site(G, p0, d, a, b, g, [0, 0, 1, 1, 1, 0, 0, 0], L=40)
    assert abs(E3 - Er3) < 1e-8 * max(1.0, abs(Er3)), (E3, Er3)
    assert abs(plbo.site_energy(G, plbo.transformed_ops(p3, d, a, b, g, L=120)) - E3) < 1e-9 * max(1.0, abs(E3))


def test_plbo_adam_steps_match_the_oracle():
    """Five Adam steps from the same start: the library (exact gradients)
    and the oracle (five-point differences, Kingma & Ba's update) agree."""
    import paper_2410_18740_amd as P
    from oracle import plbo
    G, a, b, g = _plbo_site_G(seed=13)
    d = G.shape[1]
    mask = [0, 0, 1, 1, 1, 1, 0, 0]
    p0 = np.array([0, 0, 0.05, 0.1, 0.05, 0.02, 0, 0])
    o = P.PlboOpts(steps=5, lr=0.01, optimizer=P.PLBO_ADAM, mask=0b111100)
    p, _ = P.plbo_minimize(G, p0, a, b, g, o)
    pr, _ = plbo.adam(p0, lambda q: plbo.param_gradient(G, q, d, a, b, g, L=40, which=[2, 3, 4, 5]), 5, 0.01,
                      mask=mask)
    assert np.abs(p - pr).max() < 1e-9, (p, pr)
    with pytest.raises(P.TnError):
        P.plbo_minimize(G, p0, a, b, g, P.PlboOpts(optimizer=7))


def test_williamson_split_matches_oracle():
    """General split of mixed covariances (uniform loss plus thermal noise):
    the library's pure part reproduces the oracle's Q = S S^T / 2 through
    covariance(r, U), its factor the oracle's C; a pure V gives K = 0 and
    its own squeezing back; an unphysical V is rejected."""
    import paper_2410_18740_amd as P
    import workloads as W
    from oracle import noisy, gbs
    for N, seed, th in ((3, 1, 0.1), (6, 2, 0.0), (10, 3, 0.3)):
        r, U = W.make_problem(N, seed, (0.3, 1.1))
        V = noisy.lossy_covariance(r, U, 0.7) + th * np.eye(2 * N)
        rp, Up, L = P.noise_williamson(V)
        Q, C = noisy.decompose_williamson(V)
        assert np.abs(gbs.covariance(rp, Up) - Q).max() < 1e-12
        assert np.abs(L @ L.T - C).max() < 1e-12
        assert np.abs(Up @ Up.conj().T - np.eye(N)).max() < 1e-12
    r, U = W.make_problem(4, 5, (0.3, 1.1))
    rp, Up, L = P.noise_williamson(gbs.covariance(r, U))
    assert L.shape == (8, 0) and np.abs(np.sort(rp) - np.sort(r)).max() < 1e-10
    with pytest.raises(P.TnError):
        P.noise_williamson(0.3 * np.eye(4))


def test_plbo_effective_cutoff_matches_oracle():
    """Effective cutoff of pLBO bases: library (banded Taylor exponentials)
    against the oracle (dense expm), for the Fock basis, squeezes and
    composite parameters."""
    import paper_2410_18740_amd as P
    from oracle import plbo
    rng = np.random.default_rng(31)
    cases = [np.zeros(8), np.array([0, 0, 0.6, 0.4, 0, 0, 0, 0])] + [_plbo_params(rng) for _ in range(3)]
    for p in cases:
        for d in (1, 4):
            assert P.plbo_effective_cutoff(d, p, 120, 1e-10) == plbo.effective_cutoff(p, d, 120, 1e-10), (d, p)
    with pytest.raises(P.TnError):
        P.plbo_effective_cutoff(4, np.zeros(8), 3)
