"""GPU parity of noisy-GBS sampling (Sec. II.F, eq. CovarianceDecomposition):
the pure part of a lossy instance is solved by DMRG, and photon-number samples
of D(alpha)|psi> with alpha from the classical part follow the oracle's
displaced sampler stream; their single-mode histograms and mean photon numbers
match the lossy Gaussian state."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import noisy, gbs, sampler as osampler

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2410_18740_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _pure_state(ctx, r, U, D, chi, sweeps=6):
    import paper_2410_18740_amd as P
    m = P.MPO(ctx, r, U, D)
    N = len(r)
    mp = P.MPS(ctx, W.random_mps(N, D, chi, 1234))
    for _ in range(sweeps):
        st = P.dmrg_sweep(ctx, m, mp, P.SweepOpts(chi_max=chi, tol=1e-12))
    return m, mp, st["energy"]


@pytest.mark.parametrize("N,D,chi", [(4, 6, 36), (3, 18, 24)])
def test_displaced_samples_follow_the_oracle_stream(ctx, N, D, chi):
    """Same z, same factor L and seed: the library's patterns equal the
    oracle's displaced sampler (displacement matrices by expm there, by the
    row recurrence in LDS here) on all but rounding ties; D = 6 takes the
    register path of the displacement kernel, D = 18 the general one."""
    import paper_2410_18740_amd as P
    r, U = W.make_problem(N, 0, (0.5, 0.5))
    eta = 0.7
    rp, Lc = P.noise_uniform_loss(r, U, eta)
    rp_o, C, Lo = noisy.decompose_uniform_loss(r, U, eta)
    assert np.abs(rp - rp_o).max() < 1e-14 and np.abs(Lc @ Lc.T - C).max() < 1e-14
    m, mp, E = _pure_state(ctx, rp, U, D, chi)
    assert E < 1e-3
    z = np.random.default_rng(9).standard_normal((300, N))
    smp = P.sample_displaced(ctx, mp, m, 300, 77, Lc, z=z).cpu().numpy()
    ref, tie = noisy.sample_displaced(mp.export(), noisy.alphas(z, Lo), 77, L=D + 60, with_ties=True)
    bad, nties = osampler.stream_mismatches(smp, ref, tie)
    print(f"displaced stream N={N} D={D}: {bad} mismatches outside ties, {nties} samples with a tie")
    assert bad == 0
    # no displacement: the plain sampler's stream
    plain = P.sample(ctx, mp, m, 300, 77).cpu().numpy()
    zero = P.sample_displaced(ctx, mp, m, 300, 77, np.zeros((2 * N, N)), z=z).cpu().numpy()
    assert np.array_equal(plain, zero)


def test_displaced_samples_through_an_lbo_basis(ctx):
    """d < D_raw: after LBO sweeps the Fock tensors are W_s A_s, and the
    displaced stream equals the oracle's run on those tensors."""
    import paper_2410_18740_amd as P
    from oracle import mps as omps
    N, D, d, chi = 4, 10, 5, 25
    r, U = W.make_problem(N, 8, (0.5, 0.7))
    rp, Lc = P.noise_uniform_loss(r, U, 0.6)
    _, _, Lo = noisy.decompose_uniform_loss(r, U, 0.6)
    m = P.MPO(ctx, rp, U, D, d)
    mp = P.MPS(ctx, W.random_mps(N, d, chi, 99))
    o = P.SweepOpts()
    o.chi_max, o.tol, o.lbo = chi, 1e-12, 1
    for _ in range(4):
        P.dmrg_sweep(ctx, m, mp, o)
    z = np.random.default_rng(3).standard_normal((300, N))
    smp = P.sample_displaced(ctx, mp, m, 300, 5, Lc, z=z).cpu().numpy()
    F = omps.fock_tensors(mp.export(), list(m.isometries()))
    ref, tie = noisy.sample_displaced(F, noisy.alphas(z, Lo), 5, L=D + 60, with_ties=True)
    bad, nties = osampler.stream_mismatches(smp, ref, tie)
    assert bad == 0, (bad, nties)


def test_noisy_marginals_match_the_lossy_gaussian_state(ctx):
    """400k noisy samples of a 4-mode instance with eta = 0.6: every mode's
    photon-number histogram matches the photon distribution of the 2 x 2 block
    of V_eta = eta V + (1 - eta) I/2 (5 sigma plus the cutoff's weight), and
    so do the mean photon numbers (V_jj + V_{N+j,N+j} - 1)/2."""
    import paper_2410_18740_amd as P
    r, U = W.make_problem(4, 5, (0.4, 0.6))
    eta, D, n = 0.6, 10, 400000
    rp, Lc = P.noise_uniform_loss(r, U, eta)
    m, mp, E = _pure_state(ctx, rp, U, D, 64)
    assert E < 1e-6
    smp = P.sample_displaced(ctx, mp, m, n, 4242, Lc).cpu().numpy()
    V = noisy.lossy_covariance(r, U, eta)
    N = 4
    for j in range(N):
        V2 = V[np.ix_([j, N + j], [j, N + j])]
        want = noisy.gaussian_photon_distribution(V2, D)
        tail = 1.0 - want.sum()
        hist = np.bincount(smp[:, j], minlength=D)[:D] / n
        sig = np.sqrt(want * (1 - want) / n)
        assert np.all(np.abs(hist - want) <= 5 * sig + 2 * tail + 1e-6), (j, hist, want)
        mean = 0.5 * (V[j, j] + V[N + j, N + j] - 1.0)
        assert abs(smp[:, j].mean() - mean) < 5 * math.sqrt(want @ (np.arange(D) ** 2) / n) + D * tail + 1e-4


def test_noise_entry_points_reject_bad_arguments(ctx):
    import paper_2410_18740_amd as P
    r, U = W.make_problem(3, 0, (0.5, 0.5))
    for eta in (0.0, 1.5, float("nan")):
        with pytest.raises(P.TnError):
            P.noise_uniform_loss(r, U, eta)
    with pytest.raises(P.TnError):
        P.noise_uniform_loss(np.array([0.3, -0.1, 0.2]), U, 0.5)
    m, mp, _ = _pure_state(ctx, r, U, 4, 8, sweeps=1)
    bad = np.zeros((6, 3))
    bad[0, 0] = np.inf
    with pytest.raises(P.TnError):
        P.sample_displaced(ctx, mp, m, 10, 1, bad)
    with pytest.raises(ValueError):
        P.sample_displaced(ctx, mp, m, 10, 1, np.zeros((5, 3)))


def test_displaced_stream_at_the_benchmark_size(ctx):
    """The benchmark configuration of the noisy mode (32 modes, D_raw 16 -> d 8,
    chi 128, eta = 0.5, FP32 + LBO sweeps of the pure part): 24 displaced
    samples against the oracle's displaced sampler run on the exported Fock
    tensors W_s A_s with the same z, factor and seed."""
    import paper_2410_18740_amd as P
    from oracle import mps as omps
    w = W.WORKLOADS["gbs_n32_d16to8_chi128"]
    r, U = W.workload_problem("gbs_n32_d16to8_chi128")
    rp, Lc = P.noise_uniform_loss(r, U, 0.5)
    _, _, Lo = noisy.decompose_uniform_loss(r, U, 0.5)
    m = P.MPO(ctx, rp, U, w.D_raw, w.d)
    mp = P.MPS(ctx, W.random_mps(w.N, w.d, w.chi, w.mps_seed))
    o = P.SweepOpts(chi_max=w.chi, tol=1e-6, krylov_max=24, max_matvecs=16, precision=P.FP32, lbo=1)
    for _ in range(2):
        P.dmrg_sweep(ctx, m, mp, o)
    z = np.random.default_rng(31).standard_normal((24, w.N))
    smp = P.sample_displaced(ctx, mp, m, 24, 8, Lc, z=z).cpu().numpy()
    F = omps.fock_tensors(mp.export(), list(m.isometries()))
    ref, tie = noisy.sample_displaced(F, noisy.alphas(z, Lo), 8, L=w.D_raw + 60, with_ties=True)
    bad, nties = osampler.stream_mismatches(smp, ref, tie)
    assert bad == 0, (bad, nties)


def test_williamson_split_samples_match_a_general_mixed_state(ctx):
    """A mixed covariance that is not uniform loss (loss 0.7 plus thermal
    noise 0.05 on every mode): the Williamson split's pure part (r, U) is
    solved by DMRG, the displacement factor has rank 2N, the stream follows
    the oracle's, and 400k samples reproduce each mode's photon distribution
    of V."""
    import paper_2410_18740_amd as P
    r, U = W.make_problem(4, 6, (0.4, 0.6))
    N, D, n = 4, 12, 400000
    V = noisy.lossy_covariance(r, U, 0.7) + 0.05 * np.eye(2 * N)
    rp, Up, Lc = P.noise_williamson(V)
    assert Lc.shape == (2 * N, 2 * N)
    # the Williamson pure part is more squeezed than the minimal one: the
    # Fock box leaves a larger <H>
    m, mp, E = _pure_state(ctx, rp, Up, D, 64)
    assert E < 1e-4
    z = np.random.default_rng(12).standard_normal((200, 2 * N))
    smp = P.sample_displaced(ctx, mp, m, 200, 21, Lc, z=z).cpu().numpy()
    ref, tie = noisy.sample_displaced(mp.export(), noisy.alphas(z, Lc), 21, L=D + 60, with_ties=True)
    bad, nties = osampler.stream_mismatches(smp, ref, tie)
    assert bad == 0, (bad, nties)
    smp = P.sample_displaced(ctx, mp, m, n, 4343, Lc).cpu().numpy()
    for j in range(N):
        want = noisy.gaussian_photon_distribution(V[np.ix_([j, N + j], [j, N + j])], D)
        tail = 1.0 - want.sum()
        hist = np.bincount(smp[:, j], minlength=D)[:D] / n
        sig = np.sqrt(want * (1 - want) / n)
        assert np.all(np.abs(hist - want) <= 5 * sig + 2 * tail + 1e-6), (j, hist, want)


def test_displaced_samples_through_gate_parameterised_bases(ctx):
    """The pure part solved in pLBO bases: the sampler's Fock tensors use the
    Fock image of the learned bases, and the displaced stream equals the
    oracle's run on U(p)[:D, :d] A_s with U(p) from the oracle's gate
    exponentials."""
    import paper_2410_18740_amd as P
    from oracle import mps as omps, plbo
    N, D, d, chi = 4, 12, 3, 9
    r, U = W.make_problem(N, 10, (0.4, 0.6))
    rp, Lc = P.noise_uniform_loss(r, U, 0.7)
    _, _, Lo = noisy.decompose_uniform_loss(r, U, 0.7)
    m = P.MPO(ctx, rp, U, D, d)
    P.plbo_enable(ctx, m)
    mp = P.MPS(ctx, W.random_mps(N, d, chi, 4))
    o = P.SweepOpts()
    o.chi_max, o.tol = chi, 1e-11
    for _ in range(4):
        P.plbo_sweep(ctx, m, mp, o, P.PlboOpts(steps=15, lr=0.03, matvecs=8))
    p = P.plbo_params(ctx, m)
    z = np.random.default_rng(2).standard_normal((200, N))
    smp = P.sample_displaced(ctx, mp, m, 200, 9, Lc, z=z).cpu().numpy()
    F = omps.fock_tensors(mp.export(), [plbo.fock_isometry(p[s], D, d) for s in range(N)])
    ref, tie = noisy.sample_displaced(F, noisy.alphas(z, Lo), 9, L=D + 60, with_ties=True)
    bad, nties = osampler.stream_mismatches(smp, ref, tie)
    assert bad == 0, (bad, nties)


def test_library_noise_draws_follow_the_oracle_generator(ctx):
    """With no z passed, the library draws the noise itself (Philox4x32-10 and
    the Box-Muller transform, counter (sample, column, 1)): the stream equals
    the oracle's displaced sampler fed with the oracle's own draws of the same
    generator, outside rounding ties, and a second call with the same seed
    repeats it bit for bit."""
    import paper_2410_18740_amd as P
    N, D, chi = 4, 6, 36
    r, U = W.make_problem(N, 3, (0.5, 0.6))
    rp, Lc = P.noise_uniform_loss(r, U, 0.65)
    _, _, Lo = noisy.decompose_uniform_loss(r, U, 0.65)
    m, mp, E = _pure_state(ctx, rp, U, D, chi)
    n, seed = 300, 2024
    smp = P.sample_displaced(ctx, mp, m, n, seed, Lc).cpu().numpy()
    again = P.sample_displaced(ctx, mp, m, n, seed, Lc).cpu().numpy()
    assert np.array_equal(smp, again)
    z = noisy.library_normals(n, Lc.shape[1], seed)
    ref, tie = noisy.sample_displaced(mp.export(), noisy.alphas(z, Lo), seed, L=D + 60, with_ties=True)
    bad, nties = osampler.stream_mismatches(smp, ref, tie)
    print(f"library noise: {bad} mismatches outside ties, {nties} samples with a tie")
    assert bad == 0
    # the same draws passed explicitly give the same stream
    expl = P.sample_displaced(ctx, mp, m, n, seed, Lc, z=z).cpu().numpy()
    bad2, _ = osampler.stream_mismatches(expl, ref, tie)
    assert bad2 == 0
