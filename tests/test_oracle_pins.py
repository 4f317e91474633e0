"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test ties an oracle function to something other than itself: a second
independent construction, a closed form, a printed value of the paper, a
brute-force count, or an invariant the paper states.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import gbs, operators, dense, mpo, mps as M, dmrg, flops, lbo

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _small_problem(N=3, seed=0, r=(0.5, 0.3, 0.7)):
    U = W.haar_unitary(N, np.random.default_rng(seed))
    return np.array(r[:N], dtype=float), U


# --------------------------------------------------------------- Hamiltonian
@pytest.mark.parametrize("D", [3, 4])
def test_quadrature_form_equals_bogoliubov_form(D):
    """eq. GBSHamiltonian (quadratures) == eq. CentralEquation (sum b^dag b)."""
    r, U = _small_problem()
    al, be, ga = gbs.coefficients(r, U)
    Hq = dense.php_quadrature(al, be, ga, D)
    Hb = dense.php_bogoliubov(r, U, D)
    assert np.abs(Hq - Hb).max() < 1e-12


def test_hamiltonian_annihilates_output_state():
    """H|psi> = 0 (eq. CentralEquation): H built on a (D+2)-box, applied to the
    exact amplitudes, vanishes on the inner D-box (H moves each n_k by <= 2)."""
    r, U = _small_problem()
    al, be, ga = gbs.coefficients(r, U)
    D = 4
    H = dense.php_quadrature(al, be, ga, D + 2)
    psi = gbs.exact_amplitudes(r, U, D + 2).reshape(-1)
    res = (H @ psi).reshape((D + 2,) * 3)[:D, :D, :D]
    assert np.abs(res).max() < 1e-12
    assert np.abs(psi).max() > 0.1


def test_commutator_defect_golden():
    """SM Sec. 5 prints [X, P] = i diag(1, ..., 1, 1-D) for D x D matrices."""
    for line in open(os.path.join(GOLD, "commutator_defect.txt")):
        if line.startswith("#") or not line.strip():
            continue
        vals = [float(v) for v in line.split()]
        D, diag = int(vals[0]), np.array(vals[1:])
        X, P = operators.quadratures(D)
        C = X @ P - P @ X
        assert np.abs(C - 1j * np.diag(diag)).max() < 1e-12


def test_local_square_uses_d_plus_4():
    """SM Sec. 5: X^2 built at D+4 then truncated equals the exact compression
    P X^2 P (tridiagonal band of the infinite matrix), unlike (PXP)^2."""
    D = 5
    Xb, _ = operators.quadratures(D + 4)
    X, _, S = operators.local_operators(D, 2.0, 0.0, 0.0)
    # S = 1/2 * 2 X^2 - 1/2 -> X^2 = S + 1/2
    X2 = S + 0.5 * np.eye(D)
    exact = np.zeros((D, D))
    for n in range(D):
        exact[n, n] = n + 0.5
        if n + 2 < D:
            exact[n, n + 2] = exact[n + 2, n] = 0.5 * math.sqrt((n + 1) * (n + 2))
    assert np.abs(X2 - exact).max() < 1e-13
    assert np.abs((X @ X) - exact).max() > 0.1   # the naive square differs


# --------------------------------------------------------------- amplitudes
def test_recursion_matches_hafnian():
    """Amplitude recursion == brute-force hafnian <n|psi> (Sec. II.A)."""
    for N, r in ((3, (0.5, 0.3, 0.7)), (4, (0.4, 0.6, 0.5, 0.8))):
        r_, U = _small_problem(N, seed=N, r=r)
        psi = gbs.exact_amplitudes(r_, U, 4)
        rng = np.random.default_rng(7)
        checked = 0
        for _ in range(40):
            n = tuple(int(v) for v in rng.integers(0, 4, N))
            if sum(n) > 10:
                continue
            h = gbs.amplitude_hafnian(n, r_, U)
            assert abs(psi[n] - h) < 1e-12
            checked += 1
        assert checked > 20


def test_single_mode_closed_form():
    """N = 1: P(2n) = (2n)!/(4^n n!^2) tanh^{2n} r / cosh r, P(odd) = 0; ED of
    the truncated single-mode H at D = 40 gives E0 ~ 0 and the same vector."""
    r = np.array([0.5])
    U = np.eye(1, dtype=complex)
    psi = gbs.exact_amplitudes(r, U, 30)
    P = np.abs(psi) ** 2
    Pc = gbs.single_mode_probabilities(0.5, 30)
    assert np.abs(P - Pc).max() < 1e-14
    assert abs(psi[2] / psi[0] - (-math.tanh(0.5)) * math.sqrt(2) / 2) < 1e-14
    al, be, ga = gbs.coefficients(r, U)
    H = dense.php_quadrature(al, be, ga, 40)
    ev, vec = dense.ground_states(H, 4)
    assert abs(ev[0]) < 1e-11
    # harmonic spectrum (eq. generalizedCCR): 0, 1, 2, 3
    assert np.abs(ev - np.arange(4)).max() < 1e-7   # truncation raises them slightly
    v = vec[:, 0] * np.sign(vec[0, 0].real)
    assert np.abs(np.abs(v[:30]) ** 2 - Pc).max() < 1e-11


# --------------------------------------------------------------- MPO
def test_mpo_bond_dimensions_and_boundary_cores():
    """SM Sec. 8: w_s = 2 + 2 min(s, N-s); boundary cores as printed."""
    gold = {}
    for line in open(os.path.join(GOLD, "mpo_boundary_cores.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        gold[k] = [int(x) for x in v]
    for N in range(2, 12):
        w, kinds = mpo.structure(N)
        assert w[0] == 1 and w[N] == 1
        for s in range(1, N):
            assert w[s] == 2 + 2 * min(s, N - s)
        # L_1 = (X_1, P_1, 1, S_1): row S of core 1 over columns X_1, P_1, S, F
        if N >= 3:
            assert list(kinds[0][0]) == gold["L1"]
        # R_N^T = (X_N, P_N, 1, S_N): column F of core N over rows Xw_N, Pw_N, F, S
        if N >= 2:
            assert list(kinds[N - 1][:, 0]) == gold["RN"]


@pytest.mark.parametrize("N,D", [(1, 5), (2, 4), (3, 4), (4, 3), (5, 3)])
def test_mpo_contracts_to_php(N, D):
    """The MPO (SM Sec. 8) contracts to the dense PHP of eq. GBSHamiltonian,
    including the paper's worked N = 5 case."""
    U = W.haar_unitary(N, np.random.default_rng(N + 10))
    r = np.linspace(0.3, 0.8, N)
    al, be, ga = gbs.coefficients(r, U)
    ops = [operators.local_operators(D, al[s, s], be[s, s], ga[s, s]) for s in range(N)]
    Hm = mpo.to_dense(mpo.cores(al, be, ga, ops))
    Hq = dense.php_quadrature(al, be, ga, D)
    assert np.abs(Hm - Hq).max() < 1e-12


def test_mpo_vacuum_is_number_operator():
    """r = 0: H = sum_k a_k^dag a_k for any interferometer (Sec. II.C.1,
    H_|0>): the MPO contracts to diag(sum n) with integer entries."""
    N, D = 4, 3
    U = W.haar_unitary(N, np.random.default_rng(3))
    al, be, ga = gbs.coefficients(np.zeros(N), U)
    ops = [operators.local_operators(D, al[s, s], be[s, s], ga[s, s]) for s in range(N)]
    Hm = mpo.to_dense(mpo.cores(al, be, ga, ops))
    n = np.indices((D,) * N).reshape(N, -1).sum(0)
    assert np.abs(Hm - np.diag(n)).max() < 1e-12


def test_mpo_kind_table_is_positional():
    """U = identity makes every cross coefficient vanish; the kind table is
    unchanged (a zero coefficient never removes a block)."""
    N = 6
    w, kinds = mpo.structure(N)
    al, be, ga = gbs.coefficients(np.full(N, 0.4), np.eye(N, dtype=complex))
    for s in range(1, N + 1):
        rows, cols, E = mpo.core_entries(N, s, al, be, ga)
        K = np.zeros((len(rows), len(cols)), dtype=np.int8)
        for (rl, cl), (kind, _, _) in E.items():
            K[rows.index(rl), cols.index(cl)] = kind
        assert np.array_equal(K, kinds[s - 1])


def test_core_counts():
    N = 9
    m = mpo.middle_site(N)
    w, kinds = mpo.structure(N)
    for s in range(1, N + 1):
        n_op, n_sc = flops.core_counts(kinds[s - 1])
        if s < m:
            assert (n_op, n_sc) == (2 * s + 1, 0)
        elif s == m:
            assert (n_op, n_sc) == (1 + 2 * (m - 1) + 2 * (N - m), 4 * (m - 1) * (N - m))
        else:
            assert (n_op, n_sc) == (2 * (N - s) + 3, 0)


# --------------------------------------------------------------- ED + truncation
def _cfg_n4():
    r, U = W.workload_problem("gbs_n4_d6_chi16")
    return r, U, gbs.coefficients(r, U)


def test_ed_truncation_properties():
    """SM Sec. 1 and Sec. II.E: E0 >= 0, non-increasing in D (interlacing),
    matches the oracle-written golden values, E0 <= <Ppsi|H|Ppsi>/|Ppsi|^2,
    F >= 1 - E0, and the ground state has even total photon number."""
    r, U, (al, be, ga) = _cfg_n4()
    gold = {}
    for line in open(os.path.join(GOLD, "cfg_n4_ed.txt")):
        if line.startswith("#") or not line.strip():
            continue
        D, e = line.split()
        gold[int(D)] = float(e)
    prev = np.inf
    for D in (3, 4, 5, 6):
        H = dense.php_quadrature(al, be, ga, D)
        ev, vec = dense.ground_states(H, 2)
        assert ev[0] >= -1e-12
        assert ev[0] <= prev + 1e-12
        prev = ev[0]
        assert abs(ev[0] - gold[D]) < 1e-10
    psiP = gbs.exact_amplitudes(r, U, 6).reshape(-1)
    ray = float(np.vdot(psiP, H @ psiP).real / np.vdot(psiP, psiP).real)
    assert ev[0] <= ray
    F = abs(np.vdot(psiP, vec[:, 0])) ** 2
    assert F >= 1 - ev[0]
    n = np.indices((6,) * 4).reshape(4, -1).sum(0)
    assert np.sum(np.abs(vec[n % 2 == 1, 0]) ** 2) < 1e-20
    # first excitation near 1 (harmonic spectrum, raised by truncation)
    assert 0.99 < ev[1] < 1.2


# --------------------------------------------------------------- DMRG
def _cfg_n4_mpo(D=6):
    r, U, (al, be, ga) = _cfg_n4()
    ops = [operators.local_operators(D, al[s, s], be[s, s], ga[s, s]) for s in range(4)]
    return r, U, mpo.cores(al, be, ga, ops), dense.php_quadrature(al, be, ga, D)


def test_dmrg_full_rank_matches_ed():
    """chi = 36 is the full Schmidt rank for N = 4, D = 6: two-site DMRG
    reaches the ED ground energy and distribution (Sec. II.D, II.E)."""
    r, U, Ws, H = _cfg_n4_mpo()
    ev, vec = dense.ground_states(H, 1)
    m0 = W.random_mps(4, 6, 36, 1000)
    out, st = dmrg.dmrg(m0, Ws, 36, 3, tol=1e-12)
    assert abs(st[-1]["energy"] - ev[0]) < 1e-12
    P = M.probabilities(out)
    assert np.abs(P - np.abs(vec[:, 0]) ** 2).max() < 1e-12


def test_dmrg_truncated_is_variational():
    """chi = 16: E_DMRG >= E_ED, the excess bounded by 50x the ED discarded
    Schmidt weight at the middle cut (eq. SurrogateEpsChi), sweep energies
    non-increasing up to the discarded weight."""
    r, U, Ws, H = _cfg_n4_mpo()
    ev, vec = dense.ground_states(H, 1)
    sv = np.linalg.svd(vec[:, 0].reshape(36, 36), compute_uv=False)
    tail = float(np.sum(sv[16:] ** 2))
    m0 = W.random_mps(4, 6, 16, 1000)
    out, st = dmrg.dmrg(m0, Ws, 16, 4, tol=1e-12)
    E = st[-1]["energy"]
    assert E >= ev[0] - 1e-12
    assert E - ev[0] <= 50 * tail
    for a, b in zip(st, st[1:]):
        assert b["energy"] <= a["energy"] + max(a["max_discarded"], 1e-12)


def test_dmrg_vacuum_product_state():
    """r = 0: the vacuum is exact at chi = 1 with <H> = 0."""
    N, D = 5, 4
    U = W.haar_unitary(N, np.random.default_rng(5))
    al, be, ga = gbs.coefficients(np.zeros(N), U)
    ops = [operators.local_operators(D, al[s, s], be[s, s], ga[s, s]) for s in range(N)]
    Ws = mpo.cores(al, be, ga, ops)
    m0 = W.random_mps(N, D, 1, 3)
    out, st = dmrg.dmrg(m0, Ws, 1, 2, tol=1e-13)
    assert abs(st[-1]["energy"]) < 1e-12


def test_energy_two_ways():
    """<H> by environment contraction == sum_k ||b_k psi||^2 (eq.
    CentralEquation as a sum of squares); both non-negative."""
    r, U = _small_problem()
    al, be, ga = gbs.coefficients(r, U)
    D = 4
    ops = [operators.local_operators(D, al[s, s], be[s, s], ga[s, s]) for s in range(3)]
    Ws = mpo.cores(al, be, ga, ops)
    for seed in (1, 2):
        m = W.random_mps(3, D, 8, seed)
        e1 = dmrg.energy(m, Ws)
        e2 = dmrg.energy_bogoliubov(m, r, U, D)
        assert e1 > 0 and e2 > 0
        assert abs(e1 - e2) < 1e-12 * max(1.0, abs(e1))


def test_fidelity_bound_from_energy():
    """F >= 1 - <H> (Sec. II.E) for DMRG states of the full-space H."""
    r, U, Ws, H = _cfg_n4_mpo()
    m0 = W.random_mps(4, 6, 16, 1000)
    out, st = dmrg.dmrg(m0, Ws, 16, 2, tol=1e-12)
    c = M.to_dense(out)
    c = c / np.linalg.norm(c)
    psi = gbs.exact_amplitudes(r, U, 6).reshape(-1)
    F = abs(np.vdot(psi, c)) ** 2
    assert F >= 1 - st[-1]["energy"]


def test_marginals_match_dense():
    r, U, Ws, H = _cfg_n4_mpo(D=4)
    m = W.random_mps(4, 4, 8, 11)
    P = np.abs(M.to_dense(m)) ** 2
    P = (P / P.sum()).reshape((4,) * 4)
    marg = M.marginals(m)
    for j in range(4):
        axes = tuple(a for a in range(4) if a != j)
        assert np.abs(marg[j] - P.sum(axis=axes)).max() < 1e-13


def test_lanczos_matches_eigh():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((60, 60)) + 1j * rng.standard_normal((60, 60))
    A = A + A.conj().T
    lam, x, k, conv = dmrg.lanczos_lowest(lambda v: A @ v, rng.standard_normal(60) + 0j, tol=1e-12)
    assert conv
    assert abs(lam - np.linalg.eigvalsh(A)[0]) < 1e-10
    assert np.linalg.norm(A @ x - lam * x) < 1e-10


def _haar_isometry(m, k, rng):
    Z = rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))
    Q, R = np.linalg.qr(Z)
    return Q * (np.diag(R) / np.abs(np.diag(R)))[None, :]


def test_truncation_keeps_the_known_singular_values():
    """theta = V1 diag(sigma) V2^dag with chosen sigma (Sec. II.C truncation):
    the kept values are sigma[:chi] renormalised, the discarded weight is
    sum sigma[chi:]^2 / sum sigma^2, and by Eckart-Young the kept factors
    rebuild the best rank-chi approximation, whose squared error is exactly
    the discarded sum; a relative cut sigma_cut keeps the values above
    sigma_cut * sigma_0, and at least one."""
    rng = np.random.default_rng(21)
    cl, d, cr = 5, 3, 4
    m, n = cl * d, d * cr
    sigma = np.sort(rng.uniform(0.05, 2.0, 12))[::-1]
    V1, V2 = _haar_isometry(m, 12, rng), _haar_isometry(n, 12, rng)
    M0 = (V1 * sigma) @ V2.conj().T
    theta = M0.reshape(cl, d, d, cr)
    tot = float(np.sum(sigma ** 2))
    for chi in (1, 5, 12, 20):
        U, S, Vh, disc = dmrg.truncate(theta, chi)
        k = min(chi, 12)
        assert len(S) == k
        kept = sigma[:k]
        assert np.abs(S - kept / np.linalg.norm(kept)).max() < 1e-12
        assert abs(disc - float(np.sum(sigma[k:] ** 2)) / tot) < 1e-13
        assert np.abs(U.conj().T @ U - np.eye(k)).max() < 1e-12
        assert np.abs(Vh @ Vh.conj().T - np.eye(k)).max() < 1e-12
        err = np.linalg.norm(M0 - (U * (S * np.linalg.norm(kept))) @ Vh) ** 2
        assert abs(err - float(np.sum(sigma[k:] ** 2))) < 1e-11
    cut = 0.5 * (sigma[3] + sigma[4]) / sigma[0]
    assert len(dmrg.truncate(theta, 12, sigma_cut=cut)[1]) == 4
    assert len(dmrg.truncate(theta, 12, sigma_cut=2.0)[1]) == 1


def test_two_site_matvec_matches_brute_force_loops():
    """eq. of the two-site effective Hamiltonian: theta' = L W1 W2 R theta,
    each output element summed by explicit loops over every index on a tiny
    case with all dimensions distinct, so a transposed or swapped leg fails;
    with Hermitian L, R (in their bra/ket legs) and W (in s, s') the map is
    Hermitian."""
    rng = np.random.default_rng(5)
    a, wl, wm, wr, d, b = 2, 3, 2, 4, 3, 2
    c = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    L, W1, W2, R, th = c(wl, a, a), c(wl, wm, d, d), c(wm, wr, d, d), c(wr, b, b), c(a, d, d, b)
    got = dmrg.heff_matvec(L, W1, W2, R, th)
    want = np.zeros((a, d, d, b), dtype=np.complex128)
    for i in range(a):
        for s in range(d):
            for t in range(d):
                for j in range(b):
                    acc = 0j
                    for l in range(wl):
                        for m_ in range(wm):
                            for n_ in range(wr):
                                for i2 in range(a):
                                    for s2 in range(d):
                                        for t2 in range(d):
                                            for j2 in range(b):
                                                acc += (L[l, i, i2] * W1[l, m_, s, s2] * W2[m_, n_, t, t2]
                                                        * R[n_, j, j2] * th[i2, s2, t2, j2])
                    want[i, s, t, j] = acc
    assert np.abs(got - want).max() < 1e-12
    # single-site form: L W1 R1 on A, with R1 on W1's right bond
    A, R1 = c(a, d, b), R[:wm]
    want1 = np.zeros((a, d, b), dtype=np.complex128)
    for i, s, j in np.ndindex(a, d, b):
        want1[i, s, j] = sum(L[l, i, i2] * W1[l, m_, s, s2] * R1[m_, j, j2] * A[i2, s2, j2]
                             for l in range(wl) for m_ in range(wm)
                             for i2 in range(a) for s2 in range(d) for j2 in range(b))
    assert np.abs(dmrg.heff_matvec_single(L, W1, R1, A) - want1).max() < 1e-12
    herm = lambda X: X + np.conj(np.swapaxes(X, -1, -2))
    L, W1, W2, R = herm(L), herm(W1), herm(W2), herm(R)
    n = a * d * d * b
    H = np.stack([dmrg.heff_matvec(L, W1, W2, R, e.reshape(a, d, d, b)).ravel() for e in np.eye(n)], axis=1)
    assert np.abs(H - H.conj().T).max() < 1e-12


def test_environment_updates_match_brute_force_loops():
    """Left and right environment updates (Sec. II.C sweeps): every element
    summed by explicit loops over the bra site tensor conj(A), the MPO core W
    and the ket A, all dimensions distinct; contracting a left environment
    with the right one of the same bond gives the same number at any bond."""
    rng = np.random.default_rng(6)
    a, wl, wr, d, b = 2, 3, 4, 3, 5
    c = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    L, R, W, A = c(wl, a, a), c(wr, b, b), c(wl, wr, d, d), c(a, d, b)
    wantL = np.zeros((wr, b, b), dtype=np.complex128)
    for m_, j, j2 in np.ndindex(wr, b, b):
        wantL[m_, j, j2] = sum(np.conj(A[i, s, j]) * L[l, i, i2] * W[l, m_, s, s2] * A[i2, s2, j2]
                               for l in range(wl) for i in range(a) for i2 in range(a)
                               for s in range(d) for s2 in range(d))
    assert np.abs(dmrg.env_left_update(L, A, W) - wantL).max() < 1e-12
    wantR = np.zeros((wl, a, a), dtype=np.complex128)
    for l, i, i2 in np.ndindex(wl, a, a):
        wantR[l, i, i2] = sum(np.conj(A[i, s, j]) * W[l, n_, s, s2] * R[n_, j, j2] * A[i2, s2, j2]
                              for n_ in range(wr) for j in range(b) for j2 in range(b)
                              for s in range(d) for s2 in range(d))
    assert np.abs(dmrg.env_right_update(R, A, W) - wantR).max() < 1e-12
    # <L_s, R_s> is the same scalar at every bond s of a chain
    N, dd, chi = 4, 3, 3
    mps_ = [c(1 if s == 0 else chi, dd, 1 if s == N - 1 else chi) for s in range(N)]
    Ws = [c(1 if s == 0 else 2, 1 if s == N - 1 else 2, dd, dd) for s in range(N)]
    Ls, Rs = dmrg.left_envs(mps_, Ws), dmrg.right_envs(mps_, Ws)
    vals = [np.sum(Ls[s] * Rs[s]) for s in range(N + 1)]
    assert max(abs(v - vals[0]) for v in vals) < 1e-10 * abs(vals[0])


# --------------------------------------------------------------- flops
def test_flop_formula_counts_naive_contraction():
    """The matvec formula equals the multiply-adds of the naive 4-stage
    contraction (L, W_s, W_{s+1}, R) with identity blocks free and scalar
    blocks costing one multiply per element, counted by explicit loops."""
    N = 5
    w, kinds = mpo.structure(N)
    d, cl, cr = 3, 4, 5
    for s in range(1, N):
        Ks, Ks1 = kinds[s - 1], kinds[s]
        wl, wr = w[s - 1], w[s + 1]
        macs = wl * cl * cl * d * d * cr          # L x theta
        for K in (Ks, Ks1):
            for v in K.reshape(-1):
                if 2 <= v <= 5:
                    macs += d * d * d * cl * cr   # d x d operator on one leg
                elif v == 6:
                    macs += d * d * cl * cr
        macs += wr * cl * d * d * cr * cr         # x R
        assert flops.matvec_flops(d, cl, cr, wl, wr, Ks, Ks1) == 8 * macs


# --------------------------------------------------------------- sampler
def test_philox_known_answers():
    """Published Philox4x32-10 known-answer vectors (Salmon et al., SC'11)."""
    from oracle import sampler
    n = 0
    for line in open(os.path.join(GOLD, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        assert sampler.philox4x32_10(v[:4], v[4:6]) == tuple(v[6:])
        n += 1
    assert n == 3


def test_sampler_statistics_match_exact_marginals():
    """Histogram of oracle samples vs exact MPS marginals: every cell within 5
    sigma (binomial) on a 3-mode state."""
    from oracle import sampler
    r, U = _small_problem()
    al, be, ga = gbs.coefficients(r, U)
    D = 4
    ops = [operators.local_operators(D, al[s, s], be[s, s], ga[s, s]) for s in range(3)]
    Ws = mpo.cores(al, be, ga, ops)
    out, _ = dmrg.dmrg(W.random_mps(3, D, 16, 4), Ws, 16, 2, tol=1e-12)
    n = 3000
    smp = sampler.sample(out, n, seed=2004)
    marg = M.marginals(out)
    for j in range(3):
        h = np.bincount(smp[:, j], minlength=D) / n
        sig = np.sqrt(marg[j] * (1 - marg[j]) / n) + 1e-12
        assert np.all(np.abs(h - marg[j]) <= 5 * sig + 1e-3)
    # joint distribution of the first two modes
    P = np.abs(M.to_dense(out)) ** 2
    P = (P / P.sum()).reshape(D, D, D).sum(axis=2)
    H = np.zeros((D, D))
    for a, b in smp[:, :2]:
        H[a, b] += 1
    H /= n
    sig = np.sqrt(P * (1 - P) / n) + 1e-12
    assert np.all(np.abs(H - P) <= 5 * sig + 1e-3)


# --------------------------------------------------------------- local basis
def test_gaussian_reduced_state_spectrum():
    """Sec. III.A.1: the spectrum of rho_i of a Gaussian state is
    nbar^k / (nbar+1)^(k+1); checked on rho_i from the exact amplitudes of a
    3-mode state (large box), and the truncation bounds N eps >= eps_D >= eps
    of eq. SpecWfromSDsums at a small cutoff."""
    from oracle import lbo
    r, U = _small_problem()
    Db = 22
    psi = gbs.exact_amplitudes(r, U, Db)
    V = gbs.covariance(r, U)
    for i in range(3):
        rho = lbo.rdm_from_dense(psi, i)
        ev = np.sort(np.linalg.eigvalsh(rho))[::-1][:6]
        ref = lbo.gaussian_rdm_spectrum(V, i, 6)
        # the box [0, 22)^3 holds all but ~1e-7 of the state
        assert np.abs(ev - ref).max() < 2 * (1 - float(np.vdot(psi, psi).real)) + 1e-12
    # bounds at cutoff D = 4 in the optimal local basis, with eps from the spectra
    d = 4
    eps = 1 - np.mean([lbo.gaussian_rdm_spectrum(V, i, d).sum() for i in range(3)])
    # eps_D of the optimal-basis truncation: project each mode on its top-d eigenvectors
    proj = psi
    for i in range(3):
        rho = lbo.rdm_from_dense(psi, i)
        w, Z = np.linalg.eigh(rho)
        Pi = Z[:, -d:] @ Z[:, -d:].conj().T
        proj = np.moveaxis(np.tensordot(Pi, proj, axes=([1], [i])), 0, i)
    epsD = 1 - float(np.vdot(psi, proj).real) / float(np.vdot(psi, psi).real)
    assert 3 * eps >= epsD - 1e-12 and epsD >= eps - 1e-12


def test_lbo_step_finds_product_state_basis():
    """U = identity: the state is a product of single-mode squeezed vacua, so
    one local basis vector per site (d = 1) suffices; after LBO + DMRG the
    energy is that of the cutoff-D single-mode problems and the basis vector is
    the single-mode ground state."""
    from oracle import lbo
    N, D, d = 3, 10, 1
    r = np.array([0.3, 0.5, 0.4])
    U = np.eye(N, dtype=complex)
    al, be, ga, raw = lbo.local_ops(r, U, D)
    iso = [np.eye(D)[:, :d].astype(complex) for _ in range(N)]
    mps_ = [np.ones((1, d, 1), dtype=complex) for _ in range(N)]
    for s in range(N):
        cores = lbo.cores_in_basis(al, be, ga, raw, iso)
        raw_cores = mpo.cores(al, be, ga, raw)
        # centre at s: with chi = 1 every tensor is a normalised scalar
        Wn, A, disc, lam = lbo.lbo_site(mps_, cores, raw_cores[s], iso[s], s)
        iso[s] = Wn
        mps_[s] = A
    cores = lbo.cores_in_basis(al, be, ga, raw, iso)
    E = dmrg.energy(mps_, cores)
    E_single = sum(np.linalg.eigvalsh(raw[s][2])[0] for s in range(N))
    assert abs(E - E_single) < 1e-10
    for s in range(N):
        gs = np.linalg.eigh(raw[s][2])[1][:, 0]
        assert abs(abs(np.vdot(gs, iso[s][:, 0])) - 1.0) < 1e-8


# --------------------------------------------------------------- learned warm start
def test_mlp_gradients_match_finite_differences():
    """Backward pass == central finite differences of the MSE (FP64)."""
    from oracle import mlp
    rng = np.random.default_rng(0)
    params = mlp.init_params(rng, in_dim=7, hidden=9, out_dim=3)
    X = rng.standard_normal((5, 7))
    T = rng.standard_normal((5, 3))
    L, grads = mlp.loss_and_grads(params, X, T)
    p0, g0 = mlp.flatten(params), mlp.flatten(grads)
    h = 1e-6
    idx = rng.choice(len(p0), 40, replace=False)
    for i in idx:
        pp, pm = p0.copy(), p0.copy()
        pp[i] += h
        pm[i] -= h
        Lp, _ = mlp.loss_and_grads(mlp.unflatten(pp, 7, 9, 3), X, T)
        Lm, _ = mlp.loss_and_grads(mlp.unflatten(pm, 7, 9, 3), X, T)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g0[i]) <= 1e-6 * max(1e-3, abs(g0[i])) + 1e-9


def test_squeezed_basis_closed_form_and_targets():
    """The squeezed basis is an isometry whose first column is the squeezed
    vacuum (closed form); a single-mode squeezed state's moments give back its
    squeezing parameter and nbar = 0 (eq. diagReducedGaussianDM with one term)."""
    from oracle import mlp
    zeta = 0.4 * np.exp(0.7j)
    Wb = mlp.squeezed_basis(zeta, 30, 6)
    assert np.abs(Wb.conj().T @ Wb - np.eye(6)).max() < 1e-12
    t, e = np.tanh(0.4), np.exp(0.7j)
    for q in range(5):
        ref = (-e * t) ** q * math.sqrt(math.factorial(2 * q)) / (2 ** q * math.factorial(q)) / math.sqrt(np.cosh(0.4))
        assert abs(Wb[2 * q, 0] - ref) < 1e-9
    rho = np.outer(Wb[:, 0], Wb[:, 0].conj())
    n, m = mlp.moments(rho)
    tg = mlp.targets_from_moments(n, m)
    assert abs(tg[0] + 1j * tg[1] - zeta) < 1e-8
    assert abs(tg[2]) < 1e-8
    # the basis spans the eigenvectors of a squeezed thermal state
    nbar = 0.3
    lam = np.array([nbar ** k / (nbar + 1) ** (k + 1) for k in range(40)])
    Wbig = mlp.squeezed_basis(zeta, 60, 40)
    rho = (Wbig * lam) @ Wbig.conj().T
    tg = mlp.targets_from_moments(*mlp.moments(rho))
    assert abs(tg[0] + 1j * tg[1] - zeta) < 1e-6 and abs(tg[2] - math.log1p(nbar)) < 1e-6


def test_squeezed_basis_matches_matrix_exponential():
    """Columns of the squeezed basis equal S(zeta)|k> with S(zeta) =
    exp(1/2 (zeta* a^2 - zeta a^dag^2)) taken by scipy's expm on a large box."""
    import scipy.linalg
    from oracle import mlp
    zeta = 0.55 * np.exp(-1.1j)
    Db = 240
    a = np.diag(np.sqrt(np.arange(1, Db)), 1).astype(complex)
    S = scipy.linalg.expm(0.5 * (np.conj(zeta) * a @ a - zeta * a.T @ a.T))
    Wb = mlp.squeezed_basis(zeta, 110, 8)   # tails beyond row 110 are below 1e-13
    assert np.abs(Wb - S[:110, :8]).max() < 1e-10


def test_reduced_density_matrices_match_dense_partial_trace():
    """rho_j from the MPS contraction == brute-force partial trace of the dense
    state; Hermitian, unit trace, diagonal == the marginals."""
    from oracle import lbo
    m = W.random_mps(4, 3, 5, 21)
    psi = M.to_dense(m).reshape((3,) * 4)
    psi = psi / np.linalg.norm(psi)
    rho = M.reduced_density_matrices(m)
    marg = M.marginals(m)
    for j in range(4):
        ref = lbo.rdm_from_dense(psi, j)
        assert np.abs(rho[j] - ref).max() < 1e-13
        assert abs(np.trace(rho[j]) - 1) < 1e-13
        assert np.abs(rho[j] - rho[j].conj().T).max() < 1e-14
        assert np.abs(np.real(np.diag(rho[j])) - marg[j]).max() < 1e-13


def test_reduced_state_depends_on_doubled_angle_only():
    """The learned start's features use 2 arg U_jk: flipping the sign of any
    input mode (U -> U diag(+-1), an even squeezed vacuum is unchanged) leaves
    the Gaussian covariance, hence every reduced state, and the features alike."""
    from oracle import mlp
    r, U = W.make_problem(7, 5, (0.3, 1.2))
    s = np.array([1, -1, -1, 1, -1, 1, 1])
    U2 = U * s[None, :]
    assert np.abs(gbs.covariance(r, U) - gbs.covariance(r, U2)).max() < 1e-13
    for j in range(7):
        assert np.abs(mlp.features(r, U, j) - mlp.features(r, U2, j)).max() < 1e-13


def test_gaussian_params_reproduce_the_exact_reduced_state():
    """The squeezed thermal state built from a mode's reduced covariance equals
    that mode's reduced density matrix of the exact GBS state (dense, large
    cutoff), and its spectrum is the Williamson one (eq. diagReducedGaussianDM)."""
    from oracle import mlp, lbo
    r, U = W.make_problem(3, 8, (0.3, 0.6))
    V = gbs.covariance(r, U)
    D = 16
    psi = gbs.exact_amplitudes(r, U, D)
    psi = psi / np.linalg.norm(psi)
    for j in range(3):
        y = mlp.gaussian_params(V, j)
        zeta, nbar = y[0] + 1j * y[1], math.expm1(y[2])
        Wb = mlp.squeezed_basis(zeta, 60, 40)
        lam = np.array([nbar ** k / (nbar + 1) ** (k + 1) for k in range(40)])
        rho_model = ((Wb * lam) @ Wb.conj().T)[:D, :D]
        rho = lbo.rdm_from_dense(psi, j)
        assert np.abs(rho - rho_model).max() < 1e-6
        assert np.abs(lam[:6] - lbo.gaussian_rdm_spectrum(V, j, 6)).max() < 1e-12


def test_two_mode_cutoff_error_equals_the_discarded_weight():
    """A pure two-mode Gaussian state is, in the two optimal local bases, a
    Schmidt sum over |k>|k> with weights sigma_k^2 (Sec. III.A.1), so keeping d
    states per mode gives eps_D = eps exactly (the lower bound of eq.
    SpecWfromSDsums met).  eps_D here is computed by brute force: exact
    amplitudes on a 40-photon box, each mode's top-d reduced eigenvectors,
    1 - |projection|^2."""
    from oracle import cutoff
    for seed in (1, 2, 3):
        r, U = W.make_problem(2, seed, (0.4, 0.8))
        V = gbs.covariance(r, U)
        psi = gbs.exact_amplitudes(r, U, 40)
        box_loss = 1.0 - np.linalg.norm(psi) ** 2
        assert box_loss < 1e-10
        for d in (2, 4):
            Ws = []
            for i in range(2):
                _, v = np.linalg.eigh(lbo.rdm_from_dense(psi, i))
                Ws.append(v[:, ::-1][:, :d])
            eps_D = 1.0 - np.linalg.norm(Ws[0].conj().T @ psi @ Ws[1].conj()) ** 2
            tails, eps, (lo, hi) = cutoff.eps_bounds(V, d)
            assert abs(eps_D - eps) < 1e-10 and abs(tails[0] - tails[1]) < 1e-12
            assert lo == eps and abs(hi - 2 * eps) < 1e-15


def test_cutoff_error_bounds_hold_for_three_modes():
    """eps <= eps_D <= N eps (eq. SpecWfromSDsums) with eps_D by brute force on
    a 22-photon box for three-mode Haar instances; the ratio eps / eps_D lies
    strictly inside [1/N, 1] for these generic states, as in Fig. 2."""
    from oracle import cutoff
    for seed in (4, 5, 6):
        r, U = W.make_problem(3, seed, (0.3, 0.6))
        V = gbs.covariance(r, U)
        psi = gbs.exact_amplitudes(r, U, 22)
        assert 1.0 - np.linalg.norm(psi) ** 2 < 1e-8       # far below eps_D (1e-4 .. 1e-2 here)
        Ws = []
        for i in range(3):
            _, v = np.linalg.eigh(lbo.rdm_from_dense(psi, i))
            Ws.append(v[:, ::-1][:, :3])
        proj = np.einsum("am,bn,co,abc->mno", Ws[0].conj(), Ws[1].conj(), Ws[2].conj(), psi)
        eps_D = 1.0 - np.linalg.norm(proj) ** 2
        _, eps, (lo, hi) = cutoff.eps_bounds(V, 3)
        assert lo < eps_D < hi
        assert 1 / 3 < eps / eps_D < 1


def test_effective_cutoff_of_the_squeezed_vacuum_closed_form():
    """With one kept vector the isometry defect at cutoff D is the squeezed
    vacuum's weight beyond D, sum_{2q >= D} tanh(r)^{2q} (2q)! / (4^q q!^2) /
    cosh r; the effective cutoff is the first D where that tail is within tol.
    With r = 0 the squeezed basis is the Fock basis: the effective cutoff is
    d itself."""
    from oracle import cutoff
    for r, tol in ((0.6, 1e-12), (1.1, 1e-10)):
        t = math.tanh(r)
        w = [t ** (2 * q) * math.comb(2 * q, q) / 4 ** q / math.cosh(r) for q in range(400)]
        tail = lambda D: 1.0 - sum(w[q] for q in range(400) if 2 * q < D)
        D_ref = next(D for D in range(1, 600) if tail(D) <= tol)
        zeta = r * np.exp(0.7j)
        assert cutoff.effective_cutoff(zeta, 1, 300, tol) == D_ref
    for d in (1, 3, 8):
        assert cutoff.effective_cutoff(0.0, d, 40, 1e-14) == d


def _split_dense(psi, d, N):
    """Exact MPS of a dense state by successive SVDs (no truncation)."""
    out, rest, cl = [], psi.reshape(1, -1), 1
    for s in range(N - 1):
        Uu, S, Vh = np.linalg.svd(rest.reshape(cl * d, -1), full_matrices=False)
        out.append(Uu.reshape(cl, d, -1))
        cl = len(S)
        rest = S[:, None] * Vh
    out.append(rest.reshape(cl, d, 1))
    return out


def test_energy_variance_against_dense_states():
    """<H^2> of the two-layer MPO contraction equals ||H psi||^2 with H the dense
    quadrature-form PHP (a separate construction), on random MPS, also with
    isometries where (PHP)^2 acts in the raw box; an eigenvector of PHP has
    sigma_H = 0 (Sec. II.E.2)."""
    for N, D, seed in ((3, 4, 1), (4, 3, 2)):
        r, U = W.make_problem(N, seed, (0.4, 0.8))
        al, be, ga = gbs.coefficients(r, U)
        ops = [operators.local_operators(D, al[s, s], be[s, s], ga[s, s]) for s in range(N)]
        Ws = mpo.cores(al, be, ga, ops)
        H = dense.php_quadrature(al, be, ga, D)
        state = W.random_mps(N, D, 4, seed + 10)
        psi = M.to_dense(state).reshape(-1)
        n2 = np.vdot(psi, psi).real
        e_ref = np.vdot(psi, H @ psi).real / n2
        h2_ref = np.linalg.norm(H @ psi) ** 2 / n2
        e, h2, var = dmrg.energy_variance(state, Ws)
        assert abs(e - e_ref) < 1e-10 * max(1, abs(e_ref)) and abs(h2 - h2_ref) < 1e-10 * h2_ref
        assert var > 1e-3
        # an eigenvector of PHP as an exact MPS
        w, v = np.linalg.eigh(H)
        e0, h20, var0 = dmrg.energy_variance(_split_dense(v[:, 0], D, N), Ws)
        assert abs(e0 - w[0]) < 1e-10 and abs(var0) < 1e-10
    # isometries: the physical state lives in the raw box, D = 5 -> d = 3
    N, D, d = 3, 5, 3
    r, U = W.make_problem(N, 7, (0.4, 0.8))
    al, be, ga = gbs.coefficients(r, U)
    ops = [operators.local_operators(D, al[s, s], be[s, s], ga[s, s]) for s in range(N)]
    Ws = mpo.cores(al, be, ga, ops)
    H = dense.php_quadrature(al, be, ga, D)
    rng = np.random.default_rng(3)
    iso = [np.linalg.qr(rng.normal(size=(D, d)) + 1j * rng.normal(size=(D, d)))[0] for _ in range(N)]
    state = W.random_mps(N, d, 4, 17)
    Psi = M.to_dense([np.einsum("im,amb->aib", Wi, A) for Wi, A in zip(iso, state)]).reshape(-1)
    n2 = np.vdot(Psi, Psi).real
    e_ref = np.vdot(Psi, H @ Psi).real / n2
    h2_ref = np.linalg.norm(H @ Psi) ** 2 / n2
    e, h2, var = dmrg.energy_variance(state, Ws, iso)
    assert abs(e - e_ref) < 1e-10 * max(1, abs(e_ref)) and abs(h2 - h2_ref) < 1e-10 * h2_ref


def test_cz_hamiltonian_annihilates_the_transformed_gaussian_state():
    """Sec. II.C.2: exp(-i kappa prod X) maps the Gaussian state to the zero
    mode of the literal Hamiltonian with y = (X, P + xi).  On a 14-photon box
    (three modes, r <= 0.35) <H> of the transformed exact amplitudes is at the
    box's truncation level, while the opposite sign of kappa, or the
    untransformed state, leave an energy of order kappa^2."""
    from oracle import cz
    N, B, kappa = 3, 14, 0.3
    r, U = W.make_problem(N, 12, (0.2, 0.35))
    al, be, ga = gbs.coefficients(r, U)
    psi = gbs.exact_amplitudes(r, U, B).reshape(-1)
    x, V = np.linalg.eigh(operators.quadratures(B)[0])
    V3 = np.kron(np.kron(V, V), V)
    phase = np.exp(-1j * kappa * np.einsum("a,b,c->abc", x, x, x)).reshape(-1)
    phi = V3 @ (phase * (V3.conj().T @ psi))
    assert abs(cz.expectation_literal(al, be, ga, kappa, B, phi)) < 1e-6
    assert cz.expectation_literal(al, be, ga, -kappa, B, phi) > 0.05
    assert cz.expectation_literal(al, be, ga, kappa, B, psi) > 0.01
    assert abs(cz.expectation_literal(al, be, ga, 0.0, B, psi)) < 1e-9


def test_cz_mpo_contracts_to_the_dense_hamiltonian():
    """The block MPO (Gaussian middle-site MPO + the H_1 and H_2 automata)
    contracts to PHP of the literal form; at kappa = 0 it is the Gaussian
    quadrature-form PHP; the integer structure has the stated bond dimensions."""
    from oracle import cz
    for N, D in ((3, 4), (4, 3), (2, 5)):
        r, U = W.make_problem(N, 11, (0.3, 0.6))
        al, be, ga, ops = cz.site_operators(r, U, D)
        for kappa in (0.0, 0.35):
            Hm = mpo.to_dense(cz.cores(al, be, ga, kappa, ops))
            Hd = cz.dense_php(al, be, ga, kappa, D)
            assert np.abs(Hm - Hd).max() < 1e-12
        assert np.abs(cz.dense_php(al, be, ga, 0.0, D) - dense.php_quadrature(al, be, ga, D)).max() < 1e-12
        w, kinds = cz.structure(N)
        wg = mpo.bond_dims(N)
        assert w == [wg[t] + (0 if t in (0, N) else 4 + 4 * t) for t in range(N + 1)]
        assert all(k.shape == (w[s], w[s + 1]) for s, k in enumerate(kinds))


# ------------------------------------------------------------------ pLBO (Sec. III.B)
def _plbo_blocks(d):
    from oracle import plbo
    return plbo.quadratic_blocks(d)


def test_plbo_single_gates_have_their_closed_forms():
    """Each gate of eq. pLBOUnitary alone, built by expm of its generator,
    transforms the quadratures as the textbook relations say: displacement
    shifts X, P by sqrt2 alpha; squeezing (phi = 0) scales X by e^-r and P by
    e^r; rotation turns (X, P); the quadratic phase adds s X to P; the cubic
    phase adds sqrt2 gamma X^2 to P; the Kerr gate multiplies <m|X|n> by
    exp(i kappa (n^2 - m^2)).  A wrong sign or factor in any generator fails."""
    from oracle import plbo
    d = 7
    X, P, X2, P2, Pt = _plbo_blocks(d)
    I = np.eye(d)

    def one(j, v):
        q = np.zeros(8)
        q[j] = v
        return plbo.transformed_ops(q, d, 1.0, 1.0, 0.0)

    Xt, Ptl, _, X2t, _ = one(0, 0.3)
    assert np.abs(Xt - (X + math.sqrt(2) * 0.3 * I)).max() < 1e-12
    assert np.abs(X2t - (X2 + 2 * math.sqrt(2) * 0.3 * X + 0.18 * I)).max() < 1e-12
    Xt, Ptl, *_ = one(1, -0.25)
    assert np.abs(Ptl - (P - math.sqrt(2) * 0.25 * I)).max() < 1e-12
    Xt, Ptl, *_ = one(2, 0.4)
    assert np.abs(Xt - math.exp(-0.4) * X).max() < 1e-12 and np.abs(Ptl - math.exp(0.4) * P).max() < 1e-12
    Xt, Ptl, *_ = one(4, 0.7)
    c, s = math.cos(0.7), math.sin(0.7)
    assert np.abs(Xt - (c * X - s * P)).max() < 1e-12 and np.abs(Ptl - (c * P + s * X)).max() < 1e-12
    Xt, Ptl, *_ = one(5, 0.3)
    assert np.abs(Xt - X).max() < 1e-12 and np.abs(Ptl - (P + 0.3 * X)).max() < 1e-12
    Xt, Ptl, *_ = one(6, 0.1)
    assert np.abs(Xt - X).max() < 1e-12 and np.abs(Ptl - (P + math.sqrt(2) * 0.1 * X2)).max() < 1e-12
    n = np.arange(d)
    Xt, *_ = one(7, 0.2)
    assert np.abs(Xt - X * np.exp(1j * 0.2 * (n[None, :] ** 2 - n[:, None] ** 2))).max() < 1e-12
    # a squeeze along phi = pi/2 exchanges the roles: X rotated by 45 degrees mixes
    Xt, Ptl, *_ = plbo.transformed_ops([0, 0, 0.4, math.pi, 0, 0, 0, 0], d, 1.0, 1.0, 0.0)
    assert np.abs(Xt - math.exp(0.4) * X).max() < 1e-12 and np.abs(Ptl - math.exp(-0.4) * P).max() < 1e-12


def test_plbo_composite_transform_matches_the_papers_closed_form():
    """eq. SymplecticBasisTransformation: U^dag a U written out with the
    Kerr phases, built at d + 4 and truncated (SM Sec. 5), gives the same
    X, P, X^2, P^2-bearing S and XP + PX as the definition (product of gate
    exponentials in 200 levels) for composite parameters, to 1e-10."""
    from oracle import plbo
    d, Db = 8, 12
    rng = np.random.default_rng(3)
    a = np.zeros((Db, Db), complex)
    for k in range(1, Db):
        a[k - 1, k] = math.sqrt(k)
    ad = a.conj().T
    nn = np.arange(Db, dtype=float)
    for _ in range(3):
        ax, ap, r, phi, th, s, g, kap = rng.uniform(-1, 1, 8) * [0.4, 0.4, 0.5, 3, 3, 0.3, 0.1, 0.1]
        e1, e2 = np.exp(1j * th), np.exp(1j * (phi - th))
        c1 = (1 + 0.5j * s) * e1 * math.cosh(r) + 0.5j * s * e2 * math.sinh(r)
        c2 = (1 - 0.5j * s) * e2 * math.sinh(r) - 0.5j * s * e1 * math.cosh(r)
        c3 = e1 * math.cosh(r) + e2 * math.sinh(r)
        K1 = np.diag(np.exp(1j * kap * (2 * nn - 1)))
        K3 = np.diag(np.exp(4j * kap * (nn - 1)))
        At = (c1 * a @ K1 - c2 * K1.conj() @ ad
              + 0.5j * g * c3 * (np.diag(2 * nn + 1) + a @ a @ K3 + K3.conj() @ ad @ ad)
              + (ax + 1j * ap) * np.eye(Db))
        Xb = (At + At.conj().T) / math.sqrt(2)
        Pb = -1j * (At - At.conj().T) / math.sqrt(2)
        cut = lambda M: M[:d, :d]
        want = (cut(Xb), cut(Pb), cut(0.5 * (1.1 * Xb @ Xb + 0.8 * Pb @ Pb + 0.3 * (Xb @ Pb + Pb @ Xb)) - 0.5 * np.eye(Db)),
                cut(Xb @ Xb), cut(Xb @ Pb + Pb @ Xb))
        got = plbo.transformed_ops([ax, ap, r, phi, th, s, g, kap], d, 1.1, 0.8, 0.3)
        for w, o in zip(want, got):
            assert np.abs(w - o).max() < 1e-10


def test_plbo_definition_is_converged_in_the_fock_cutoff():
    """The d x d transformed operators do not move when the expm space grows
    from 200 (the default) to 256 levels, at the edge of the test parameter
    range (the cubic phase spreads the basis states most)."""
    from oracle import plbo
    p = [0.3, -0.2, 0.45, 0.7, 0.5, 0.2, 0.1, 0.06]
    a = plbo.transformed_ops(p, 10, 1.2, 0.9, 0.2)
    b = plbo.transformed_ops(p, 10, 1.2, 0.9, 0.2, L=256)
    assert max(np.abs(x - y).max() for x, y in zip(a, b)) < 1e-10


@pytest.mark.parametrize("kappa", [0.0, 0.3])
def test_plbo_slot_environments_reproduce_the_energy(kappa):
    """E = sum_k <G_k, O_k>: with G_k from the core environment of a site and
    the slot coefficients of its core, the site energy equals <psi|H|psi> of
    the dense MPO and MPS, for the Fock operators and for pLBO operators at
    that site (Gaussian and global-CZ MPOs)."""
    from oracle import plbo, cz
    N, d, site = 4, 4, 2
    r, U = W.make_problem(N, 5, (0.3, 0.6))
    al, be, ga = gbs.coefficients(r, U)
    rng = np.random.default_rng(8)
    dims = [1, 3, 5, 3, 1]
    mps = [rng.normal(size=(dims[s], d, dims[s + 1])) + 1j * rng.normal(size=(dims[s], d, dims[s + 1]))
           for s in range(N)]
    p = [0.2, -0.1, 0.3, 0.4, 0.2, 0.1, 0.05, 0.04]
    ops = [cz.local_ops(d, al[s, s], be[s, s], ga[s, s]) for s in range(N)]
    ops[site] = plbo.transformed_ops(p, d, al[site, site], be[site, site], ga[site, site])
    Ws = cz.cores(al, be, ga, kappa, ops) if kappa else mpo.cores(al, be, ga, [o[:3] for o in ops])
    psi = M.to_dense(mps)
    E = np.real(psi.conj() @ mpo.to_dense(Ws) @ psi)
    Ls = dmrg.left_envs(mps, Ws)
    Rs = dmrg.right_envs(mps, Ws)
    Gf = plbo.core_environment(Ls[site], mps[site], Rs[site + 1])
    mk = (plbo.cz_core_maker(al, be, ga, kappa, site) if kappa else plbo.gaussian_core_maker(al, be, ga, site))
    G = plbo.slot_gradients(Gf, plbo.slot_coefficients(mk, d))
    assert abs(plbo.site_energy(G, ops[site]) - E) < 1e-9 * max(1.0, abs(E))


def test_plbo_parameter_gradient_closed_forms():
    """At p = 0 the derivatives of the operators are closed forms: d/dalpha_x
    gives (sqrt2 I, 0, S', 2 sqrt2 X, 2 sqrt2 P) and d/dtheta gives
    (-P, X, ., -(XP+PX), 2(X^2 - P^2)).  The five-point difference of the
    site energy matches Re <G, dO> for a random G."""
    from oracle import plbo
    d, a_ss, b_ss, g_ss = 6, 1.3, 0.7, 0.2
    rng = np.random.default_rng(4)
    G = rng.normal(size=(6, d, d)) + 1j * rng.normal(size=(6, d, d))
    X, P, X2, P2, Pt = _plbo_blocks(d)
    g = plbo.param_gradient(G, np.zeros(8), d, a_ss, b_ss, g_ss, L=64)
    r2 = math.sqrt(2)

    def dE(dX, dP, dX2, dP2, dPt):
        dS = 0.5 * (a_ss * dX2 + b_ss * dP2 + g_ss * dPt)
        return sum(np.real(np.sum(G[k + 1] * o)) for k, o in enumerate((dX, dP, dS, dX2, dPt)))

    Z = np.zeros((d, d))
    assert abs(g[0] - dE(r2 * np.eye(d), Z, 2 * r2 * X, Z, 2 * r2 * P)) < 1e-8
    assert abs(g[1] - dE(Z, r2 * np.eye(d), Z, 2 * r2 * P, 2 * r2 * X)) < 1e-8
    assert abs(g[4] - dE(-P, X, -Pt, Pt, 2 * (X2 - P2))) < 1e-8


def test_plbo_adam_first_step_moves_each_free_parameter_by_lr():
    """Adam's bias correction makes the first update lr * g / (|g| + eps): a
    step of lr against the sign of every free gradient component, none on
    masked ones."""
    from oracle import plbo
    g0 = np.array([0.5, -2.0, 1e-3, 3.0, -0.1, 0.2, 7.0, -4.0])
    mask = [1, 1, 1, 1, 0, 1, 1, 1]
    p, st = plbo.adam(np.zeros(8), lambda q: g0, 1, 0.01, mask=mask)
    want = np.where(np.array(mask, bool), -0.01 * np.sign(g0), 0.0)
    assert np.abs(p - want).max() < 1e-7 and st[2] == 1


def test_plbo_product_of_squeezed_vacua_is_exact_with_one_basis_state():
    """With no interferometer the output state is a product of squeezed vacua,
    so a one-state pLBO basis S(r_i e^{i phi})|0> on every mode is exact and
    its energy is 0 for the right orientation of the squeeze, while the Fock
    vacuum (p = 0) sits at the sum of the single-mode energies > 0."""
    from oracle import plbo
    r = np.array([0.5, 0.3])
    U = np.eye(2, dtype=complex)
    al, be, ga = gbs.coefficients(r, U)
    best = []
    for phi in (0.0, math.pi):
        ops = [plbo.transformed_ops([0, 0, r[s], phi, 0, 0, 0, 0], 1, al[s, s], be[s, s], ga[s, s]) for s in range(2)]
        Ws = mpo.cores(al, be, ga, [o[:3] for o in ops])
        best.append(np.real(mpo.to_dense(Ws)[0, 0]))
    assert min(best) < 1e-10 and max(best) > 0.1
    ops0 = [plbo.transformed_ops(np.zeros(8), 1, al[s, s], be[s, s], ga[s, s]) for s in range(2)]
    assert np.real(mpo.to_dense(mpo.cores(al, be, ga, [o[:3] for o in ops0]))[0, 0]) > 0.1


# ------------------------------------------------------------------ noisy GBS (Sec. II.F)
def test_noisy_decomposition_is_pure_plus_classical():
    """eq. CovarianceDecomposition for uniform loss: Q = covariance(r', U) is
    pure (all symplectic eigenvalues 1/2), C = V_eta - Q is positive
    semidefinite with rank N, C = L L^T, and eta = 1 gives Q = V, C = 0."""
    from oracle import noisy
    r, U = W.make_problem(5, 3, (0.4, 1.1))
    for eta in (1.0, 0.9, 0.5):
        rp, C, L = noisy.decompose_uniform_loss(r, U, eta)
        Q = gbs.covariance(rp, U)
        V = noisy.lossy_covariance(r, U, eta)
        assert np.abs(Q + C - V).max() < 1e-12
        assert np.abs(noisy.symplectic_eigenvalues(Q) - 0.5).max() < 1e-10
        ev = np.linalg.eigvalsh(C)
        assert ev.min() > -1e-12
        assert np.abs(L @ L.T - C).max() < 1e-12
        if eta == 1.0:
            assert np.abs(rp - r).max() < 1e-14 and np.abs(C).max() < 1e-14
        else:
            assert (rp < r).all() and (rp > 0).all()
            assert np.sum(ev > 1e-12) == 5
    # the symplectic eigenvalues of the lossy V exceed 1/2 (it is mixed)
    assert noisy.symplectic_eigenvalues(noisy.lossy_covariance(r, U, 0.7)).max() > 0.55


def test_noisy_pure_part_has_the_smallest_trace_per_mode():
    """Per input mode, every pure Q_i = 1/2 diag(q, 1/q) below V_i (V_i - Q_i
    >= 0) has a trace no smaller than the closed-form choice (scan over q)."""
    from oracle import noisy
    for r, eta in ((0.8, 0.6), (0.3, 0.9), (1.2, 0.3)):
        rp, C, _ = noisy.decompose_uniform_loss(np.array([r]), np.eye(1, dtype=complex), eta)
        vx, vp = eta * math.exp(-2 * r) + 1 - eta, eta * math.exp(2 * r) + 1 - eta
        q0 = math.exp(-2 * rp[0])
        assert q0 <= vx + 1e-14 and 1 / q0 <= vp + 1e-14           # feasible
        qs = np.linspace(1e-3, 10, 200001)
        feas = (qs <= vx) & (1 / qs <= vp)
        best = np.min(qs[feas] + 1 / qs[feas])
        assert best >= q0 + 1 / q0 - 1e-12 and best - (q0 + 1 / q0) < 1e-3


def test_displacement_matrix_closed_forms():
    """<n|D(alpha)|0> is the coherent state e^{-|a|^2/2} a^n/sqrt(n!);
    D(a) D(b) = e^{(a b^* - a^* b)/2} D(a + b) and D(a) D(-a) = I on the kept
    levels (expm in 160 levels, |alpha| <= 0.8, 12 kept)."""
    from oracle import noisy
    a, b = 0.5 - 0.3j, -0.2 + 0.6j
    Dm = noisy.displacement_matrix(a, 12)
    coh = np.array([np.exp(-abs(a) ** 2 / 2) * a ** n / math.sqrt(math.factorial(n)) for n in range(12)])
    assert np.abs(Dm[:, 0] - coh).max() < 1e-13
    big = 40
    Da, Db = noisy.displacement_matrix(a, big), noisy.displacement_matrix(b, big)
    Dab = noisy.displacement_matrix(a + b, big)
    ph = np.exp(0.5 * (a * np.conj(b) - np.conj(a) * b))
    assert np.abs((Da @ Db)[:12, :12] - ph * Dab[:12, :12]).max() < 1e-12
    assert np.abs((Da @ noisy.displacement_matrix(-a, big))[:12, :12] - np.eye(12)).max() < 1e-12


def test_gaussian_photon_distribution_closed_forms():
    """Squeezed vacuum: the closed form of gbs; thermal: geometric; a rotated
    squeezed thermal state has the photon numbers of the unrotated one."""
    from oracle import noisy
    r = 0.7
    P = noisy.gaussian_photon_distribution(0.5 * np.diag([math.exp(-2 * r), math.exp(2 * r)]), 20)
    assert np.abs(P - gbs.single_mode_probabilities(r, 20)).max() < 1e-13
    nb = 0.8
    P = noisy.gaussian_photon_distribution((nb + 0.5) * np.eye(2), 20)
    q = nb / (nb + 1)
    assert np.abs(P - (1 - q) * q ** np.arange(20)).max() < 1e-13
    V = np.diag([0.4, 1.9])
    c, s = math.cos(0.7), math.sin(0.7)
    R = np.array([[c, -s], [s, c]])
    assert np.abs(noisy.gaussian_photon_distribution(R @ V @ R.T, 20)
                  - noisy.gaussian_photon_distribution(V, 20)).max() < 1e-12


def test_displaced_pure_part_averages_to_the_lossy_state():
    """One lossy squeezed mode: averaging the photon distribution of
    D(alpha)|psi_Q> over alpha ~ N(0, C) (Gauss-Hermite, 80 nodes along the
    noisy quadrature) gives the photon distribution of V_eta = Q + C."""
    from oracle import noisy
    r, eta = np.array([0.9]), 0.6
    U = np.eye(1, dtype=complex)
    rp, C, L = noisy.decompose_uniform_loss(r, U, eta)
    Lb = 120
    psi = np.zeros(Lb, dtype=complex)
    psi[:] = 0.0
    x, wts = np.polynomial.hermite_e.hermegauss(80)        # weight exp(-x^2/2)
    wts = wts / wts.sum()
    # pure squeezed vacuum of Q in the x-squeezed convention: S(r') with the
    # oracle's squeezing sign is checked through its covariance below
    a = np.zeros((Lb, Lb), dtype=complex)
    for n in range(1, Lb):
        a[n - 1, n] = math.sqrt(n)
    import scipy.linalg as sla
    vac = np.zeros(Lb, dtype=complex)
    vac[0] = 1.0
    psi = sla.expm(0.5 * rp[0] * (a @ a - a.conj().T @ a.conj().T)) @ vac
    X = (a + a.conj().T) / math.sqrt(2)
    P_ = -1j * (a - a.conj().T) / math.sqrt(2)
    Q = gbs.covariance(rp, U)
    assert abs(np.real(psi.conj() @ (X @ X)[:, :] @ psi) - Q[0, 0]) < 1e-10
    assert abs(np.real(psi.conj() @ (P_ @ P_) @ psi) - Q[1, 1]) < 1e-10
    mix = np.zeros(30)
    for xi, wi in zip(x, wts):
        alpha = noisy.alphas(np.array([[xi]]), L)[0, 0]
        phi = noisy.displacement_matrix(alpha, Lb, L=Lb + 80) @ psi
        mix += wi * np.abs(phi[:30]) ** 2
    want = noisy.gaussian_photon_distribution(noisy.lossy_covariance(r, U, eta), 30)
    assert np.abs(mix - want).max() < 1e-10


def test_displaced_sampler_reduces_to_the_plain_sampler():
    """alpha = 0 leaves the sequential sampler unchanged (same Philox stream);
    for one mode its empirical distribution is |<n|D(alpha)|psi>|^2."""
    from oracle import noisy, sampler
    rng = np.random.default_rng(6)
    t = [rng.normal(size=(1, 5, 3)) + 1j * rng.normal(size=(1, 5, 3)),
         rng.normal(size=(3, 5, 2)) + 1j * rng.normal(size=(3, 5, 2)),
         rng.normal(size=(2, 5, 1)) + 1j * rng.normal(size=(2, 5, 1))]
    t = M.right_canonicalize(t)
    a = np.zeros((40, 3), dtype=complex)
    assert np.array_equal(noisy.sample_displaced(t, a, 17, L=40), sampler.sample(t, 40, 17))
    psi = np.array([0.8, 0.0, 0.6, 0.0], dtype=complex)
    al = 0.3 + 0.2j
    smp = noisy.sample_displaced([psi.reshape(1, 4, 1)], np.full((3000, 1), al), 5, L=60)[:, 0]
    p = np.abs(noisy.displacement_matrix(al, 4, 60) @ psi) ** 2
    p /= p.sum()
    hist = np.bincount(smp, minlength=4) / 3000.0
    assert np.abs(hist - p).max() < 4 * math.sqrt(0.25 / 3000)


def test_plbo_site_minimiser_finds_the_squeezed_vacuum():
    """One squeezed mode, one basis state: the oracle's site minimiser over
    (r, phi) drives the energy to 0 with |r| equal to the instance's squeezing."""
    from oracle import plbo
    r = np.array([0.5])
    al, be, ga = gbs.coefficients(r, np.eye(1, dtype=complex))
    G = np.zeros((6, 1, 1), dtype=complex)
    G[3, 0, 0] = 1.0                        # N = 1: the Hamiltonian is the site operator S
    mask = [0, 0, 1, 1, 0, 0, 0, 0]
    p, E = plbo.minimize_site(G, [0, 0, 0.1, 0.3, 0, 0, 0, 0], 1, al[0, 0], be[0, 0], ga[0, 0], mask, L=40)
    assert abs(E) < 1e-10 and abs(abs(p[2]) - 0.5) < 1e-5


def test_williamson_split_of_a_general_mixed_state():
    """Williamson decomposition V = S diag(nu, nu) S^T of a mixed covariance
    (uniform loss plus thermal noise): S is symplectic, nu are the symplectic
    eigenvalues (moduli of eig(i Omega V)), Q = S S^T/2 is pure and
    C = V - Q >= 0; for uniform loss alone the pure part's squeezing is the
    closed form r_W = ln(v_p / v_x)/4 per input mode, and it carries more
    photons than the minimal-trace split (the order of the paper's table)."""
    from oracle import noisy
    r, U = W.make_problem(5, 3, (0.4, 1.1))
    V = noisy.lossy_covariance(r, U, 0.6) + 0.1 * np.eye(10)
    nu, S = noisy.williamson(V)
    Om = noisy._omega(5)
    assert np.abs(S @ Om @ S.T - Om).max() < 1e-12
    assert np.abs(S @ np.diag(np.concatenate([nu, nu])) @ S.T - V).max() < 1e-12
    assert np.abs(np.sort(nu) - noisy.symplectic_eigenvalues(V)[::2]).max() < 1e-10
    Q, C = noisy.decompose_williamson(V)
    assert np.abs(noisy.symplectic_eigenvalues(Q) - 0.5).max() < 1e-10
    assert np.linalg.eigvalsh(C).min() > -1e-12 and np.abs(Q + C - V).max() < 1e-12
    L = noisy.factor_psd(C)
    assert np.abs(L @ L.T - C).max() < 1e-12
    Vl = noisy.lossy_covariance(r, U, 0.6)
    Ql, _ = noisy.decompose_williamson(Vl)
    rw, Uw = noisy.pure_state_parameters(Ql)
    vx, vp = 0.6 * np.exp(-2 * r) + 0.4, 0.6 * np.exp(2 * r) + 0.4
    assert np.abs(np.sort(rw) - np.sort(0.25 * np.log(vp / vx))).max() < 1e-10
    rk, _, _ = noisy.decompose_uniform_loss(r, U, 0.6)
    assert np.sum(np.sinh(rw) ** 2) > np.sum(np.sinh(rk) ** 2)


def test_pure_state_parameters_invert_the_covariance():
    """(r, U) from a pure covariance: covariance(r, U) reproduces it, U is
    unitary and r matches the squeezing as a set; also with unsqueezed modes
    (a degenerate eigenvalue 1/2)."""
    from oracle import noisy
    for r0, seed in (((0.3, 0.8, 0.5, 1.1), 2), ((0.0, 0.6, 0.0), 4)):
        r0 = np.array(r0)
        U0 = W.make_problem(len(r0), seed, (0.5, 0.5))[1]
        Q = gbs.covariance(r0, U0)
        r, U = noisy.pure_state_parameters(Q)
        assert np.abs(gbs.covariance(r, U) - Q).max() < 1e-12
        assert np.abs(U @ U.conj().T - np.eye(len(r0))).max() < 1e-12
        assert np.abs(np.sort(r) - np.sort(r0)).max() < 1e-10


def test_plbo_effective_cutoff_special_cases():
    """The pLBO basis's effective cutoff: the Fock basis (p = 0) needs exactly
    d levels; a pure squeeze S(r e^{i phi}) gives the squeezed basis's
    effective cutoff of the analytic-basis report (cutoff.effective_cutoff,
    built independently); a displacement needs more levels than no
    displacement."""
    from oracle import plbo, cutoff
    assert plbo.effective_cutoff(np.zeros(8), 5, 60, 1e-10) == 5
    for r, phi in ((0.5, 0.0), (0.8, 1.1)):
        p = np.zeros(8)
        p[2], p[3] = r, phi
        assert plbo.effective_cutoff(p, 4, 120, 1e-10) == cutoff.effective_cutoff(r * np.exp(1j * phi), 4, 120, 1e-10)
    q = np.zeros(8)
    q[0] = 0.5
    assert plbo.effective_cutoff(q, 4, 120, 1e-10) > 4


# --------------------------------------------------------------- pins of the
# optimiser, the joint LBO sweep and the learned product state
def test_adam_steps_follow_the_kingma_ba_closed_forms():
    """Adam (Kingma & Ba, Algorithm 1) with bias correction: under a constant
    gradient every step moves each parameter by exactly lr * g / (|g| + eps),
    so t steps move it t times that; after one gradient g and then a zero
    gradient, the second step is lr * (b1 / (1 + b1)) / sqrt(b2 / (1 + b2)) *
    sign(g) (0.670059 lr for 0.9 / 0.999), and the update is unchanged when
    every gradient is scaled by a constant (up to eps)."""
    from oracle import mlp
    rng = np.random.default_rng(5)
    params = mlp.init_params(rng, in_dim=5, hidden=7, out_dim=3)
    p0 = mlp.flatten(params)
    g = rng.standard_normal(p0.size) * rng.choice([1e-3, 1.0, 30.0], p0.size)
    grads = mlp.unflatten(g, 5, 7, 3)
    lr = 1e-2
    state = (np.zeros_like(p0), np.zeros_like(p0), 0)
    p = params
    for t in range(1, 6):
        p, state = mlp.adam(p, grads, state, lr)
        moved = mlp.flatten(p) - p0
        assert np.abs(moved + t * lr * g / (np.abs(g) + 1e-8)).max() < 1e-13
    assert state[2] == 5
    # one gradient, then zero: the hand-derived second step
    state = (np.zeros_like(p0), np.zeros_like(p0), 0)
    p1, state = mlp.adam(params, grads, state, lr)
    p2, state = mlp.adam(p1, mlp.unflatten(np.zeros_like(g), 5, 7, 3), state, lr)
    step2 = mlp.flatten(p2) - mlp.flatten(p1)
    ratio = (0.9 / 1.9) / math.sqrt(0.999 / 1.999)
    assert abs(ratio - 0.670059) < 1e-6
    big = np.abs(g) > 1.0           # where eps is negligible against |g|
    assert np.abs(step2[big] + lr * ratio * np.sign(g[big])).max() < 1e-8 * lr
    # scale invariance over a varying gradient sequence
    seq = [rng.standard_normal(p0.size) for _ in range(4)]
    outs = []
    for c in (1.0, 1e3):
        st = (np.zeros_like(p0), np.zeros_like(p0), 0)
        q = params
        for gg in seq:
            q, st = mlp.adam(q, mlp.unflatten(c * gg, 5, 7, 3), st, lr)
        outs.append(mlp.flatten(q))
    # eps / |g| stays below 1e-5 for these draws
    assert np.abs(outs[0] - outs[1]).max() < 1e-5 * lr


def test_initial_product_state_is_thermal_in_the_squeezed_basis():
    """The learned product state: squared amplitudes are the Boltzmann weights
    exp(-beta m) / Z over the d kept levels with beta = log(1 + 1/nbar) (a
    thermal state of mean photon number nbar, eq. diagReducedGaussianDM), and
    the basis columns are S(zeta)|m> with S(zeta) = exp(1/2 (zeta* a^2 -
    zeta a^dag^2)) taken by scipy's expm on a large box."""
    import scipy.linalg
    from oracle import mlp
    D, d = 60, 5
    y = np.array([[0.30, -0.20, math.log1p(0.40)],
                  [-0.10, 0.45, math.log1p(0.05)],
                  [0.0, 0.0, math.log1p(1.30)]])
    isos, amps = mlp.initial_product_state(y, D, d)
    Db = 200
    a = np.diag(np.sqrt(np.arange(1, Db)), 1).astype(complex)
    for yj, Wj, cj in zip(y, isos, amps):
        nbar = math.expm1(yj[2])
        beta = math.log(1.0 + 1.0 / nbar)
        w = np.exp(-beta * np.arange(d))
        assert np.abs(cj ** 2 - w / w.sum()).max() < 1e-13
        assert abs(np.sum(cj ** 2) - 1.0) < 1e-14
        zeta = complex(yj[0], yj[1])
        S = scipy.linalg.expm(0.5 * (np.conj(zeta) * a @ a - zeta * a.T @ a.T))
        ref = S[:D, :d]
        # the cut to D rows is re-orthonormalised; the rows beyond D carry < 1e-12 here
        assert np.abs(Wj - ref).max() < 1e-10
        assert np.abs(Wj.conj().T @ Wj - np.eye(d)).max() < 1e-13


def test_joint_lbo_sweep_reaches_the_product_state_energy():
    """dmrg_lbo itself on U = identity with one basis state per mode: the state
    is a product of single-mode squeezed vacua, so the sweeps must end at the
    sum of the single-mode ground energies of the cutoff-D problems, with each
    basis vector the single-mode ground state (Sec. III.A: the optimal local
    basis of a product state has one element)."""
    from oracle import lbo
    N, D, d = 3, 10, 1
    r = np.array([0.3, 0.5, 0.4])
    U = np.eye(N, dtype=complex)
    iso = [np.eye(D)[:, :d].astype(complex) for _ in range(N)]
    mps_ = [np.ones((1, d, 1), dtype=complex) for _ in range(N)]
    mps_, iso, st = lbo.dmrg_lbo(mps_, r, U, D, iso, chi=1, sweeps=2)
    _, _, _, raw = lbo.local_ops(r, U, D)
    E_single = sum(np.linalg.eigvalsh(raw[s][2])[0] for s in range(N))
    assert abs(st[-1]["energy"] - E_single) < 1e-10
    for s in range(N):
        gs = np.linalg.eigh(raw[s][2])[1][:, 0]
        assert abs(abs(np.vdot(gs, iso[s][:, 0])) - 1.0) < 1e-8


def test_joint_lbo_sweep_finds_the_gaussian_optimal_bases():
    """dmrg_lbo on a three-mode Haar instance at full bond dimension:
    * the final MPS is the ground state of PHP in its final bases (dense ED of
      (W0 x W1 x W2)^dag PHP (W0 x W1 x W2)), which a sweep that built its
      environments in a stale basis would miss;
    * the kept bases are the Gaussian optimum of Sec. III.A.1: each mode's
      reduced density matrix in its kept basis has the spectrum
      nbar^k / (nbar + 1)^(k + 1) (eq. diagReducedGaussianDM), and the kept
      basis holds all but the optimal tail sum_{k >= d} lambda_k of the exact
      state's reduced density matrix (eq. SVDPhysicalDimension), far more than
      the first d Fock states hold;
    * the energy lies below the same sweeps' energy in the first d Fock states."""
    from oracle import lbo, mps as M
    N, D, d = 3, 10, 5
    r, U = _small_problem(3, 0, (0.3, 0.25, 0.35))
    V = gbs.covariance(r, U)
    al, be, ga, raw = lbo.local_ops(r, U, D)
    iso0 = [np.eye(D)[:, :d].astype(complex) for _ in range(N)]
    m0 = W.random_mps(N, d, d, 7)
    H = dense.php_quadrature(al, be, ga, D)

    def ed_in(iso):
        Wk = np.kron(np.kron(iso[0], iso[1]), iso[2])
        return np.linalg.eigvalsh(Wk.conj().T @ H @ Wk)[0]

    # after one sweep the bases still move by much at every step: the last
    # two-site update (full rank, so exact in its bases) must have used the
    # basis the LBO step just chose
    _, iso1, st1 = lbo.dmrg_lbo([a.copy() for a in m0], r, U, D, iso0, chi=d, sweeps=1)
    assert abs(st1[-1]["energy"] - ed_in(iso1)) < 1e-12
    m_lbo, iso, st = lbo.dmrg_lbo([a.copy() for a in m0], r, U, D, iso0, chi=d, sweeps=4)
    E = st[-1]["energy"]
    assert abs(E - ed_in(iso)) < 1e-12
    # the Fock-basis run of the same sweeps (no basis update) is worse
    cores_fock = lbo.cores_in_basis(al, be, ga, raw, iso0)
    _, st_fock = dmrg.dmrg([a.copy() for a in m0], cores_fock, d, 4, tol=1e-12)
    assert E < st_fock[-1]["energy"] - 1e-6
    rho = M.reduced_density_matrices(m_lbo)
    psi_x = gbs.exact_amplitudes(r, U, 40)      # the box holds all but < 1e-12
    psi_x = psi_x / np.linalg.norm(psi_x)
    tail_all = sum(lbo.gaussian_rdm_spectrum(V, i, 60)[d:].sum() for i in range(N))
    for i in range(N):
        lam = lbo.gaussian_rdm_spectrum(V, i, d)
        ev = np.sort(np.linalg.eigvalsh(rho[i]))[::-1]
        tail = lbo.gaussian_rdm_spectrum(V, i, 60)[d:].sum()
        # the truncated ground state differs from P psi at first order in the
        # discarded amplitude, sqrt of all modes' tails together
        assert np.abs(ev - lam / lam.sum()).max() < 0.1 * math.sqrt(tail_all)
        rho_x = lbo.rdm_from_dense(psi_x, i)[:D, :D]
        lost = 1.0 - np.trace(iso[i].conj().T @ rho_x @ iso[i]).real
        lost_fock = 1.0 - np.trace(rho_x[:d, :d]).real
        assert lost < 1e-6 + 2 * tail and lost < 0.02 * lost_fock


def test_noise_normals_are_standard_normal():
    """The oracle's noise draws (Box-Muller of Philox blocks): 20000 draws pass
    a Kolmogorov-Smirnov test against N(0, 1) and have its first four moments;
    the blocks with last counter word 1 are not the photon-number draws."""
    import scipy.stats
    from oracle import sampler
    z = np.array([sampler.normal(b, i, 77) for b in range(5000) for i in range(4)])
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(np.mean(z ** 3)) < 5 * math.sqrt(15.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 5 * math.sqrt(96.0 / n)
    u = np.array([sampler.uniform(b, i, 77) for b in range(200) for i in range(4)])
    zz = z[:800]
    assert abs(np.corrcoef(u, zz)[0, 1]) < 5 / math.sqrt(800)


def test_sampler_reports_rounding_ties():
    """pick_outcome flags a draw as a tie exactly when u lies within 1e-12 of
    a cumulative sum; the stream comparison ignores a sample only from its
    first tie on."""
    from oracle import sampler
    p = np.array([0.25, 0.25, 0.5])
    assert sampler.pick_outcome(p, 0.25) == (0, True)
    assert sampler.pick_outcome(p, 0.25 + 1e-9) == (1, False)
    assert sampler.pick_outcome(p, 0.1) == (0, False)
    assert sampler.pick_outcome(np.array([0.0, 0.5, 0.5]), 0.0) == (1, True)
    ref = np.array([[1, 2, 3], [1, 2, 3]])
    got = np.array([[1, 2, 4], [1, 0, 3]])
    assert sampler.stream_mismatches(got, ref, np.array([2, 3])) == (0 + 1, 1)
    assert sampler.stream_mismatches(got, ref, np.array([2, 1])) == (0, 2)
