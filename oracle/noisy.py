"""Noisy GBS as a pure state plus classical displacements (oracle; test
infrastructure only).

Two splits are kept: the closed form for uniform loss below, and for a
general mixed covariance the Williamson decomposition V = S diag(nu, nu) S^T
with Q = S S^T/2 and C = S (diag(nu, nu) - I/2) S^T (the pure states of the
first column of the paper's photon table); the pure part's (r, U) comes from
its eigenvectors (Bloch-Messiah form).

Sec. II.F, eq. CovarianceDecomposition: a mixed covariance V is split as
V = Q + C with Q the covariance of a pure state and C >= 0 the covariance of
zero-mean Gaussian random displacements; a sample of the noisy experiment is a
photon-number sample of D(alpha)|psi_Q> with alpha drawn from N(0, C).

Noise model of the synthetic instances: uniform loss eta after the squeezers
(it commutes with the passive interferometer), V_eta = eta V + (1 - eta) I/2
with V = 1/2 O diag(e^{-2r}, e^{2r}) O^T.  Per input mode the lossy variances
are v_x = (eta e^{-2r} + 1 - eta)/2 and v_p = (eta e^{2r} + 1 - eta)/2.  The
paper finds Q by semi-definite programming (the pure state with the fewest
photons); for this model the decomposition is taken in closed form: keep the
squeezed variance, Q_i = 1/2 diag(e^{-2r'}, e^{2r'}) with e^{-2r'} = 2 v_x,
and put the rest in the anti-squeezed quadrature, C_i = diag(0, v_p - e^{2r'}/2).
Among pure single-mode Q_i <= V_i this Q_i has the smallest trace (checked
by a scan in the tests).  Quadrature order (x_1..x_N, p_1..p_N); a
displacement d = (d_x, d_p) of mode j is alpha_j = (d_x + i d_p)/sqrt(2).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import gbs, sampler


def lossy_covariance(r, U, eta: float) -> np.ndarray:
    """V_eta = eta V + (1 - eta) I/2 (uniform loss channel on every mode)."""
    V = gbs.covariance(r, U)
    return eta * V + (1.0 - eta) * 0.5 * np.eye(V.shape[0])


def decompose_uniform_loss(r, U, eta: float):
    """(r_pure, C, L) with Q = covariance(r_pure, U), C = V_eta - Q >= 0 and
    C = L L^T, L of shape (2N, N)."""
    r = np.asarray(r, dtype=np.float64)
    N = len(r)
    vx = eta * np.exp(-2 * r) + 1 - eta          # 2 v_x
    vp = eta * np.exp(2 * r) + 1 - eta           # 2 v_p
    rp = -0.5 * np.log(vx)
    c = 0.5 * (vp - np.exp(2 * rp))              # variance added to p of input mode i
    O = gbs.quadrature_rotation(U)
    L = O[:, N:] * np.sqrt(np.maximum(c, 0.0))[None, :]
    return rp, L @ L.T, L


def symplectic_eigenvalues(V: np.ndarray) -> np.ndarray:
    """Moduli of the eigenvalues of i Omega V (each appears twice)."""
    N = V.shape[0] // 2
    Om = np.block([[np.zeros((N, N)), np.eye(N)], [-np.eye(N), np.zeros((N, N))]])
    ev = np.abs(np.linalg.eigvals(1j * Om @ V))
    return np.sort(ev)


def displacement_matrix(alpha: complex, D: int, L: int = 160) -> np.ndarray:
    """<n|D(alpha)|k>, n, k < D, from expm(alpha a^dag - alpha^* a) in L levels."""
    a = np.zeros((L, L), dtype=np.complex128)
    for n in range(1, L):
        a[n - 1, n] = math.sqrt(n)
    return sla.expm(alpha * a.conj().T - np.conj(alpha) * a)[:D, :D].copy()


def alphas(z, L):
    """alpha[b, j] = (d_x + i d_p)/sqrt2 with d = L z_b (z: (B, N) standard normals)."""
    d = np.asarray(z) @ np.asarray(L).T           # (B, 2N)
    N = d.shape[1] // 2
    return (d[:, :N] + 1j * d[:, N:]) / math.sqrt(2.0)


def sample_displaced(fock_tensors, alpha, seed: int, L: int = 160, with_ties: bool = False):
    """Samples of D(alpha_b)|psi> for each row alpha_b: the sequential
    conditional sampler of oracle.sampler (same Philox uniforms and inverse-CDF
    rule) with each site's Fock tensor replaced by D(alpha_{b,s}) A^F_s over the
    D kept Fock levels.  With with_ties, also each sample's first rounding-tie
    site (N if none), as in oracle.sampler.sample."""
    alpha = np.asarray(alpha)
    B, N = alpha.shape
    out = np.zeros((B, N), dtype=np.int64)
    first_tie = np.full(B, N, dtype=np.int64)
    cache = {}
    for b in range(B):
        v = np.ones(1, dtype=np.complex128)
        for s, A in enumerate(fock_tensors):
            D = A.shape[1]
            T = np.tensordot(v, A, axes=([0], [0]))                 # (D, chi_r)
            key = (complex(alpha[b, s]), D)
            if key not in cache:
                cache[key] = displacement_matrix(alpha[b, s], D, L)
            T = cache[key] @ T
            p = np.sum(np.abs(T) ** 2, axis=1)
            u = sampler.uniform(b, s, seed) * p.sum()
            pick, tie = sampler.pick_outcome(p, u)
            if tie and first_tie[b] == N:
                first_tie[b] = s
            out[b, s] = pick
            v = T[pick] / np.sqrt(p[pick])
    return (out, first_tie) if with_ties else out


def library_normals(n_samples: int, K: int, seed: int):
    """z[b][i] = oracle.sampler.normal(b, i, seed): the noise draws the library
    makes itself when the caller passes none."""
    return np.array([[sampler.normal(b, i, seed) for i in range(K)] for b in range(n_samples)])


def gaussian_photon_distribution(V2: np.ndarray, nmax: int, L: int = 160) -> np.ndarray:
    """P(n), n < nmax, of the zero-mean single-mode Gaussian state with
    covariance V2 (2 x 2, vacuum = I/2).  The state is a rotated squeezed
    thermal state, nbar = sqrt(det V2) - 1/2 and e^{4r} = ratio of the
    eigenvalues of V2; photon numbers do not see the rotation, so
    S(r) rho_th S(r)^dag is built in L levels (expm) and its diagonal read."""
    nbar = max(math.sqrt(np.linalg.det(V2)) - 0.5, 0.0)
    w = np.linalg.eigvalsh(V2)
    r = 0.25 * math.log(w[1] / w[0])
    a = np.zeros((L, L), dtype=np.complex128)
    for n in range(1, L):
        a[n - 1, n] = math.sqrt(n)
    ad = a.conj().T
    S = sla.expm(0.5 * r * (a @ a - ad @ ad))
    q = nbar / (nbar + 1.0)
    th = np.diag([(1 - q) * q ** k for k in range(L)])
    rho = S @ th @ S.conj().T
    return np.real(np.diag(rho))[:nmax].copy()


# ---------------------------------------------------------------- general split
def _omega(N):
    return np.block([[np.zeros((N, N)), np.eye(N)], [-np.eye(N), np.zeros((N, N))]])


def williamson(V):
    """(nu, S) with V = S diag(nu, nu) S^T, S symplectic (S Omega S^T = Omega),
    quadrature order (x_1..x_N, p_1..p_N): with A = V^{-1/2} Omega V^{-1/2}
    (real antisymmetric, eigenvalues +-i/nu), an orthogonal K that brings A
    to [[0, diag(1/nu)], [-diag(1/nu), 0]] gives S = V^{1/2} K diag(nu)^{-1/2}.
    K's columns come from the eigenvectors of the Hermitian i A (numpy eigh)."""
    N = V.shape[0] // 2
    w, E = np.linalg.eigh(V)
    Vh = (E * np.sqrt(w)) @ E.T
    Vmh = (E / np.sqrt(w)) @ E.T
    A = Vmh @ _omega(N) @ Vmh
    mu, Uc = np.linalg.eigh(1j * A)
    pos = np.argsort(-mu)[:N]                    # the N positive eigenvalues 1/nu
    K = np.zeros((2 * N, 2 * N))
    for c, k in enumerate(pos):
        K[:, c] = math.sqrt(2.0) * Uc[:, k].real
        K[:, N + c] = -math.sqrt(2.0) * Uc[:, k].imag
    nu = 1.0 / mu[pos]
    S = Vh @ K @ np.diag(np.concatenate([nu, nu]) ** -0.5)
    return nu, S


def decompose_williamson(V):
    """Pure part Q = S S^T / 2 of the Williamson decomposition and the
    classical part C = S (diag(nu, nu) - I/2) S^T >= 0 (Sec. II.F, the
    decomposition of the first column of the paper's photon table)."""
    nu, S = williamson(V)
    Q = 0.5 * S @ S.T
    C = S @ np.diag(np.concatenate([nu, nu]) - 0.5) @ S.T
    return Q, C


def pure_state_parameters(Q):
    """(r, U) with Q = covariance(r, U) for a pure covariance Q
    (Bloch-Messiah form): eigenvectors of Q with eigenvalue e^{-2r}/2 <= 1/2
    give the x-columns (X; Y) of the passive O = [[X, -Y], [Y, X]], their
    partners -Omega x are the p-columns; a degenerate eigenspace at 1/2 is
    split into such pairs by Gram-Schmidt."""
    N = Q.shape[0] // 2
    Om = _omega(N)
    w, E = np.linalg.eigh(Q)
    cols, rs = [], []
    used = np.zeros((2 * N, 0))
    for k in np.argsort(w):
        if len(cols) == N:
            break
        v = E[:, k].copy()
        if used.shape[1]:
            v -= used @ (used.T @ v)
        nv = np.linalg.norm(v)
        if nv < 1e-6 or w[k] > 0.5 + 1e-9:
            continue
        v /= nv
        cols.append(v)
        rs.append(-0.5 * math.log(2.0 * min(w[k], 0.5)))
        used = np.column_stack([used, v, -Om @ v])
    X = np.array([c[:N] for c in cols]).T
    Y = np.array([c[N:] for c in cols]).T
    return np.array(rs), X + 1j * Y


def factor_psd(C, tol=1e-12):
    """L (2N x K) with C = L L^T over the eigenvalues above tol * max."""
    w, E = np.linalg.eigh(0.5 * (C + C.T))
    keep = w > tol * max(w.max(), 1e-300)
    return E[:, keep] * np.sqrt(w[keep])[None, :]
