"""Dense truncated Hamiltonian PHP for tiny sizes, and exact diagonalisation
(oracle; test infrastructure only).

PHP is the compression of H onto the Fock box [0, D)^N (eq. ProjectionOperator;
"we simply consider PHP", Sec. II.E.1).  Two independent constructions:
  * quadrature form, eq. GBSHamiltonian: sum of single-site S_j plus
    X/P cross terms, with the squares built at D+4 and truncated (SM Sec. 5);
  * Bogoliubov form, eq. CentralEquation: H = sum_k b_k^dag b_k with the
    circuit-transformed annihilators, assembled on a (D+2)-box with sparse
    matrices and restricted to the inner D-box (each quadratic term moves a
    photon number by at most 2, so the restriction is exact).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import gbs, operators


def _kron_list(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def _embed(op, site, N, D):
    mats = [np.eye(D, dtype=np.complex128)] * N
    mats = list(mats)
    mats[site] = op
    return _kron_list(mats)


def php_quadrature(alpha, beta, gamma, D: int) -> np.ndarray:
    """PHP from eq. GBSHamiltonian: H = sum_s S_s + sum_{k<s} [X_k (alpha_ks X_s
    + gamma_ks P_s) + P_k (gamma_sk X_s + beta_ks P_s)], S_s as in SM Sec. 8."""
    N = alpha.shape[0]
    X, P = operators.quadratures(D)
    H = np.zeros((D ** N, D ** N), dtype=np.complex128)
    for s in range(N):
        _, _, S = operators.local_operators(D, alpha[s, s], beta[s, s], gamma[s, s])
        H += _embed(S, s, N, D)
    for k in range(N):
        for s in range(k + 1, N):
            Xk, Pk = _embed(X, k, N, D), _embed(P, k, N, D)
            Xs, Ps = _embed(X, s, N, D), _embed(P, s, N, D)
            H += Xk @ (alpha[k, s] * Xs + gamma[k, s] * Ps)
            H += Pk @ (gamma[s, k] * Xs + beta[k, s] * Ps)
    return H


def php_bogoliubov(r, U, D: int) -> np.ndarray:
    """PHP from eq. CentralEquation: sum_k b_k^dag b_k, b_k = sum_j (c_jk a_j +
    s_jk a_j^dag), assembled on the (D+2)-box and restricted to [0, D)^N."""
    N = len(r)
    Db = D + 2
    c, s = gbs.bogoliubov_modes(np.asarray(r), U)
    a = sp.csr_matrix(operators.ladder(Db))
    ad = sp.csr_matrix(a.conj().T)
    I = sp.identity(Db, dtype=np.complex128, format="csr")

    def emb(op, site):
        out = None
        for t in range(N):
            m = op if t == site else I
            out = m if out is None else sp.kron(out, m, format="csr")
        return out

    A = [emb(a, j) for j in range(N)]
    Ad = [emb(ad, j) for j in range(N)]
    dim = Db ** N
    H = sp.csr_matrix((dim, dim), dtype=np.complex128)
    for k in range(N):
        b = sp.csr_matrix((dim, dim), dtype=np.complex128)
        for j in range(N):
            b = b + c[j, k] * A[j] + s[j, k] * Ad[j]
        H = H + b.conj().T @ b
    # indices of the inner box
    grids = np.indices((Db,) * N).reshape(N, -1)
    inner = np.all(grids < D, axis=0)
    sel = np.nonzero(inner)[0]
    Hin = H[sel][:, sel].toarray()
    return Hin


def ground_states(H: np.ndarray, k: int = 2):
    """Lowest k eigenpairs of a dense Hermitian matrix (numpy eigh)."""
    w, v = np.linalg.eigh(0.5 * (H + H.conj().T))
    return w[:k], v[:, :k]


def truncated_exact_state(r, U, D: int) -> np.ndarray:
    """P|psi> in the box (flattened, row-major over modes), NOT renormalised."""
    return gbs.exact_amplitudes(r, U, D).reshape(-1)
