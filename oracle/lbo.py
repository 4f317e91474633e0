"""Local basis optimisation (oracle; test infrastructure only).

Sec. III.A: the optimal local basis of site i is spanned by the top
eigenvectors of the reduced density matrix rho_i (eq. ReducedDensityMatrix);
keeping d of them discards sum_{k >= d} lambda_k (eq. SVDPhysicalDimension).
SM Sec. 6: the basis is an isometry W (D x d) per site, optimised site by site
against its effective Hamiltonian, starting from [I; 0].  Reading taken here:
with the orthogonality centre at site s, the raw-basis tensor B = W_s A_s is
re-optimised by a single-site solve with the site's operators in the raw Fock
basis, rho_s = sum_{a,b} B[a,:,b] B[a,:,b]^dag, W_s = its top-d eigenvectors
(each column's largest-modulus entry made real positive), A_s = W_s^dag B.

Sec. III.A.1 gives the Gaussian closed form used as a pin: the reduced state
of mode i is thermal in a squeezed basis with
lambda_k = nbar^k / (nbar + 1)^(k+1), nbar = sqrt(det V_i) - 1/2 (hbar = 1).
"""
from __future__ import annotations

import numpy as np

from . import dmrg, operators, mpo as ompo, gbs


def reduced_covariance(V: np.ndarray, i: int) -> np.ndarray:
    N = V.shape[0] // 2
    idx = [i, N + i]
    return V[np.ix_(idx, idx)]


def gaussian_rdm_spectrum(V: np.ndarray, i: int, K: int) -> np.ndarray:
    """lambda_k = nbar^k / (nbar+1)^(k+1) for k < K (eq. diagReducedGaussianDM),
    nbar from the symplectic eigenvalue sqrt(det V_i) = nbar + 1/2 (eq.
    WilliamsonDecomposition)."""
    nbar = np.sqrt(np.linalg.det(reduced_covariance(V, i))) - 0.5
    k = np.arange(K)
    return nbar ** k / (nbar + 1.0) ** (k + 1)


def rdm_from_dense(psi: np.ndarray, i: int) -> np.ndarray:
    """rho_i = Tr_{k != i} |psi><psi| for a dense state of shape (D,)*N."""
    N = psi.ndim
    t = np.moveaxis(psi, i, 0).reshape(psi.shape[i], -1)
    return t @ t.conj().T


def local_ops(r, U, D):
    al, be, ga = gbs.coefficients(r, U)
    return al, be, ga, [operators.local_operators(D, al[s, s], be[s, s], ga[s, s]) for s in range(len(r))]


def cores_in_basis(al, be, ga, raw_ops, iso):
    ops = [tuple(operators.project(o, W) for o in raw) for raw, W in zip(raw_ops, iso)]
    return ompo.cores(al, be, ga, ops)


def lbo_site(mps, cores, raw_core, W, s, tol=1e-12, krylov_max=32, max_iter=400):
    """One local basis update of site s (orthogonality centre at s).
    mps: tensors in the current local bases; cores: MPO cores in those bases;
    raw_core: the MPO core of site s in the raw Fock basis; W: isometry of s.
    Returns (W_new, A_new, discarded, lambda)."""
    L = dmrg.boundary_env()
    for t in range(s):
        L = dmrg.env_left_update(L, mps[t], cores[t])
    R = dmrg.boundary_env()
    for t in range(len(mps) - 1, s, -1):
        R = dmrg.env_right_update(R, mps[t], cores[t])
    B = np.tensordot(W, mps[s], axes=([1], [1])).transpose(1, 0, 2)   # (chi_l, D, chi_r)
    shp = B.shape
    mv = lambda v: dmrg.heff_matvec_single(L, raw_core, R, v.reshape(shp)).reshape(-1)
    lam, x, _, _ = dmrg.lanczos_lowest(mv, B.reshape(-1), tol, krylov_max, max_iter)
    B = x.reshape(shp)
    rho = np.tensordot(B, B.conj(), axes=([0, 2], [0, 2]))           # (D, D)
    ev, Z = np.linalg.eigh(0.5 * (rho + rho.conj().T))
    ev, Z = ev[::-1], Z[:, ::-1]
    d = W.shape[1]
    Wn = Z[:, :d].copy()
    for j in range(d):
        i = int(np.argmax(np.abs(Wn[:, j])))
        Wn[:, j] *= np.conj(Wn[i, j]) / abs(Wn[i, j])
    A = np.tensordot(Wn.conj(), B, axes=([0], [1])).transpose(1, 0, 2)
    A /= np.linalg.norm(A)
    disc = float(np.sum(np.maximum(ev[d:], 0.0)) / np.sum(np.maximum(ev, 0.0)))
    return Wn, A, disc, lam


def dmrg_lbo(mps, r, U, D, iso, chi, sweeps, tol=1e-12, krylov_max=32, max_iter=400):
    """Two-site DMRG sweeps with the local basis of the centre site re-optimised
    (lbo_site) before each two-site update: site s on the left-to-right half,
    site s+1 on the right-to-left half (the joint optimisation of SM Sec. 6
    carried out inside the sweep).  The input MPS is right-canonicalised first.
    Returns (mps, iso, stats)."""
    from . import mps as mpsmod
    al, be, ga, raw = local_ops(r, U, D)
    raw_cores = ompo.cores(al, be, ga, raw)
    iso = [W.copy() for W in iso]
    N = len(mps)
    mps = mpsmod.right_canonicalize(mps)
    stats = []
    for sw in range(sweeps):
        disc_lbo = 0.0
        order = [(s, +1) for s in range(N - 1)] + [(s, -1) for s in range(N - 2, -1, -1)]
        for s, direction in order:
            c = s if direction > 0 else s + 1
            cores = cores_in_basis(al, be, ga, raw, iso)
            Wn, A, disc, _ = lbo_site(mps, cores, raw_cores[c], iso[c], c, tol, krylov_max, max_iter)
            iso[c] = Wn
            mps[c] = A
            disc_lbo += disc
            cores = cores_in_basis(al, be, ga, raw, iso)
            L = dmrg.boundary_env()
            for t in range(s):
                L = dmrg.env_left_update(L, mps[t], cores[t])
            R = dmrg.boundary_env()
            for t in range(N - 1, s + 1, -1):
                R = dmrg.env_right_update(R, mps[t], cores[t])
            theta = np.tensordot(mps[s], mps[s + 1], axes=([2], [0]))
            shp = theta.shape
            mv = lambda v: dmrg.heff_matvec(L, cores[s], cores[s + 1], R, v.reshape(shp)).reshape(-1)
            lam, x, _, _ = dmrg.lanczos_lowest(mv, theta.reshape(-1), tol, krylov_max, max_iter)
            Uu, S, Vh, disc = dmrg.truncate(x.reshape(shp), chi)
            cl, d1, d2, cr = shp
            k = len(S)
            if direction > 0:
                mps[s] = Uu.reshape(cl, d1, k)
                mps[s + 1] = (S[:, None] * Vh).reshape(k, d2, cr)
            else:
                mps[s] = (Uu * S[None, :]).reshape(cl, d1, k)
                mps[s + 1] = Vh.reshape(k, d2, cr)
        cores = cores_in_basis(al, be, ga, raw, iso)
        stats.append(dict(sweep=sw, energy=dmrg.energy(mps, cores), lbo_discarded=disc_lbo))
    return mps, iso, stats
