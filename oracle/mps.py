"""Matrix product state utilities (oracle; test infrastructure only).

Open-boundary MPS, eq. MPSAnsatz: c_n = M1_{n1}^T M2_{n2} ... MN_{nN}, with
site tensors A_s of shape (chi_{s-1}, d, chi_s) and chi_0 = chi_N = 1
(Sec. II.D).  Canonical forms use numpy's QR; environments and the energy
live in the dmrg module.
"""
from __future__ import annotations

import numpy as np


def to_dense(mps) -> np.ndarray:
    """Full coefficient vector c_n, row-major over sites (tiny N only)."""
    T = mps[0]                       # (1, d, chi)
    T = T.reshape(-1, T.shape[-1])
    for A in mps[1:]:
        T = T @ A.reshape(A.shape[0], -1)
        T = T.reshape(-1, A.shape[-1])
    return T.reshape(-1)


def norm2(mps) -> float:
    E = np.ones((1, 1), dtype=np.complex128)
    for A in mps:
        E = np.tensordot(np.tensordot(E, A.conj(), axes=([0], [0])), A, axes=([0, 1], [0, 1]))
    return float(E[0, 0].real)


def right_canonicalize(mps):
    """Right-canonical form from site N down to 2 by LQ (QR of the adjoint);
    the norm ends up on site 1, which is then normalised."""
    mps = [A.copy() for A in mps]
    N = len(mps)
    for s in range(N - 1, 0, -1):
        A = mps[s]
        cl, d, cr = A.shape
        M = A.reshape(cl, d * cr)
        Q, R = np.linalg.qr(M.conj().T)          # M^dag = Q R  ->  M = R^dag Q^dag
        k = Q.shape[1]
        mps[s] = Q.conj().T.reshape(k, d, cr)
        mps[s - 1] = np.tensordot(mps[s - 1], R.conj().T, axes=([2], [0]))
    nrm = np.linalg.norm(mps[0])
    mps[0] = mps[0] / nrm
    return mps


def is_left_canonical(A, tol=1e-10) -> bool:
    M = A.reshape(-1, A.shape[-1])
    return np.abs(M.conj().T @ M - np.eye(M.shape[1])).max() < tol


def is_right_canonical(A, tol=1e-10) -> bool:
    M = A.reshape(A.shape[0], -1)
    return np.abs(M @ M.conj().T - np.eye(M.shape[0])).max() < tol


def probabilities(mps) -> np.ndarray:
    """P(n) = |<n|psi>|^2 / <psi|psi> inside the box (Sec. II.A)."""
    c = to_dense(mps)
    p = np.abs(c) ** 2
    return p / p.sum()


def fock_tensors(mps, isometries):
    """Site tensors in the raw Fock basis: A^F_s[n] = sum_m W_s[n, m] A_s[m]
    (eq. InverseBasisTransformation)."""
    if isometries is None:
        return [A.copy() for A in mps]
    return [np.einsum("nm,amb->anb", W, A) for W, A in zip(isometries, mps)]


def _env_left(L, A):
    """L'[c, d] = sum_{a,b,s} L[a, b] conj(A[a, s, c]) A[b, s, d]."""
    T = np.tensordot(L, A, axes=([1], [0]))              # (a, s, d)
    return np.tensordot(A.conj(), T, axes=([0, 1], [0, 1]))


def _env_right(R, A):
    """R'[a, b] = sum_{c,d,s} conj(A[a, s, c]) A[b, s, d] R[c, d]."""
    T = np.tensordot(A, R.T, axes=([2], [0]))            # (b, s, c)
    return np.tensordot(A.conj(), T, axes=([1, 2], [1, 2]))


def marginals(mps, isometries=None, n_modes=None) -> np.ndarray:
    """Single-mode photon-number marginals P_j(n) by contracting the reduced
    density matrix rho_j (eq. ReducedDensityMatrix), shape (n_modes, D_raw)."""
    F = fock_tensors(mps, isometries)
    N = len(F)
    n_modes = N if n_modes is None else n_modes
    left = [np.ones((1, 1), dtype=np.complex128)]
    for A in F[:n_modes]:
        left.append(_env_left(left[-1], A))
    right = [np.ones((1, 1), dtype=np.complex128)]
    for A in reversed(F):
        right.append(_env_right(right[-1], A))
    right = right[::-1]
    # <psi|psi> from the full right environment of site 0
    nrm = right[0][0, 0].real
    D = F[0].shape[1]
    out = np.zeros((n_modes, D))
    for j in range(n_modes):
        A = F[j]
        # rho_j[s, s] = sum L[a, b] conj(A[a, s, c]) A[b, s, d] R[c, d]
        T = np.tensordot(left[j], A, axes=([1], [0]))    # (a, s, d)
        T = np.tensordot(T, right[j + 1], axes=([2], [1]))  # (a, s, c)
        out[j] = np.real(np.einsum("asc,asc->s", A.conj(), T)) / nrm
    return out


def reduced_density_matrices(mps, isometries=None) -> np.ndarray:
    """rho_j[n, n'] = <n|rho_j|n'> = sum over the other modes of psi_n conj(psi_n')
    / <psi|psi> (eq. ReducedDensityMatrix), in the raw Fock basis, shape
    (N, D_raw, D_raw)."""
    F = fock_tensors(mps, isometries)
    N = len(F)
    left = [np.ones((1, 1), dtype=np.complex128)]
    for A in F:
        # left[x, y] = sum over left modes of psi_x conj(psi_y)
        left.append(np.einsum("ab,asc,bsd->cd", left[-1], A, A.conj()))
    right = [np.ones((1, 1), dtype=np.complex128)]
    for A in reversed(F):
        right.append(np.einsum("cd,asc,bsd->ab", right[-1], A, A.conj()))
    right = right[::-1]
    nrm = left[-1][0, 0].real
    D = F[0].shape[1]
    out = np.zeros((N, D, D), dtype=np.complex128)
    for j, A in enumerate(F):
        out[j] = np.einsum("ab,asc,btd,cd->st", left[j], A, A.conj(), right[j + 1]) / nrm
    return out
