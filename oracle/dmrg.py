"""Two-site DMRG for the parent Hamiltonian (oracle; test infrastructure only).

The variational problem of Sec. II.B/II.D: minimise <psi|PHP|psi> over MPS of
bond dimension <= chi, by sweeping two-site updates (the paper ran single-site
DMRG; two sites is the reading taken here).  Each update:
  theta = A_s A_{s+1};  lowest eigenpair of H_eff by Lanczos (FP64, full
  reorthogonalisation);  SVD of theta reshaped (chi_l d) x (d chi_r), keep
  k = min(chi, #{sigma_i > sigma_cut sigma_1}), discarded weight
  sum_{i>k} sigma_i^2 (eq. SurrogateEpsChi), renormalise;  split and update
  the environment.
Environments: L_t[l, b, b'] (b bra, b' ket) covers sites 1..t; R_t[n, b, b']
covers sites t+1..N.
"""
from __future__ import annotations

import numpy as np

from . import mps as mpsmod


# ---------------------------------------------------------------- environments
def env_left_update(L, A, W):
    """L_s[m,b,b'] = sum conj(A[a,s,b]) L[l,a,a'] W[l,m,s,s'] A[a',s',b']."""
    T = np.tensordot(L, A, axes=([2], [0]))                 # l a t c
    T = np.tensordot(T, W, axes=([0, 2], [0, 3]))           # a c m s
    T = np.tensordot(A.conj(), T, axes=([0, 1], [0, 3]))    # b c m
    return np.ascontiguousarray(T.transpose(2, 0, 1))


def env_right_update(R, A, W):
    """R_{s-1}[l,a,a'] = sum conj(A[a,s,b]) W[l,n,s,s'] R[n,b,b'] A[a',s',b']."""
    T = np.tensordot(A, R, axes=([2], [2]))                 # y t n b
    T = np.tensordot(T, W, axes=([1, 2], [3, 1]))           # y b l s
    T = np.tensordot(A.conj(), T, axes=([1, 2], [3, 1]))    # a y l
    return np.ascontiguousarray(T.transpose(2, 0, 1))


def boundary_env():
    return np.ones((1, 1, 1), dtype=np.complex128)


def left_envs(mps, Ws):
    out = [boundary_env()]
    for A, W in zip(mps, Ws):
        out.append(env_left_update(out[-1], A, W))
    return out


def right_envs(mps, Ws):
    N = len(mps)
    out = [None] * (N + 1)
    out[N] = boundary_env()
    for s in range(N - 1, -1, -1):
        out[s] = env_right_update(out[s + 1], mps[s], Ws[s])
    return out


# ----------------------------------------------------------------- energy
def energy(mps, Ws) -> float:
    """<psi|H|psi>/<psi|psi> by a full FP64 environment contraction (the error
    measure of eq. MagOfSimError)."""
    L = left_envs(mps, Ws)[-1]
    return float(L[0, 0, 0].real) / mpsmod.norm2(mps)


def env2_left_update(L, A, W):
    """Two-layer left environment of <psi|H H|psi>:
    L'[b,u',v',b'] = sum conj(A[a,n,b]) W[u,u',n,m] W[v,v',m,k] A[a',k,b'] L[a,u,v,a']."""
    T = np.tensordot(L, A, axes=([3], [0]))                  # a u v k b'
    T = np.tensordot(T, W, axes=([2, 3], [0, 3]))            # a u b' v' m
    T = np.tensordot(T, W, axes=([1, 4], [0, 3]))            # a b' v' u' n
    T = np.tensordot(A.conj(), T, axes=([0, 1], [0, 4]))     # b b' v' u'
    return np.ascontiguousarray(T.transpose(0, 3, 2, 1))


def energy_variance(mps, Ws, iso=None):
    """(<H>, <H^2>, sigma_H^2) of the normalised state for the MPO Ws of PHP in
    the raw Fock box (Sec. II.E.2: sigma_H^2 = <(PHP)^2> - <PHP>^2).  With
    isometries iso[s] (D x d) the physical state has site tensors W_s A_s, so
    (PHP)^2 is taken in the raw box, not in the kept basis."""
    if iso is not None:
        mps = [np.einsum("im,amb->aib", W, A) for W, A in zip(iso, mps)]
    L = np.ones((1, 1, 1, 1), dtype=np.complex128)
    for A, W in zip(mps, Ws):
        L = env2_left_update(L, A, W)
    n2 = mpsmod.norm2(mps)
    e = energy(mps, Ws)
    h2 = float(L[0, 0, 0, 0].real) / n2
    return e, h2, h2 - e * e


def energy_bogoliubov(mps, r, U, D) -> float:
    """<H> = sum_k ||b_k psi||^2 / <psi|psi> (eq. CentralEquation read as a sum
    of squares), evaluated on the dense state with b_k restricted to the box
    and the vector embedded in a (D+1)-box.  Dense; tiny N only."""
    from . import gbs, operators
    N = len(mps)
    psi = mpsmod.to_dense(mps).reshape((D,) * N)
    Db = D + 1
    big = np.zeros((Db,) * N, dtype=np.complex128)
    big[tuple(slice(0, D) for _ in range(N))] = psi
    c, s = gbs.bogoliubov_modes(np.asarray(r), U)
    a = operators.ladder(Db)
    ad = a.conj().T
    tot = 0.0
    for k in range(N):
        out = np.zeros_like(big)
        for j in range(N):
            out += c[j, k] * np.moveaxis(np.tensordot(a, big, axes=([1], [j])), 0, j)
            out += s[j, k] * np.moveaxis(np.tensordot(ad, big, axes=([1], [j])), 0, j)
        # PHP: only the components inside the box of H applied to P psi count;
        # H = sum b^dag b, <Ppsi|H|Ppsi> = sum_k ||b_k P psi||^2 with b_k on the full space
        tot += float(np.vdot(out, out).real)
    return tot / float(np.vdot(psi, psi).real)


# ----------------------------------------------------------------- local problem
def heff_matvec(L, W1, W2, R, theta):
    """theta'[a,s,t,b] = sum L[l,a,a'] W1[l,m,s,s'] W2[m,n,t,t'] R[n,b,b']
    theta[a',s',t',b'] (the two-site effective Hamiltonian)."""
    T = np.tensordot(L, theta, axes=([2], [0]))             # l a u v y
    T = np.tensordot(T, W1, axes=([0, 2], [0, 3]))          # a v y m s
    T = np.tensordot(T, W2, axes=([3, 1], [0, 3]))          # a y s n t
    T = np.tensordot(T, R, axes=([1, 3], [2, 0]))           # a s t b
    return T


def heff_matvec_single(L, W, R, A):
    """Single-site effective Hamiltonian applied to A[a, s, b]."""
    T = np.tensordot(L, A, axes=([2], [0]))                 # l a u y
    T = np.tensordot(T, W, axes=([0, 2], [0, 3]))           # a y n s
    T = np.tensordot(T, R, axes=([1, 2], [2, 0]))           # a s b
    return T


def lanczos_lowest(matvec, x0, tol=1e-12, krylov_max=32, max_iter=200):
    """Lowest eigenpair by Lanczos with full (two-pass classical Gram-Schmidt)
    reorthogonalisation and explicit restart from the Ritz vector.
    Returns (lambda, x, matvecs, converged)."""
    x = x0 / np.linalg.norm(x0)
    matvecs = 0
    lam = np.nan
    while True:
        V = [x]
        alphas, betas = [], []
        for j in range(krylov_max):
            w = matvec(V[j])
            matvecs += 1
            a = float(np.vdot(V[j], w).real)
            alphas.append(a)
            w = w - a * V[j]
            if j > 0:
                w = w - betas[-1] * V[j - 1]
            for _ in range(2):
                for v in V:
                    w = w - np.vdot(v, w) * v
            b = float(np.linalg.norm(w))
            T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
            evals, evecs = np.linalg.eigh(T)
            lam, y = evals[0], evecs[:, 0]
            res = b * abs(y[-1])
            if res <= tol or b < 1e-300 or matvecs >= max_iter:
                xr = sum(yi * v for yi, v in zip(y, V))
                xr = xr / np.linalg.norm(xr)
                return lam, xr, matvecs, res <= tol or b < 1e-300
            betas.append(b)
            V.append(w / b)
        xr = sum(yi * v for yi, v in zip(y, V[:len(y)]))
        x = xr / np.linalg.norm(xr)


def truncate(theta, chi, sigma_cut=0.0):
    """SVD truncation of theta (chi_l, d, d, chi_r) -> (U, S, Vh, discarded),
    S renormalised to unit norm; discarded weight relative to ||theta||^2."""
    cl, d1, d2, cr = theta.shape
    M = theta.reshape(cl * d1, d2 * cr)
    U, S, Vh = np.linalg.svd(M, full_matrices=False)
    tot = float(np.sum(S ** 2))
    keep = min(chi, len(S))
    if sigma_cut > 0:
        keep = min(keep, int(np.sum(S > sigma_cut * S[0])))
    keep = max(keep, 1)
    disc = float(np.sum(S[keep:] ** 2)) / tot
    Sk = S[:keep] / np.sqrt(float(np.sum(S[:keep] ** 2)))
    return U[:, :keep], Sk, Vh[:keep], disc


# ----------------------------------------------------------------- sweeps
def dmrg(mps, Ws, chi, sweeps, tol=1e-12, krylov_max=32, max_iter=200,
         sigma_cut=0.0, callback=None):
    """Two-site DMRG sweeps (L->R then R->L, 2(N-1) updates each).  The input
    MPS is right-canonicalised first.  Returns (mps, stats_per_sweep)."""
    N = len(mps)
    mps = mpsmod.right_canonicalize(mps)
    R = right_envs(mps, Ws)
    L = [None] * (N + 1)
    L[0] = boundary_env()
    stats = []
    for sw in range(sweeps):
        disc_max, disc_sum, nmv, unconv = 0.0, 0.0, 0, 0
        order = [(s, +1) for s in range(N - 1)] + [(s, -1) for s in range(N - 2, -1, -1)]
        for s, direction in order:
            theta = np.tensordot(mps[s], mps[s + 1], axes=([2], [0]))
            Le, Re = L[s], R[s + 2]
            shp = theta.shape
            mv = lambda v: heff_matvec(Le, Ws[s], Ws[s + 1], Re, v.reshape(shp)).reshape(-1)
            lam, x, k, conv = lanczos_lowest(mv, theta.reshape(-1), tol, krylov_max, max_iter)
            nmv += k
            unconv += (not conv)
            U, S, Vh, disc = truncate(x.reshape(shp), chi, sigma_cut)
            disc_max = max(disc_max, disc)
            disc_sum += disc
            cl, d1, d2, cr = shp
            k_ = len(S)
            if direction > 0:
                mps[s] = U.reshape(cl, d1, k_)
                mps[s + 1] = (S[:, None] * Vh).reshape(k_, d2, cr)
                L[s + 1] = env_left_update(L[s], mps[s], Ws[s])
            else:
                mps[s] = (U * S[None, :]).reshape(cl, d1, k_)
                mps[s + 1] = Vh.reshape(k_, d2, cr)
                R[s + 1] = env_right_update(R[s + 2], mps[s + 1], Ws[s + 1])
        E = energy(mps, Ws)
        st = dict(sweep=sw, energy=E, last_eig=lam, max_discarded=disc_max,
                  sum_discarded=disc_sum, matvecs=nmv, unconverged=unconv)
        stats.append(st)
        if callback:
            callback(st)
    return mps, stats
