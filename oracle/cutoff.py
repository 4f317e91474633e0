"""Cutoff errors of the Gaussian optimal local basis (oracle; test infrastructure only).

Sec. II.E.1 defines the cutoff error eps_D = 1 - <psi|P|psi> (eq. epsilonD),
P projecting every mode on its kept local states.  Sec. III.A.2 bounds it by
the discarded weights of the single-mode reduced density matrices (eq.
SpecWfromSDsums, proof in SM Sec. 4): with
    eps = 1 - (1/N) sum_i sum_{k < d_i} sigma_k^(i)2,
the spectrum sigma_k^(i)2 = nbar_i^k / (nbar_i + 1)^(k+1) of eq.
diagReducedGaussianDM, N eps >= eps_D >= eps.  Reading taken: the inner sum
runs over the d_i kept states k = 0 .. d_i - 1.

The effective cutoff (eq. Effectivecutoff) is the smallest Fock cutoff D at
which the matrix V_nm = <n|S^dag|m> (n < D, m < d) of the squeezed basis is an
isometry, here to a stated tolerance on max |V^dag V - 1|.  S is built by
scipy's matrix exponential of the squeezing generator on a box far larger than
any cutoff asked about.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import lbo, operators


def eps_bounds(V: np.ndarray, d: int):
    """(discarded weight per mode, eps, (lower, upper) bounds on eps_D) for the
    Gaussian state of covariance V with d kept states per mode."""
    N = V.shape[0] // 2
    tails = np.array([1.0 - lbo.gaussian_rdm_spectrum(V, i, d).sum() for i in range(N)])
    eps = float(tails.mean())
    return tails, eps, (eps, N * eps)


def squeeze_columns(zeta: complex, d: int, D: int, box: int = 400) -> np.ndarray:
    """<n|S|m> for n < D, m < d, S = exp(1/2 (zeta* a^2 - zeta a^dag^2))
    exponentiated on a Fock box of size max(box, D + 200)."""
    Db = max(box, D + 200)
    a = operators.ladder(Db)
    ad = a.conj().T
    G = 0.5 * (np.conj(zeta) * (a @ a) - zeta * (ad @ ad))
    S = scipy.linalg.expm(G)
    return S[:D, :d]


def effective_cutoff(zeta: complex, d: int, D_max: int, tol: float) -> int:
    """Smallest D in [d, D_max] with max |V_D^dag V_D - 1| <= tol, V_D the
    first D rows of the first d squeezed basis vectors; -1 if none."""
    V = squeeze_columns(zeta, d, D_max)
    for D in range(d, D_max + 1):
        Vd = V[:D]
        if np.abs(Vd.conj().T @ Vd - np.eye(d)).max() <= tol:
            return D
    return -1
