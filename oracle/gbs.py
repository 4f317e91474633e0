"""Gaussian boson sampling problem definition (oracle; test infrastructure only).

Conventions (hbar = 1, Sec. II):
  a = (X + iP)/sqrt(2),  X = (a + a^dag)/sqrt(2),  P = -i (a - a^dag)/sqrt(2).
  Quadrature vector x = (X_1..X_N, P_1..P_N) ("xxpp" order).
  Squeezing D = diag(e^{-r}, e^{r}) (Sec. II.C.1); r > 0 squeezes X.
  Interferometer in the Heisenberg picture a_j -> sum_k U_jk a_k, whose
  quadrature rotation is O = [[Re U, -Im U], [Im U, Re U]].
  Covariance V = 1/2 O D^2 O^T (Sec. II.C.1), vacuum V = I/2.
  H = x^T (V^{-1}/4) x - N/2 (eq. GBSHamiltonian), i.e. H = 1/2 x^T M x - N/2
  with M = V^{-1}/2 = [[alpha, gamma], [gamma^T, beta]] (SM Sec. 8 defines
  alpha_ij, beta_ij, gamma_ij as halves of blocks of V^{-1}).
"""
from __future__ import annotations

import itertools
import math
import numpy as np


def quadrature_rotation(U: np.ndarray) -> np.ndarray:
    """Orthogonal-symplectic O of the passive interferometer (Sec. II.C.1)."""
    Ur, Ui = U.real, U.imag
    return np.block([[Ur, -Ui], [Ui, Ur]])


def covariance(r: np.ndarray, U: np.ndarray) -> np.ndarray:
    """V = 1/2 O D^2 O^T with D = diag(e^{-r}, e^{r}) (Sec. II.C.1)."""
    r = np.asarray(r, dtype=np.float64)
    O = quadrature_rotation(U)
    D2 = np.concatenate([np.exp(-2.0 * r), np.exp(2.0 * r)])
    return 0.5 * (O * D2[None, :]) @ O.T


def coefficients(r: np.ndarray, U: np.ndarray):
    """alpha, beta, gamma = halves of the blocks of V^{-1} (SM Sec. 8), so that
    H = 1/2 x^T [[alpha, gamma], [gamma^T, beta]] x - N/2 (eq. GBSHamiltonian)."""
    N = len(r)
    V = covariance(r, U)
    Vinv = np.linalg.inv(V)
    M = 0.5 * Vinv
    M = 0.5 * (M + M.T)
    return M[:N, :N].copy(), M[N:, N:].copy(), M[:N, N:].copy()


def bogoliubov_matrix(r: np.ndarray, U: np.ndarray) -> np.ndarray:
    """B = -U diag(tanh r) U^T: the output state is prop. to
    exp(1/2 sum_jk B_jk a_j^dag a_k^dag)|0> (the output of Sec. II.C.1)."""
    return -(U * np.tanh(r)[None, :]) @ U.T


def bogoliubov_modes(r: np.ndarray, U: np.ndarray):
    """Coefficients of b_k = sum_j (c_jk a_j + s_jk a_j^dag), the circuit-
    transformed annihilators A_n of eq. CentralEquation:
    c_jk = cosh(r_k) conj(U_jk), s_jk = sinh(r_k) U_jk."""
    c = np.conj(U) * np.cosh(r)[None, :]
    s = U * np.sinh(r)[None, :]
    return c, s


def exact_amplitudes(r: np.ndarray, U: np.ndarray, D: int) -> np.ndarray:
    """<n|psi> for every n in the box [0, D)^N (the untruncated state; the
    distribution of Sec. II.A restricted to the box).

    Uses a_j|psi> = sum_k B_jk a_k^dag |psi>, i.e.
      sqrt(n_j + 1) psi(n + e_j) = sum_l B_jl sqrt(n_l) psi(n - e_l),
    with psi(0) = prod_k cosh(r_k)^{-1/2}.  Entries are filled in order of
    total photon number, each from the first nonzero coordinate."""
    r = np.asarray(r, dtype=np.float64)
    N = len(r)
    B = bogoliubov_matrix(r, U)
    psi = np.zeros((D,) * N, dtype=np.complex128)
    psi[(0,) * N] = np.prod(np.cosh(r)) ** -0.5
    # visit in order of total photon number so all predecessors exist
    idx = sorted(itertools.product(range(D), repeat=N), key=lambda t: sum(t))
    for n in idx:
        if sum(n) == 0:
            continue
        j = next(i for i, v in enumerate(n) if v > 0)
        m = list(n)
        m[j] -= 1                       # psi(n) with n = m + e_j
        acc = 0.0 + 0.0j
        for l in range(N):
            if m[l] > 0:
                p = list(m)
                p[l] -= 1
                acc += B[j, l] * math.sqrt(m[l]) * psi[tuple(p)]
        psi[n] = acc / math.sqrt(m[j] + 1)
    return psi


def hafnian(A: np.ndarray) -> complex:
    """Hafnian by brute-force recursion over perfect matchings (Sec. II.A;
    exponential, for tiny matrices only)."""
    n = A.shape[0]
    if n == 0:
        return 1.0 + 0.0j
    if n % 2:
        return 0.0 + 0.0j
    total = 0.0 + 0.0j
    rest = list(range(1, n))
    for k, j in enumerate(rest):
        others = rest[:k] + rest[k + 1:]
        sub = A[np.ix_(others, others)]
        total += A[0, j] * hafnian(sub)
    return total


def amplitude_hafnian(n, r: np.ndarray, U: np.ndarray) -> complex:
    """<n|psi> = Haf(B_n) / sqrt(prod n_j! prod cosh r_k), B_n = B with row and
    column j repeated n_j times."""
    B = bogoliubov_matrix(r, U)
    rows = [j for j, c in enumerate(n) for _ in range(c)]
    Bn = B[np.ix_(rows, rows)]
    norm = math.sqrt(float(np.prod([math.factorial(c) for c in n]))) * math.sqrt(float(np.prod(np.cosh(r))))
    return hafnian(Bn) / norm


def single_mode_probabilities(r: float, nmax: int) -> np.ndarray:
    """Photon-number distribution of a squeezed vacuum (closed form):
    P(2n) = (2n)! / (4^n (n!)^2) tanh^{2n}(r) / cosh(r), P(odd) = 0."""
    P = np.zeros(nmax)
    t = math.tanh(r)
    for k in range(0, nmax, 2):
        n = k // 2
        P[k] = math.factorial(2 * n) / (4 ** n * math.factorial(n) ** 2) * t ** (2 * n) / math.cosh(r)
    return P


def mean_photons(r: np.ndarray, U: np.ndarray) -> np.ndarray:
    """<n_j> = 1/2 (V_{x_j x_j} + V_{p_j p_j}) - 1/2 per output mode (hbar = 1,
    vacuum V = I/2)."""
    V = covariance(r, U)
    N = len(r)
    return 0.5 * (V[np.arange(N), np.arange(N)] + V[N + np.arange(N), N + np.arange(N)]) - 0.5
