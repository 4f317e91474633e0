"""Local Fock-space operators (oracle; test infrastructure only).

X = (a + a^dag)/sqrt(2), P = -i(a - a^dag)/sqrt(2) with a_{n-1,n} = sqrt(n)
(Sec. II.C.1).  Products of quadratures are formed at dimension D+4 and then
truncated to D (SM Sec. 5), which discards the entries spoiled by the
[X, P] defect of a finite matrix and leaves exactly the compression P O P of
each quadratic operator.
"""
from __future__ import annotations

import numpy as np


def ladder(D: int) -> np.ndarray:
    a = np.zeros((D, D), dtype=np.complex128)
    for n in range(1, D):
        a[n - 1, n] = np.sqrt(n)
    return a


def quadratures(D: int):
    a = ladder(D)
    ad = a.conj().T
    X = (a + ad) / np.sqrt(2.0)
    P = -1j * (a - ad) / np.sqrt(2.0)
    return X, P


def local_operators(D: int, a_ss: float, b_ss: float, g_ss: float):
    """(X, P, S) truncated to D, where
    S = 1/2 (a_ss X^2 + b_ss P^2 + g_ss (XP + PX)) - 1/2 (single-site operator
    of SM Sec. 8), built at D+4 and truncated (SM Sec. 5)."""
    Xb, Pb = quadratures(D + 4)
    Sb = 0.5 * (a_ss * Xb @ Xb + b_ss * Pb @ Pb + g_ss * (Xb @ Pb + Pb @ Xb)) - 0.5 * np.eye(D + 4)
    return Xb[:D, :D].copy(), Pb[:D, :D].copy(), Sb[:D, :D].copy()


def project(op: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Operator in a local basis given by the isometry W (D x d): W^dag op W
    (Sec. III.A, the Hamiltonian cast in the optimised local basis)."""
    return W.conj().T @ op @ W
