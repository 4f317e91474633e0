"""Global-CZ (non-Gaussian) parent Hamiltonian (oracle; test infrastructure only).

Sec. II.C.2: after the Gaussian circuit a fully connected phase gate
exp(-i kappa prod_k X_k) acts (eq. GlobalCZgate).  It leaves X unchanged and
maps P_i -> P_i + xi_i with xi_i = kappa prod_{n != i} X_n, so the parent
Hamiltonian is H = y^T (V^{-1}/4) y - N/2 with y = (X, P + xi) (eq.
nonGBSHamiltonian).  With M = V^{-1}/2 = [[alpha, gamma], [gamma^T, beta]] (the
Gaussian coefficients) the expansion is H = H_G + kappa H_1 + kappa^2 H_2,
  H_1 = Tr(gamma) prod_n X_n + sum_i beta_ii P_i prod_{n!=i} X_n
        + sum_{i!=j} (gamma_ij X_i^2 + beta_ij/2 Pt_i) prod_{n!=i,j} X_n,
  H_2 = 1/2 sum_i beta_ii prod_{n!=i} X_n^2
        + sum_{i<j} beta_ij X_i X_j prod_{n!=i,j} X_n^2,
with Pt = XP + PX: the terms of the purple, blue and magenta MPOs of SM Sec. 8.
Same-site products (X^2, Pt, S) are formed at D + 4 and truncated to D, so the
operator is the compression PHP (SM Sec. 5).

MPO reading (recorded in the design notes): the block sum of the Gaussian
middle-site MPO and two left-to-right automata, one for H_1 (background X) and
one for H_2 (background X^2).  Bond t of the H_1 block holds
[A0, AF, (AX2 i, APt i, AI i) for i = 1..t]: A0 = only background so far,
AF = the term is complete, AX2 i / APt i = X^2 / Pt placed at site i and its
identity partner still to come, AI i = the identity placed at site i and its
X^2 / Pt partner still to come.  Bond t of the H_2 block holds
[B0, BF, (BX i) for i = 1..t].  Bonds 0 and N are the Gaussian [S] and [F].

Kind codes extend the Gaussian ones: 7 X^2, 8 Pt, 9 c_X2 X^2 + c_Pt Pt.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import mpo as ompo, operators, gbs

KIND_X2, KIND_PT, KIND_COMBO2 = 7, 8, 9


def local_ops(D: int, a_ss: float, b_ss: float, g_ss: float):
    """(X, P, S, X^2, Pt) truncated to D; S, X^2, Pt formed at D + 4."""
    X, P, S = operators.local_operators(D, a_ss, b_ss, g_ss)
    Xb, Pb = operators.quadratures(D + 4)
    X2 = (Xb @ Xb)[:D, :D].copy()
    Pt = (Xb @ Pb + Pb @ Xb)[:D, :D].copy()
    return X, P, S, X2, Pt


def _kron_all(ops):
    out = sp.csr_matrix(np.array([[1.0 + 0j]]))
    for op in ops:
        out = sp.kron(out, sp.csr_matrix(op), format="csr")
    return out


def y_operators(N: int, kappa: float, B: int):
    """The 2N operators y = (X_1..X_N, P_1 + xi_1 .. P_N + xi_N) on the box
    [0, B)^N (sparse), every factor the B x B truncated quadrature."""
    X, P = operators.quadratures(B)
    I = np.eye(B, dtype=np.complex128)
    Y = []
    for k in range(N):
        ops = [I] * N
        ops[k] = X
        Y.append(_kron_all(ops))
    for i in range(N):
        ops = [I] * N
        ops[i] = P
        xi_ops = [X] * N
        xi_ops[i] = I
        Y.append(_kron_all(ops) + kappa * _kron_all(xi_ops))
    return Y


def dense_literal(alpha, beta, gamma, kappa, B: int) -> np.ndarray:
    """1/2 y^T M y - N/2 with y = (X, P + xi), products taken as matrix
    products in the box [0, B)^N."""
    N = alpha.shape[0]
    Y = y_operators(N, kappa, B)
    M = np.block([[alpha, gamma], [gamma.T, beta]])
    H = -0.5 * N * sp.identity(B ** N, dtype=np.complex128, format="csr")
    for a in range(2 * N):
        for b in range(2 * N):
            if M[a, b] != 0.0:
                H = H + 0.5 * M[a, b] * (Y[a] @ Y[b])
    return H.toarray()


def expectation_literal(alpha, beta, gamma, kappa, B: int, v: np.ndarray) -> float:
    """<v|H|v>/<v|v> of the same literal form, from w_a = y_a v:
    1/2 sum_ab M_ab <w_a, w_b> - N/2 (the y_a are Hermitian)."""
    N = alpha.shape[0]
    Y = y_operators(N, kappa, B)
    M = np.block([[alpha, gamma], [gamma.T, beta]])
    w = [y @ v for y in Y]
    e = -0.5 * N * np.vdot(v, v)
    for a in range(2 * N):
        for b in range(2 * N):
            e += 0.5 * M[a, b] * np.vdot(w[a], w[b])
    return float(e.real / np.vdot(v, v).real)


def dense_php(alpha, beta, gamma, kappa, D: int) -> np.ndarray:
    """PHP on [0, D)^N: the literal form in the box [0, D + 2)^N (every term has
    per-site degree <= 2, so its entries inside [0, D)^N are exact there),
    restricted to [0, D)^N."""
    N = alpha.shape[0]
    B = D + 2
    Hb = dense_literal(alpha, beta, gamma, kappa, B)
    keep = [int(np.ravel_multi_index(n, (B,) * N)) for n in itertools.product(range(D), repeat=N)]
    return Hb[np.ix_(keep, keep)]


def bond_labels(N: int, t: int):
    """Channel labels of bond t: the Gaussian labels, then the H_1 block, then the H_2 block."""
    g = ompo.bond_labels(N, t)
    if t == 0 or t == N:
        return g
    a = [("A0",), ("AF",)]
    for i in range(1, t + 1):
        a += [("AX2", i), ("APt", i), ("AI", i)]
    b = [("B0",), ("BF",)]
    for i in range(1, t + 1):
        b += [("BX", i)]
    return g + a + b


def bond_dims(N: int):
    return [len(bond_labels(N, t)) for t in range(N + 1)]


def core_entries(N: int, s: int, alpha, beta, gamma, kappa):
    """Entries of core s (1-based) as {(row_label, col_label): (kind, c1, c2)}:
    c1, c2 are (c_X, c_P) for kind 5, the scalar (in c1) for kind 6 and
    (c_X2, c_Pt) for kind 9."""
    if N < 2:
        raise ValueError("the global CZ Hamiltonian needs N >= 2")
    _, _, E = ompo.core_entries(N, s, alpha, beta, gamma)
    rows = bond_labels(N, s - 1)
    cols = bond_labels(N, s)
    rset, cset = set(rows), set(cols)
    b = lambda i, j: beta[i - 1, j - 1]
    g = lambda i, j: gamma[i - 1, j - 1]
    k = kappa

    def put(r, c, kind, c1=0.0, c2=0.0):
        if r in rset and c in cset:
            assert (r, c) not in E
            E[(r, c)] = (kind, c1, c2)

    last = s == N
    # H_1 block (background X)
    src0 = ("S",) if s == 1 else ("A0",)
    dstF = ("F",) if last else ("AF",)
    if not last:
        put(src0, ("A0",), ompo.KIND_X)
        put(src0, ("AX2", s), KIND_X2)
        put(src0, ("APt", s), KIND_PT)
        put(src0, ("AI", s), ompo.KIND_I)
    trg = k * float(np.trace(gamma)) if s == 1 else 0.0
    put(src0, dstF, ompo.KIND_COMBO, trg, k * b(s, s))
    if s > 1:
        put(("AF",), dstF, ompo.KIND_X)
    for i in range(1, s):
        if not last:
            put(("AX2", i), ("AX2", i), ompo.KIND_X)
            put(("APt", i), ("APt", i), ompo.KIND_X)
            put(("AI", i), ("AI", i), ompo.KIND_X)
        put(("AX2", i), dstF, ompo.KIND_SCALAR, k * g(i, s))
        put(("APt", i), dstF, ompo.KIND_SCALAR, 0.5 * k * b(i, s))
        put(("AI", i), dstF, KIND_COMBO2, k * g(s, i), 0.5 * k * b(s, i))
    # H_2 block (background X^2)
    src0 = ("S",) if s == 1 else ("B0",)
    dstF = ("F",) if last else ("BF",)
    if not last:
        put(src0, ("B0",), KIND_X2)
        put(src0, ("BX", s), ompo.KIND_X)
    put(src0, dstF, ompo.KIND_SCALAR, 0.5 * k * k * b(s, s))
    if s > 1:
        put(("BF",), dstF, KIND_X2)
    for i in range(1, s):
        if not last:
            put(("BX", i), ("BX", i), KIND_X2)
        put(("BX", i), dstF, ompo.KIND_COMBO, k * k * b(i, s), 0.0)
    return rows, cols, E


def structure(N: int):
    """(w[0..N], kinds) with kinds[s-1] an int8 (w_{s-1}, w_s) table."""
    z = np.zeros((N, N))
    w = bond_dims(N)
    kinds = []
    for s in range(1, N + 1):
        rows, cols, E = core_entries(N, s, z, z, z, 0.0)
        K = np.zeros((len(rows), len(cols)), dtype=np.int8)
        for (rl, cl), (kind, _, _) in E.items():
            K[rows.index(rl), cols.index(cl)] = kind
        kinds.append(K)
    return w, kinds


def cores(alpha, beta, gamma, kappa, site_ops):
    """Dense cores W_s (w_{s-1}, w_s, d, d); site_ops[s-1] = (X, P, S, X^2, Pt)
    truncated (and projected, with a local basis) for site s."""
    N = alpha.shape[0]
    out = []
    for s in range(1, N + 1):
        X, P, Sop, X2, Pt = site_ops[s - 1]
        d = X.shape[0]
        I = np.eye(d, dtype=np.complex128)
        rows, cols, E = core_entries(N, s, alpha, beta, gamma, kappa)
        W = np.zeros((len(rows), len(cols), d, d), dtype=np.complex128)
        for (rl, cl), (kind, c1, c2) in E.items():
            i, j = rows.index(rl), cols.index(cl)
            W[i, j] = {ompo.KIND_I: I, ompo.KIND_X: X, ompo.KIND_P: P, ompo.KIND_S: Sop, KIND_X2: X2, KIND_PT: Pt,
                       ompo.KIND_COMBO: c1 * X + c2 * P, ompo.KIND_SCALAR: c1 * I,
                       KIND_COMBO2: c1 * X2 + c2 * Pt}[kind]
        out.append(W)
    return out


def site_operators(r, U, D: int):
    """Per-site (X, P, S, X^2, Pt) of the instance (r, U)."""
    al, be, ga = gbs.coefficients(r, U)
    return al, be, ga, [local_ops(D, al[s, s], be[s, s], ga[s, s]) for s in range(len(r))]
