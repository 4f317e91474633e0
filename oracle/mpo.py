"""Middle-site algebraic MPO of the GBS Hamiltonian (oracle; test
infrastructure only).  Follows SM Sec. 8 ("H_Gaussian MPO"): left cores L_s
collect X/P operator strings, the middle core M_{N_m} collapses them with the
coefficients, right cores R_s collect the strings from the right.

Bond bases (position 0 first; each name describes the left part of the bond):
  bond 0: [S]                              bond N: [F]
  left bonds t = 1..m-1:  [X_t, P_t, X_{t-1}, P_{t-1}, ..., X_1, P_1, S, F]
  right bonds t = m..N-1: [Xw_{t+1}, Pw_{t+1}, ..., Xw_N, Pw_N, F, S]
with m = ceil(N/2) the middle site (the paper's N_m = (N+1)/2 for odd N;
the even case is a reading, recorded in the design notes).  X_k means "an X
placed at site k, waiting for its partner", Xw_j "waiting for X_j", S "nothing
placed yet", F "a finished term".  This reproduces the paper's
L_1 = (X_1, P_1, 1, S_1) and R_N^T = (X_N, P_N, 1, S_N).

Kind codes of a core entry: 0 absent, 1 identity, 2 X, 3 P, 4 S_s,
5 c_X X + c_P P, 6 scalar * identity.
"""
from __future__ import annotations

import numpy as np

KIND_ABSENT, KIND_I, KIND_X, KIND_P, KIND_S, KIND_COMBO, KIND_SCALAR = range(7)


def middle_site(N: int) -> int:
    return (N + 1) // 2


def bond_labels(N: int, t: int):
    """Channel labels of bond t as tuples ('X', k), ('P', k), ('Xw', j),
    ('Pw', j), ('S',), ('F',) with 1-based sites."""
    m = middle_site(N)
    if t == 0:
        return [("S",)]
    if t == N:
        return [("F",)]
    if t < m:
        out = []
        for k in range(t, 0, -1):
            out += [("X", k), ("P", k)]
        return out + [("S",), ("F",)]
    out = []
    for j in range(t + 1, N + 1):
        out += [("Xw", j), ("Pw", j)]
    return out + [("F",), ("S",)]


def bond_dims(N: int):
    return [len(bond_labels(N, t)) for t in range(N + 1)]


def core_entries(N: int, s: int, alpha, beta, gamma):
    """Entries of core s (1-based) as {(row_label, col_label): (kind, cX, cP)};
    cX/cP hold the combination coefficients (kind 5) or the scalar (kind 6, in cX)."""
    m = middle_site(N)
    rows = bond_labels(N, s - 1)
    cols = bond_labels(N, s)
    rset, cset = set(rows), set(cols)
    a = lambda i, j: alpha[i - 1, j - 1]
    b = lambda i, j: beta[i - 1, j - 1]
    g = lambda i, j: gamma[i - 1, j - 1]
    E = {}

    def put(r, c, kind, cx=0.0, cp=0.0):
        if r in rset and c in cset:
            E[(r, c)] = (kind, cx, cp)

    S, F = ("S",), ("F",)
    put(S, S, KIND_I)
    put(F, F, KIND_I)
    put(S, F, KIND_S)
    if s < m:
        put(S, ("X", s), KIND_X)
        put(S, ("P", s), KIND_P)
        for k in range(1, s):
            put(("X", k), ("X", k), KIND_I)
            put(("P", k), ("P", k), KIND_I)
            put(("X", k), F, KIND_COMBO, a(k, s), g(k, s))
            put(("P", k), F, KIND_COMBO, g(s, k), b(k, s))
    elif s == m:
        for k in range(1, s):
            put(("X", k), F, KIND_COMBO, a(k, s), g(k, s))
            put(("P", k), F, KIND_COMBO, g(s, k), b(k, s))
        for j in range(s + 1, N + 1):
            put(S, ("Xw", j), KIND_COMBO, a(s, j), g(j, s))
            put(S, ("Pw", j), KIND_COMBO, g(s, j), b(s, j))
            for k in range(1, s):
                put(("X", k), ("Xw", j), KIND_SCALAR, a(k, j))
                put(("X", k), ("Pw", j), KIND_SCALAR, g(k, j))
                put(("P", k), ("Xw", j), KIND_SCALAR, g(j, k))
                put(("P", k), ("Pw", j), KIND_SCALAR, b(k, j))
    else:
        put(("Xw", s), F, KIND_X)
        put(("Pw", s), F, KIND_P)
        for j in range(s + 1, N + 1):
            put(("Xw", j), ("Xw", j), KIND_I)
            put(("Pw", j), ("Pw", j), KIND_I)
            put(S, ("Xw", j), KIND_COMBO, a(s, j), g(j, s))
            put(S, ("Pw", j), KIND_COMBO, g(s, j), b(s, j))
    return rows, cols, E


def structure(N: int):
    """(w[0..N], kinds) with kinds[s-1] an int8 (w_{s-1}, w_s) table."""
    z = np.zeros((N, N))
    w = bond_dims(N)
    kinds = []
    for s in range(1, N + 1):
        rows, cols, E = core_entries(N, s, z, z, z)
        K = np.zeros((len(rows), len(cols)), dtype=np.int8)
        for (rl, cl), (kind, _, _) in E.items():
            K[rows.index(rl), cols.index(cl)] = kind
        kinds.append(K)
    return w, kinds


def cores(alpha, beta, gamma, site_ops):
    """Dense cores W_s of shape (w_{s-1}, w_s, d, d).  site_ops[s-1] = (X, P, S)
    already truncated (and projected, with LBO) for site s."""
    N = alpha.shape[0]
    out = []
    for s in range(1, N + 1):
        X, P, Sop = site_ops[s - 1]
        d = X.shape[0]
        I = np.eye(d, dtype=np.complex128)
        rows, cols, E = core_entries(N, s, alpha, beta, gamma)
        W = np.zeros((len(rows), len(cols), d, d), dtype=np.complex128)
        for (rl, cl), (kind, cx, cp) in E.items():
            i, j = rows.index(rl), cols.index(cl)
            if kind == KIND_I:
                W[i, j] = I
            elif kind == KIND_X:
                W[i, j] = X
            elif kind == KIND_P:
                W[i, j] = P
            elif kind == KIND_S:
                W[i, j] = Sop
            elif kind == KIND_COMBO:
                W[i, j] = cx * X + cp * P
            elif kind == KIND_SCALAR:
                W[i, j] = cx * I
        out.append(W)
    return out


def to_dense(Ws) -> np.ndarray:
    """Contract the MPO to a dense matrix (row index = output/bra Fock string,
    row-major over sites)."""
    T = Ws[0][0]                       # (w_1, d, d)
    T = T.reshape(T.shape[0], T.shape[1], T.shape[2])
    # T[l, out, in] with out/in accumulated multi-indices
    for W in Ws[1:]:
        # T[l, O, I] W[l, m, o, i] -> T'[m, O o, I i]
        Tn = np.einsum("lOI,lmoi->mOoIi", T, W)
        wm = Tn.shape[0]
        T = Tn.reshape(wm, Tn.shape[1] * Tn.shape[2], Tn.shape[3] * Tn.shape[4])
    return T[0]
