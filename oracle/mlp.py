"""Learned warm start (oracle; test infrastructure only).  Not in the paper:
the network is the hot path's learned part; its physical targets follow
Sec. III.A.1 (the optimal local basis of a Gaussian reduced state is a
squeezed Fock basis, eq. OLB / eq. diagReducedGaussianDM).

Reading taken here:
* features of output mode j of an instance (r, U): [j/N, N/64] and, for the 16
  largest |U_jk|, (r_k, |U_jk|, cos 2 arg U_jk, sin 2 arg U_jk) in descending
  order of |U_jk|, zero-padded (66 numbers).  The doubled angle: a squeezed
  vacuum is unchanged by a_k -> -a_k, so the reduced state of mode j of the
  Gaussian state depends on U_jk only through |U_jk| and U_jk^2;
* targets from a converged state's single-mode reduced density matrix rho_j:
  n = <a^dag a>, m = <a^2>; the state is S(zeta) tau S(zeta)^dag with tau
  thermal, S(zeta) = exp(1/2 (zeta* a^2 - zeta a^dag^2)), which gives
  (2 nbar + 1)^2 = (2n + 1)^2 - 4|m|^2, tanh(2|zeta|) = 2|m| / (2n + 1),
  zeta / |zeta| = -m / |m|; targets (Re zeta, Im zeta, log(1 + nbar));
* the basis W = first d columns of <n|S(zeta)|k>, from S(zeta)|0> (closed form)
  and S|k> = (a^dag cosh r + e^{-i phi} sinh r a) S|k-1> / sqrt(k), built on a
  larger box, cut to D rows and re-orthonormalised (Gram-Schmidt);
* the network: 3 dense layers (tanh, tanh, linear), mean-squared error, Adam.
"""
from __future__ import annotations

import math

import numpy as np

K_TOP = 16
IN_DIM = 2 + 4 * K_TOP
OUT_DIM = 3


def features(r, U, j):
    N = len(r)
    row = U[j]
    order = sorted(range(N), key=lambda k: (-abs(row[k]), k))[:K_TOP]
    f = [j / N, N / 64.0]
    for k in order:
        z = row[k]
        a = abs(z)
        th = math.atan2(z.imag, z.real)
        f += [float(r[k]), a, math.cos(2 * th) if a > 0 else 1.0, math.sin(2 * th) if a > 0 else 0.0]
    f += [0.0] * (IN_DIM - len(f))
    return np.array(f)


def moments(rho):
    """n = <a^dag a>, m = <a^2> for rho[n, n'] = <n|rho|n'>."""
    D = rho.shape[0]
    n = float(sum(k * rho[k, k].real for k in range(D)))
    # Tr(rho a^2) = sum_k <k|rho|k-2> sqrt(k (k-1)), since (a^2)_{k-2,k} = sqrt(k (k-1))
    m = complex(sum(rho[k, k - 2] * math.sqrt(k * (k - 1)) for k in range(2, D)))
    return n, m


def targets_from_moments(n, m):
    s = 2 * n + 1
    am = abs(m)
    nu2 = max(s * s - 4 * am * am, 1.0)
    nbar = 0.5 * (math.sqrt(nu2) - 1.0)
    r = 0.5 * math.atanh(min(2 * am / s, 1 - 1e-15)) if am > 0 else 0.0
    ph = (-m / am) if am > 0 else 1.0
    zeta = r * ph
    return np.array([zeta.real, zeta.imag, math.log1p(max(nbar, 0.0))])


def gaussian_params(V, j):
    """(Re zeta, Im zeta, log(1 + nbar)) of output mode j read off the reduced
    covariance V_j (2 x 2 block of V in xxpp order): <a^dag a> =
    (Vxx + Vpp)/2 - 1/2 and <a^2> = (Vxx - Vpp + 2i Vxp)/2 for a = (X + iP)/sqrt 2;
    the reduced state is exactly the squeezed thermal state with these moments
    (eq. diagReducedGaussianDM, eq. OLB)."""
    N = V.shape[0] // 2
    vxx, vpp, vxp = V[j, j], V[N + j, N + j], V[j, N + j]
    n = 0.5 * (vxx + vpp) - 0.5
    m = 0.5 * (vxx - vpp) + 1j * vxp
    return targets_from_moments(n, m)


def squeezed_basis(zeta, D, d, margin=64):
    """W (D x d): first d columns of <n|S(zeta)|k>, built on a (D + margin) box,
    cut to D rows, orthonormalised column by column."""
    Db = D + margin
    r = abs(zeta)
    e = zeta / r if r > 0 else 1.0
    t = math.tanh(r)
    v = np.zeros(Db, dtype=complex)
    for k in range(0, Db, 2):
        q = k // 2
        v[k] = (-e * t) ** q * math.sqrt(math.factorial(k)) / (2 ** q * math.factorial(q)) / math.sqrt(math.cosh(r)) \
            if k < 170 else 0.0
    cols = [v]
    ch, sh = math.cosh(r), math.sinh(r)
    for k in range(1, d):
        prev = cols[-1]
        nxt = np.zeros(Db, dtype=complex)
        for i in range(Db):
            acc = 0.0
            if i >= 1:
                acc += ch * math.sqrt(i) * prev[i - 1]           # a^dag
            if i + 1 < Db:
                acc += np.conj(e) * sh * math.sqrt(i + 1) * prev[i + 1]  # a
            nxt[i] = acc
        cols.append(nxt / math.sqrt(k))
    Wm = np.stack([c[:D] for c in cols], axis=1)
    for j in range(d):
        for i in range(j):
            Wm[:, j] -= np.vdot(Wm[:, i], Wm[:, j]) * Wm[:, i]
        Wm[:, j] /= np.linalg.norm(Wm[:, j])
    return Wm


def initial_product_state(y, D, d):
    """Warm-start state from outputs y[j] = (Re zeta, Im zeta, log(1 + nbar)):
    the squeezed basis of zeta_j and thermal amplitudes sqrt(lambda_m),
    lambda_m = nbar^m / (nbar + 1)^(m + 1) renormalised over m < d (the
    eigenvalues of a thermal state, eq. diagReducedGaussianDM)."""
    isos, amps = [], []
    for yj in y:
        zeta = complex(yj[0], yj[1])
        nbar = max(math.expm1(float(yj[2])), 0.0)
        lam = np.array([nbar ** m / (nbar + 1.0) ** (m + 1) for m in range(d)])
        isos.append(squeezed_basis(zeta, D, d))
        amps.append(np.sqrt(lam / lam.sum()))
    return isos, amps


# ------------------------------------------------------------------ network
def init_params(rng, in_dim=IN_DIM, hidden=256, out_dim=OUT_DIM):
    def lin(o, i):
        lim = math.sqrt(6.0 / (i + o))
        return rng.uniform(-lim, lim, (o, i)), rng.uniform(-0.1, 0.1, o)
    W1, b1 = lin(hidden, in_dim)
    W2, b2 = lin(hidden, hidden)
    W3, b3 = lin(out_dim, hidden)
    return [W1, b1, W2, b2, W3, b3]


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    H1 = np.tanh(X @ W1.T + b1)
    H2 = np.tanh(H1 @ W2.T + b2)
    Y = H2 @ W3.T + b3
    return Y, (X, H1, H2)


def loss_and_grads(params, X, T):
    """MSE = mean over batch and outputs of (Y - T)^2 and its gradients."""
    W1, b1, W2, b2, W3, b3 = params
    Y, (X, H1, H2) = forward(params, X)
    B, O = Y.shape
    L = float(np.mean((Y - T) ** 2))
    dY = 2.0 * (Y - T) / (B * O)
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * (1.0 - H2 ** 2)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * (1.0 - H1 ** 2)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(axis=0)
    return L, [dW1, db1, dW2, db2, dW3, db3]


def flatten(params):
    return np.concatenate([p.reshape(-1) for p in params])


def unflatten(vec, in_dim=IN_DIM, hidden=256, out_dim=OUT_DIM):
    shapes = [(hidden, in_dim), (hidden,), (hidden, hidden), (hidden,), (out_dim, hidden), (out_dim,)]
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(vec[o:o + n].reshape(s))
        o += n
    return out


def adam(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on flat arrays; state = (m, v, t)."""
    p, g = flatten(params), flatten(grads)
    m, v, t = state
    t += 1
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = p - lr * mh / (np.sqrt(vh) + eps)
    return unflatten(p, params[0].shape[1], params[0].shape[0], params[4].shape[0]), (m, v, t)
