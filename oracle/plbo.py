"""Parameterised local basis optimisation, pLBO (oracle; test infrastructure only).

Sec. III.B: the local basis of mode i is the image of the first d Fock states
under a gate sequence with eight real parameters per mode,
    U = D(alpha) S(r e^{i phi}) R(theta) P2(s) P3(gamma) K(kappa),
    p = (alpha_x, alpha_p, r, phi, theta, s, gamma, kappa),  alpha = alpha_x + i alpha_p,
(eq. pLBOUnitary gives U^dag as the reversed product of the inverses), and the
Hamiltonian is cast in that basis through the transformed operators
<m| U^dag O U |n>, m, n < d.  Gate conventions (those of the StrawberryFields
gates the paper names, with hbar = 2 in their quadrature):
    D(alpha)  = exp(alpha a^dag - alpha^* a)
    S(z)      = exp((z^* a^2 - z a^dag^2) / 2)
    R(theta)  = exp(i theta n)
    P2(s)     = exp(i s (a + a^dag)^2 / 4)
    P3(gamma) = exp(i gamma (a + a^dag)^3 / 6)
    K(kappa)  = exp(i kappa n^2)
Under these U^dag a U is the closed form of eq. SymplecticBasisTransformation.

Everything here follows the DEFINITION, not that closed form: every gate is the
matrix exponential (scipy.linalg.expm) of its generator in a Fock space of
L >> d levels, U is their product, and the transformed operator is the d x d
block of B^dag O B with B = U[:, :d] and O the L x L block of the quadratic
operator (formed at L + 4, SM Sec. 5).  For the parameter ranges of the tests
the columns of B carry a negligible weight near level L (checked by comparing
two values of L).

The energy of a site is linear in its five operators (X, P, S, X^2, XP + PX;
S = (a_ss X^2 + b_ss P^2 + g_ss (XP + PX))/2 - 1/2), so with the MPS held
fixed E(p) = Re sum_k <G_k, O_k(p)> + const, where G_k = dE/dO_k is the
environment of the operator slot k (core_environment + slot_gradients).  The
gradient in p is taken by a five-point central difference of that exact
function (the paper uses automatic differentiation; any exact derivative is
the same number).  The optimiser is Adam (Kingma & Ba, Algorithm 1), the one
the paper reports using per site (Sec. V, optimisation strategies).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import mpo as ompo, cz as ocz

NPARAM = 8
PARAM_NAMES = ("alpha_x", "alpha_p", "r", "phi", "theta", "s", "gamma", "kappa")


def _ladder(L: int) -> np.ndarray:
    a = np.zeros((L, L), dtype=np.complex128)
    for n in range(1, L):
        a[n - 1, n] = np.sqrt(n)
    return a


def _poly_block(L: int, power: int) -> np.ndarray:
    """L x L block of (a + a^dag)^power, formed at L + power and cut."""
    a = _ladder(L + power)
    y = a + a.conj().T
    out = np.eye(L + power, dtype=np.complex128)
    for _ in range(power):
        out = out @ y
    return out[:L, :L].copy()


def gate_unitary(p, L: int) -> np.ndarray:
    """U = D S R P2 P3 K on L Fock levels, each factor expm of its generator."""
    ax, ap, r, phi, th, s, g, k = [float(v) for v in p]
    a = _ladder(L)
    ad = a.conj().T
    n = np.arange(L, dtype=np.float64)
    al = ax + 1j * ap
    z = r * np.exp(1j * phi)
    I = np.eye(L, dtype=np.complex128)
    # a gate with a zero parameter is the identity (exp of the zero matrix)
    Dg = sla.expm(al * ad - np.conj(al) * a) if al != 0 else I
    Sg = sla.expm(0.5 * (np.conj(z) * (a @ a) - z * (ad @ ad))) if z != 0 else I
    Rg = np.diag(np.exp(1j * th * n))
    P2 = sla.expm(1j * s * _poly_block(L, 2) / 4.0) if s != 0 else I
    P3 = sla.expm(1j * g * _poly_block(L, 3) / 6.0) if g != 0 else I
    Kg = np.diag(np.exp(1j * k * n * n))
    return Dg @ Sg @ Rg @ P2 @ P3 @ Kg


def quadratic_blocks(L: int):
    """(X, P, X^2, P^2, XP + PX) on L levels, products formed at L + 4."""
    Lb = L + 4
    a = _ladder(Lb)
    ad = a.conj().T
    X = (a + ad) / np.sqrt(2.0)
    P = -1j * (a - ad) / np.sqrt(2.0)
    cut = lambda M: M[:L, :L].copy()
    return cut(X), cut(P), cut(X @ X), cut(P @ P), cut(X @ P + P @ X)


def transformed_ops(p, d: int, a_ss: float, b_ss: float, g_ss: float, L: int = 200):
    """(X, P, S, X^2, XP + PX) in the pLBO basis of parameters p, each the
    d x d block of U^dag O U (Sec. III.B; S is the single-site operator of the
    parent Hamiltonian, SM Sec. 8)."""
    U = gate_unitary(p, L)
    B = U[:, :d]
    X, P, X2, P2, Pt = quadratic_blocks(L)
    tr = lambda O: B.conj().T @ O @ B
    Xt, Pt_, X2t, P2t, PXt = tr(X), tr(P), tr(X2), tr(P2), tr(Pt)
    S = 0.5 * (a_ss * X2t + b_ss * P2t + g_ss * PXt) - 0.5 * np.eye(d)
    return Xt, Pt_, S, X2t, PXt


def fock_isometry(p, D: int, d: int, L: int = 200) -> np.ndarray:
    """U_{nm} = <n|U|m> for n < D, m < d: the map from the pLBO basis to the
    Fock basis used for photon-number observables (SM Sec. 5 figure)."""
    return gate_unitary(p, L)[:D, :d].copy()


# ------------------------------------------------------------ operator environments
def core_environment(Lenv, A, Renv):
    """Gfull[l, n, s, s'] = sum conj(A[a,s,b]) L[l,a,a'] A[a',s',b'] R[n,b,b'],
    the derivative of <A|H_eff|A> with respect to the core W[l, n, s, s']
    (environments in the oracle's convention: L[l, bra, ket], R[n, bra, ket])."""
    T = np.tensordot(Lenv, A, axes=([2], [0]))            # l a s' b'
    T = np.tensordot(T, Renv, axes=([3], [2]))            # l a s' n b
    return np.einsum("asb,lavnb->lnsv", A.conj(), T)


def slot_coefficients(make_core, d: int):
    """C_k[l, n] for the operator slots k = 0..5 (I, X, P, S, X^2, XP + PX) of a
    core that is linear in its site operators: make_core(ops) builds the core
    from a 5-tuple of d x d matrices; with d = 1 and unit/zero operators the
    core entries are the slot coefficients."""
    z = [np.zeros((1, 1), dtype=np.complex128)] * 5
    base = make_core(tuple(z))[..., 0, 0]
    out = [base]
    for k in range(5):
        ops = list(z)
        ops[k] = np.ones((1, 1), dtype=np.complex128)
        out.append(make_core(tuple(ops))[..., 0, 0] - base)
    return out


def gaussian_core_maker(alpha, beta, gamma, site: int):
    """make_core for site (0-based) of the Gaussian middle-site MPO (kappa = 0)."""
    N = alpha.shape[0]

    def make(ops):
        X, P, S, _, _ = ops
        site_ops = [(X, P, S) if t == site else (np.zeros_like(X),) * 3 for t in range(N)]
        return ompo.cores(alpha, beta, gamma, site_ops)[site]
    return make


def cz_core_maker(alpha, beta, gamma, kappa, site: int):
    """make_core for site (0-based) of the global-CZ MPO."""
    N = alpha.shape[0]

    def make(ops):
        site_ops = [ops if t == site else (np.zeros_like(ops[0]),) * 5 for t in range(N)]
        return ocz.cores(alpha, beta, gamma, kappa, site_ops)[site]
    return make


def slot_gradients(Gfull, coeffs):
    """G_k[s, s'] = sum_{l,n} C_k[l,n] Gfull[l,n,s,s'] for k = 0..5."""
    return np.stack([np.einsum("ln,lnst->st", C, Gfull) for C in coeffs])


def site_energy(G, ops) -> float:
    """Re sum_{k=0..5} <G_k, O_k> with O_0 = I and ops = (X, P, S, X^2, XP+PX)."""
    d = G.shape[1]
    full = [np.eye(d)] + list(ops)
    return float(sum(np.real(np.sum(G[k] * full[k])) for k in range(6)))


def param_gradient(G, p, d: int, a_ss: float, b_ss: float, g_ss: float, L: int = 200, h: float = 2e-4,
                   which=range(NPARAM)):
    """dE/dp_j by the five-point central difference
    (-f(+2h) + 8 f(+h) - 8 f(-h) + f(-2h)) / (12 h), truncation error O(h^4).
    The Kerr parameter enters through phases exp(i kappa n^2), so its
    derivatives grow like n^2 per order; h = 2e-4 keeps the truncation term
    below 1e-10 relative for d <= 10 while the rounding term stays ~1e-11."""
    p = np.asarray(p, dtype=np.float64)
    f = lambda q: site_energy(G, transformed_ops(q, d, a_ss, b_ss, g_ss, L))
    g = np.zeros(NPARAM)
    for j in which:
        e = np.zeros(NPARAM)
        e[j] = h
        g[j] = (-f(p + 2 * e) + 8 * f(p + e) - 8 * f(p - e) + f(p - 2 * e)) / (12 * h)
    return g


def adam(p, grad_fn, steps: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, mask=None, state=None):
    """Adam (Kingma & Ba, Algorithm 1) on the masked parameters; returns
    (p, (m, v, t)).  state carries the moment estimates between calls."""
    p = np.array(p, dtype=np.float64)
    m, v, t = (np.zeros(NPARAM), np.zeros(NPARAM), 0) if state is None else (state[0].copy(), state[1].copy(), state[2])
    mk = np.ones(NPARAM, bool) if mask is None else np.asarray(mask, bool)
    for _ in range(steps):
        g = np.where(mk, grad_fn(p), 0.0)
        t += 1
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p = p - np.where(mk, lr * mh / (np.sqrt(vh) + eps), 0.0)
    return p, (m, v, t)


def minimize_site(G, p0, d: int, a_ss: float, b_ss: float, g_ss: float, mask, L: int = 200):
    """Local minimum of the site energy over the masked parameters from p0 by
    scipy's L-BFGS-B (the optimiser family the paper also reports), with the
    five-point-difference gradient; returns (p, E)."""
    import scipy.optimize as so
    p0 = np.asarray(p0, dtype=np.float64)
    mk = np.asarray(mask, bool)
    free = np.flatnonzero(mk)

    def full(x):
        q = p0.copy()
        q[free] = x
        return q

    f = lambda x: site_energy(G, transformed_ops(full(x), d, a_ss, b_ss, g_ss, L))
    jac = lambda x: param_gradient(G, full(x), d, a_ss, b_ss, g_ss, L, which=free)[free]
    res = so.minimize(f, p0[free], jac=jac, method="L-BFGS-B", options={"maxiter": 100, "ftol": 1e-15, "gtol": 1e-8})
    return full(res.x), float(res.fun)


def effective_cutoff(p, d: int, D_max: int, tol: float, L: int = 200) -> int:
    """Effective cutoff of a pLBO basis (Sec. III.A, eq. Effectivecutoff, as
    used for the pLBO bases of the paper's pLBO figure): the smallest D in
    [d, D_max] at which the first d basis vectors U|m>, cut to D Fock rows,
    are orthonormal within tol; -1 if none."""
    V = fock_isometry(p, D_max, d, L=max(L, D_max + 64))
    for D in range(d, D_max + 1):
        Vd = V[:D]
        if np.abs(Vd.conj().T @ Vd - np.eye(d)).max() <= tol:
            return D
    return -1
