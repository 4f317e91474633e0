"""Pythonic wrappers with the C ABI's names (marshalling only)."""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np

from . import _lib as L
from ._lib import TnError, TN_FP64 as FP64, TN_FP32 as FP32, TN_BF16X3 as BF16X3


def _check(ctx, status):
    if status != L.TN_OK:
        msg = L.lib().tn_last_error(ctx).decode() if ctx else ""
        raise TnError(status, msg)


def _torch():
    import torch
    return torch


class Context:
    """A library context on one GPU, enqueueing on torch's current stream and
    allocating through torch's caching allocator."""

    def __init__(self, device: int = 0, use_torch_allocator: bool = False, alloc_gate=None):
        """alloc_gate (with use_torch_allocator): a callable taking the byte
        count; when it returns False the allocator reports failure, which
        lets tests drive the library's out-of-memory path from the host."""
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library needs an MI355X")
        torch.cuda.set_device(device)
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self._alloc = None
        ap = None
        if use_torch_allocator:
            dev = device

            @C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
            def _a(nbytes, user):
                if alloc_gate is not None and not alloc_gate(int(nbytes)):
                    return None
                try:
                    return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev))
                except Exception:
                    return None

            @C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
            def _f(ptr, user):
                if ptr:
                    torch.cuda.caching_allocator_delete(int(ptr))

            self._alloc = L.tn_allocator(_a, _f, None)
            ap = C.byref(self._alloc)
        h = C.c_void_p()
        _check(None, L.lib().tn_ctx_create(device, C.c_void_p(self.stream.cuda_stream), ap, C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            for obj in list(self._children):
                obj._release()
            L.lib().tn_ctx_destroy(self.h)
            self.h = None

    @property
    def _children(self):
        import weakref
        if not hasattr(self, "_kids"):
            self._kids = weakref.WeakSet()
        return self._kids

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, status):
        _check(self.h, status)

    def profile(self, mode: int = -1) -> dict:
        """mode -1 read, 0 stop+reset, 1 start (reset first)."""
        out = np.zeros(16)
        self.check(L.lib().tn_profile(self.h, mode, L.dptr(out)))
        keys = ["ms_convert", "ms_gemm_l", "ms_ops", "ms_gemm_r", "ms_reduce", "matvecs",
                "flops_l", "flops_r", "flops_matvec", "bytes_l", "bytes_r",
                "ms_tridiag", "tridiag_launches", "bytes_tridiag", "lanczos_iters", "lanczos_full_passes"]
        return dict(zip(keys, out.tolist()))

    @property
    def last_error(self) -> str:
        return L.lib().tn_last_error(self.h).decode()


class MPO:
    """Middle-site MPO of PHP for per-mode squeezing r and interferometer U."""

    def __init__(self, ctx: Context, r, U, D_raw: int, d: int | None = None, iso=None, kappa: float = 0.0):
        self.ctx = ctx
        r = np.ascontiguousarray(r, dtype=np.float64)
        U = np.ascontiguousarray(U, dtype=np.complex128)
        N = len(r)
        d = D_raw if d is None else d
        self.N, self.D_raw, self.d = N, D_raw, d
        self._r = r
        self._U = U.view(np.float64).copy()
        self._iso = None if iso is None else np.ascontiguousarray(iso, dtype=np.complex128).view(np.float64).copy()
        self.kappa = float(kappa)
        prob = L.tn_problem(N, D_raw, d, L.dptr(self._r), L.dptr(self._U),
                            None if self._iso is None else L.dptr(self._iso), self.kappa)
        h = C.c_void_p()
        ctx.check(L.lib().tn_mpo_build(ctx.h, C.byref(prob), C.byref(h)))
        self.h = h
        ctx._children.add(self)

    def structure(self):
        w = np.zeros(self.N + 1, dtype=np.int32)
        L.lib().tn_mpo_structure(self.h, L.dptr(w, C.c_int32), None)
        tot = int(sum(int(w[s]) * int(w[s + 1]) for s in range(self.N)))
        k = np.zeros(tot, dtype=np.int8)
        L.lib().tn_mpo_structure(self.h, L.dptr(w, C.c_int32), L.dptr(k, C.c_int8))
        kinds, off = [], 0
        for s in range(self.N):
            n = int(w[s]) * int(w[s + 1])
            kinds.append(k[off:off + n].reshape(int(w[s]), int(w[s + 1])))
            off += n
        return w, kinds

    def coefficients(self):
        a = np.zeros((self.N, self.N)); b = np.zeros_like(a); g = np.zeros_like(a)
        L.lib().tn_mpo_coefficients(self.h, L.dptr(a), L.dptr(b), L.dptr(g))
        return a, b, g

    def isometries(self):
        out = np.zeros((self.N, self.D_raw, self.d), dtype=np.complex128)
        L.lib().tn_mpo_isometries(self.h, L.dptr(out.view(np.float64)))
        return out

    def site_ops(self, s: int):
        """(X, P, S, X^2, XP + PX) of site s in the current basis."""
        out = np.zeros((5, self.d, self.d), dtype=np.complex128)
        self.ctx.check(L.lib().tn_mpo_site_ops(self.h, s, L.dptr(out.view(np.float64))))
        return out

    def _release(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            L.lib().tn_mpo_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self._release()
        except Exception:
            pass


class MPS:
    """Device MPS created from host site tensors (chi_{s}, d, chi_{s+1})."""

    def __init__(self, ctx: Context, tensors):
        self.ctx = ctx
        N = len(tensors)
        d = tensors[0].shape[1]
        dims = [1] + [int(t.shape[2]) for t in tensors]
        self.N, self.d = N, d
        flat = np.concatenate([np.ascontiguousarray(t, dtype=np.complex128).reshape(-1) for t in tensors])
        flat = flat.view(np.float64)
        dims = np.asarray(dims, dtype=np.int32)
        h = C.c_void_p()
        ctx.check(L.lib().tn_mps_create(ctx.h, N, d, L.dptr(dims, C.c_int32), L.dptr(flat), C.byref(h)))
        self.h = h
        ctx._children.add(self)

    def bond_dims(self):
        w = np.zeros(self.N + 1, dtype=np.int32)
        L.lib().tn_mps_bond_dims(self.h, L.dptr(w, C.c_int32))
        return w

    def export(self):
        need = C.c_size_t()
        self.ctx.check(L.lib().tn_mps_export(self.ctx.h, self.h, None, 0, C.byref(need)))
        buf = np.zeros(need.value, dtype=np.float64)
        self.ctx.check(L.lib().tn_mps_export(self.ctx.h, self.h, L.dptr(buf), need.value, C.byref(need)))
        z = buf.view(np.complex128)
        dims = self.bond_dims()
        out, off = [], 0
        for s in range(self.N):
            n = int(dims[s]) * self.d * int(dims[s + 1])
            out.append(z[off:off + n].reshape(int(dims[s]), self.d, int(dims[s + 1])).copy())
            off += n
        return out

    def canonicalize(self):
        self.ctx.check(L.lib().tn_mps_canonicalize(self.ctx.h, self.h))

    @property
    def sweeps(self) -> int:
        n = C.c_int64()
        self.ctx.check(L.lib().tn_mps_sweeps(self.h, C.byref(n)))
        return n.value

    def checkpoint(self, mpo: "MPO | None" = None) -> np.ndarray:
        """The flat FP64 checkpoint buffer (tensors, centre, sweep counter and,
        with mpo, its isometries)."""
        need = C.c_size_t()
        mh = None if mpo is None else mpo.h
        self.ctx.check(L.lib().tn_mps_checkpoint(self.ctx.h, self.h, mh, None, 0, C.byref(need)))
        buf = np.zeros(need.value, dtype=np.float64)
        self.ctx.check(L.lib().tn_mps_checkpoint(self.ctx.h, self.h, mh, L.dptr(buf), need.value, C.byref(need)))
        return buf

    @classmethod
    def from_checkpoint(cls, ctx: Context, buf):
        """(MPS, isometries [N][D_raw][d] or None) from a checkpoint buffer."""
        buf = np.ascontiguousarray(buf, dtype=np.float64)
        N, d, D = int(buf[2]), int(buf[3]), int(buf[6])
        iso = np.zeros((N, max(D, 1), d), dtype=np.complex128)
        info = np.zeros(2, dtype=np.int32)
        h = C.c_void_p()
        ctx.check(L.lib().tn_mps_import(ctx.h, L.dptr(buf), buf.size, C.byref(h), L.dptr(iso.view(np.float64)),
                                        L.dptr(info, C.c_int32)))
        self = cls.__new__(cls)
        self.ctx, self.N, self.d, self.h = ctx, N, d, h
        ctx._children.add(self)
        return self, (iso if D > 0 else None)

    def _release(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            L.lib().tn_mps_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self._release()
        except Exception:
            pass


@dataclasses.dataclass
class SweepOpts:
    chi_max: int = 16
    sigma_cut: float = 0.0
    tol: float = 1e-12
    krylov_max: int = 32
    max_matvecs: int = 200
    precision: int = FP64
    lbo: int = 0
    compute_energy: int = 1
    lbo_matvecs: int = 0

    def c(self):
        return L.tn_sweep_opts(self.chi_max, self.sigma_cut, self.tol, self.krylov_max,
                               self.max_matvecs, self.precision, self.lbo, self.compute_energy, self.lbo_matvecs)


def dmrg_sweep(ctx: Context, mpo: MPO, mps: MPS, opts: SweepOpts) -> dict:
    st = L.tn_sweep_stats()
    o = opts.c()
    ctx.check(L.lib().tn_dmrg_sweep(ctx.h, mpo.h, mps.h, C.byref(o), C.byref(st)))
    return st.as_dict()


def dmrg_solve(ctx: Context, mpo: MPO, mps: MPS, sweep: SweepOpts, max_sweeps: int = 20,
               bulk_precision: int = FP32, max_refine: int = 2, target: float = 1e-8,
               switch_tol: float = 1e-5, conv_tol: float = 1e-12, bulk_tol: float = 1e-6,
               refine_tol: float = 1e-9, lbo_bulk: int = 1, lbo_refine: int = 0) -> dict:
    """Sweeps with the precision schedule until <H> <= target (see tn_dmrg_solve)."""
    so = L.tn_solve_opts(max_sweeps, bulk_precision, max_refine, lbo_bulk, lbo_refine, 0, target, switch_tol,
                         conv_tol, bulk_tol, refine_tol, sweep.c())
    res = L.tn_solve_result()
    et = np.full(max_sweeps, np.nan)
    tt = np.full(max_sweeps, np.nan)
    ctx.check(L.lib().tn_dmrg_solve(ctx.h, mpo.h, mps.h, C.byref(so), C.byref(res), L.dptr(et), L.dptr(tt)))
    d = res.as_dict()
    d["energy_trace"] = et[:res.sweeps].tolist()
    d["time_trace"] = tt[:res.sweeps].tolist()
    return d


def energy(ctx: Context, mpo: MPO, mps: MPS):
    e = C.c_double()
    n = C.c_double()
    ctx.check(L.lib().tn_energy(ctx.h, mpo.h, mps.h, C.byref(e), C.byref(n)))
    return e.value, n.value


def energy_variance(ctx: Context, mpo: MPO, mps: MPS):
    """(<H>, <H^2>, sigma_H^2) of the normalised state, FP64."""
    e, h2, v = C.c_double(), C.c_double(), C.c_double()
    ctx.check(L.lib().tn_energy_variance(ctx.h, mpo.h, mps.h, C.byref(e), C.byref(h2), C.byref(v)))
    return e.value, h2.value, v.value


def lbo_step(ctx: Context, mpo: MPO, mps: MPS, site: int, opts: SweepOpts) -> float:
    disc = C.c_double()
    o = opts.c()
    ctx.check(L.lib().tn_lbo_step(ctx.h, mpo.h, mps.h, site, C.byref(o), C.byref(disc)))
    return disc.value


PLBO_NPARAM = 8


PLBO_ADAM, PLBO_LBFGS = 0, 1


class PlboOpts:
    """Per-visit pLBO step: Lanczos matvecs on the centre tensor, then Adam
    steps or L-BFGS iterations on the masked parameters (bit j of mask:
    parameter j)."""
    steps: int = 10
    matvecs: int = 0
    lr: float = 0.02
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    mask: int = 0xFF
    optimizer: int = PLBO_ADAM

    def __init__(self, **kw):
        for k, v in kw.items():
            if not hasattr(self, k):
                raise AttributeError(k)
            setattr(self, k, v)

    def c(self):
        return L.tn_plbo_opts(self.steps, self.matvecs, self.lr, self.beta1, self.beta2, self.eps, self.mask,
                              self.optimizer)


def plbo_ops(d: int, params, a_ss: float, b_ss: float, g_ss: float, derivatives: bool = False):
    """(X, P, S, X^2, XP + PX) in the gate-parameterised basis, [5][d][d]
    complex; with derivatives also d/dp_j of each, [8][5][d][d]."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    ops = np.zeros((5, d, d), dtype=np.complex128)
    dops = np.zeros((PLBO_NPARAM, 5, d, d), dtype=np.complex128) if derivatives else None
    st = L.lib().tn_plbo_ops(d, L.dptr(p), a_ss, b_ss, g_ss, L.dptr(ops.view(np.float64)),
                             L.dptr(dops.view(np.float64)) if derivatives else None)
    if st != L.TN_OK:
        raise TnError(st, "tn_plbo_ops: bad arguments")
    return (ops, dops) if derivatives else ops


def plbo_fock_isometry(D: int, d: int, params, levels: int | None = None):
    """<n|U|m> for n < D, m < d, [D][d] complex."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    W = np.zeros((D, d), dtype=np.complex128)
    lv = max(D, d) + 192 if levels is None else levels
    st = L.lib().tn_plbo_fock_isometry(D, d, L.dptr(p), lv, L.dptr(W.view(np.float64)))
    if st != L.TN_OK:
        raise TnError(st, "tn_plbo_fock_isometry: bad arguments")
    return W


def plbo_minimize(G, params, a_ss: float, b_ss: float, g_ss: float, opts: PlboOpts):
    """Host-side optimisation of one site's parameters with its slot
    environments G ([6][d][d]) fixed: (params [8], final site energy)."""
    G = np.ascontiguousarray(G, dtype=np.complex128)
    d = G.shape[1]
    p = np.array(params, dtype=np.float64)
    e = C.c_double()
    o = opts.c()
    st = L.lib().tn_plbo_minimize(d, L.dptr(G.view(np.float64)), a_ss, b_ss, g_ss, C.byref(o), L.dptr(p), C.byref(e))
    if st != L.TN_OK:
        raise TnError(st, "tn_plbo_minimize: bad arguments")
    return p, e.value


def plbo_effective_cutoff(d: int, params, D_max: int = 256, tol: float = 1e-10) -> int:
    """Smallest Fock cutoff at which the first d pLBO basis vectors are
    orthonormal within tol (-1 if none up to D_max)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    out = C.c_int32()
    st = L.lib().tn_plbo_effective_cutoff(d, L.dptr(p), D_max, tol, C.byref(out))
    if st != L.TN_OK:
        raise TnError(st, "tn_plbo_effective_cutoff: bad arguments")
    return out.value


def plbo_enable(ctx: Context, mpo: MPO, params=None):
    """Switch mpo to gate-parameterised bases ([N][8] parameters, None: zeros)."""
    if params is None:
        ctx.check(L.lib().tn_plbo_enable(mpo.h, None))
    else:
        p = np.ascontiguousarray(params, dtype=np.float64).reshape(mpo.N, PLBO_NPARAM)
        ctx.check(L.lib().tn_plbo_enable(mpo.h, L.dptr(p)))


def plbo_linear(ctx: Context, mpo: MPO):
    """Put a linear isometry (D_raw x d, optimised by the LBO step) on top of
    the gate-parameterised bases (SM Sec. 6)."""
    ctx.check(L.lib().tn_plbo_linear(mpo.h))


def plbo_linear_isometries(ctx: Context, mpo: MPO):
    W = np.zeros((mpo.N, mpo.D_raw, mpo.d), dtype=np.complex128)
    ctx.check(L.lib().tn_plbo_linear_isometries(mpo.h, L.dptr(W.view(np.float64))))
    return W


def plbo_params(ctx: Context, mpo: MPO):
    p = np.zeros((mpo.N, PLBO_NPARAM))
    ctx.check(L.lib().tn_plbo_params(mpo.h, L.dptr(p)))
    return p


def plbo_site_gradient(ctx: Context, mpo: MPO, mps: MPS, site: int, precision: int = FP64):
    """(G [6][d][d] complex, energy, grad [8]) at the orthogonality centre."""
    G = np.zeros((6, mpo.d, mpo.d), dtype=np.complex128)
    e = C.c_double()
    g = np.zeros(PLBO_NPARAM)
    ctx.check(L.lib().tn_plbo_site_gradient(ctx.h, mpo.h, mps.h, site, precision, L.dptr(G.view(np.float64)),
                                            C.byref(e), L.dptr(g)))
    return G, e.value, g


def plbo_sweep(ctx: Context, mpo: MPO, mps: MPS, opts: SweepOpts, popts: PlboOpts) -> dict:
    """One two-site sweep with a pLBO step at every centre visit; the stats
    dict gains "plbo_gain" (summed site-energy decrease of the parameter steps)."""
    st = L.tn_sweep_stats()
    o = opts.c()
    po = popts.c()
    g = C.c_double()
    ctx.check(L.lib().tn_plbo_sweep(ctx.h, mpo.h, mps.h, C.byref(o), C.byref(po), C.byref(st), C.byref(g)))
    out = st.as_dict()
    out["plbo_gain"] = g.value
    return out


def marginals(ctx: Context, mps: MPS, mpo: MPO, n_modes: int | None = None):
    n = mps.N if n_modes is None else n_modes
    out = np.zeros((n, mpo.D_raw))
    ctx.check(L.lib().tn_marginals(ctx.h, mps.h, mpo.h, n, L.dptr(out)))
    return out


def sample(ctx: Context, mps: MPS, mpo: MPO, n_samples: int, seed: int):
    torch = _torch()
    out = torch.empty((n_samples, mps.N), dtype=torch.int32, device=f"cuda:{ctx.device}")
    ctx.check(L.lib().tn_sample(ctx.h, mps.h, mpo.h, n_samples, C.c_uint64(seed), C.c_void_p(out.data_ptr())))
    return out


def noise_uniform_loss(r, U, eta: float):
    """(r_pure [N], L [2N][N]): the pure part and the displacement factor
    C = L L^T of uniform loss eta (eq. CovarianceDecomposition)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    Uf = np.ascontiguousarray(U, dtype=np.complex128).view(np.float64)
    N = len(r)
    rp = np.zeros(N)
    Lc = np.zeros((2 * N, N))
    st = L.lib().tn_noise_uniform_loss(N, L.dptr(r), L.dptr(Uf), eta, L.dptr(rp), L.dptr(Lc))
    if st != L.TN_OK:
        raise TnError(st, "tn_noise_uniform_loss: bad arguments")
    return rp, Lc


def noise_williamson(V):
    """(r_pure [N], U_pure [N][N], L [2N][K]): the Williamson split of a mixed
    covariance V = Q + C with Q = covariance(r_pure, U_pure) and C = L L^T."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    N = V.shape[0] // 2
    rp = np.zeros(N)
    Up = np.zeros((N, N), dtype=np.complex128)
    Lc = np.zeros(4 * N * N)
    K = C.c_int32()
    st = L.lib().tn_noise_williamson(N, L.dptr(V), L.dptr(rp), L.dptr(Up.view(np.float64)), L.dptr(Lc), C.byref(K))
    if st != L.TN_OK:
        raise TnError(st, "tn_noise_williamson: bad covariance")
    return rp, Up, Lc[: 2 * N * K.value].reshape(2 * N, K.value).copy()


def sample_displaced(ctx: Context, mps: MPS, mpo: MPO, n_samples: int, seed: int, Lc, z=None):
    """Noisy-GBS samples: photon numbers of D(alpha_b)|psi> with alpha_b from
    d = Lc z_b, Lc of shape (2N, K).  z: (n_samples, K) standard normals
    (device or host); when None the library draws them from its counter-based
    generator seeded with `seed` (Philox4x32-10 and the Box-Muller transform)."""
    torch = _torch()
    dev = f"cuda:{ctx.device}"
    Lh = np.ascontiguousarray(Lc, dtype=np.float64)
    if Lh.ndim != 2 or Lh.shape[0] != 2 * mps.N:
        raise ValueError("Lc must have shape (2N, K)")
    K = Lh.shape[1]
    zp = None
    if z is not None:
        z = torch.as_tensor(np.ascontiguousarray(z, dtype=np.float64) if not hasattr(z, "device") else z,
                            dtype=torch.float64).to(dev).contiguous()
        if tuple(z.shape) != (n_samples, K):
            raise ValueError("z must have shape (n_samples, K)")
        zp = z.data_ptr()
    out = torch.empty((n_samples, mps.N), dtype=torch.int32, device=dev)
    ctx.check(L.lib().tn_sample_displaced(ctx.h, mps.h, mpo.h, n_samples, C.c_uint64(seed), K,
                                          C.c_void_p(zp), L.dptr(Lh), C.c_void_p(out.data_ptr())))
    return out


def _dev(x):
    torch = _torch()
    assert x.is_cuda and x.dtype == torch.complex128 and x.is_contiguous()
    return C.c_void_p(x.data_ptr())


def heff_apply(ctx: Context, mpo: MPO, site: int, Lenv, Renv, theta, precision: int = FP64):
    """theta' = H_eff theta for the window (site, site+1); torch complex128 cuda tensors."""
    torch = _torch()
    chi_l, chi_r = int(theta.shape[0]), int(theta.shape[-1])
    out = torch.empty_like(theta)
    ctx.check(L.lib().tn_heff_apply(ctx.h, mpo.h, site, chi_l, chi_r, _dev(Lenv), _dev(Renv), _dev(theta),
                                    _dev(out), precision))
    return out


def env_update(ctx: Context, mpo: MPO, site: int, direction: int, env_in, A, precision: int = FP64):
    torch = _torch()
    chi_l, chi_r = int(A.shape[0]), int(A.shape[2])
    w = int(mpo.structure()[0][site + 1] if direction > 0 else mpo.structure()[0][site])
    chi = chi_r if direction > 0 else chi_l
    out = torch.empty((w, chi, chi), dtype=torch.complex128, device=A.device)
    ctx.check(L.lib().tn_env_update(ctx.h, mpo.h, site, direction, chi_l, chi_r, _dev(env_in), _dev(A),
                                    _dev(out), precision))
    return out


def truncate(ctx: Context, theta, chi: int, sigma_cut: float = 0.0, direction: int = 1):
    """SVD truncation of the m x n device matrix theta (complex128)."""
    torch = _torch()
    m, n = int(theta.shape[0]), int(theta.shape[1])
    kmax = max(1, min(chi, m, n))
    left = torch.empty((m, kmax), dtype=torch.complex128, device=theta.device)
    right = torch.empty((kmax, n), dtype=torch.complex128, device=theta.device)
    k = C.c_int32()
    sv = np.zeros(kmax)
    disc = C.c_double()
    ctx.check(L.lib().tn_truncate(ctx.h, m, n, _dev(theta), chi, sigma_cut, direction, _dev(left), _dev(right),
                                  C.byref(k), L.dptr(sv), C.byref(disc)))
    kk = k.value
    return left[:, :kk].contiguous() if kk < kmax else left, \
        right[:kk].contiguous(), sv[:kk], disc.value


def cgemm(ctx: Context, A, B, precision: int = FP64, trans_a: bool = False, trans_b: bool = False):
    """C = op(A) op(B) on the matrix cores (torch complex cuda tensors: complex128
    for FP64, complex64 for FP32 / BF16x3)."""
    torch = _torch()
    M = A.shape[1] if trans_a else A.shape[0]
    K = A.shape[0] if trans_a else A.shape[1]
    N = B.shape[0] if trans_b else B.shape[1]
    C_ = torch.empty((M, N), dtype=A.dtype, device=A.device)
    ctx.check(L.lib().tn_cgemm(ctx.h, precision, int(trans_a), int(trans_b), M, N, K, C.c_void_p(A.data_ptr()),
                               A.shape[1], C.c_void_p(B.data_ptr()), B.shape[1], C.c_void_p(C_.data_ptr()), N))
    return C_


def philox4x32_10(ctx: Context, ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros_like(ctr)
    ctx.check(L.lib().tn_philox4x32_10(ctx.h, L.dptr(ctr, C.c_uint32), L.dptr(key, C.c_uint32),
                                       L.dptr(out, C.c_uint32), len(ctr)))
    return out


def matvec_flops(mpo: MPO, site: int, chi_l: int, chi_r: int) -> float:
    return L.lib().tn_matvec_flops(mpo.h, site, chi_l, chi_r)


def env_flops(mpo: MPO, site: int, chi_l: int, chi_r: int) -> float:
    return L.lib().tn_env_flops(mpo.h, site, chi_l, chi_r)


def rdm(ctx: Context, mps: MPS, mpo: MPO, n_modes: int | None = None):
    """Single-site reduced density matrices [n_modes][D_raw][D_raw] (FP64)."""
    n = mps.N if n_modes is None else n_modes
    out = np.zeros((n, mpo.D_raw, mpo.D_raw), dtype=np.complex128)
    ctx.check(L.lib().tn_rdm(ctx.h, mps.h, mpo.h, n, L.dptr(out.view(np.float64))))
    return out


def squeezed_basis(zeta: complex, D: int, d: int, margin: int = 64):
    out = np.zeros((D, d), dtype=np.complex128)
    st = L.lib().tn_squeezed_basis(float(np.real(zeta)), float(np.imag(zeta)), D, d, margin,
                                   L.dptr(out.view(np.float64)))
    if st != L.TN_OK:
        raise TnError(st, "tn_squeezed_basis: bad arguments")
    return out


def _fdev(x):
    torch = _torch()
    assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
    return C.c_void_p(x.data_ptr())


class MLP:
    """3-layer FP32 perceptron trained by the library's kernels (tn_mlp_*)."""

    def __init__(self, ctx: Context, in_dim: int, hidden: int, out_dim: int, seed: int = 0):
        self.ctx = ctx
        self.in_dim, self.hidden, self.out_dim = in_dim, hidden, out_dim
        h = C.c_void_p()
        ctx.check(L.lib().tn_mlp_create(ctx.h, in_dim, hidden, out_dim, C.c_uint64(seed), C.byref(h)))
        self.h = h
        ctx._children.add(self)

    @property
    def num_params(self) -> int:
        return int(L.lib().tn_mlp_num_params(self.h))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.num_params, dtype=np.float32)
        self.ctx.check(L.lib().tn_mlp_params(self.ctx.h, self.h, L.dptr(out, C.c_float), None))
        return out

    def set_params(self, flat) -> None:
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        if flat.size != self.num_params:
            raise ValueError("parameter vector has the wrong length")
        self.ctx.check(L.lib().tn_mlp_params(self.ctx.h, self.h, None, L.dptr(flat, C.c_float)))

    def forward(self, X):
        torch = _torch()
        Y = torch.empty((X.shape[0], self.out_dim), dtype=torch.float32, device=X.device)
        self.ctx.check(L.lib().tn_mlp_forward(self.ctx.h, self.h, _fdev(X), int(X.shape[0]), _fdev(Y)))
        return Y

    def grad(self, X, T):
        g = np.zeros(self.num_params, dtype=np.float32)
        loss = C.c_float()
        self.ctx.check(L.lib().tn_mlp_grad(self.ctx.h, self.h, _fdev(X), _fdev(T), int(X.shape[0]),
                                           L.dptr(g, C.c_float), C.byref(loss)))
        return loss.value, g

    def train_step(self, X, T, lr: float) -> float:
        loss = C.c_float()
        self.ctx.check(L.lib().tn_mlp_train_step(self.ctx.h, self.h, _fdev(X), _fdev(T), int(X.shape[0]),
                                                 C.c_float(lr), C.byref(loss)))
        return loss.value

    def _release(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            L.lib().tn_mlp_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self._release()
        except Exception:
            pass


def ws_features(r, U):
    """Network inputs [N][66] of every output mode (tn_ws_features)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    Uf = np.ascontiguousarray(U, dtype=np.complex128).view(np.float64)
    out = np.zeros((len(r), 66), dtype=np.float32)
    st = L.lib().tn_ws_features(len(r), L.dptr(r), L.dptr(Uf), L.dptr(out, C.c_float))
    if st != L.TN_OK:
        raise TnError(st, "tn_ws_features: bad arguments")
    return out


def ws_targets(rho):
    """Training targets [n][3] from reduced density matrices [n][D][D]."""
    rho = np.ascontiguousarray(rho, dtype=np.complex128)
    out = np.zeros((rho.shape[0], 3), dtype=np.float32)
    st = L.lib().tn_ws_targets(rho.shape[0], rho.shape[1], L.dptr(rho.view(np.float64)), L.dptr(out, C.c_float))
    if st != L.TN_OK:
        raise TnError(st, "tn_ws_targets: bad arguments")
    return out


def ws_gaussian_params(r, U):
    """Analytic local-basis parameters [N][3] from each mode's reduced covariance."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    Uf = np.ascontiguousarray(U, dtype=np.complex128).view(np.float64)
    out = np.zeros((len(r), 3), dtype=np.float32)
    st = L.lib().tn_ws_gaussian_params(len(r), L.dptr(r), L.dptr(Uf), L.dptr(out, C.c_float))
    if st != L.TN_OK:
        raise TnError(st, "tn_ws_gaussian_params: bad arguments")
    return out


def cutoff_report(r, U, d: int, D_max: int = 256, tol: float = 1e-12):
    """Cutoff errors of the Gaussian optimal basis with d kept states per mode:
    {"eps_mode": [N], "eps": eps, "eps_D_bounds": (eps, N eps), "D_eff": [N]}."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    Uf = np.ascontiguousarray(U, dtype=np.complex128).view(np.float64)
    N = len(r)
    eps = np.zeros(N)
    deff = np.zeros(N, dtype=np.int32)
    b = np.zeros(2)
    st = L.lib().tn_cutoff_report(N, L.dptr(r), L.dptr(Uf), d, D_max, tol, L.dptr(eps), L.dptr(deff, C.c_int32),
                                  L.dptr(b))
    if st != L.TN_OK:
        raise TnError(st, "tn_cutoff_report: bad arguments")
    return {"eps_mode": eps, "eps": float(b[0]), "eps_D_bounds": (float(b[0]), float(b[1])), "D_eff": deff}


def ws_initial_state(y, D: int, d: int, chi: int, seed: int, noise: float = 1e-3):
    """(isometries [N][D][d], site tensors) of the learned warm start."""
    y = np.ascontiguousarray(y, dtype=np.float32)
    N = y.shape[0]
    dims = np.zeros(N + 1, dtype=np.int32)
    need = C.c_size_t()
    iso = np.zeros((N, D, d), dtype=np.complex128)
    lib = L.lib()
    st = lib.tn_ws_initial_state(N, D, d, chi, L.dptr(y, C.c_float), C.c_uint64(seed), noise,
                                 L.dptr(iso.view(np.float64)), L.dptr(dims, C.c_int32), None, 0, C.byref(need))
    if st != L.TN_OK:
        raise TnError(st, "tn_ws_initial_state: bad arguments")
    buf = np.zeros(need.value, dtype=np.float64)
    st = lib.tn_ws_initial_state(N, D, d, chi, L.dptr(y, C.c_float), C.c_uint64(seed), noise,
                                 L.dptr(iso.view(np.float64)), L.dptr(dims, C.c_int32), L.dptr(buf), need.value,
                                 C.byref(need))
    if st != L.TN_OK:
        raise TnError(st, "tn_ws_initial_state: bad outputs")
    z = buf.view(np.complex128)
    out, off = [], 0
    for s in range(N):
        n = int(dims[s]) * d * int(dims[s + 1])
        out.append(z[off:off + n].reshape(int(dims[s]), d, int(dims[s + 1])).copy())
        off += n
    return iso, out
