"""Learned warm start of the DMRG + local-basis-optimisation solve.

A 3-layer FP32 perceptron (the library's tn_mlp_* kernels) maps the features
of output mode j of an instance (r, U) to the parameters of a squeezed thermal
single-mode state: the squeezing zeta_j, whose squeezed Fock basis is the
optimal local basis of a Gaussian reduced state (Sec. III.A.1), and the
thermal occupation nbar_j, whose eigenvalues give a product-state initial MPS.
Training targets come from the solver itself: plain DMRG + LBO runs, their
single-site reduced density matrices (tn_rdm) and the moment map
tn_ws_targets.  <H> after the first sweep decides whether the learned start
is kept; when it is worse than the plain start's first sweep, or not finite,
the plain start is used (and its time is counted).

This module only orders calls into the library; every arithmetic step runs in
libtn.so (kernels, or host helpers that do no GPU work).
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import api

HIDDEN = 256
IN_DIM = 66
OUT_DIM = 3


@dataclasses.dataclass
class RunTrace:
    energies: list
    seconds: list          # cumulative wall seconds after each sweep
    init_seconds: float    # building the start (network, basis, MPO, MPS)
    phases: dict = dataclasses.field(default_factory=dict)   # summed sweep statistics

    def time_to(self, target: float):
        """(sweeps, seconds) until <H> <= target, or (None, None)."""
        for k, e in enumerate(self.energies):
            if e <= target:
                return k + 1, self.init_seconds + self.seconds[k]
        return None, None

    @property
    def final(self) -> float:
        return self.energies[-1]


def sweep_opts(chi: int, tol: float = 1e-8, max_matvecs: int = 30, lbo: bool = True) -> api.SweepOpts:
    return api.SweepOpts(chi_max=chi, tol=tol, krylov_max=24, max_matvecs=max_matvecs, precision=api.FP64,
                         lbo=int(lbo), compute_energy=1)


def run_sweeps(ctx, mpo, mps, opts, max_sweeps: int, conv_tol: float = 0.0, stop_at: float | None = None,
               init_seconds: float = 0.0) -> RunTrace:
    """Joint DMRG + LBO sweeps; stops at max_sweeps, when the energy changes by
    less than conv_tol * max(1, E), or when <H> <= stop_at."""
    import torch
    es, ts = [], []
    ph = {}
    t0 = time.perf_counter()
    for _ in range(max_sweeps):
        st = api.dmrg_sweep(ctx, mpo, mps, opts)
        torch.cuda.synchronize()
        for k in ("t_heff", "t_lanczos", "t_svd", "t_env", "t_lbo", "t_energy", "t_total", "matvecs"):
            ph[k] = ph.get(k, 0.0) + float(st[k])
        es.append(float(st["energy"]))
        ts.append(time.perf_counter() - t0)
        if not math.isfinite(es[-1]):
            break
        if stop_at is not None and es[-1] <= stop_at:
            break
        if len(es) > 1 and abs(es[-1] - es[-2]) <= conv_tol * max(1.0, abs(es[-1])):
            break
    return RunTrace(es, ts, init_seconds, ph)


def plain_start(ctx, r, U, D: int, d: int, tensors):
    """MPO with the first d Fock states as local basis and the given MPS."""
    return api.MPO(ctx, r, U, D, d), api.MPS(ctx, tensors)


def learned_start(ctx, net: api.MLP, r, U, D: int, d: int, chi: int, seed: int, noise: float = 1e-3,
                  tensors=None):
    """Learned local bases; the learned product state unless `tensors` (an
    MPS in the learned bases) is given."""
    import torch
    X = torch.from_numpy(api.ws_features(r, U)).cuda()
    y = net.forward(X).cpu().numpy()
    return start_from_params(ctx, y, r, U, D, d, chi, seed, noise, tensors)


def analytic_start(ctx, r, U, D: int, d: int, chi: int, seed: int, noise: float = 1e-3, tensors=None):
    """The same start with the parameters read off each mode's reduced
    covariance (tn_ws_gaussian_params) instead of the network: exact for a
    Gaussian state, so the ceiling of what the network can learn."""
    return start_from_params(ctx, api.ws_gaussian_params(r, U), r, U, D, d, chi, seed, noise, tensors)


def start_from_params(ctx, y, r, U, D: int, d: int, chi: int, seed: int, noise: float = 1e-3, tensors=None):
    """MPO in the squeezed bases given by y [N][3] and the product state of
    their thermal weights (or `tensors`)."""
    iso, prod = api.ws_initial_state(y, D, d, chi, seed, noise)
    return api.MPO(ctx, r, U, D, d, iso=iso), api.MPS(ctx, prod if tensors is None else tensors)


def instance_data(ctx, r, U, D: int, d: int, chi: int, tensors, max_sweeps: int = 8, conv_tol: float = 1e-9):
    """(features, targets) of one solved instance."""
    mpo, mps = plain_start(ctx, r, U, D, d, tensors)
    tr = run_sweeps(ctx, mpo, mps, sweep_opts(chi), max_sweeps, conv_tol)
    rho = api.rdm(ctx, mps, mpo)
    return api.ws_features(r, U), api.ws_targets(rho), tr


def train(ctx, X, T, epochs: int = 200, batch: int = 256, lr: float = 1e-3, seed: int = 0, val_frac: float = 0.1,
          check_every: int = 10):
    """Adam on the mean-squared error with a held-out validation split; the
    parameters with the lowest validation loss (checked every check_every
    epochs) are kept.  Returns (net, train losses, best validation loss)."""
    import torch
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    perm = rng.permutation(n)
    nv = max(1, int(val_frac * n))
    vi, ti = perm[:nv], perm[nv:]
    net = api.MLP(ctx, X.shape[1], HIDDEN, T.shape[1], seed=seed)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).cuda()
    Xv, Tv = Xd[torch.from_numpy(vi).cuda()].contiguous(), Td[torch.from_numpy(vi).cuda()].contiguous()
    losses = []
    best, best_p = float("inf"), None
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(ti)).cuda()
        tot = 0.0
        for b0 in range(0, len(ti), batch):
            idx = order[b0:b0 + batch]
            tot += net.train_step(Xd[idx].contiguous(), Td[idx].contiguous(), lr) * len(idx)
        losses.append(tot / len(ti))
        if (ep + 1) % check_every == 0 or ep + 1 == epochs:
            vl, _ = net.grad(Xv, Tv)
            if vl < best:
                best, best_p = float(vl), net.get_params()
    if best_p is not None:
        net.set_params(best_p)
    return net, losses, best


def solve_with_fallback(ctx, net, r, U, D: int, d: int, chi: int, seed: int, plain_tensors, plain_first: float,
                        max_sweeps: int, conv_tol: float = 1e-9, stop_at: float | None = None,
                        learned_state: bool = True, lbo: bool = True, params=None):
    """Learned start accepted or rejected by <H> after its first sweep against
    the plain start's first-sweep energy plain_first; on failure the plain start runs
    and the learned sweep's time is added.  With learned_state False the
    learned bases start from plain_tensors instead of the learned product
    state; with lbo False the learned bases stay fixed (no local basis
    optimisation; the fallback still uses it).  Returns (trace, used_learned,
    learned first-sweep energy).  With params ([N][3] basis parameters) given
    instead of net, the start uses those parameters (the analytic ones of
    tn_ws_gaussian_params: the network's ceiling) under the same acceptance test."""
    import torch
    t0 = time.perf_counter()
    tens = None if learned_state else plain_tensors
    if params is not None:
        mpo, mps = start_from_params(ctx, params, r, U, D, d, chi, seed, tensors=tens)
    else:
        mpo, mps = learned_start(ctx, net, r, U, D, d, chi, seed, tensors=tens)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    opts = sweep_opts(chi, lbo=lbo)
    first = run_sweeps(ctx, mpo, mps, opts, 1, init_seconds=t_init)
    e1 = first.energies[0]
    if math.isfinite(e1) and e1 <= plain_first:
        rest = run_sweeps(ctx, mpo, mps, opts, max_sweeps - 1, conv_tol, stop_at) if max_sweeps > 1 else None
        es = first.energies + (rest.energies if rest else [])
        ts = first.seconds + ([first.seconds[-1] + s for s in rest.seconds] if rest else [])
        ph = {k: first.phases.get(k, 0.0) + (rest.phases.get(k, 0.0) if rest else 0.0) for k in first.phases}
        return RunTrace(es, ts, t_init, ph), True, e1
    lost = t_init + first.seconds[-1]
    t1 = time.perf_counter()
    mpo, mps = plain_start(ctx, r, U, D, d, plain_tensors)
    torch.cuda.synchronize()
    tr = run_sweeps(ctx, mpo, mps, sweep_opts(chi), max_sweeps, conv_tol, stop_at,
                    init_seconds=lost + time.perf_counter() - t1)
    return tr, False, e1


def solve_hybrid(ctx, net, r, U, D: int, d: int, chi: int, seed: int, plain_tensors, bulk_sweeps: int,
                 max_sweeps: int, conv_tol: float = 1e-9, stop_at: float | None = None):
    """Learned local bases held fixed for bulk_sweeps sweeps (no local basis
    optimisation, about half the cost of a joint sweep), then joint DMRG + LBO
    sweeps.  No fallback.  Returns the trace."""
    import torch
    t0 = time.perf_counter()
    mpo, mps = learned_start(ctx, net, r, U, D, d, chi, seed, tensors=plain_tensors)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    a = run_sweeps(ctx, mpo, mps, sweep_opts(chi, lbo=False), bulk_sweeps, init_seconds=t_init)
    b = run_sweeps(ctx, mpo, mps, sweep_opts(chi), max_sweeps - bulk_sweeps, conv_tol, stop_at)
    es = a.energies + b.energies
    ts = a.seconds + [a.seconds[-1] + x for x in b.seconds]
    ph = {k: a.phases.get(k, 0.0) + b.phases.get(k, 0.0) for k in a.phases}
    return RunTrace(es, ts, t_init, ph)
