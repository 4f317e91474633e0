"""Sampling and marginals at the full 48-mode size (cutoff 24 compressed to a
10-dim local basis, chi = 256, Haar U from seed 4, r ~ U[1.0, 1.5]) on a
right-canonicalised random MPS: marginals of the first 8 modes against the
oracle's contraction, 10^5 samples against those marginals (5 sigma per cell),
and the oracle's sequential sampler replaying the first samples on the same
Philox stream."""
import time

import numpy as np
import pytest

import workloads as W
from oracle import mps as omps, sampler as osampler

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def state():
    import paper_2410_18740_amd as P
    ctx = P.Context(0)
    w = W.WORKLOADS["gbs_n48_d24to10_chi256"]
    r, U = W.workload_problem("gbs_n48_d24to10_chi256")
    mpo = P.MPO(ctx, r, U, w.D_raw, w.d)
    mps = P.MPS(ctx, W.random_mps(w.N, w.d, w.chi, w.mps_seed))
    t0 = time.perf_counter()
    mps.canonicalize()
    print(f"canonicalised N={w.N} chi={w.chi} in {time.perf_counter() - t0:.2f} s", flush=True)
    yield ctx, mpo, mps
    ctx.close()


def test_marginals_match_oracle_at_scale(state):
    import paper_2410_18740_amd as P
    ctx, mpo, mps = state
    marg = P.marginals(ctx, mps, mpo, 8)
    ref = omps.marginals(mps.export(), list(mpo.isometries()), n_modes=8)
    assert np.abs(marg - ref).max() < 1e-12
    assert np.abs(marg.sum(axis=1) - 1.0).max() < 1e-12


def test_samples_match_marginals_at_scale(state):
    import torch
    import paper_2410_18740_amd as P
    ctx, mpo, mps = state
    n = 100_000
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp = P.sample(ctx, mps, mpo, n, 2004)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"{n} samples x {mps.N} modes in {dt:.3f} s ({n / dt:.0f} samples/s)", flush=True)
    smp = smp.cpu().numpy()
    D = mpo.D_raw
    assert smp.min() >= 0 and smp.max() < D
    marg = P.marginals(ctx, mps, mpo, 8)
    for j in range(8):
        h = np.bincount(smp[:, j], minlength=D) / n
        sig = np.sqrt(marg[j] * (1 - marg[j]) / n) + 1e-12
        assert np.all(np.abs(h - marg[j]) <= 5 * sig + 2.0 / n), j


def test_oracle_replays_the_first_samples(state):
    import paper_2410_18740_amd as P
    ctx, mpo, mps = state
    smp = P.sample(ctx, mps, mpo, 8, 2004).cpu().numpy()
    fock = omps.fock_tensors(mps.export(), list(mpo.isometries()))
    ref, tie = osampler.sample(fock, 8, 2004, with_ties=True)
    # a draw may differ only where u lands within rounding of a CDF step
    bad, nties = osampler.stream_mismatches(smp, ref, tie)
    assert bad == 0, (bad, nties)
