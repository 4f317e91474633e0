"""The allocation-free sampling entry point (tn_sample_noalloc) against
tn_sample through the raw C ABI: two calls in a row, the second with a
smaller MPS and fewer samples, must give the same samples bit for bit; a
state beyond the scratch limit is refused."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _state(P, ctx, N, D, chi, seed, sweeps=3):
    r, U = W.make_problem(N, seed, (0.4, 0.7))
    m = P.MPO(ctx, r, U, D)
    mp = P.MPS(ctx, W.random_mps(N, D, chi, seed + 100))
    for _ in range(sweeps):
        P.dmrg_sweep(ctx, m, mp, P.SweepOpts(chi_max=chi, tol=1e-10))
    return m, mp


def _draw(fn, ctx, mp, m, n, seed, N):
    import torch
    out = torch.full((n, N), -1, dtype=torch.int32, device=f"cuda:{ctx.device}")
    st = fn(ctx.h, mp.h, m.h, n, C.c_uint64(seed), C.c_void_p(out.data_ptr()))
    return st, out.cpu().numpy()


def test_noalloc_sampler_matches_tn_sample_on_two_calls():
    import paper_2410_18740_amd as P
    from paper_2410_18740_amd import _lib as L
    ctx = P.Context(0)          # torch's HIP runtime first, then the library (the binding's order)
    lib = L.lib()
    try:
        cases = [(5, 6, 36, 1, 700, 2024), (3, 4, 8, 2, 90, 7)]   # the second call is smaller
        for N, D, chi, seed, n, sseed in cases:
            m, mp = _state(P, ctx, N, D, chi, seed)
            st_a, a = _draw(lib.tn_sample, ctx, mp, m, n, sseed, N)
            st_b, b = _draw(lib.tn_sample_noalloc, ctx, mp, m, n, sseed, N)
            print(f"noalloc N={N} D={D} chi={chi} n={n}: status {st_a} {st_b}, "
                  f"{int(np.sum(a != b))} differing entries", flush=True)
            assert st_a == 0 and st_b == 0
            assert a.min() >= 0 and a.max() < D
            assert np.array_equal(a, b)
        # a state whose Fock-basis tensors exceed the 64 MiB scratch (12 modes,
        # D 16, chi 256: 134 MB) is refused before any work; the MPS comes from
        # a checkpoint buffer that records its centre at site 0
        N, D, chi = 12, 16, 256
        t = W.random_mps(N, D, chi, 9)
        dims = [1] + [x.shape[2] for x in t]
        buf = np.concatenate([[1414415184.0, 1.0, N, D, 0, 0, 0, 0], np.array(dims, dtype=float),
                              np.concatenate([x.reshape(-1) for x in t]).view(np.float64)])
        big, _ = P.MPS.from_checkpoint(ctx, buf)
        r, U = W.make_problem(N, 3, (0.4, 0.7))
        mbig = P.MPO(ctx, r, U, D)
        st, _ = _draw(lib.tn_sample_noalloc, ctx, big, mbig, 4, 1, N)
        assert st == L.TN_EINVAL
        assert "scratch" in ctx.last_error
        # and the entry point still works after the refusal
        m, mp = _state(P, ctx, 4, 5, 25, 4)
        st_a, a = _draw(lib.tn_sample, ctx, mp, m, 50, 3, 4)
        st_b, b = _draw(lib.tn_sample_noalloc, ctx, mp, m, 50, 3, 4)
        assert st_a == 0 and st_b == 0 and np.array_equal(a, b)
    finally:
        ctx.close()
