"""Shared set-up for the GPU parity tests (inputs from workloads/, references
from oracle/)."""
import numpy as np

import workloads as W
from oracle import gbs, operators, mpo as omp


def problem(name):
    w = W.WORKLOADS[name]
    r, U = W.workload_problem(name)
    return w, r, U


def oracle_cores(r, U, D, iso=None):
    al, be, ga = gbs.coefficients(r, U)
    N = len(r)
    ops = []
    for s in range(N):
        X, P, S = operators.local_operators(D, al[s, s], be[s, s], ga[s, s])
        if iso is not None:
            X, P, S = (operators.project(o, iso[s]) for o in (X, P, S))
        ops.append((X, P, S))
    return omp.cores(al, be, ga, ops)


def rand_env(w, chi, rng, hermitian=True):
    E = rng.standard_normal((w, chi, chi)) + 1j * rng.standard_normal((w, chi, chi))
    if hermitian:
        E = 0.5 * (E + np.conj(np.transpose(E, (0, 2, 1))))
    return E


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).cuda()


def from_dev(x):
    return x.cpu().numpy()
