"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method itself: it only draws random
numbers (interferometer unitaries, squeezing parameters, initial MPS tensors)
and names the workload shapes.  Both the CPU oracle and the GPU path receive
the arrays produced here, so neither side generates its own inputs.

Shapes follow the paper's GBS workloads: per-mode squeezing r_j and an N x N
interferometer unitary U (Sec. II.C.1), a Fock cutoff D, a local basis size d
(Sec. III.A) and a bond dimension chi (Sec. II.E).  The paper measures on
random pure covariance matrices and on Borealis data; neither is available, so
seeded Haar-random interferometers (and, for the literal 1e-8 target, a
shallow beamsplitter mesh) stand in for them.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "haar_unitary",
    "brickwork_unitary",
    "make_problem",
    "random_mps",
    "bond_dims",
]


def haar_unitary(N: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random N x N unitary: QR of a complex Gaussian matrix followed by
    the diagonal phase fix of Mezzadri (Notices AMS 54, 2007)."""
    Z = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    ph = np.diag(R) / np.abs(np.diag(R))
    return Q * ph[None, :]


def brickwork_unitary(N: int, layers: int, rng: np.random.Generator,
                      t_scale: float = 0.6) -> np.ndarray:
    """Shallow nearest-neighbour beamsplitter mesh.

    Layer l acts on pairs (i, i+1) with i = l mod 2, l mod 2 + 2, ...; each
    beamsplitter is [[cos t, -e^{-i phi} sin t], [e^{i phi} sin t, cos t]] with
    t = t_scale * uniform(0.5, 1) and phi = uniform(0, 2 pi), drawn in that
    order.  U = B_last ... B_first.
    """
    U = np.eye(N, dtype=np.complex128)
    for layer in range(layers):
        B = np.eye(N, dtype=np.complex128)
        for i in range(layer % 2, N - 1, 2):
            t = t_scale * rng.uniform(0.5, 1.0)
            phi = rng.uniform(0.0, 2.0 * np.pi)
            c, s = np.cos(t), np.sin(t)
            B[i, i] = c
            B[i, i + 1] = -np.exp(-1j * phi) * s
            B[i + 1, i] = np.exp(1j * phi) * s
            B[i + 1, i + 1] = c
        U = B @ U
    return U


def bond_dims(N: int, d: int, chi: int) -> list[int]:
    """Open-boundary bond dimensions min(chi, d^s, d^(N-s)) for s = 0..N."""
    out = []
    for s in range(N + 1):
        left = d ** min(s, 40)
        right = d ** min(N - s, 40)
        out.append(int(min(chi, left, right)))
    return out


def random_mps(N: int, d: int, chi: int, seed: int) -> list[np.ndarray]:
    """Random-normal complex MPS: Re, Im ~ N(0, 1) i.i.d., site tensors of
    shape (chi_{s-1}, d, chi_s) drawn in site order from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    dims = bond_dims(N, d, chi)
    out = []
    for s in range(N):
        shape = (dims[s], d, dims[s + 1])
        re = rng.standard_normal(shape)
        im = rng.standard_normal(shape)
        out.append(re + 1j * im)
    return out


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    N: int
    D_raw: int          # raw Fock cutoff (levels 0..D_raw-1)
    d: int              # local basis size (== D_raw without LBO)
    chi: int
    seed: int
    r_range: tuple      # (lo, hi) for uniform draws; lo == hi means constant
    kind: str = "haar"  # "haar" or "brickwork"
    mps_seed: int = 0
    sweeps: int = 6
    tol: float = 1e-12


WORKLOADS = {
    # 4 modes, cutoff 6, chi 16, r = 0.5 on every mode, Haar U from seed 0.
    "gbs_n4_d6_chi16": Workload("gbs_n4_d6_chi16", 4, 6, 6, 16, 0, (0.5, 0.5),
                                mps_seed=1000, sweeps=6, tol=1e-12),
    # 16 modes, cutoff 12, chi 64, r ~ U[0.5, 1.0].
    "gbs_n16_d12_chi64": Workload("gbs_n16_d12_chi64", 16, 12, 12, 64, 1, (0.5, 1.0),
                                  mps_seed=1001, sweeps=4, tol=1e-10),
    # 32 modes, raw cutoff 16 compressed to an 8-dim local basis, chi 128.
    "gbs_n32_d16to8_chi128": Workload("gbs_n32_d16to8_chi128", 32, 16, 8, 128, 2, (0.8, 1.2),
                                      mps_seed=1002, sweeps=4, tol=1e-10),
    # Same shapes as above on a 4-layer beamsplitter mesh with weak squeezing,
    # where <H> <= 1e-8 is reachable at chi 128.
    "mesh_n32_d16to8_chi128": Workload("mesh_n32_d16to8_chi128", 32, 16, 8, 128, 2, (0.1, 0.2),
                                       kind="brickwork", mps_seed=1002, sweeps=4, tol=1e-10),
    # Basis-limited case for the gate-parameterised basis: a 4-layer mesh keeps
    # the entanglement low enough for chi 32, while r ~ U[0.6, 0.9] puts a few
    # per cent of each mode's weight beyond the first 4 Fock states.
    "mesh_n32_d4_chi32": Workload("mesh_n32_d4_chi32", 32, 16, 4, 32, 3, (0.6, 0.9),
                                  kind="brickwork", mps_seed=1003, sweeps=4, tol=1e-10),
    # 48 modes, raw cutoff 24 compressed to 10, chi 256.
    "gbs_n48_d24to10_chi256": Workload("gbs_n48_d24to10_chi256", 48, 24, 10, 256, 4, (1.0, 1.5),
                                       mps_seed=1004, sweeps=4, tol=1e-10),
}


def make_problem(N: int, seed: int, r_range=(0.5, 0.5), kind: str = "haar",
                 layers: int = 4):
    """(r, U) for a seeded instance.  U is drawn first, then r from the same
    generator (no draw when r_range is a single value)."""
    rng = np.random.default_rng(seed)
    if kind == "haar":
        U = haar_unitary(N, rng)
    elif kind == "brickwork":
        U = brickwork_unitary(N, layers, rng)
    else:
        raise ValueError(kind)
    lo, hi = r_range
    if lo == hi:
        r = np.full(N, float(lo))
    else:
        r = rng.uniform(lo, hi, N)
    return np.ascontiguousarray(r, dtype=np.float64), np.ascontiguousarray(U, dtype=np.complex128)


def workload_problem(name: str):
    w = WORKLOADS[name]
    return make_problem(w.N, w.seed, w.r_range, w.kind)
