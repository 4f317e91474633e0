"""Sequential conditional sampling of photon-number patterns from an MPS
(oracle; test infrastructure only).

The distribution is P(n) = |<n|psi>|^2 (Sec. II.A).  With the MPS
right-canonical and its norm on site 0, the conditional of n_s given the
earlier outcomes is p(n) = ||v A^F_s[n]||^2 with v the normalised left
vector; n is the smallest index whose cumulative probability reaches u * sum p
(the paper does not state a sampling algorithm; this is the reading taken).
Uniform draws come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11) with counter
(sample lo, sample hi, site, 0) and key (seed lo, seed hi); u takes 53 bits
as (x0 >> 5) * 2^26 + (x1 >> 6), divided by 2^53.
"""
from __future__ import annotations

import math

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Ten Philox-4x32 rounds; the key is bumped by the Weyl constants before
    every round after the first."""
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return (c0, c1, c2, c3)


def uniform(sample: int, site: int, seed: int) -> float:
    out = philox4x32_10((sample & MASK, (sample >> 32) & MASK, site, 0), (seed & MASK, (seed >> 32) & MASK))
    a, b = out[0] >> 5, out[1] >> 6
    return (a * 67108864.0 + b) / 9007199254740992.0


def normal(sample: int, col: int, seed: int) -> float:
    """A standard normal draw for noise column `col` of sample `sample`: the
    Box-Muller transform (Box & Muller, Ann. Math. Statist. 29, 1958)
    z = sqrt(-2 ln u1) cos(2 pi u2) of the uniforms u1 in (0, 1] (words 0-1,
    53 bits, plus one) and u2 in [0, 1) (words 2-3) of the Philox block with
    counter (sample lo, sample hi, col, 1); the last counter word keeps these
    blocks apart from the photon-number draws."""
    out = philox4x32_10((sample & MASK, (sample >> 32) & MASK, col, 1), (seed & MASK, (seed >> 32) & MASK))
    u1 = ((out[0] >> 5) * 67108864.0 + (out[1] >> 6) + 1.0) / 9007199254740992.0
    u2 = ((out[2] >> 5) * 67108864.0 + (out[3] >> 6)) / 9007199254740992.0
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


TIE = 1e-12


def pick_outcome(p, u):
    """The smallest n whose cumulative probability reaches u (u already scaled
    by sum p), skipping zero-probability outcomes; and whether the draw is a
    rounding tie, i.e. u lies within TIE * sum p of a cumulative sum, where a
    different rounding of the probabilities may pick the neighbour."""
    cum = np.cumsum(p)
    pick = len(p) - 1
    for n in range(len(p)):
        if cum[n] >= u and p[n] > 0:
            pick = n
            break
    while pick > 0 and not p[pick] > 0:
        pick -= 1
    tie = bool(np.min(np.abs(cum - u)) < TIE * max(float(cum[-1]), 1e-300))
    return pick, tie


def sample(fock_tensors, n_samples: int, seed: int, with_ties: bool = False):
    """Samples (n_samples x N ints) from right-canonical Fock-basis tensors
    A^F_s[a, n, b] with the norm on site 0; probabilities in FP64.  With
    with_ties, also the first site of each sample whose draw is a rounding
    tie (N if none): outcomes up to that site are determined exactly."""
    N = len(fock_tensors)
    out = np.zeros((n_samples, N), dtype=np.int64)
    first_tie = np.full(n_samples, N, dtype=np.int64)
    for b in range(n_samples):
        v = np.ones(1, dtype=np.complex128)
        for s, A in enumerate(fock_tensors):
            T = np.tensordot(v, A, axes=([0], [0]))      # (D, chi_r)
            p = np.sum(np.abs(T) ** 2, axis=1)
            u = uniform(b, s, seed) * p.sum()
            pick, tie = pick_outcome(p, u)
            if tie and first_tie[b] == N:
                first_tie[b] = s
            out[b, s] = pick
            v = T[pick] / np.sqrt(p[pick])
    return (out, first_tie) if with_ties else out


def stream_mismatches(got, ref, first_tie):
    """Samples of `got` that differ from the oracle stream `ref` before the
    oracle's first rounding tie in that sample (the count that must be 0),
    and the number of samples that hold a tie at all."""
    got = np.asarray(got)
    bad = 0
    for b in range(ref.shape[0]):
        t = int(first_tie[b])
        if np.any(got[b, :t] != ref[b, :t]):
            bad += 1
    return bad, int(np.sum(first_tie < ref.shape[1]))
