"""Algorithmic FLOP accounting for the two-site matvec and the environment
update (oracle; test infrastructure only).  A complex multiply-add counts 8
real flops.  Counts depend only on shapes and on the MPO kind table:
  matvec(s):  8 d^2 chi_l chi_r (w_{s-1} chi_l + w_{s+1} chi_r)
              + sum_{t in {s, s+1}} [8 d^3 chi_l chi_r n_op(t) + 8 d^2 chi_l chi_r n_sc(t)]
  env(s):     8 (w_{s-1} chi_l^2 d chi_r + n_op(s) d^2 chi_l chi_r
                 + n_sc(s) d chi_l chi_r + w_s chi_l d chi_r^2)
where n_op counts operator blocks (kinds 2-5, and 7-9 of the global-CZ
Hamiltonian: X^2, XP + PX and their combinations) and n_sc scalar blocks
(kind 6) of the core; identity blocks count nothing.  chi_l, chi_r are the outer bonds
of the window (the matvec) or of the site (the environment update).
"""
from __future__ import annotations


def core_counts(kind_table):
    n_op = int(sum(1 for v in kind_table.reshape(-1) if 2 <= int(v) <= 5 or 7 <= int(v) <= 9))
    n_sc = int(sum(1 for v in kind_table.reshape(-1) if int(v) == 6))
    return n_op, n_sc


def matvec_flops(d, chi_l, chi_r, w_left, w_right, kinds_s, kinds_s1) -> int:
    f = 8 * d * d * chi_l * chi_r * (w_left * chi_l + w_right * chi_r)
    for K in (kinds_s, kinds_s1):
        n_op, n_sc = core_counts(K)
        f += 8 * d ** 3 * chi_l * chi_r * n_op + 8 * d * d * chi_l * chi_r * n_sc
    return int(f)


def env_flops(d, chi_l, chi_r, w_left, w_right, kinds) -> int:
    n_op, n_sc = core_counts(kinds)
    return int(8 * (w_left * chi_l * chi_l * d * chi_r + n_op * d * d * chi_l * chi_r
                    + n_sc * d * chi_l * chi_r + w_right * chi_l * d * chi_r * chi_r))
