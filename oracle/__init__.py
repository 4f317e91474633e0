"""Plain, slow FP64 CPU oracle for the GBS parent-Hamiltonian DMRG path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
execute anything under ``oracle/``; only the tests, the smoke check and the
CPU-baseline leg of the benchmark do.  The oracle shares no code with the GPU
library: it is written from the paper (arXiv 2410.18740) with NumPy complex128
and plain loops, each function citing the section or equation it follows.

Modules
  gbs        problem -> covariance -> quadratic-form coefficients; exact
             amplitudes by recursion and by hafnians; closed forms
  operators  Fock-space operator matrices built at D+4 and truncated
  dense      dense truncated Hamiltonian PHP, two constructions, ED
  mpo        middle-site algebraic MPO (structure + values)
  mps        MPS utilities: canonical forms, dense contraction, marginals
  dmrg       two-site DMRG: H_eff matvec, Lanczos, SVD truncation,
             environments, sweeps, <H> two ways
  lbo        local basis optimisation (Gaussian optimal basis, linear sweep)
  sampler    Philox4x32-10 and sequential conditional sampling
  mlp        learned warm-start network, forward/backward in FP64
  flops      algorithmic FLOP accounting
  cutoff     Fock-cutoff error bounds and the effective cutoff
  cz         global-CZ (non-Gaussian) parent Hamiltonian and its MPO
  noisy      noisy GBS: uniform-loss covariance, V = Q + C split, displacement
             matrices, displaced sequential sampling
  plbo       gate-parameterised local basis: transformed operators by
             the definition, slot environments, gradients, Adam

Parity status: every function is pinned by a CPU test in tests/ except those
whose module docstring says "parity unpinned".
"""
