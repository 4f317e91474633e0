/* tn.h -- C ABI of the gfx950 two-site DMRG library for the parent Hamiltonian
 * of Gaussian boson sampling (Vinther & Kastoryano, "Variational Tensor Network
 * Simulation of Gaussian Boson Sampling and Beyond", arXiv 2410.18740).
 *
 * The output state |psi> = U V |0> of a squeezer bank V (per-mode squeezing r_j)
 * followed by an interferometer U is the unique zero-energy ground state of the
 * positive semidefinite H = sum_n A_n^dag A_n (Sec. II.B, eq. CentralEquation);
 * for GBS, H = x^T (V^{-1}/4) x - N/2 in quadratures (Sec. II.C.1, eq.
 * GBSHamiltonian).  The library writes the compression PHP of H onto a Fock box
 * (Sec. II.E.1) as the middle-site MPO of SM Sec. 8, optionally in an optimised
 * local basis (Sec. III.A, SM Sec. 6), and finds its ground state variationally
 * with two-site DMRG on one MI355X.  <H> >= 0 is the simulation error
 * (eq. MagOfSimError).
 *
 * Conventions: hbar = 1; a = (X + iP)/sqrt(2); quadrature order (X_1..X_N,
 * P_1..P_N); the interferometer acts as a_j -> sum_k U_jk a_k; D = diag(e^{-r},
 * e^{r}) so r > 0 squeezes X.  Complex numbers are interleaved (re, im) doubles.
 * All arrays are row-major.  Site and bond indices in this header are 0-based.
 *
 * Ownership and threading: the caller owns every array it passes; inputs are
 * copied during the call.  Handles own their device memory until *_destroy.
 * Device memory comes from the context allocator (hipMalloc when none is given).
 * Work is enqueued on the context's HIP stream; calls that return host values
 * synchronise that stream.  A context is not thread-safe: use one per thread.
 *
 * Errors: every function returns tn_status.  Invalid arguments are rejected
 * before any work, with no side effects, and tn_last_error() describes them.
 */
#ifndef TN_H
#define TN_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tn_status;
#define TN_OK 0
#define TN_EINVAL (-1)   /* invalid argument; nothing was done */
#define TN_ENOMEM (-2)   /* allocation failed; the handle stays valid */
#define TN_EHIP (-3)     /* a HIP runtime call failed */
#define TN_ENUMERIC (-4) /* NaN/Inf met; the MPS is left at the last completed step */
#define TN_ESTATE (-5)   /* handle in the wrong state for this call */

enum { TN_FP64 = 0, TN_FP32 = 1, TN_BF16X3 = 2 };

typedef struct tn_ctx tn_ctx;
typedef struct tn_mpo tn_mpo;
typedef struct tn_mps tn_mps;
typedef struct tn_mlp tn_mlp;

/* Device allocator hooks.  alloc(bytes, user) returns device memory or NULL;
 * free(ptr, user) releases it.  Used for every device allocation of the
 * context and its handles (PyTorch's caching allocator from the binding). */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} tn_allocator;

/* Library version string (static storage). */
const char* tn_version(void);

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  alloc may be NULL.
 * Makes `device` current.  TN_EINVAL for a bad device index or allocator;
 * TN_EHIP if the device, or the per-device scratch array of
 * tn_sample_noalloc, cannot be reached. */
tn_status tn_ctx_create(int device, void* hip_stream, const tn_allocator* alloc, tn_ctx** out);
/* Close a context: drain its stream and free its workspaces.  MPO, MPS and
 * network handles made on it may be destroyed before or after this call, in
 * any order: the context's host object lives until the last of them is
 * destroyed, and destroying a handle after the context touches no stream.
 * The allocator's callbacks must stay callable until then.  Every other call
 * that is given a closed context, or a handle whose context is closed where it
 * would touch the device, returns TN_ESTATE.  Passing the pointer after the
 * context and all its handles are gone is undefined, as for any freed object. */
void tn_ctx_destroy(tn_ctx* ctx);
/* Message of the last failing call on this context ("" if none). */
const char* tn_last_error(const tn_ctx* ctx);
/* Kernel timing of the window matvec.  When profiling is on, every matvec
 * records HIP events around its launches on the context stream and waits for
 * them (so it serialises the host).  out (may be NULL, 16 doubles) receives the
 * accumulated milliseconds of [convert, left contraction GEMM, operator kernel,
 * right contraction GEMM, split-K reduction], the matvec count, the
 * algorithmic flops of the left contraction, of the right contraction and of
 * the whole matvec (the integer formula), the algorithmic bytes of the two
 * GEMMs, and for the truncation's Householder tridiagonalisation (one event
 * pair around each sequence of column launches) the milliseconds, the launch
 * count and the algorithmic bytes (32 (p - j - 1)^2 for column j: the
 * trailing block read and written once), then the Lanczos iterations and how
 * many of them orthogonalised against the whole Krylov basis (these two are
 * counted whether or not profiling is on). 
 * mode: -1 read only, 0 stop and reset, 1 start (after reset). */
tn_status tn_profile(tn_ctx* ctx, int32_t mode, double* out);

/* ------------------------------------------------------------------ problem / MPO
 * Sec. II.C.1: per-mode squeezing r_j and interferometer U define
 * V = 1/2 O D^2 O^T; SM Sec. 8: alpha, beta, gamma = halves of the blocks of
 * V^{-1}.  Local quadratic operators are built at D_raw + 4 and truncated to
 * D_raw (SM Sec. 5), so the MPO is exactly PHP.  With a local basis
 * (d < D_raw, or iso given) each site operator O becomes W_s^dag O W_s. */
typedef struct {
  int32_t N;          /* modes = sites, N >= 1 */
  int32_t D_raw;      /* Fock cutoff: levels 0..D_raw-1, 1 <= D_raw <= 64 */
  int32_t d;          /* local basis size, 1 <= d <= D_raw (d == D_raw: Fock basis) */
  const double* r;    /* [N] host, finite */
  const double* U;    /* [N*N*2] host, interleaved complex, unitary to 1e-10 */
  const double* iso;  /* NULL (initial basis = first d Fock states, SM Sec. 6) or
                         [N][D_raw][d] complex host isometries, W^dag W = I to 1e-10 */
  double kappa;       /* 0: GBS.  Otherwise the global CZ gate exp(-i kappa prod X)
                         follows the Gaussian circuit (Sec. II.C.2, eq. GlobalCZgate):
                         P_i -> P_i + kappa prod_{n != i} X_n in the parent Hamiltonian
                         (eq. nonGBSHamiltonian); finite, and N >= 2 */
} tn_problem;

tn_status tn_mpo_build(tn_ctx* ctx, const tn_problem* prob, tn_mpo** out);
/* Integer structure: w[N+1] bond dimensions; kinds (may be NULL) receives the
 * concatenated per-site kind tables (w[s] x w[s+1], row-major): 0 absent,
 * 1 identity, 2 X, 3 P, 4 S_s, 5 c_X X + c_P P, 6 scalar * identity, and for
 * kappa != 0: 7 X^2, 8 XP + PX, 9 c_1 X^2 + c_2 (XP + PX).  With kappa != 0 the
 * MPO is the block sum of the Gaussian middle-site MPO (SM Sec. 8) and two
 * left-to-right blocks for the terms of order kappa and kappa^2; bond t (0 < t
 * < N) holds the Gaussian channels, then [A0, AF, (AX2 i, APt i, AI i), i <= t],
 * then [B0, BF, (BX i), i <= t]: w_t = w_t(Gaussian) + 4 + 4 t. */
tn_status tn_mpo_structure(const tn_mpo* mpo, int32_t* w, int8_t* kinds);
/* Coefficients alpha, beta, gamma (each N*N doubles; any pointer may be NULL). */
tn_status tn_mpo_coefficients(const tn_mpo* mpo, double* alpha, double* beta, double* gamma);
/* Current isometries [N][D_raw][d] complex (host). */
tn_status tn_mpo_isometries(const tn_mpo* mpo, double* iso);
/* Local operators of site s in the current basis: [5][d][d] complex
 * (X, P, S, X^2, XP + PX; products formed at D_raw + 4, SM Sec. 5). */
tn_status tn_mpo_site_ops(const tn_mpo* mpo, int32_t site, double* ops);
void tn_mpo_destroy(tn_mpo* mpo);

/* ------------------------------------------------------------------ MPS
 * Open-boundary MPS (Sec. II.D, eq. MPSAnsatz), site tensors A_s of shape
 * (chi_s, d, chi_{s+1}), chi_0 = chi_N = 1, stored FP64 on the device.
 * bond_dims[N+1]; init = host complex128 tensors concatenated in site order. */
tn_status tn_mps_create(tn_ctx* ctx, int32_t N, int32_t d, const int32_t* bond_dims, const double* init,
                        tn_mps** out);
tn_status tn_mps_bond_dims(const tn_mps* mps, int32_t* bond_dims);
/* Copy all site tensors to host (complex128, concatenated).  cap in doubles;
 * *needed receives the required size (call with host_buf = NULL to query). */
tn_status tn_mps_export(tn_ctx* ctx, const tn_mps* mps, double* host_buf, size_t cap, size_t* needed);
/* Checkpoint and resume (the state of a run that a later process continues):
 * tn_mps_checkpoint writes one flat host buffer of doubles: a header [magic
 * 1414415184, format 1, N, d, orthogonality centre (-1 unknown), completed
 * sweeps, D_raw (0 when mpo is NULL), 0], the bond dimensions [N + 1], the site
 * tensors (complex128, concatenated in site order) and, when mpo is given,
 * that MPO's isometries [N][D_raw][d] complex (as tn_mpo_isometries gives
 * them; gate parameters of a pLBO basis are saved with tn_plbo_params).
 * cap in doubles; *needed receives the size (buf = NULL to query).  Synchronises
 * the stream.  TN_EINVAL if mpo and mps do not match or cap is too small.
 * tn_mps_import rebuilds an MPS handle from such a buffer of exactly `len`
 * doubles, with the same tensors, centre and sweep counter, so a sweep on it
 * continues the saved run; iso (NULL or host [N][D_raw][d] complex) receives
 * the isometries for tn_problem.iso, and info (NULL or [2]) receives D_raw and
 * the centre.  The tensors are taken to be in the canonical form the header
 * records.  TN_EINVAL for a bad magic, format, size or non-finite tensor.
 * tn_mps_sweeps: completed sweeps of this MPS (tn_dmrg_sweep, tn_dmrg_solve
 * and tn_plbo_sweep count), restored by tn_mps_import. */
tn_status tn_mps_checkpoint(tn_ctx* ctx, const tn_mps* mps, const tn_mpo* mpo, double* buf, size_t cap,
                            size_t* needed);
tn_status tn_mps_import(tn_ctx* ctx, const double* buf, size_t len, tn_mps** out, double* iso, int32_t* info);
tn_status tn_mps_sweeps(const tn_mps* mps, int64_t* sweeps);
/* Right-canonicalise (sites N-1..1) and normalise; orthogonality centre at 0. */
tn_status tn_mps_canonicalize(tn_ctx* ctx, tn_mps* mps);
void tn_mps_destroy(tn_mps* mps);

/* ------------------------------------------------------------------ DMRG sweep
 * One sweep = left-to-right over windows (0,1)..(N-2,N-1), then right-to-left,
 * i.e. 2(N-1) two-site updates.  Each update: theta = A_s A_{s+1}; lowest
 * eigenpair of H_eff by Lanczos (FP64 vectors, full re-orthogonalisation, H_eff
 * applied in `precision`); FP64 SVD truncation keeping
 * min(chi_max, #{sigma_i > sigma_cut sigma_1}) values (eq. SurrogateEpsChi
 * gives the discarded weight); environment update in `precision`.
 * With lbo != 0 the local basis of the centre site is re-optimised before each
 * update (raw single-site solve, top-d eigenvectors of rho_s; Sec. III.A,
 * SM Sec. 6).  The energy is the FP64 <H> after the sweep. */
typedef struct {
  int32_t chi_max;
  double sigma_cut;
  double tol;              /* Lanczos residual tolerance ||H x - l x|| (||x|| = 1) */
  int32_t krylov_max;      /* Krylov vectors before an explicit restart, 2..64 */
  int32_t max_matvecs;     /* per local solve */
  int32_t precision;       /* TN_FP64 / TN_FP32 / TN_BF16X3 */
  int32_t lbo;             /* 0 / 1 */
  int32_t compute_energy;  /* 0 / 1: FP64 <H> after the sweep */
  int32_t lbo_matvecs;     /* per LBO raw single-site solve; 0 = max_matvecs */
} tn_sweep_opts;

typedef struct {
  double energy;               /* FP64 <H> after the sweep (NaN if not computed) */
  double last_eigenvalue;      /* last local Lanczos eigenvalue */
  double max_discarded, sum_discarded;
  double lbo_discarded;        /* sum over sites of the local-basis discarded weight */
  int64_t matvecs;
  int32_t unconverged_steps;
  int32_t pad_;
  double heff_flops;           /* algorithmic flops of all two-site matvecs */
  double env_flops;            /* algorithmic flops of all environment updates */
  double t_heff, t_lanczos, t_svd, t_env, t_lbo, t_energy, t_total; /* seconds */
  double svd_flops;            /* implementation flops of the truncations' dense stages:
                                  Gram GEMM, Householder tridiagonalisation of the full
                                  trailing block, back-transform and second factor
                                  (bisection, inverse iteration and Jacobi not counted) */
} tn_sweep_stats;

tn_status tn_dmrg_sweep(tn_ctx* ctx, tn_mpo* mpo, tn_mps* mps, const tn_sweep_opts* opts, tn_sweep_stats* out);

/* Sweeps with the precision schedule until a target energy.  Bulk sweeps run
 * in bulk_precision (TN_FP64 for the plain form); once the FP64 <H> after a
 * sweep changes by less than switch_tol (relative to max(1, <H>)) or rises
 * twice, up to max_refine FP64 refinement sweeps follow.  The run stops as soon
 * as <H> <= target, when an FP64 sweep changes <H> by less than conv_tol, or
 * after max_sweeps.  Wall time starts at the call (inputs already on the GPU). */
typedef struct {
  int32_t max_sweeps;
  int32_t bulk_precision;
  int32_t max_refine;
  int32_t lbo_bulk;         /* local basis optimisation in bulk sweeps */
  int32_t lbo_refine;       /* ... and in refinement sweeps */
  int32_t pad_;
  double target;            /* stop when <H> <= target */
  double switch_tol;
  double conv_tol;
  double bulk_tol;          /* Lanczos tolerance of bulk sweeps */
  double refine_tol;        /* Lanczos tolerance of refinement sweeps */
  tn_sweep_opts sweep;      /* chi_max, sigma_cut, krylov_max, max_matvecs (precision/tol/lbo set per sweep) */
} tn_solve_opts;

typedef struct {
  int32_t sweeps;           /* total sweeps run */
  int32_t refine_sweeps;
  int32_t reached;          /* 1 if <H> <= target */
  int32_t pad_;
  double energy;            /* final FP64 <H> */
  double seconds;           /* wall time of the whole call */
  double t_target;          /* wall time when <H> <= target first held (NaN if never) */
  double heff_flops, t_heff;
} tn_solve_result;

/* energy_trace / time_trace (may be NULL): FP64 <H> and elapsed seconds after
 * each sweep, capacity max_sweeps. */
tn_status tn_dmrg_solve(tn_ctx* ctx, tn_mpo* mpo, tn_mps* mps, const tn_solve_opts* opts, tn_solve_result* out,
                        double* energy_trace, double* time_trace);

/* <psi|PHP|psi>/<psi|psi> in FP64 by a full environment sweep (eq.
 * MagOfSimError); norm2 (may be NULL) receives <psi|psi>. */
tn_status tn_energy(tn_ctx* ctx, const tn_mpo* mpo, const tn_mps* mps, double* energy, double* norm2);

/* Energy variance sigma_H^2 = <(PHP)^2> - <PHP>^2 of the normalised state
 * (Sec. II.E.2), in FP64: ~0 when the state is an eigenstate, so it separates
 * the bond-dimension error from the cutoff error.  <(PHP)^2> comes from a
 * two-layer environment contraction with the product operators taken in the
 * raw Fock box (with a local basis W the physical state is W A, and W W^dag is
 * not inserted between the two copies of PHP).  Outputs are host doubles;
 * h2 (may be NULL) receives <(PHP)^2>.  The variance is returned as computed
 * (it may be slightly negative from rounding).  Workspace: two environments of
 * w^2 chi^2 complex doubles at the widest bond, plus GEMM buffers up to 8 GiB.
 * TN_EINVAL on NULL handles or outputs, TN_ESTATE on an MPS/MPO mismatch,
 * TN_ENUMERIC on a non-finite result. */
tn_status tn_energy_variance(tn_ctx* ctx, const tn_mpo* mpo, const tn_mps* mps, double* energy, double* h2,
                             double* variance);

/* Local basis optimisation.  site >= 0: re-optimise W_site (the orthogonality
 * centre must be at `site`, else TN_ESTATE); site == -1: one joint LBO + DMRG
 * sweep.  discarded (may be NULL) receives the local discarded weight
 * sum_{k >= d} lambda_k of rho_site (site >= 0) or its sum over sites. */
tn_status tn_lbo_step(tn_ctx* ctx, tn_mpo* mpo, tn_mps* mps, int32_t site, const tn_sweep_opts* opts,
                      double* discarded);

/* ------------------------------------------------------------------ gate-parameterised local basis
 * Sec. III.B (eq. pLBOUnitary, eq. SymplecticBasisTransformation; SM Sec. 5).
 * The basis of mode i is U_i|m>, m < d, with
 *   U = D(alpha) S(r e^{i phi}) R(theta) P2(s) P3(gamma) K(kappa),
 * parameters p = (alpha_x, alpha_p, r, phi, theta, s, gamma, kappa), alpha =
 * alpha_x + i alpha_p, in the gate conventions D = exp(alpha a^dag - alpha^* a),
 * S(z) = exp((z^* a^2 - z a^dag^2)/2), R = exp(i theta n),
 * P2 = exp(i s (a + a^dag)^2 / 4), P3 = exp(i gamma (a + a^dag)^3 / 6),
 * K = exp(i kappa n^2).  The site operators are the blocks <m|U^dag O U|n>
 * built from the closed form of U^dag a U at d + 4 levels and truncated to d.
 * Parameter arrays are host doubles [N][TN_PLBO_NPARAM]. */
#define TN_PLBO_NPARAM 8

typedef struct {
  int32_t steps;      /* Adam steps on the site's parameters per visit, >= 0 */
  int32_t matvecs;    /* single-site Lanczos matvecs in the current basis before them (0: none) */
  double lr;          /* Adam step size > 0 */
  double beta1, beta2;/* Adam moment decays in [0, 1) */
  double eps;         /* Adam denominator guard > 0 */
  uint32_t mask;      /* bit j set: parameter j is optimised (0xFF: all eight) */
  int32_t optimizer;  /* TN_PLBO_ADAM: `steps` Adam steps, moments kept per site;
                         TN_PLBO_LBFGS: `steps` L-BFGS iterations (8 pairs, Armijo
                         backtracking on the exact site energy, first step at most lr
                         per parameter), started afresh at every visit */
} tn_plbo_opts;
#define TN_PLBO_ADAM 0
#define TN_PLBO_LBFGS 1

/* Host only, no GPU work.  ops: [5][d][d] complex (interleaved doubles) =
 * (X, P, S, X^2, XP + PX) in the basis of params (8 doubles), S =
 * (a_ss X^2 + b_ss P^2 + g_ss (XP + PX))/2 - 1/2; dops (may be NULL):
 * [8][5][d][d] complex, their derivatives in the parameters.  TN_EINVAL on
 * d outside [1, 64], NULL params/ops or non-finite inputs. */
tn_status tn_plbo_ops(int32_t d, const double* params, double a_ss, double b_ss, double g_ss, double* ops,
                      double* dops);
/* Host only.  iso: [D][d] complex, <n|U|m> for n < D, m < d: the gates applied
 * to |m> in `levels` Fock levels (levels >= D; each exponential by a Taylor
 * series over sub-steps of unit norm), then cut to D rows.  TN_EINVAL on
 * d < 1, D < d, D > 4096, levels outside [D, 8192] or non-finite params. */
tn_status tn_plbo_fock_isometry(int32_t D, int32_t d, const double* params, int32_t levels, double* iso);
/* Host only.  Effective cutoff of the basis of params (Sec. III.A, eq.
 * Effectivecutoff): *D_eff = the smallest D <= D_max at which the first d
 * basis vectors, cut to D Fock rows, are orthonormal within tol
 * (max |V^dag V - 1|), or -1 if none.  TN_EINVAL on d < 1, D_max outside
 * [d, 4096], tol <= 0 or non-finite params. */
tn_status tn_plbo_effective_cutoff(int32_t d, const double* params, int32_t D_max, double tol, int32_t* D_eff);
/* Host only, no GPU work.  Runs opts' optimiser on the energy of one site as a
 * function of its parameters with the slot environments G (host [6][d][d]
 * complex, as from tn_plbo_site_gradient) held fixed: params (8, in/out) from
 * their input values, Adam moments from zero; energy receives the final site
 * energy.  TN_EINVAL on bad sizes, options or non-finite params. */
tn_status tn_plbo_minimize(int32_t d, const double* G, double a_ss, double b_ss, double g_ss, const tn_plbo_opts* opts,
                           double* params, double* energy);
/* Switch the MPO to gate-parameterised bases with the given parameters (NULL:
 * all zero, i.e. the Fock basis) and reset the Adam moments.  From then on the
 * site operators follow the parameters, linear LBO is refused (TN_ESTATE)
 * until tn_plbo_linear puts an isometry on top, and
 * the Fock image of each basis (tn_mpo_isometries, observables) is recomputed
 * on demand.  TN_EINVAL on a NULL handle or non-finite parameters. */
tn_status tn_plbo_enable(tn_mpo* mpo, const double* params);
/* SM Sec. 6: put a linear isometry W (D_raw x d) on top of the gate-
 * parameterised bases.  The raw basis of site i becomes U_i|m>, m < D_raw,
 * with the pLBO operators on those D_raw states as the raw operators; W
 * starts at the first d of them (so <H> is unchanged) and is what the LBO
 * step of tn_dmrg_sweep / tn_plbo_sweep (opts->lbo = 1) optimises, while the
 * pLBO steps move the parameters with W fixed (gradients through W^dag O W).
 * Observables use the Fock image U[:D_raw, :D_raw] W.  One-way: TN_ESTATE if
 * the MPO has no parameterised basis or the isometry is already on. */
tn_status tn_plbo_linear(tn_mpo* mpo);
/* W of every site, host [N][D_raw][d] complex; TN_ESTATE unless tn_plbo_linear ran. */
tn_status tn_plbo_linear_isometries(const tn_mpo* mpo, double* W);
/* Current parameters [N][8]; TN_ESTATE if the MPO has no parameterised basis. */
tn_status tn_plbo_params(const tn_mpo* mpo, double* params);
/* Slot environments and gradient at `site` in `precision`, for x = the site
 * tensor divided by its norm and the environments of the other tensors as
 * they are (when `site` is the orthogonality centre, E below is <H>):
 *   G (may be NULL): host [6][d][d] complex, G_k[n'][n] = dE/dO_k[n'][n] for
 *     the slots (I, X, P, S, X^2, XP + PX), so E = Re sum_k <G_k, O_k>;
 *   energy: E = <x|H_eff|x> at the current parameters;
 *   grad (may be NULL): host [8], dE/dp_j.
 * Environments are built or reused as for tn_lbo_step. */
tn_status tn_plbo_site_gradient(tn_ctx* ctx, tn_mpo* mpo, tn_mps* mps, int32_t site, int32_t precision, double* G,
                                double* energy, double* grad);
/* One two-site sweep (as tn_dmrg_sweep, opts->lbo must be 0) in which every
 * visit of a centre site first runs the pLBO step: popts->matvecs Lanczos
 * matvecs on the single-site tensor, its slot environments, and popts->steps
 * Adam steps on the site's masked parameters (moments kept per site across
 * sweeps).  gain (may be NULL) receives the sum over visits of the site-energy
 * decrease from the parameter steps.  TN_ESTATE if the MPO has no
 * parameterised basis; TN_EINVAL on bad options. */
tn_status tn_plbo_sweep(tn_ctx* ctx, tn_mpo* mpo, tn_mps* mps, const tn_sweep_opts* opts, const tn_plbo_opts* popts,
                        tn_sweep_stats* out, double* gain);

/* ------------------------------------------------------------------ observables
 * Single-mode photon-number marginals P_j(n), j < n_modes, n < D_raw, in FP64
 * (eq. ReducedDensityMatrix, eq. InverseBasisTransformation).  out: host
 * [n_modes][D_raw].  The MPS must be normalised and right-canonical with the
 * centre at site 0 (the state after a sweep). */
tn_status tn_marginals(tn_ctx* ctx, const tn_mps* mps, const tn_mpo* mpo, int32_t n_modes, double* out);

/* Photon-number samples by sequential conditional sampling in the Fock basis
 * (Sec. II.A): p(n_s | n_<s) = ||v A^F_s[n]||^2 in FP64, u from
 * Philox4x32-10 with counter (sample, site, 0, 0) and key (seed lo, seed hi),
 * n = smallest index whose cumulative probability reaches u * sum p.
 * out: device int32 [n_samples][N] (caller-owned).  Same centre requirement
 * as tn_marginals. */
tn_status tn_sample(tn_ctx* ctx, const tn_mps* mps, const tn_mpo* mpo, int64_t n_samples, uint64_t seed,
                    int32_t* out);
/* tn_sample_noalloc: tn_sample for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, outputs (bit for bit) and errors as tn_sample;
 * it calls no hipMalloc, hipFree or other allocating routine.  Its buffers
 * (GEMM descriptors, the Fock-basis site tensors W_s A_s, the per-chunk
 * contractions and left vectors) live in one 64 MiB device array per GPU that
 * the library holds until the process ends.  Limit: 64 KiB of descriptors plus
 * sum_s chi_s D_raw chi_{s+1} * 16 bytes of site tensors plus at least one
 * sample's (D_raw + 2) chi_max * 16 bytes must fit in 64 MiB, else TN_EINVAL
 * (chunks of samples are sized to what remains).  A gate-parameterised MPO
 * whose Fock image is stale gives TN_ESTATE (tn_mpo_isometries refreshes it).
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (several host threads or streams) race and must be serialised by the
 * caller. */
tn_status tn_sample_noalloc(tn_ctx* ctx, const tn_mps* mps, const tn_mpo* mpo, int64_t n_samples, uint64_t seed,
                            int32_t* out);

/* ------------------------------------------------------------------ noisy GBS
 * Sec. II.F, eq. CovarianceDecomposition: a mixed covariance V = Q + C, Q pure,
 * C >= 0 the covariance of zero-mean random displacements; a noisy sample is a
 * photon-number sample of D(alpha)|psi_Q> with alpha ~ N(0, C).
 *
 * tn_noise_uniform_loss (host only): for uniform loss eta in (0, 1] after the
 * squeezers r (N) of the interferometer U (host complex [N][N], interleaved),
 * V_eta = eta V + (1 - eta) I/2.  The pure part keeps each input mode's
 * squeezed variance: r_pure[i] = -ln(eta e^{-2 r_i} + 1 - eta)/2, so the MPO
 * of the pure state is built from (r_pure, U).  L (host [2N][N], quadrature
 * order x_1..x_N, p_1..p_N) factors C = L L^T.  TN_EINVAL on N outside
 * [1, 4096], eta outside (0, 1], negative or non-finite r, non-finite U or NULL
 * pointers.
 *
 * tn_noise_williamson (host only): the general split of a mixed covariance V
 * (host [2N][2N], symmetric, vacuum = I/2) by the Williamson decomposition
 * V = S diag(nu, nu) S^T: Q = S S^T / 2 (pure; r_pure [N] and U_pure, host
 * complex [N][N], with Q = 1/2 O diag(e^{-2r}, e^{2r}) O^T as for an ideal
 * instance) and C = S (diag(nu, nu) - I/2) S^T = L L^T with L host
 * [2N][K] row-major (capacity 4 N^2 doubles), K = *K columns (the eigenvalues
 * of C above 1e-12 of the largest eigenvalue of V; K = 0 for a pure V).
 * TN_EINVAL on N outside [1, 512],
 * non-finite or non-symmetric V, V not positive definite, or a symplectic
 * eigenvalue below 1/2 (not a physical state); TN_ENUMERIC if the pure part
 * cannot be brought to that form.
 *
 * tn_sample_displaced: as tn_sample for the state D(alpha_b)|psi>, with
 * alpha_b,j = (d_x + i d_p)/sqrt2, d = L z_b (Sec. II.F: a noisy sample is a
 * sample of a randomly displaced pure state, alpha ~ N(0, C), C = L L^T).
 * z: device doubles [n_samples][K] of standard normal draws supplied by the
 * caller, or NULL: the library then draws z[b][i] itself by the Box-Muller
 * transform z = sqrt(-2 ln u1) cos(2 pi u2) of one Philox4x32-10 block with
 * counter (sample lo, sample hi, i, 1) and key (seed lo, seed hi), u1 =
 * (53 bits of words 0-1 + 1) / 2^53 in (0, 1], u2 = (53 bits of words 2-3) /
 * 2^53 (the bit layout of tn_sample's uniforms).  L: host [2N][K],
 * 1 <= K <= 2N.  The displacement acts on the D_raw
 * kept Fock levels of each mode (weight it moves beyond them is dropped and
 * the conditional probabilities renormalised).  Uniform draws and the
 * inverse-CDF rule are tn_sample's.  Same centre requirement as tn_sample. */
tn_status tn_noise_uniform_loss(int32_t N, const double* r, const double* U, double eta, double* r_pure, double* L);
tn_status tn_noise_williamson(int32_t N, const double* V, double* r_pure, double* U_pure, double* L, int32_t* K);
tn_status tn_sample_displaced(tn_ctx* ctx, const tn_mps* mps, const tn_mpo* mpo, int64_t n_samples, uint64_t seed,
                              int32_t K, const double* z, const double* L, int32_t* out);

/* Single-site reduced density matrices rho_j[n][n'] = <n|rho_j|n'> (eq.
 * ReducedDensityMatrix) in the raw Fock basis, FP64, for j < n_modes.  out:
 * host [n_modes][D_raw][D_raw] complex.  Same centre requirement as
 * tn_marginals. */
tn_status tn_rdm(tn_ctx* ctx, const tn_mps* mps, const tn_mpo* mpo, int32_t n_modes, double* out);

/* ------------------------------------------------------------------ learned warm start
 * A 3-layer perceptron in FP32 (tanh, tanh, linear), trained with a
 * mean-squared error and Adam by the library's own kernels.  It maps the
 * per-site features of an instance to the parameters of a squeezed local
 * basis (tn_squeezed_basis) and the local thermal occupation; the learned
 * basis and a product-state initial MPS warm-start the DMRG, and <H> after the
 * first sweep decides whether the start is kept (plain start as fallback).
 * x, y, t below are device float arrays, row-major [batch][dim]. */
tn_status tn_mlp_create(tn_ctx* ctx, int32_t in_dim, int32_t hidden, int32_t out_dim, uint64_t seed, tn_mlp** out);
void tn_mlp_destroy(tn_mlp* mlp);
int64_t tn_mlp_num_params(const tn_mlp* mlp);
/* get (host, may be NULL) receives all parameters [W1 b1 W2 b2 W3 b3]
 * (W_l row-major out x in); set (host, may be NULL) replaces them and resets
 * the optimiser state. */
tn_status tn_mlp_params(tn_ctx* ctx, tn_mlp* mlp, float* get, const float* set);
tn_status tn_mlp_forward(tn_ctx* ctx, tn_mlp* mlp, const float* x, int32_t batch, float* y);
/* gradients of mean((y - t)^2) into grads (host, may be NULL); loss to host */
tn_status tn_mlp_grad(tn_ctx* ctx, tn_mlp* mlp, const float* x, const float* t, int32_t batch, float* grads,
                      float* loss);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the mean-squared error */
tn_status tn_mlp_train_step(tn_ctx* ctx, tn_mlp* mlp, const float* x, const float* t, int32_t batch, float lr,
                            float* loss);
/* Squeezed local basis: out (host, D x d complex) = first d columns of
 * <n|S(zeta)|k>, S(zeta) = exp(1/2 (zeta* a^2 - zeta a^dag^2)), the optimal
 * local basis of a squeezed thermal reduced state (Sec. III.A.1), built on a
 * (D + margin) box, cut to D rows and orthonormalised. */
tn_status tn_squeezed_basis(double zeta_re, double zeta_im, int32_t D, int32_t d, int32_t margin, double* out);

/* Host helpers of the warm start (no GPU work).
 * tn_ws_features: out (host float [N][66]) = per output mode j: j/N, N/64, then
 * for the 16 largest |U_jk| (ties by k) the tuple (r_k, |U_jk|, cos 2 arg U_jk,
 * sin 2 arg U_jk), zero-padded; U host complex N x N row-major.
 * tn_ws_targets: out (host float [n_modes][3]) = (Re zeta, Im zeta,
 * log(1 + nbar)) of the squeezed thermal state with the same <a^dag a> and
 * <a^2> as rho_j (host complex [n_modes][D][D], as from tn_rdm); the
 * diagonal form of a Gaussian reduced state (Sec. III.A.1) motivates it.
 * tn_ws_initial_state: from outputs y (host float [N][3]) writes iso (host
 * complex [N][D][d], squeezed bases) and a product-state MPS with thermal
 * amplitudes in bond channel (0, 0) plus seeded complex Gaussian noise of
 * scale `noise`; dims (N + 1) receives min(chi, d^s, d^(N-s)); tensors (host,
 * `cap` doubles) receives the site tensors (chi_s, d, chi_s+1) back to back,
 * complex interleaved; with tensors NULL only *need is set. */
tn_status tn_ws_features(int32_t N, const double* r, const double* U, float* out);
tn_status tn_ws_targets(int32_t n_modes, int32_t D, const double* rho, float* out);
/* The same (Re zeta, Im zeta, log(1 + nbar)) read off each output mode's
 * reduced covariance (the 2 x 2 block of V = 1/2 O D^2 O^T, Sec. II.C.1): for
 * a Gaussian state the reduced state is exactly squeezed thermal, so these are
 * the optimal local basis (eq. OLB, eq. WilliamsonDecomposition) and the
 * network's ceiling.  out: host float [N][3]; U as in tn_ws_features. */
tn_status tn_ws_gaussian_params(int32_t N, const double* r, const double* U, float* out);
/* Cutoff errors of the Gaussian optimal local basis with d kept states per
 * mode (Sec. II.E.1 eq. epsilonD, Sec. III.A.2 eq. SpecWfromSDsums and eq.
 * Effectivecutoff).  Host only, no GPU work.  For output mode j of (r, U):
 *   eps_mode[j] = (nbar_j / (nbar_j + 1))^d, the thermal weight beyond the d
 *                 kept states, nbar_j = sqrt(det V_j) - 1/2;
 *   D_eff[j]    = the smallest Fock cutoff D <= D_max at which the first d
 *                 squeezed basis vectors, cut to D rows, are orthonormal
 *                 within tol (max |V^dag V - 1|), or -1 if none is;
 *   bounds[0]   = eps = mean_j eps_mode[j], bounds[1] = N eps: the bounds
 *                 eps <= eps_D <= N eps on eps_D = 1 - <psi|P|psi>.
 * Outputs are host arrays of N (eps_mode, D_eff) and 2 (bounds) entries.
 * TN_EINVAL on N or D_max outside [1, 4096], d > D_max, tol <= 0, NULL
 * pointers or non-finite inputs. */
tn_status tn_cutoff_report(int32_t N, const double* r, const double* U, int32_t d, int32_t D_max, double tol,
                           double* eps_mode, int32_t* D_eff, double* bounds);
tn_status tn_ws_initial_state(int32_t N, int32_t D, int32_t d, int32_t chi, const float* y, uint64_t seed,
                              double noise, double* iso, int32_t* dims, double* tensors, size_t cap, size_t* need);

/* ------------------------------------------------------------------ step entry points
 * Building blocks of the sweep, on caller-owned device buffers (FP64 complex):
 *   theta: [chi_l][d][d][chi_r] for the window (site, site+1);
 *   L: [w_site][chi_l][chi_l] left environment (bra index first);
 *   R: [w_{site+2}][chi_r][chi_r] right environment (bra index first).
 * tn_heff_apply writes theta_out = H_eff theta computed in `precision`. */
tn_status tn_heff_apply(tn_ctx* ctx, const tn_mpo* mpo, int32_t site, int32_t chi_l, int32_t chi_r,
                        const double* L, const double* R, const double* theta_in, double* theta_out,
                        int32_t precision);
/* Environment update across site `site` (FP64 device buffers):
 * direction +1: env_out[w_{site+1}][chi_r][chi_r] from env_in = L[w_site][chi_l][chi_l];
 * direction -1: env_out[w_site][chi_l][chi_l] from env_in = R[w_{site+1}][chi_r][chi_r].
 * A: [chi_l][d][chi_r]. */
tn_status tn_env_update(tn_ctx* ctx, const tn_mpo* mpo, int32_t site, int32_t direction, int32_t chi_l,
                        int32_t chi_r, const double* env_in, const double* A, double* env_out, int32_t precision);
/* SVD truncation of the m x n matrix theta (device, FP64 complex):
 * keep k = min(chi, #{sigma_i > sigma_cut sigma_1}) values; *k_out = k.
 * direction +1: left (m x k, orthonormal columns) and right (k x n) = S V^dag;
 * direction -1: left = U S (m x k) and right (k x n, orthonormal rows).
 * Both factors renormalised so that the product has unit norm.  sv (host, may
 * be NULL, capacity min(m, n)) receives the kept singular values of the
 * normalised theta; discarded receives the discarded weight. */
tn_status tn_truncate(tn_ctx* ctx, int32_t m, int32_t n, const double* theta, int32_t chi, double sigma_cut,
                      int32_t direction, double* left, double* right, int32_t* k_out, double* sv,
                      double* discarded);
/* Complex GEMM on the matrix cores: C[M x N] = op(A) op(B) with op = identity
 * or conjugate transpose (trans_a / trans_b != 0; then A is stored K x M, B is
 * stored N x K), row-major device buffers with leading dimensions in elements.
 * precision TN_FP64 uses FP64 complex buffers, TN_FP32 / TN_BF16X3 FP32 complex
 * (interleaved float pairs). */
tn_status tn_cgemm(tn_ctx* ctx, int32_t precision, int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                   const void* A, int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc);
/* Philox4x32-10 (Salmon et al., SC'11) as used by tn_sample: out[4i..4i+3] =
 * philox(ctr[4i..4i+3], key[2i..2i+1]) for i < n, all host arrays. */
tn_status tn_philox4x32_10(tn_ctx* ctx, const uint32_t* ctr, const uint32_t* key, uint32_t* out, int32_t n);
/* Algorithmic flop counts (integer formulas of the matvec and of the
 * environment update for a window / site of the given shapes). */
double tn_matvec_flops(const tn_mpo* mpo, int32_t site, int32_t chi_l, int32_t chi_r);
double tn_env_flops(const tn_mpo* mpo, int32_t site, int32_t chi_l, int32_t chi_r);

#ifdef __cplusplus
}
#endif
#endif /* TN_H */
