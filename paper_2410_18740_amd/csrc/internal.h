// Host-side internals of the library (not part of the C ABI).
#pragma once
#include <complex>
#include <map>
#include <string>
#include <vector>
#include <array>
#include <stdexcept>
#include "common.h"
#include "../../include/tn.h"

typedef std::complex<double> cd;

// exception carrying a tn_status; converted at the ABI boundary
struct TnError : std::runtime_error {
  tn_status code;
  TnError(tn_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};
#define TN_THROW(code, msg) throw TnError((code), (msg))
#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e__ = (x);                                                                      \
    if (e__ != hipSuccess)                                                                     \
      throw TnError(TN_EHIP, std::string(#x) + ": " + hipGetErrorString(e__) + " @" + __FILE__ \
                                 + ":" + std::to_string(__LINE__));                            \
  } while (0)

struct tn_ctx {
  // lifetime: one reference for the caller's handle plus one per MPO, MPS and
  // network created on it; tn_ctx_destroy closes it and drops the caller's
  // reference, and the memory goes with the last reference
  int refs = 1;
  bool closed = false;
  int device = 0;
  hipStream_t stream = nullptr;
  tn_allocator alloc{};
  bool has_alloc = false;
  std::string err;
  std::map<std::string, std::pair<void*, size_t>> ws;  // named workspaces
  double* pinned = nullptr;                             // host pinned scratch (4096 doubles)
  hipEvent_t ev[8];
  bool ev_ok = false;
  // profiling of the window matvec: HIP events around each launch, in a ring
  // of slots read back once a slot comes round again (or at read-out), so that
  // profiling adds no wait to the matvec
  bool prof = false;
  struct ProfSlot {
    hipEvent_t e[6];
    double fl[3] = {0, 0, 0}, by[2] = {0, 0};
    bool pending = false;
  };
  static constexpr int PROF_RING = 8;
  ProfSlot pslot[PROF_RING];
  int64_t pseq = 0;
  double prof_ms[5] = {0, 0, 0, 0, 0};   // convert, GEMM-L, operators, GEMM-R, reduce
  double prof_flops[3] = {0, 0, 0};      // algorithmic: L-contraction, R-contraction, whole matvec
  int64_t prof_n = 0;
  double prof_bytes[2] = {0, 0};         // algorithmic bytes read + written by the two GEMMs
  // sampled tridiagonalisation columns (every TRI_SAMPLE-th launch): ms, count, algorithmic bytes
  std::vector<hipEvent_t> tri_ev;
  double prof_tri_ms = 0.0, prof_tri_bytes = 0.0;
  int64_t prof_tri_n = 0;
  int64_t lz_iters = 0, lz_full = 0;  // Lanczos iterations, and those orthogonalised against the whole basis
};

// add a profiling slot's event times and work counts to the totals (waits for its last event)
void prof_harvest(tn_ctx* c, tn_ctx::ProfSlot& ps);

// per-device address of tn_sample_noalloc's scratch, taken with `device` current
tn_status sample_scratch_setup(int device);
void ctx_retain(tn_ctx* c);
void ctx_release(tn_ctx* c);
// entry points taking a context refuse a closed one
#define TN_CTX_OPEN(c)                                             \
  do {                                                             \
    if ((c)->closed) {                                             \
      (c)->err = "the context has been destroyed";                 \
      return TN_ESTATE;                                            \
    }                                                              \
  } while (0)
void* dev_alloc(tn_ctx* c, size_t bytes);
void dev_free(tn_ctx* c, void* p);
void* ws_get(tn_ctx* c, const std::string& name, size_t bytes);
template <typename T> T* wsT(tn_ctx* c, const std::string& name, size_t count) {
  return reinterpret_cast<T*>(ws_get(c, name, count * sizeof(T)));
}
void upload(tn_ctx* c, void* dst, const void* src, size_t bytes);
void download(tn_ctx* c, void* dst, const void* src, size_t bytes);  // synchronising

// entry decomposition of a core block into the basis {I, X, P, S, X^2, XP + PX}
// local operators of a site: 1 X, 2 P, 3 S, 4 X^2, 5 XP + PX (index 0 is the identity)
constexpr int NOPS = 5;
struct CoreEntry {
  int row, col;
  int kind;
  double c[NOPS + 1];  // coefficients of I, X, P, S, X^2, XP + PX
};

struct tn_mpo {
  tn_ctx* ctx = nullptr;
  int N = 0, D_raw = 0, d = 0;
  std::vector<int> w;                            // N+1
  std::vector<std::vector<int8_t>> kinds;        // per site, w[s] x w[s+1]
  std::vector<std::vector<CoreEntry>> entries;   // per site
  std::vector<double> r;
  std::vector<cd> U;
  std::vector<double> alpha, beta, gamma;        // N x N
  std::vector<std::vector<cd>> iso;              // per site D_raw x d
  double kappa = 0.0;                            // global-CZ strength (0: GBS)
  std::vector<std::vector<cd>> raw_ops;          // per site NOPS x D_raw x D_raw
  std::vector<std::vector<cd>> loc_ops;          // per site NOPS x d x d
  // gate-parameterised local basis (Sec. III.B): when plbo is set, loc_ops of
  // every site come from its eight parameters and iso is their Fock image
  bool plbo = false;
  std::vector<std::array<double, TN_PLBO_NPARAM>> pp, pm, pv;  // parameters, Adam moments
  std::vector<int> pt;                                          // Adam step count per site
  std::vector<bool> iso_stale;                                  // Fock image not yet recomputed
  // pLBO with a linear isometry on top (SM Sec. 6): raw_ops are the pLBO
  // operators on D_raw basis states, iso the linear isometry W (D_raw x d)
  // the LBO step optimises, and fock / d_fock the Fock image U[:D, :D] W
  bool plbo_lin = false;
  std::vector<std::vector<cd>> fock;
  cf64* d_fock = nullptr;
  const cf64* fock_iso() const { return (plbo && plbo_lin) ? d_fock : d_iso; }
  cf64* d_ops64 = nullptr;   // [N][NOPS][d][d]
  cf32* d_ops32 = nullptr;
  cf64* d_raw64 = nullptr;   // [N][NOPS][D][D]
  cf32* d_raw32 = nullptr;
  cf64* d_iso = nullptr;     // [N][D][d]
  uint64_t version = 1;
  void upload_site(int s);
  const void* op_ptr(int prec, int site, int k, bool raw) const;  // k in 1..NOPS
};

struct tn_mps {
  tn_ctx* ctx = nullptr;
  int N = 0, d = 0;
  std::vector<int> dims;        // N+1
  std::vector<cf64*> A;         // device tensors, capacity per site
  std::vector<size_t> cap;      // elements allocated
  int center = -1;              // orthogonality centre (site), -1 unknown
  int64_t sweeps = 0;           // completed sweeps (checkpoint counter)
  // cached environments (precision env_prec): L[s] at bond s, Rt[s] at bond s (transposed)
  int env_prec = -1;
  const tn_mpo* env_mpo = nullptr;
  uint64_t env_version = 0;
  std::vector<void*> L, Rt;
  std::vector<size_t> Lcap, Rcap;
  std::vector<bool> Lok, Rok;
  void ensure_site(int s, size_t elems);
};

// ------------------------------------------------------------------ planner
struct PlanL {  // effective left channel: mixture of original channels
  std::vector<std::pair<int, double>> src;
};
struct PlanTerm {
  int ych;  // index into PlanL / Y buffers
  int a, b; // 0 I, 1 X, 2 P, 3 S, 4 X^2, 5 XP + PX on leg 0 / leg 1
  double c;
};
struct PlanT {
  std::vector<PlanTerm> terms;
};
struct PlanR {
  int kind;  // 0: Y buffer, 1: T buffer
  int idx;
  std::vector<std::pair<int, double>> env;  // mixture of right channels
};
struct Plan {
  std::vector<PlanL> L;
  std::vector<PlanT> T;
  std::vector<PlanR> R;
};
struct Term2 {
  int l, n, a, b;
  double c;
};
// terms of O[l][n] = sum_m W_s[l][m] (x) W_{s+1}[m][n] (two-site) or W_s[l][n] (one site)
std::vector<Term2> window_terms(const tn_mpo* mpo, int site, int nsites);
// transpose roles (for right environment updates): l <-> n
Plan build_plan(const std::vector<Term2>& terms, int wl, int wr, bool allow_right_fold);

// Executes the window operator for a plan.  Input x and output y are FP64
// (n = chi_l*ds*dt*chi_r); envL[l] (chi_l x chi_l) and envRt[n] (chi_r x chi_r,
// transposed) in precision prec.
struct WindowOp {
  tn_ctx* ctx = nullptr;
  int prec = 0, chi_l = 0, ds = 0, dt = 0, chi_r = 0;
  Plan plan;
  // device descriptor arrays
  GemmJob* d_jobL = nullptr; GemmSeg* d_segL = nullptr; int njobL = 0;
  OpJob* d_opjob = nullptr; OpTerm* d_opterm = nullptr; int nopjob = 0;
  GemmJob* d_jobR = nullptr; GemmSeg* d_segR = nullptr; int njobR = 0;
  void* xin = nullptr;      // input in prec (if prec != FP64)
  void* partials = nullptr; // split-K partials
  int nsplit = 1;
  size_t n = 0;
  char* ybuf = nullptr;            // left-contracted tensors Y[i] = L_i x, one per plan.L entry
  std::vector<const void*> rptr;   // right environment (plain or mixed) of each plan.R entry
  double fl_L = 0, fl_R = 0, fl_all = 0, by_L = 0, by_R = 0;
  void setup(tn_ctx* c, const tn_mpo* mpo, int site, int nsites, int prec_, int chi_l_, int chi_r_,
             const std::vector<const void*>& envL, const std::vector<const void*>& envRt, bool raw_leg0,
             const std::string& tag);
  void apply(const cf64* x, cf64* y);
  void apply_left(const cf64* x);  // only the conversion of x and the left contraction into ybuf
};

size_t elem_bytes(int prec);

// ------------------------------------------------------------------ gate-parameterised basis
// ops = (X, P, S, X^2, XP + PX) in the basis of parameters p, NOPS x d x d;
// dops (optional) = their derivatives, [TN_PLBO_NPARAM][NOPS][d][d]
void plbo_local_ops(int d, const double* p, double a_ss, double b_ss, double g_ss, std::vector<cd>& ops,
                    std::vector<cd>* dops);
// the energy of one site as a function of its parameters, the slot
// environments G ([NOPS + 1][d][d]) held fixed
struct PlboSite {
  int d;
  double a_ss, b_ss, g_ss;
  const std::vector<cd>* G;
  int D = 0;                            // with W: operators built on D basis states,
  const std::vector<cd>* W = nullptr;   // then projected, W^dag O W (W: D x d)
};
double plbo_site_energy(const PlboSite& S, const double* p, double* grad);
// po.steps Adam steps (moments m, v, count t in and out) or L-BFGS iterations
void plbo_optimise(const PlboSite& S, const tn_plbo_opts& po, double* p, double* m, double* v, int* t);
// W[n][m] = <n|U|m>, n < D, m < d, from the gates applied in `levels` Fock levels
void plbo_fock_isometry(int D, int d, const double* p, int levels, std::vector<cd>& W);
// recompute the Fock image (iso) of every gate-parameterised basis changed since the last call
void plbo_sync_iso(const tn_mpo* mpo);
struct SlotJob {
  const void* U;  // x R^H (chi_l x d x chi_r)
  const void* Y;  // L x   (chi_l x d x chi_r)
};
// out[j][n'][n] = sum_{a,b} conj(U_j[a][n'][b]) Y_j[a][n][b], FP64
hipError_t launch_slot_gram(int sprec, const SlotJob* d_jobs, int njobs, int cl, int d, int cr, cf64* out,
                            hipStream_t st);
double matvec_flops_formula(const tn_mpo* mpo, int site, int chi_l, int chi_r);
double env_flops_formula(const tn_mpo* mpo, int site, int chi_l, int chi_r);
