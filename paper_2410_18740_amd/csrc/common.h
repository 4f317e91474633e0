// Shared definitions for the gfx950 GBS-DMRG library (host + device).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

typedef float2 cf32;
typedef double2 cf64;

#define TN_HOST_DEVICE __host__ __device__ __forceinline__

// ----------------------------------------------------------------- complex helpers
template <typename C> struct real_of;
template <> struct real_of<cf32> { typedef float type; };
template <> struct real_of<cf64> { typedef double type; };

TN_HOST_DEVICE cf32 cmk(float r, float i) { return make_float2(r, i); }
TN_HOST_DEVICE cf64 cmk(double r, double i) { return make_double2(r, i); }
template <typename C> TN_HOST_DEVICE C czero();
template <> TN_HOST_DEVICE cf32 czero<cf32>() { return make_float2(0.f, 0.f); }
template <> TN_HOST_DEVICE cf64 czero<cf64>() { return make_double2(0.0, 0.0); }
TN_HOST_DEVICE cf32 cadd(cf32 a, cf32 b) { return make_float2(a.x + b.x, a.y + b.y); }
TN_HOST_DEVICE cf64 cadd(cf64 a, cf64 b) { return make_double2(a.x + b.x, a.y + b.y); }
TN_HOST_DEVICE cf32 csub(cf32 a, cf32 b) { return make_float2(a.x - b.x, a.y - b.y); }
TN_HOST_DEVICE cf64 csub(cf64 a, cf64 b) { return make_double2(a.x - b.x, a.y - b.y); }
TN_HOST_DEVICE cf32 cmul(cf32 a, cf32 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
TN_HOST_DEVICE cf64 cmul(cf64 a, cf64 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
TN_HOST_DEVICE cf32 cconj(cf32 a) { return make_float2(a.x, -a.y); }
TN_HOST_DEVICE cf64 cconj(cf64 a) { return make_double2(a.x, -a.y); }
TN_HOST_DEVICE cf32 cscale(cf32 a, float s) { return make_float2(a.x * s, a.y * s); }
TN_HOST_DEVICE cf64 cscale(cf64 a, double s) { return make_double2(a.x * s, a.y * s); }
// a*conj(b)
TN_HOST_DEVICE cf64 cmulc(cf64 a, cf64 b) { return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }
// conj(a)*b
TN_HOST_DEVICE cf64 cconjmul(cf64 a, cf64 b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
TN_HOST_DEVICE cf32 cconjmul(cf32 a, cf32 b) { return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
TN_HOST_DEVICE double cabs2(cf64 a) { return a.x * a.x + a.y * a.y; }

// ----------------------------------------------------------------- precisions
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16X3 = 2 };

// ----------------------------------------------------------------- GEMM descriptors
// C[M x N] (=|+=) sum_seg opA(A_seg)[M x K_seg] * opB(B_seg)[K_seg x N], complex,
// row-major with leading dimensions in elements.  opA = conj-transpose when
// trans_a != 0 (then A is stored K x M), likewise for B (stored N x K).
struct GemmSeg {
  const void* A;
  const void* B;
  int64_t lda, ldb;
  int32_t K;
  int32_t pad_;
};
struct GemmJob {
  void* C;
  int64_t ldc;
  int32_t M, N;
  int32_t seg0, nseg;
};

// 1/q from the hardware reciprocal refined by two Newton steps
// (r <- r + r (1 - q r)), each of which squares the relative error
static __device__ __forceinline__ double recip_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

// ------------------------------------------------------------------ wavefront reduction (DPP)
// Sum over the 64 lanes of a wavefront with data-parallel-primitive moves
// (register crossbar, no LDS traffic): quad xor 1 and 2, half-row and row
// mirrors give every lane its row-of-16 sum; row_bcast:15 and row_bcast:31
// fold rows 0..3 into row 3; lane 63 then broadcasts the total.  The
// summation order is fixed, so results are reproducible.
template <int CTRL, int ROWMASK = 0xf>
static __device__ __forceinline__ double dpp_src_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL, int ROWMASK = 0xf>
static __device__ __forceinline__ float dpp_src_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xf, false));
}
static __device__ __forceinline__ double wave_reduce_sum(double v) {
  v += dpp_src_d<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_src_d<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_src_d<0x141>(v);       // row_half_mirror
  v += dpp_src_d<0x140>(v);       // row_mirror
  v += dpp_src_d<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_src_d<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
static __device__ __forceinline__ float wave_reduce_sum(float v) {
  v += dpp_src_f<0xB1>(v);
  v += dpp_src_f<0x4E>(v);
  v += dpp_src_f<0x141>(v);
  v += dpp_src_f<0x140>(v);
  v += dpp_src_f<0x142, 0xA>(v);
  v += dpp_src_f<0x143, 0xC>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}


// Launch a batch of jobs.  All jobs share precision and transposition flags.
// d_jobs / d_segs are device arrays.  Max M/N over jobs sets the grid.
hipError_t launch_cgemm(int prec, int trans_a, int trans_b, const GemmJob* d_jobs, int njobs,
                        const GemmSeg* d_segs, int maxM, int maxN, int accumulate, hipStream_t st);

// ----------------------------------------------------------------- op-apply descriptors
// out[a][s][t][b] = sum_terms coef * sum_{s',t'} opA[s][s'] opB[t][t'] src[a][s'][t'][b]
// opA/opB == nullptr means identity on that leg.
struct OpTerm {
  const void* src;
  const void* opA;
  const void* opB;
  double coef;
};
struct OpJob {
  void* dst;
  int32_t t0, nterms;
  int32_t accumulate;  // add into existing dst
  int32_t pad_;
};
hipError_t launch_opapply(int prec, const OpJob* d_jobs, int njobs, const OpTerm* d_terms, int chi_l, int ds,
                          int dt, int chi_r, hipStream_t st);

// mixed envs: out[j] = sum_{i in list} coef_i * in_i  (each n_elem complex), prec-typed
struct MixTerm {
  const void* src;
  double coef;
};
struct MixJob {
  void* dst;
  int32_t t0, nterms;
};
hipError_t launch_envmix(int prec, const MixJob* d_jobs, int njobs, const MixTerm* d_terms, int64_t n_elem,
                         hipStream_t st);

// ----------------------------------------------------------------- vector kernels (FP64 complex)
hipError_t launch_convert(int to_prec, void* dst, int from_prec, const void* src, int64_t n, hipStream_t st);
hipError_t launch_reduce_partials(cf64* out, int prec, const void* partials, int nparts, int64_t n, hipStream_t st);
hipError_t launch_multidot(const cf64* const* vs, int nv, const cf64* w, int64_t n, cf64* partials, int nblocks,
                           hipStream_t st);
hipError_t launch_multidot_finish(const cf64* partials, int nv, int nblocks, cf64* out, hipStream_t st);
hipError_t launch_axpy_dot(cf64* w, const cf64* const* vs, int nv, const cf64* coefs, int64_t n, cf64* partials,
                           int nblocks, hipStream_t st);
hipError_t launch_axpy_scale(cf64* dst, const cf64* w, const cf64* const* vs, int nv, const cf64* coefs,
                             const double* inv, int64_t n, hipStream_t st);
hipError_t launch_lincomb(cf64* dst, const cf64* const* vs, int nv, const double* coefs_dev, int64_t n,
                          hipStream_t st);
int multidot_blocks(int64_t n);

// ----------------------------------------------------------------- eigen kernels
// batched Hermitian eigensolver, n <= 64, one workgroup per matrix, LDS resident.
// A: [batch][n][n] complex (row-major), outputs eigenvalues descending (desc=1) or
// ascending, eigenvectors as columns of V [batch][n][n].
hipError_t launch_jacobi(const cf64* A, int64_t strideA, int n, int batch, double* evals, cf64* V, int64_t strideV,
                         int descending, hipStream_t st);

// Householder tridiagonalisation of a Hermitian p x p matrix (row-major, in place).
struct TridiagWork {
  cf64* A;      // p x p
  cf64* vs;     // reflectors, (p) x p  (row j holds v_j)
  cf64* taus;   // p
  double* dg;   // diagonal p
  double* off;  // off-diagonal p
  cf64* y;      // p
  cf64* w;      // p x 2 (ping-pong)
  unsigned int* counter;  // one device counter (workgroups finished)
};
hipError_t launch_tridiag(TridiagWork& tw, int p, hipStream_t st);
hipError_t launch_bisect_top(const double* dg, const double* off, int p, int k, double* evals, hipStream_t st);
hipError_t launch_inverse_iter(const double* dg, const double* off, int p, int k, const double* evals, double* X,
                               double* scratch, hipStream_t st);
hipError_t launch_orthonormalize_real(double* X, int p, int k, int j0, double* H /* k x 16 */, hipStream_t st);
hipError_t launch_ortho_check(const double* X, int p, int k, double tol, int* bad, hipStream_t st);
hipError_t launch_backtransform(const cf64* vs, const cf64* taus, int p, const double* X, int k, cf64* U,
                                hipStream_t st);
// the same with the reflectors in blocks of 16 (compact WY); Tws holds
// backtransform_wy_workspace(p) complex entries; sizes beyond 3072 use the above
size_t backtransform_wy_workspace(int p);
hipError_t launch_backtransform_wy(const cf64* vs, const cf64* taus, int p, const double* X, int k, cf64* U,
                                   cf64* Tws, hipStream_t st);

hipError_t launch_transpose_from64(int prec, void* dst, const cf64* src, int batch, int rows, int cols, hipStream_t st);
hipError_t launch_transpose_to64(int prec, cf64* dst, const void* src, int batch, int rows, int cols, hipStream_t st);
hipError_t launch_scale_host(cf64* dst, const cf64* src, double s, int64_t n, hipStream_t st);
hipError_t launch_ctranspose(cf64* dst, const cf64* src, int n, int k, hipStream_t st);
hipError_t launch_lanczos_ab(const cf64* h1, const cf64* h2, int j, int i0, double* alpha, double* beta, double* inv,
                             double* out, hipStream_t st);
hipError_t launch_inv_norm(const cf64* h, int nv, double* inv, hipStream_t st);
hipError_t launch_finite_check(const cf64* x, int64_t n, int* flag, hipStream_t st);
hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st);
hipError_t launch_set_one(void* p, int prec, hipStream_t st);
hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st);
hipError_t launch_copy2d(cf64* dst, int64_t ldd, const cf64* src, int64_t lds, int rows, int cols, int conj_t,
                         hipStream_t st);
