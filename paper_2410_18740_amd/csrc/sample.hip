// Observables of the converged MPS in the raw Fock basis: single-mode
// photon-number marginals (contraction of rho_j) and sequential conditional
// sampling of photon-number patterns with a counter-based Philox4x32-10
// generator (Salmon, Moraes, Dror, Shaw, SC'11).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include "internal.h"

#define TN_GUARD_BEGIN try {
#define TN_GUARD_END(ctx)                                         \
  }                                                               \
  catch (const TnError& e) {                                      \
    if (ctx) (ctx)->err = e.what();                               \
    return e.code;                                                \
  }                                                               \
  catch (const std::exception& e) {                               \
    if (ctx) (ctx)->err = e.what();                               \
    return TN_EINVAL;                                             \
  }                                                               \
  if (ctx) (ctx)->err.clear();                                    \
  return TN_OK;

// ------------------------------------------------------------------ Philox4x32-10
struct u32x4 { uint32_t v[4]; };
static __device__ __forceinline__ void mulhilo32(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
  const uint64_t p = (uint64_t)a * (uint64_t)b;
  hi = (uint32_t)(p >> 32);
  lo = (uint32_t)p;
}
static __device__ u32x4 philox4x32_10(u32x4 ctr, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, ctr.v[0], hi0, lo0);
    mulhilo32(M1, ctr.v[2], hi1, lo1);
    u32x4 n;
    n.v[0] = hi1 ^ ctr.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ ctr.v[3] ^ k1;
    n.v[3] = lo0;
    ctr = n;
  }
  return ctr;
}
// u in [0, 1) with 53 random bits from the first two output words
static __device__ __forceinline__ double philox_uniform(uint64_t sample, uint32_t site, uint64_t seed) {
  u32x4 c;
  c.v[0] = (uint32_t)sample;
  c.v[1] = (uint32_t)(sample >> 32);
  c.v[2] = site;
  c.v[3] = 0u;
  const u32x4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = r.v[0] >> 5, b = r.v[1] >> 6;
  return ((double)a * 67108864.0 + (double)b) * (1.0 / 9007199254740992.0);
}

__global__ void philox_test_kernel(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u32x4 c;
  for (int j = 0; j < 4; ++j) c.v[j] = ctr[4 * i + j];
  const u32x4 r = philox4x32_10(c, key[2 * i], key[2 * i + 1]);
  for (int j = 0; j < 4; ++j) out[4 * i + j] = r.v[j];
}

// one wavefront per sample: probabilities over D outcomes, inverse CDF, gather
__global__ __launch_bounds__(256) void sample_step_kernel(const cf64* __restrict__ Tmp, int B, int D, int cr,
                                                          uint64_t sample0, int site, uint64_t seed,
                                                          cf64* __restrict__ Vnew, int32_t* __restrict__ out, int N) {
  __shared__ double p[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = blockIdx.x * 4 + wave;
  if (b >= B) return;
  const cf64* row = Tmp + (size_t)b * D * cr;
  for (int n = 0; n < D; ++n) {
    double s = 0.0;
    for (int j = lane; j < cr; j += 64) s += cabs2(row[(size_t)n * cr + j]);
    s = wave_reduce_sum(s);
    if (lane == 0) p[wave][n] = s;
  }
  // p[wave] is private to this wavefront: a wavefront-level barrier orders
  // lane 0's writes before the reads (waves past B have already returned, so
  // no workgroup barrier may follow)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double tot = 0.0;
  for (int n = 0; n < D; ++n) tot += p[wave][n];
  const double u = philox_uniform(sample0 + (uint64_t)b, (uint32_t)site, seed) * tot;
  int pick = D - 1;
  double cum = 0.0;
  for (int n = 0; n < D; ++n) {
    cum += p[wave][n];
    if (cum >= u && p[wave][n] > 0.0) { pick = n; break; }
  }
  while (pick > 0 && !(p[wave][pick] > 0.0)) --pick;
  const double inv = p[wave][pick] > 0.0 ? 1.0 / sqrt(p[wave][pick]) : 0.0;
  for (int j = lane; j < cr; j += 64) {
    const cf64 v = row[(size_t)pick * cr + j];
    Vnew[(size_t)b * cr + j] = make_double2(v.x * inv, v.y * inv);
  }
  if (lane == 0) out[(size_t)b * N + site] = pick;
}

__global__ void fill_one_kernel(cf64* V, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    V[e] = make_double2(1.0, 0.0);
}

// P[n] = sum_{a,b} Re(conj(A[a][n][b]) Y[a][n][b])
__global__ __launch_bounds__(256) void marg_kernel(const cf64* __restrict__ A, const cf64* __restrict__ Y, int cl, int D,
                                                   int cr, double* __restrict__ out) {
  __shared__ double red[4];
  const int n = blockIdx.x;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)cl * cr; e += 256) {
    const int a = (int)(e / cr), b = (int)(e % cr);
    const size_t idx = ((size_t)a * D + n) * cr + b;
    const cf64 x = A[idx], y = Y[idx];
    s += x.x * y.x + x.y * y.y;
  }
  s = wave_reduce_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[n] = red[0] + red[1] + red[2] + red[3];
}

static void gemm_jobs(tn_ctx* c, int ta, int tb, const std::vector<GemmJob>& jobs, const std::vector<GemmSeg>& segs,
                      int maxM, int maxN, const char* tag) {
  const size_t bj = ((jobs.size() * sizeof(GemmJob)) + 255) & ~size_t(255);
  char* d = (char*)ws_get(c, tag, bj + segs.size() * sizeof(GemmSeg));
  HIPCHK(hipMemcpyAsync(d, jobs.data(), jobs.size() * sizeof(GemmJob), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(d + bj, segs.data(), segs.size() * sizeof(GemmSeg), hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_cgemm(PREC_FP64, ta, tb, (GemmJob*)d, (int)jobs.size(), (GemmSeg*)(d + bj), maxM, maxN, 0, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

// A^F_s[a][n][b] = sum_m W_s[n][m] A_s[a][m][b]
static cf64* fock_tensor(tn_ctx* c, const tn_mps* m, const tn_mpo* mpo, int s) {
  const int D = mpo->D_raw, d = mpo->d, cl = m->dims[s], cr = m->dims[s + 1];
  cf64* F = wsT<cf64>(c, "obs:F", (size_t)cl * D * cr);
  std::vector<GemmJob> jobs;
  std::vector<GemmSeg> segs;
  for (int a = 0; a < cl; ++a) {
    segs.push_back({mpo->fock_iso() + (size_t)s * D * d, m->A[s] + (size_t)a * d * cr, d, cr, d, 0});
    jobs.push_back({F + (size_t)a * D * cr, cr, D, cr, a, 1});
  }
  gemm_jobs(c, 0, 0, jobs, segs, D, cr, "obs:g0");
  return F;
}

static void check_obs(const tn_mps* m, const tn_mpo* mpo) {
  if (!m || !mpo) TN_THROW(TN_EINVAL, "null handle");
  if (m->N != mpo->N || m->d != mpo->d) TN_THROW(TN_EINVAL, "MPO and MPS do not match");
  if (m->center != 0) TN_THROW(TN_ESTATE, "the MPS must be right-canonical with its centre at site 0");
  plbo_sync_iso(mpo);
}

extern "C" tn_status tn_marginals(tn_ctx* c, const tn_mps* m, const tn_mpo* mpo, int32_t n_modes, double* out) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  check_obs(m, mpo);
  if (!out || n_modes < 1 || n_modes > m->N) TN_THROW(TN_EINVAL, "bad output or n_modes");
  const int D = mpo->D_raw;
  hipStream_t st = c->stream;
  size_t mx = 1;
  for (int t = 0; t <= m->N; ++t) mx = std::max(mx, (size_t)m->dims[t] * m->dims[t]);
  cf64* Ea = wsT<cf64>(c, "obs:Ea", mx);
  cf64* Eb = wsT<cf64>(c, "obs:Eb", mx);
  size_t my = 1;
  for (int s = 0; s < n_modes; ++s) my = std::max(my, (size_t)m->dims[s] * D * m->dims[s + 1]);
  cf64* Y = wsT<cf64>(c, "obs:Y", my);
  double* P = wsT<double>(c, "obs:P", (size_t)D);
  hipLaunchKernelGGL(fill_one_kernel, dim3(1), dim3(64), 0, st, Ea, (int64_t)1);
  std::vector<double> host(D);
  double nrm = 1.0;
  for (int s = 0; s < n_modes; ++s) {
    const int cl = m->dims[s], cr = m->dims[s + 1];
    cf64* F = fock_tensor(c, m, mpo, s);
    std::vector<GemmJob> jobs{{Y, (int64_t)D * cr, cl, D * cr, 0, 1}};
    std::vector<GemmSeg> segs{{Ea, F, cl, (int64_t)D * cr, cl, 0}};
    gemm_jobs(c, 0, 0, jobs, segs, cl, D * cr, "obs:g1");
    hipLaunchKernelGGL(marg_kernel, dim3(D), dim3(256), 0, st, F, Y, cl, D, cr, P);
    download(c, host.data(), P, D * sizeof(double));
    if (s == 0) {
      nrm = 0.0;
      for (int n = 0; n < D; ++n) nrm += host[n];
      if (!(nrm > 0.0)) TN_THROW(TN_ENUMERIC, "zero norm");
    }
    for (int n = 0; n < D; ++n) out[(size_t)s * D + n] = host[n] / nrm;
    std::vector<GemmJob> j2{{Eb, cr, cr, cr, 0, 1}};
    std::vector<GemmSeg> s2{{F, Y, cr, cr, cl * D, 0}};
    gemm_jobs(c, 1, 0, j2, s2, cr, cr, "obs:g2");
    std::swap(Ea, Eb);
  }
  TN_GUARD_END(c)
}

extern "C" tn_status tn_sample(tn_ctx* c, const tn_mps* m, const tn_mpo* mpo, int64_t n_samples, uint64_t seed,
                               int32_t* out) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  check_obs(m, mpo);
  if (!out || n_samples < 1) TN_THROW(TN_EINVAL, "bad output or sample count");
  const int N = m->N, D = mpo->D_raw;
  hipStream_t st = c->stream;
  int chimax = 1;
  for (int t = 0; t <= N; ++t) chimax = std::max(chimax, m->dims[t]);
  const int64_t chunk = std::min<int64_t>(n_samples, std::max<int64_t>(64, (int64_t)(1ll << 31) / ((int64_t)D * chimax * 16)));
  cf64* Tmp = wsT<cf64>(c, "smp:T", (size_t)chunk * D * chimax);
  cf64* Va = wsT<cf64>(c, "smp:Va", (size_t)chunk * chimax);
  cf64* Vb = wsT<cf64>(c, "smp:Vb", (size_t)chunk * chimax);
  std::vector<cf64*> F(N);
  for (int s = 0; s < N; ++s) {
    const size_t nel = (size_t)m->dims[s] * D * m->dims[s + 1];
    cf64* tmpF = fock_tensor(c, m, mpo, s);
    F[s] = wsT<cf64>(c, "smp:F" + std::to_string(s), nel);
    HIPCHK(hipMemcpyAsync(F[s], tmpF, nel * sizeof(cf64), hipMemcpyDeviceToDevice, st));
  }
  for (int64_t s0 = 0; s0 < n_samples; s0 += chunk) {
    const int B = (int)std::min<int64_t>(chunk, n_samples - s0);
    hipLaunchKernelGGL(fill_one_kernel, dim3(std::max(1, (B + 255) / 256)), dim3(256), 0, st, Va, (int64_t)B);
    for (int s = 0; s < N; ++s) {
      const int cl = m->dims[s], cr = m->dims[s + 1];
      std::vector<GemmJob> jobs{{Tmp, (int64_t)D * cr, B, D * cr, 0, 1}};
      std::vector<GemmSeg> segs{{Va, F[s], cl, (int64_t)D * cr, cl, 0}};
      gemm_jobs(c, 0, 0, jobs, segs, B, D * cr, "smp:g");
      hipLaunchKernelGGL(sample_step_kernel, dim3((B + 3) / 4), dim3(256), 0, st, Tmp, B, D, cr, (uint64_t)s0, s, seed,
                         Vb, out + (size_t)s0 * N, N);
      HIPCHK(hipGetLastError());
      std::swap(Va, Vb);
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  TN_GUARD_END(c)
}

// ------------------------------------------------------------------ sampling without allocation
// tn_sample_noalloc keeps every buffer tn_sample takes from the context's
// workspace in one file-scope device array per GPU instead: the GEMM
// descriptors, the Fock-basis site tensors and the per-chunk contraction and
// left vectors.  The array's device address comes from hipGetSymbolAddress,
// taken once per device at context creation with that device current; host
// code never uses the array's name as an address.
static constexpr size_t kScratchBytes = 64ull << 20;  // the stated maximum: 64 MiB per GPU
static constexpr size_t kScratchDesc = 64ull << 10;   // GEMM descriptors at its start
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Called by tn_ctx_create with `device` current.
tn_status sample_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return TN_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return TN_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return TN_EHIP;
  }
  g_scratch_ptr[device] = p;
  return TN_OK;
}

static void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  void* p = (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
  if (!p) TN_THROW(TN_ESTATE, "no sampling scratch for this device");
  return p;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// gemm_jobs with the descriptors placed at `desc` (device) instead of a workspace
static void gemm_jobs_at(tn_ctx* c, char* desc, const std::vector<GemmJob>& jobs, const std::vector<GemmSeg>& segs,
                         int maxM, int maxN) {
  const size_t bj = align256(jobs.size() * sizeof(GemmJob));
  if (bj + segs.size() * sizeof(GemmSeg) > kScratchDesc) TN_THROW(TN_EINVAL, "too many GEMM descriptors for the scratch");
  HIPCHK(hipMemcpyAsync(desc, jobs.data(), jobs.size() * sizeof(GemmJob), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(desc + bj, segs.data(), segs.size() * sizeof(GemmSeg), hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_cgemm(PREC_FP64, 0, 0, (GemmJob*)desc, (int)jobs.size(), (GemmSeg*)(desc + bj), maxM, maxN, 0,
                      c->stream));
  // the descriptors are rewritten by the next call
  HIPCHK(hipStreamSynchronize(c->stream));
}

extern "C" tn_status tn_sample_noalloc(tn_ctx* c, const tn_mps* m, const tn_mpo* mpo, int64_t n_samples,
                                       uint64_t seed, int32_t* out) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!m || !mpo) TN_THROW(TN_EINVAL, "null handle");
  if (m->N != mpo->N || m->d != mpo->d) TN_THROW(TN_EINVAL, "MPO and MPS do not match");
  if (m->center != 0) TN_THROW(TN_ESTATE, "the MPS must be right-canonical with its centre at site 0");
  if (mpo->plbo)
    for (int s = 0; s < mpo->N; ++s)
      if (mpo->iso_stale[s]) TN_THROW(TN_ESTATE, "the Fock image of the local bases is stale (tn_mpo_isometries first)");
  if (!out || n_samples < 1) TN_THROW(TN_EINVAL, "bad output or sample count");
  const int N = m->N, D = mpo->D_raw, d = mpo->d;
  hipStream_t st = c->stream;
  int chimax = 1;
  for (int t = 0; t <= N; ++t) chimax = std::max(chimax, m->dims[t]);
  for (int t = 0; t < N; ++t)
    if (m->dims[t] > 2048) TN_THROW(TN_EINVAL, "bond dimension beyond the scratch's descriptor space");
  char* base = (char*)scratch_of(c->device);
  char* desc = base;
  size_t off = kScratchDesc;
  std::vector<cf64*> F(N);
  for (int s = 0; s < N; ++s) {
    F[s] = (cf64*)(base + off);
    off += align256((size_t)m->dims[s] * D * m->dims[s + 1] * sizeof(cf64));
  }
  const size_t per = sizeof(cf64) * ((size_t)D * chimax + 2 * (size_t)chimax) + 3 * 256;
  if (off >= kScratchBytes || (kScratchBytes - off) / per < 1)
    TN_THROW(TN_EINVAL, "the MPS needs " + std::to_string(off + per) + " bytes of scratch, beyond the " +
                            std::to_string(kScratchBytes) + " of tn_sample_noalloc");
  const int64_t chunk = std::min<int64_t>(n_samples, (int64_t)((kScratchBytes - off) / per));
  cf64* Tmp = (cf64*)(base + off);
  off += align256((size_t)chunk * D * chimax * sizeof(cf64));
  cf64* Va = (cf64*)(base + off);
  off += align256((size_t)chunk * chimax * sizeof(cf64));
  cf64* Vb = (cf64*)(base + off);
  // Fock-basis site tensors A^F_s[a][n][b] = sum_m W_s[n][m] A_s[a][m][b]
  for (int s = 0; s < N; ++s) {
    const int cl = m->dims[s], cr = m->dims[s + 1];
    std::vector<GemmJob> jobs;
    std::vector<GemmSeg> segs;
    for (int a = 0; a < cl; ++a) {
      segs.push_back({mpo->fock_iso() + (size_t)s * D * d, m->A[s] + (size_t)a * d * cr, d, cr, d, 0});
      jobs.push_back({F[s] + (size_t)a * D * cr, cr, D, cr, a, 1});
    }
    gemm_jobs_at(c, desc, jobs, segs, D, cr);
  }
  for (int64_t s0 = 0; s0 < n_samples; s0 += chunk) {
    const int B = (int)std::min<int64_t>(chunk, n_samples - s0);
    hipLaunchKernelGGL(fill_one_kernel, dim3(std::max(1, (B + 255) / 256)), dim3(256), 0, st, Va, (int64_t)B);
    for (int s = 0; s < N; ++s) {
      const int cl = m->dims[s], cr = m->dims[s + 1];
      std::vector<GemmJob> jobs{{Tmp, (int64_t)D * cr, B, D * cr, 0, 1}};
      std::vector<GemmSeg> segs{{Va, F[s], cl, (int64_t)D * cr, cl, 0}};
      gemm_jobs_at(c, desc, jobs, segs, B, D * cr);
      hipLaunchKernelGGL(sample_step_kernel, dim3((B + 3) / 4), dim3(256), 0, st, Tmp, B, D, cr, (uint64_t)s0, s, seed,
                         Vb, out + (size_t)s0 * N, N);
      HIPCHK(hipGetLastError());
      std::swap(Va, Vb);
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  TN_GUARD_END(c)
}

// ------------------------------------------------------------------ noisy GBS (Sec. II.F)
// Uniform loss eta after the squeezers: per input mode the lossy variances are
// (eta e^{-2r} + 1 - eta)/2 (x, squeezed) and (eta e^{2r} + 1 - eta)/2 (p).
// The pure part keeps the squeezed variance, e^{-2r'} = eta e^{-2r} + 1 - eta,
// and the classical part C = L L^T puts the remainder c_i on p of input
// mode i, rotated by the interferometer: L[:, i] = sqrt(c_i) O[:, N + i] with
// O = [[Re U, -Im U], [Im U, Re U]] (eq. CovarianceDecomposition).
extern "C" tn_status tn_noise_uniform_loss(int32_t N, const double* r, const double* U, double eta, double* r_pure,
                                           double* L) {
  if (N < 1 || N > 4096 || !r || !U || !r_pure || !L) return TN_EINVAL;
  if (!(eta > 0.0 && eta <= 1.0)) return TN_EINVAL;
  for (int i = 0; i < N; ++i)
    if (!std::isfinite(r[i]) || r[i] < 0.0) return TN_EINVAL;
  for (int64_t i = 0; i < 2ll * N * N; ++i)
    if (!std::isfinite(U[i])) return TN_EINVAL;
  std::vector<double> c(N);
  for (int i = 0; i < N; ++i) {
    const double vx = eta * std::exp(-2.0 * r[i]) + 1.0 - eta;
    const double vp = eta * std::exp(2.0 * r[i]) + 1.0 - eta;
    r_pure[i] = -0.5 * std::log(vx);
    c[i] = std::max(0.0, 0.5 * (vp - 1.0 / vx));
  }
  for (int j = 0; j < N; ++j)
    for (int i = 0; i < N; ++i) {
      const double ur = U[2 * ((size_t)j * N + i)], ui = U[2 * ((size_t)j * N + i) + 1];
      const double sc = std::sqrt(c[i]);
      L[(size_t)j * N + i] = -ui * sc;
      L[(size_t)(N + j) * N + i] = ur * sc;
    }
  return TN_OK;
}

// Cyclic Jacobi for a complex Hermitian n x n matrix on the host (FP64):
// A (row-major) is overwritten; w receives the eigenvalues in ascending order
// and the columns of Z the eigenvectors.  The rotation zeroing a_pq is the one
// of the device eigensolver (same angle formulas).
static void herm_eig_host(int n, std::vector<cd> A, std::vector<double>& w, std::vector<cd>& Z) {
  Z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  auto at = [&](int i, int j) -> cd& { return A[(size_t)i * n + j]; };
  for (int i = 0; i < n; ++i) at(i, i) = at(i, i).real();
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) (i == j ? tot : off) += std::norm(at(i, j));
    if (off <= 1e-30 * (tot + off) || off < 1e-300) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cd apq = at(p, q);
        const double b = std::abs(apq), app = at(p, p).real(), aqq = at(q, q).real();
        if (!(b > 1e-300) || b * b <= 1e-34 * (app * app + aqq * aqq)) continue;
        const double zeta = (aqq - app) / (2.0 * b);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        const cd em = std::conj(apq) / b, ep = apq / b;  // e^{-i phi}, e^{i phi}
        for (int r = 0; r < n; ++r) {  // columns: A <- A J, Z <- Z J
          const cd xp = at(r, p), xq = at(r, q) * em;
          at(r, p) = c * xp - sn * xq;
          at(r, q) = sn * xp + c * xq;
          const cd zp = Z[(size_t)r * n + p], zq = Z[(size_t)r * n + q] * em;
          Z[(size_t)r * n + p] = c * zp - sn * zq;
          Z[(size_t)r * n + q] = sn * zp + c * zq;
        }
        for (int k = 0; k < n; ++k) {  // rows: A <- J^H A
          const cd xp = at(p, k), xq = at(q, k) * ep;
          at(p, k) = c * xp - sn * xq;
          at(q, k) = sn * xp + c * xq;
        }
        at(p, q) = 0.0;
        at(q, p) = 0.0;
        at(p, p) = at(p, p).real();
        at(q, q) = at(q, q).real();
      }
  }
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return at(a, a).real() < at(b, b).real(); });
  w.resize(n);
  std::vector<cd> Zs((size_t)n * n);
  for (int c2 = 0; c2 < n; ++c2) {
    w[c2] = at(ord[c2], ord[c2]).real();
    for (int r = 0; r < n; ++r) Zs[(size_t)r * n + c2] = Z[(size_t)r * n + ord[c2]];
  }
  Z.swap(Zs);
}

// General split of a mixed covariance (eq. CovarianceDecomposition) by the
// Williamson decomposition V = S diag(nu, nu) S^T: with A = V^{-1/2} Omega
// V^{-1/2} (antisymmetric, Omega = [[0, I], [-I, 0]]), an eigenvector a + i b
// of i A for the eigenvalue 1/nu_k gives the pair of columns sqrt2 a, -sqrt2 b
// of an orthogonal K with K^T A K = [[0, diag(1/nu)], [-diag(1/nu), 0]], and
// S = V^{1/2} K diag(nu, nu)^{-1/2}.  Q = S S^T / 2 is pure and
// C = S (diag(nu, nu) - I/2) S^T >= 0.  The pure part's (r, U): eigenvectors
// x of Q with eigenvalue e^{-2r}/2 <= 1/2 are the columns (Re U; Im U) of the
// passive rotation, -Omega x their partners; a degenerate eigenvalue 1/2 is
// split into such pairs by Gram-Schmidt.
extern "C" tn_status tn_noise_williamson(int32_t N, const double* V, double* r_pure, double* U_pure, double* L,
                                         int32_t* K) {
  if (N < 1 || N > 512 || !V || !r_pure || !U_pure || !L || !K) return TN_EINVAL;
  const int n = 2 * N;
  for (int i = 0; i < n * n; ++i)
    if (!std::isfinite(V[i])) return TN_EINVAL;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (std::fabs(V[i * n + j] - V[j * n + i]) > 1e-10 * (std::fabs(V[i * n + j]) + 1e-300) &&
          std::fabs(V[i * n + j] - V[j * n + i]) > 1e-14)
        return TN_EINVAL;
  try {
    std::vector<cd> Vc((size_t)n * n);
    for (int i = 0; i < n * n; ++i) Vc[i] = V[i];
    std::vector<double> w;
    std::vector<cd> E;
    herm_eig_host(n, Vc, w, E);
    if (!(w[0] > 0.0)) return TN_EINVAL;
    std::vector<double> Vh((size_t)n * n, 0.0), Vmh((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < n; ++k) {
          const double e = (E[(size_t)i * n + k] * std::conj(E[(size_t)j * n + k])).real();
          a += e * std::sqrt(w[k]);
          b += e / std::sqrt(w[k]);
        }
        Vh[(size_t)i * n + j] = a;
        Vmh[(size_t)i * n + j] = b;
      }
    // A = Vmh Omega Vmh; (Omega M)[i][j] = M[i+N][j] (i < N), -M[i-N][j] (i >= N)
    std::vector<double> OmV((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) OmV[(size_t)i * n + j] = i < N ? Vmh[(size_t)(i + N) * n + j] : -Vmh[(size_t)(i - N) * n + j];
    std::vector<cd> iA((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a = 0.0;
        for (int k = 0; k < n; ++k) a += Vmh[(size_t)i * n + k] * OmV[(size_t)k * n + j];
        iA[(size_t)i * n + j] = cd(0.0, a);
      }
    std::vector<double> mu;
    std::vector<cd> Uc;
    herm_eig_host(n, iA, mu, Uc);  // ascending: the last N are the positive 1/nu
    std::vector<double> nu(N), Kmat((size_t)n * n);
    for (int c = 0; c < N; ++c) {
      const int k = n - 1 - c;
      if (!(mu[k] > 0.0)) return TN_EINVAL;
      nu[c] = 1.0 / mu[k];
      if (nu[c] < 0.5 - 1e-9) return TN_EINVAL;  // not a physical covariance
      for (int i = 0; i < n; ++i) {
        Kmat[(size_t)i * n + c] = std::sqrt(2.0) * Uc[(size_t)i * n + k].real();
        Kmat[(size_t)i * n + N + c] = -std::sqrt(2.0) * Uc[(size_t)i * n + k].imag();
      }
    }
    // S = Vh K diag(nu, nu)^{-1/2}
    std::vector<double> S((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a = 0.0;
        for (int k = 0; k < n; ++k) a += Vh[(size_t)i * n + k] * Kmat[(size_t)k * n + j];
        S[(size_t)i * n + j] = a / std::sqrt(nu[j % N]);
      }
    std::vector<cd> Q((size_t)n * n), C((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double q = 0.0, c = 0.0;
        for (int k = 0; k < n; ++k) {
          const double sk = S[(size_t)i * n + k] * S[(size_t)j * n + k];
          q += 0.5 * sk;
          c += (nu[k % N] - 0.5) * sk;
        }
        Q[(size_t)i * n + j] = q;
        C[(size_t)i * n + j] = c;
      }
    // pure part (r, U)
    std::vector<double> wq;
    std::vector<cd> Eq;
    herm_eig_host(n, Q, wq, Eq);
    std::vector<std::vector<double>> basis;
    int found = 0;
    for (int k = 0; k < n && found < N; ++k) {
      if (wq[k] > 0.5 + 1e-9) break;
      std::vector<double> v(n);
      for (int i = 0; i < n; ++i) v[i] = Eq[(size_t)i * n + k].real();
      for (const auto& u : basis) {
        double dp = 0.0;
        for (int i = 0; i < n; ++i) dp += u[i] * v[i];
        for (int i = 0; i < n; ++i) v[i] -= dp * u[i];
      }
      double nv = 0.0;
      for (double x : v) nv += x * x;
      nv = std::sqrt(nv);
      if (nv < 1e-6) continue;
      for (double& x : v) x /= nv;
      std::vector<double> pv(n);  // -Omega v
      for (int i = 0; i < n; ++i) pv[i] = i < N ? -v[i + N] : v[i - N];
      r_pure[found] = -0.5 * std::log(2.0 * std::min(wq[k], 0.5));
      for (int j = 0; j < N; ++j) {
        U_pure[2 * ((size_t)j * N + found)] = v[j];
        U_pure[2 * ((size_t)j * N + found) + 1] = v[N + j];
      }
      basis.push_back(v);
      basis.push_back(pv);
      ++found;
    }
    if (found != N) return TN_ENUMERIC;
    // C = L L^T over its eigenvalues above 1e-12 of the largest eigenvalue of V
    // (a pure V leaves K = 0: no classical noise)
    std::vector<double> wc;
    std::vector<cd> Ec;
    herm_eig_host(n, C, wc, Ec);
    const double thr = 1e-12 * w[n - 1];
    int kk = 0;
    for (int k = n - 1; k >= 0; --k)
      if (wc[k] > thr) ++kk;
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < kk; ++c) {
        const int k = n - 1 - c;
        L[(size_t)i * kk + c] = Ec[(size_t)i * n + k].real() * std::sqrt(wc[k]);
      }
    *K = kk;
  } catch (...) {
    return TN_ENOMEM;
  }
  return TN_OK;
}

// Standard normal draws of the noise: z[b][i] for samples sample0 + b, noise
// column i, by the Box-Muller transform (Box & Muller, Ann. Math. Statist. 29,
// 1958) of two uniforms from one Philox4x32-10 block with counter
// (sample lo, sample hi, i, 1) and key (seed lo, seed hi): u1 in (0, 1] from
// words 0-1 and u2 in [0, 1) from words 2-3, 53 bits each;
// z = sqrt(-2 ln u1) cos(2 pi u2).  The last counter word 1 keeps these blocks
// apart from the photon-number draws, which use 0 there.
__global__ void noise_normal_kernel(uint64_t seed, uint64_t sample0, int64_t B, int K, double* __restrict__ z) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * K) return;
  const uint64_t sample = sample0 + (uint64_t)(e / K);
  const int i = (int)(e % K);
  u32x4 c;
  c.v[0] = (uint32_t)sample;
  c.v[1] = (uint32_t)(sample >> 32);
  c.v[2] = (uint32_t)i;
  c.v[3] = 1u;
  const u32x4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double k53 = 1.0 / 9007199254740992.0;
  const double u1 = ((double)(r.v[0] >> 5) * 67108864.0 + (double)(r.v[1] >> 6) + 1.0) * k53;
  const double u2 = ((double)(r.v[2] >> 5) * 67108864.0 + (double)(r.v[3] >> 6)) * k53;
  z[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

// alpha[b][j] = (d_x + i d_p) / sqrt2 with d = L z_b (L: 2N x K, z: B x K)
__global__ void noise_alpha_kernel(const double* __restrict__ z, const double* __restrict__ L, int64_t B, int N, int K,
                                   cf64* __restrict__ alpha) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * N) return;
  const int64_t b = e / N;
  const int j = (int)(e % N);
  double dx = 0.0, dp = 0.0;
  for (int i = 0; i < K; ++i) {
    const double zi = z[b * K + i];
    dx += L[(int64_t)j * K + i] * zi;
    dp += L[(int64_t)(N + j) * K + i] * zi;
  }
  const double s = 0.70710678118654752440;
  alpha[e] = make_double2(dx * s, dp * s);
}

// T2[b][n][j] = sum_k <n|D(alpha_b)|k> T[b][k][j] over the D kept levels: one
// wavefront per sample.  The matrix is built in LDS row by row from
//   <0|D|k> = e^{-|alpha|^2/2} (-alpha^*)^k / sqrt(k!),
//   <n+1|D|k> = (sqrt(k) <n|D|k-1> + alpha <n|D|k>) / sqrt(n+1)
// (from a D(alpha) = D(alpha) (a + alpha)), lane k holding column k.
__global__ __launch_bounds__(64) void displace_rows_kernel(const cf64* __restrict__ T, const cf64* __restrict__ alpha,
                                                           int64_t astride, int B, int D, int cr,
                                                           cf64* __restrict__ T2) {
  extern __shared__ unsigned char smraw[];
  cf64* Dm = reinterpret_cast<cf64*>(smraw);  // D x D
  const int b = blockIdx.x, lane = threadIdx.x;
  if (b >= B) return;
  const cf64 al = alpha[(int64_t)b * astride];
  if (lane < D) {
    // (-alpha^*)^k / sqrt(k!) e^{-|alpha|^2/2}
    const double g = exp(-0.5 * (al.x * al.x + al.y * al.y));
    double vr = g, vi = 0.0;
    for (int q = 1; q <= lane; ++q) {
      const double sq = 1.0 / sqrt((double)q);
      const double nr = (-al.x * vr - al.y * vi) * sq;  // (-alpha^*) * v: (-ax + i ay)(vr + i vi)
      const double ni = (-al.x * vi + al.y * vr) * sq;
      vr = nr;
      vi = ni;
    }
    Dm[lane] = make_double2(vr, vi);
  }
  __syncthreads();
  for (int n = 0; n + 1 < D; ++n) {
    cf64 v = make_double2(0.0, 0.0);
    if (lane < D) {
      const cf64 cur = Dm[n * D + lane];
      const cf64 left = lane > 0 ? Dm[n * D + lane - 1] : make_double2(0.0, 0.0);
      const double sk = sqrt((double)lane), inv = 1.0 / sqrt((double)(n + 1));
      v.x = (sk * left.x + al.x * cur.x - al.y * cur.y) * inv;
      v.y = (sk * left.y + al.x * cur.y + al.y * cur.x) * inv;
    }
    __syncthreads();
    if (lane < D) Dm[(n + 1) * D + lane] = v;
    __syncthreads();
  }
  const cf64* Tb = T + (int64_t)b * D * cr;
  cf64* T2b = T2 + (int64_t)b * D * cr;
  if (D <= 16) {
    // column j of T held in registers, read once; Dm entries are LDS broadcasts
    for (int j = lane; j < cr; j += 64) {
      cf64 t[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) t[k] = k < D ? Tb[(int64_t)k * cr + j] : make_double2(0.0, 0.0);
      for (int n = 0; n < D; ++n) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          if (k < D) {
            const cf64 m = Dm[n * D + k];
            sr += m.x * t[k].x - m.y * t[k].y;
            si += m.x * t[k].y + m.y * t[k].x;
          }
        }
        T2b[(int64_t)n * cr + j] = make_double2(sr, si);
      }
    }
    return;
  }
  for (int j = lane; j < cr; j += 64) {
    for (int n = 0; n < D; ++n) {
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < D; ++k) {
        const cf64 m = Dm[n * D + k], t = Tb[(int64_t)k * cr + j];
        sr += m.x * t.x - m.y * t.y;
        si += m.x * t.y + m.y * t.x;
      }
      T2b[(int64_t)n * cr + j] = make_double2(sr, si);
    }
  }
}

extern "C" tn_status tn_sample_displaced(tn_ctx* c, const tn_mps* m, const tn_mpo* mpo, int64_t n_samples,
                                         uint64_t seed, int32_t K, const double* z, const double* L, int32_t* out) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  check_obs(m, mpo);
  if (!out || !L || n_samples < 1) TN_THROW(TN_EINVAL, "bad output, noise factor or sample count");
  const int N = m->N, D = mpo->D_raw;
  if (K < 1 || K > 2 * N) TN_THROW(TN_EINVAL, "the noise factor needs 1 <= K <= 2N columns");
  for (int64_t i = 0; i < 2ll * N * K; ++i)
    if (!std::isfinite(L[i])) TN_THROW(TN_EINVAL, "non-finite noise factor");
  hipStream_t st = c->stream;
  int chimax = 1;
  for (int t = 0; t <= N; ++t) chimax = std::max(chimax, m->dims[t]);
  const int64_t chunk = std::min<int64_t>(n_samples, std::max<int64_t>(64, (int64_t)(1ll << 31) / ((int64_t)D * chimax * 16)));
  cf64* Tmp = wsT<cf64>(c, "smp:T", (size_t)chunk * D * chimax);
  cf64* T2 = wsT<cf64>(c, "smp:T2", (size_t)chunk * D * chimax);
  cf64* Va = wsT<cf64>(c, "smp:Va", (size_t)chunk * chimax);
  cf64* Vb = wsT<cf64>(c, "smp:Vb", (size_t)chunk * chimax);
  cf64* al = wsT<cf64>(c, "smp:al", (size_t)chunk * N);
  double* dL = wsT<double>(c, "smp:L", 2 * (size_t)N * K);
  double* zdraw = z ? nullptr : wsT<double>(c, "smp:z", (size_t)chunk * K);
  upload(c, dL, L, 2 * (size_t)N * K * sizeof(double));
  std::vector<cf64*> F(N);
  for (int s = 0; s < N; ++s) {
    const size_t nel = (size_t)m->dims[s] * D * m->dims[s + 1];
    cf64* tmpF = fock_tensor(c, m, mpo, s);
    F[s] = wsT<cf64>(c, "smp:F" + std::to_string(s), nel);
    HIPCHK(hipMemcpyAsync(F[s], tmpF, nel * sizeof(cf64), hipMemcpyDeviceToDevice, st));
  }
  for (int64_t s0 = 0; s0 < n_samples; s0 += chunk) {
    const int B = (int)std::min<int64_t>(chunk, n_samples - s0);
    const int64_t ne = (int64_t)B * N;
    const double* zb = z ? z + s0 * K : zdraw;
    if (!z) {
      const int64_t nz = (int64_t)B * K;
      hipLaunchKernelGGL(noise_normal_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, seed, (uint64_t)s0,
                         (int64_t)B, K, zdraw);
      HIPCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(noise_alpha_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, zb, dL,
                       (int64_t)B, N, K, al);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(fill_one_kernel, dim3(std::max(1, (B + 255) / 256)), dim3(256), 0, st, Va, (int64_t)B);
    for (int s = 0; s < N; ++s) {
      const int cl = m->dims[s], cr = m->dims[s + 1];
      std::vector<GemmJob> jobs{{Tmp, (int64_t)D * cr, B, D * cr, 0, 1}};
      std::vector<GemmSeg> segs{{Va, F[s], cl, (int64_t)D * cr, cl, 0}};
      gemm_jobs(c, 0, 0, jobs, segs, B, D * cr, "smp:g");
      hipLaunchKernelGGL(displace_rows_kernel, dim3(B), dim3(64), (size_t)D * D * sizeof(cf64), st, Tmp, al + s,
                         (int64_t)N, B, D, cr, T2);
      HIPCHK(hipGetLastError());
      hipLaunchKernelGGL(sample_step_kernel, dim3((B + 3) / 4), dim3(256), 0, st, T2, B, D, cr, (uint64_t)s0, s, seed,
                         Vb, out + (size_t)s0 * N, N);
      HIPCHK(hipGetLastError());
      std::swap(Va, Vb);
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  TN_GUARD_END(c)
}

// Philox known-answer entry point (device generator check): n counters/keys on host.
extern "C" tn_status tn_philox4x32_10(tn_ctx* c, const uint32_t* ctr, const uint32_t* key, uint32_t* out, int32_t n) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!ctr || !key || !out || n < 1) TN_THROW(TN_EINVAL, "bad arguments");
  uint32_t* dc = wsT<uint32_t>(c, "px:c", 4 * (size_t)n);
  uint32_t* dk = wsT<uint32_t>(c, "px:k", 2 * (size_t)n);
  uint32_t* dout = wsT<uint32_t>(c, "px:o", 4 * (size_t)n);
  upload(c, dc, ctr, 16 * (size_t)n);
  upload(c, dk, key, 8 * (size_t)n);
  hipLaunchKernelGGL(philox_test_kernel, dim3((n + 63) / 64), dim3(64), 0, c->stream, dc, dk, dout, n);
  HIPCHK(hipGetLastError());
  download(c, out, dout, 16 * (size_t)n);
  TN_GUARD_END(c)
}
