// Learned warm start: a 3-layer perceptron (tanh, tanh, linear) in FP32 with
// hand-written forward, backward and Adam kernels, plus the parameterised
// local basis it predicts (a squeezed Fock basis) and single-site reduced
// density matrices used to build its training targets.
#include <algorithm>
#include <cmath>
#include <cstring>
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

// ------------------------------------------------------------------ kernels
// C[M x N] = op(A) op(B) (+ bias[N]) (then tanh if act), FP32, 64x64 tiles,
// 256 threads with a 4x4 register block each.  op(A) = A^T if ta (A stored K x M).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void sgemm_kernel(int M, int N, int K, const float* __restrict__ A, int lda,
                                                    const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                    int ldc, const float* __restrict__ bias, int act, int accumulate) {
  __shared__ float As[16][64 + 1];
  __shared__ float Bs[16][64 + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      int mm, kk;
      if (!TA) { mm = e / 16; kk = e % 16; } else { kk = e / 64; mm = e % 64; }
      const int gm = m0 + mm, gk = k0 + kk;
      float v = 0.f;
      if (gm < M && gk < K) v = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      As[kk][mm] = v;
      int nn;
      if (!TB) { kk = e / 64; nn = e % 64; } else { nn = e / 16; kk = e % 16; }
      const int gn = n0 + nn;
      const int gk2 = k0 + kk;
      float w = 0.f;
      if (gn < N && gk2 < K) w = TB ? B[(int64_t)gn * ldb + gk2] : B[(int64_t)gk2 * ldb + gn];
      Bs[kk][nn] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
      if (m < M && n < N) {
        float v = acc[i][j];
        if (bias) v += bias[n];
        if (act) v = tanhf(v);
        float* p = C + (int64_t)m * ldc + n;
        if (accumulate) v += *p;
        *p = v;
      }
    }
}

static void sgemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B,
                  int ldb, float* C, int ldc, const float* bias, int act) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  if (!ta && !tb) hipLaunchKernelGGL((sgemm_kernel<false, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, bias, act, 0);
  else if (ta && !tb) hipLaunchKernelGGL((sgemm_kernel<true, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, bias, act, 0);
  else if (!ta && tb) hipLaunchKernelGGL((sgemm_kernel<false, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, bias, act, 0);
  else hipLaunchKernelGGL((sgemm_kernel<true, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, bias, act, 0);
  HIPCHK(hipGetLastError());
}

// dY = 2 (Y - T) / (B O); per-block partial sums of (Y - T)^2 (fixed order)
__global__ __launch_bounds__(256) void mse_kernel(const float* Y, const float* T, int n, float scale, float* dY,
                                                  double* partial) {
  __shared__ double red[4];
  double s = 0.0;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const float d = Y[e] - T[e];
    dY[e] = 2.f * d * scale;
    s += (double)d * d;
  }
  s = wave_reduce_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}
__global__ void sum_partials_kernel(const double* partial, int n, double scale, float* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    out[0] = (float)(s * scale);
  }
}
// dZ = dH * (1 - H^2)
__global__ void dtanh_kernel(float* dH, const float* H, int n) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) dH[e] *= 1.f - H[e] * H[e];
}
// db[j] = sum_b dZ[b][j]
__global__ void colsum_kernel(const float* dZ, int B, int O, float* db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= O) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * O + j];
  db[j] = s;
}
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// ------------------------------------------------------------------ model
struct tn_mlp {
  tn_ctx* ctx = nullptr;
  int in = 0, hid = 0, out = 0;
  int64_t np = 0;
  float* p = nullptr;  // W1 b1 W2 b2 W3 b3
  float* g = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  int64_t t = 0;
  int64_t off[6];
};

static void mlp_offsets(tn_mlp* M) {
  const int64_t sz[6] = {(int64_t)M->hid * M->in, M->hid, (int64_t)M->hid * M->hid, M->hid, (int64_t)M->out * M->hid,
                         M->out};
  int64_t o = 0;
  for (int i = 0; i < 6; ++i) { M->off[i] = o; o += sz[i]; }
  M->np = o;
}

// deterministic seeded initialisation (splitmix64 -> uniform), Xavier ranges
static uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

extern "C" void tn_mlp_destroy(tn_mlp* M);

extern "C" tn_status tn_mlp_create(tn_ctx* c, int32_t in_dim, int32_t hidden, int32_t out_dim, uint64_t seed,
                                   tn_mlp** out) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  tn_mlp* M = nullptr;
  TN_GUARD_BEGIN
  struct Free { tn_mlp*& h; ~Free() { if (h) tn_mlp_destroy(h); } } free_on_error{M};
  if (!out) TN_THROW(TN_EINVAL, "null output");
  *out = nullptr;
  if (in_dim < 1 || hidden < 1 || out_dim < 1 || in_dim > 4096 || hidden > 4096 || out_dim > 4096)
    TN_THROW(TN_EINVAL, "layer sizes out of range");
  M = new tn_mlp();
  M->ctx = c;
  ctx_retain(c);
  M->in = in_dim; M->hid = hidden; M->out = out_dim;
  mlp_offsets(M);
  M->p = (float*)dev_alloc(c, M->np * sizeof(float));
  M->g = (float*)dev_alloc(c, M->np * sizeof(float));
  M->m = (float*)dev_alloc(c, M->np * sizeof(float));
  M->v = (float*)dev_alloc(c, M->np * sizeof(float));
  std::vector<float> h(M->np, 0.f);
  uint64_t s = seed;
  auto fill = [&](int64_t o, int64_t n, double lim) {
    for (int64_t i = 0; i < n; ++i) h[o + i] = (float)((((splitmix(s) >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0) * lim);
  };
  fill(M->off[0], (int64_t)hidden * in_dim, std::sqrt(6.0 / (in_dim + hidden)));
  fill(M->off[2], (int64_t)hidden * hidden, std::sqrt(6.0 / (2.0 * hidden)));
  fill(M->off[4], (int64_t)out_dim * hidden, std::sqrt(6.0 / (hidden + out_dim)));
  HIPCHK(hipMemcpy(M->p, h.data(), M->np * sizeof(float), hipMemcpyHostToDevice));
  std::vector<float> z(M->np, 0.f);
  HIPCHK(hipMemcpy(M->m, z.data(), M->np * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(M->v, z.data(), M->np * sizeof(float), hipMemcpyHostToDevice));
  *out = M;
  M = nullptr;
  TN_GUARD_END(c)
}

extern "C" void tn_mlp_destroy(tn_mlp* M) {
  if (!M) return;
  tn_ctx* c = M->ctx;
  if (c) {
    if (!c->closed) (void)hipStreamSynchronize(c->stream);
    dev_free(c, M->p); dev_free(c, M->g); dev_free(c, M->m); dev_free(c, M->v);
  }
  delete M;
  if (c) ctx_release(c);
}

extern "C" int64_t tn_mlp_num_params(const tn_mlp* M) { return M ? M->np : -1; }

extern "C" tn_status tn_mlp_params(tn_ctx* c, tn_mlp* M, float* get, const float* set) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!M) TN_THROW(TN_EINVAL, "null model");
  if (set) {
    for (int64_t i = 0; i < M->np; ++i)
      if (!std::isfinite(set[i])) TN_THROW(TN_EINVAL, "non-finite parameter");
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(M->p, set, M->np * sizeof(float), hipMemcpyHostToDevice));
    std::vector<float> z(M->np, 0.f);
    HIPCHK(hipMemcpy(M->m, z.data(), M->np * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(M->v, z.data(), M->np * sizeof(float), hipMemcpyHostToDevice));
    M->t = 0;
  }
  if (get) download(c, get, M->p, M->np * sizeof(float));
  TN_GUARD_END(c)
}

// forward into workspace activations; returns pointers to H1, H2, Y
static void mlp_forward(tn_ctx* c, tn_mlp* M, const float* X, int B, float** H1, float** H2, float** Y) {
  hipStream_t st = c->stream;
  *H1 = wsT<float>(c, "mlp:H1", (size_t)B * M->hid);
  *H2 = wsT<float>(c, "mlp:H2", (size_t)B * M->hid);
  *Y = wsT<float>(c, "mlp:Y", (size_t)B * M->out);
  const float* W1 = M->p + M->off[0]; const float* b1 = M->p + M->off[1];
  const float* W2 = M->p + M->off[2]; const float* b2 = M->p + M->off[3];
  const float* W3 = M->p + M->off[4]; const float* b3 = M->p + M->off[5];
  sgemm(st, false, true, B, M->hid, M->in, X, M->in, W1, M->in, *H1, M->hid, b1, 1);
  sgemm(st, false, true, B, M->hid, M->hid, *H1, M->hid, W2, M->hid, *H2, M->hid, b2, 1);
  sgemm(st, false, true, B, M->out, M->hid, *H2, M->hid, W3, M->hid, *Y, M->out, b3, 0);
}

extern "C" tn_status tn_mlp_forward(tn_ctx* c, tn_mlp* M, const float* X, int32_t B, float* Yout) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!M || !X || !Yout || B < 1) TN_THROW(TN_EINVAL, "bad arguments");
  float *H1, *H2, *Y;
  mlp_forward(c, M, X, B, &H1, &H2, &Y);
  HIPCHK(hipMemcpyAsync(Yout, Y, (size_t)B * M->out * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  TN_GUARD_END(c)
}

// gradients of the mean-squared error into M->g; loss to host
static float mlp_backward(tn_ctx* c, tn_mlp* M, const float* X, const float* T, int B) {
  hipStream_t st = c->stream;
  float *H1, *H2, *Y;
  mlp_forward(c, M, X, B, &H1, &H2, &Y);
  const int n = B * M->out;
  float* dY = wsT<float>(c, "mlp:dY", (size_t)n);
  const int nb = std::max(1, std::min(64, (n + 255) / 256));
  double* part = wsT<double>(c, "mlp:part", nb);
  float* lossd = wsT<float>(c, "mlp:loss", 1);
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, st, Y, T, n, 1.f / (float)n, dY, part);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, st, part, nb, 1.0 / n, lossd);
  float* g = M->g;
  const float* W2 = M->p + M->off[2];
  const float* W3 = M->p + M->off[4];
  float* dH2 = wsT<float>(c, "mlp:dH2", (size_t)B * M->hid);
  float* dH1 = wsT<float>(c, "mlp:dH1", (size_t)B * M->hid);
  // layer 3
  sgemm(st, true, false, M->out, M->hid, B, dY, M->out, H2, M->hid, g + M->off[4], M->hid, nullptr, 0);
  hipLaunchKernelGGL(colsum_kernel, dim3((M->out + 255) / 256), dim3(256), 0, st, dY, B, M->out, g + M->off[5]);
  sgemm(st, false, false, B, M->hid, M->out, dY, M->out, W3, M->hid, dH2, M->hid, nullptr, 0);
  hipLaunchKernelGGL(dtanh_kernel, dim3(std::max(1, std::min(1024, (B * M->hid + 255) / 256))), dim3(256), 0, st, dH2, H2, B * M->hid);
  // layer 2
  sgemm(st, true, false, M->hid, M->hid, B, dH2, M->hid, H1, M->hid, g + M->off[2], M->hid, nullptr, 0);
  hipLaunchKernelGGL(colsum_kernel, dim3((M->hid + 255) / 256), dim3(256), 0, st, dH2, B, M->hid, g + M->off[3]);
  sgemm(st, false, false, B, M->hid, M->hid, dH2, M->hid, W2, M->hid, dH1, M->hid, nullptr, 0);
  hipLaunchKernelGGL(dtanh_kernel, dim3(std::max(1, std::min(1024, (B * M->hid + 255) / 256))), dim3(256), 0, st, dH1, H1, B * M->hid);
  // layer 1
  sgemm(st, true, false, M->hid, M->in, B, dH1, M->hid, X, M->in, g + M->off[0], M->in, nullptr, 0);
  hipLaunchKernelGGL(colsum_kernel, dim3((M->hid + 255) / 256), dim3(256), 0, st, dH1, B, M->hid, g + M->off[1]);
  HIPCHK(hipGetLastError());
  float loss = 0.f;
  download(c, &loss, lossd, sizeof(float));
  return loss;
}

extern "C" tn_status tn_mlp_grad(tn_ctx* c, tn_mlp* M, const float* X, const float* T, int32_t B, float* grads,
                                 float* loss) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!M || !X || !T || B < 1) TN_THROW(TN_EINVAL, "bad arguments");
  const float L = mlp_backward(c, M, X, T, B);
  if (loss) *loss = L;
  if (grads) download(c, grads, M->g, M->np * sizeof(float));
  TN_GUARD_END(c)
}

extern "C" tn_status tn_mlp_train_step(tn_ctx* c, tn_mlp* M, const float* X, const float* T, int32_t B, float lr,
                                       float* loss) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!M || !X || !T || B < 1 || !(lr > 0.f)) TN_THROW(TN_EINVAL, "bad arguments");
  const float L = mlp_backward(c, M, X, T, B);
  if (!std::isfinite(L)) TN_THROW(TN_ENUMERIC, "non-finite loss");
  M->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)M->t), c2 = 1.f - std::pow(b2, (float)M->t);
  hipLaunchKernelGGL(adam_kernel, dim3(std::max<int64_t>(1, std::min<int64_t>(2048, (M->np + 255) / 256))), dim3(256), 0,
                     c->stream, M->p, M->g, M->m, M->v, M->np, lr, b1, b2, 1e-8f, c1, c2);
  HIPCHK(hipGetLastError());
  if (loss) *loss = L;
  TN_GUARD_END(c)
}

// ------------------------------------------------------------------ parameterised local basis
// W (D x d, host, complex interleaved): first d columns of <n|S(zeta)|k>,
// S(zeta) = exp(1/2 (zeta* a^2 - zeta a^dag^2)), built on a (D + margin) box
// from the squeezed vacuum and S|k> = (a^dag cosh r + e^{-i phi} sinh r a) S|k-1> / sqrt(k),
// cut to D rows and orthonormalised column by column.
// Columns k < d of <n|S(zeta)|k> on a box of Db rows; row i of column k is
// exact for i < Db - k (each ladder step reads one row further down).
static std::vector<std::vector<cd>> squeezed_columns(cd zeta, int Db, int d) {
  const double r = std::abs(zeta);
  const cd e = r > 0 ? zeta / r : cd(1.0, 0.0);
  const double t = std::tanh(r), ch = std::cosh(r), sh = std::sinh(r);
  std::vector<cd> v(Db, 0.0);
  // squeezed vacuum via the ratio recursion c_{2q+2} / c_{2q} = -e t sqrt((2q+1)/(2q+2))
  v[0] = 1.0 / std::sqrt(ch);
  for (int k = 2; k < Db; k += 2) v[k] = v[k - 2] * (-e * t) * std::sqrt((double)(k - 1) / (double)k);
  std::vector<std::vector<cd>> cols{v};
  for (int k = 1; k < d; ++k) {
    const auto& p = cols.back();
    std::vector<cd> nx(Db, 0.0);
    for (int i = 0; i < Db; ++i) {
      cd acc = 0.0;
      if (i >= 1) acc += ch * std::sqrt((double)i) * p[i - 1];
      if (i + 1 < Db) acc += std::conj(e) * sh * std::sqrt((double)(i + 1)) * p[i + 1];
      nx[i] = acc / std::sqrt((double)k);
    }
    cols.push_back(nx);
  }
  return cols;
}

extern "C" tn_status tn_squeezed_basis(double zeta_re, double zeta_im, int32_t D, int32_t d, int32_t margin,
                                       double* out) {
  if (!out || D < 1 || d < 1 || d > D || margin < 0 || D + margin > 4096) return TN_EINVAL;
  if (!std::isfinite(zeta_re) || !std::isfinite(zeta_im)) return TN_EINVAL;
  if (std::hypot(zeta_re, zeta_im) > 20.0) return TN_EINVAL;
  const std::vector<std::vector<cd>> cols = squeezed_columns(cd(zeta_re, zeta_im), D + margin, d);
  std::vector<cd> Wm((size_t)D * d);
  for (int j = 0; j < d; ++j)
    for (int i = 0; i < D; ++i) Wm[(size_t)i * d + j] = cols[j][i];
  for (int j = 0; j < d; ++j) {
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q < j; ++q) {
        cd h = 0.0;
        for (int i = 0; i < D; ++i) h += std::conj(Wm[(size_t)i * d + q]) * Wm[(size_t)i * d + j];
        for (int i = 0; i < D; ++i) Wm[(size_t)i * d + j] -= h * Wm[(size_t)i * d + q];
      }
    double nr = 0.0;
    for (int i = 0; i < D; ++i) nr += std::norm(Wm[(size_t)i * d + j]);
    nr = std::sqrt(nr);
    if (!(nr > 1e-300)) return TN_ENUMERIC;
    for (int i = 0; i < D; ++i) Wm[(size_t)i * d + j] /= nr;
  }
  for (size_t i = 0; i < Wm.size(); ++i) { out[2 * i] = Wm[i].real(); out[2 * i + 1] = Wm[i].imag(); }
  return TN_OK;
}

// ------------------------------------------------------------------ single-site reduced density matrices
// rho_j[n][n'] = <n|rho_j|n'> in the raw Fock basis for sites j < n_modes; the MPS
// must be right-canonical with its centre at site 0.  out: host [n_modes][D][D] complex.
// C[n][n'] = sum_{a,b} Y[a][n][b] conj(F[a][n'][b]) = psi_n conj(psi_n') summed over the rest
__global__ void rho_scale_kernel(const cf64* C, int D, double s, cf64* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < D * D) out[e] = make_double2(C[e].x * s, C[e].y * s);
}
extern "C" tn_status tn_rdm(tn_ctx* c, const tn_mps* m, const tn_mpo* mpo, int32_t n_modes, double* out) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (mpo) plbo_sync_iso(mpo);
  if (!m || !mpo || !out) TN_THROW(TN_EINVAL, "null argument");
  if (m->N != mpo->N || m->d != mpo->d) TN_THROW(TN_EINVAL, "MPO and MPS do not match");
  if (m->center != 0) TN_THROW(TN_ESTATE, "the MPS must be right-canonical with its centre at site 0");
  if (n_modes < 1 || n_modes > m->N) TN_THROW(TN_EINVAL, "bad n_modes");
  const int D = mpo->D_raw, d = mpo->d;
  hipStream_t st = c->stream;
  size_t mx = 1, my = 1;
  for (int t = 0; t <= m->N; ++t) mx = std::max(mx, (size_t)m->dims[t] * m->dims[t]);
  for (int s = 0; s < n_modes; ++s) my = std::max(my, (size_t)m->dims[s] * D * m->dims[s + 1]);
  cf64* Ea = wsT<cf64>(c, "rdm:Ea", mx);
  cf64* Eb = wsT<cf64>(c, "rdm:Eb", mx);
  cf64* Y = wsT<cf64>(c, "rdm:Y", my);
  cf64* F = wsT<cf64>(c, "rdm:F", my);
  cf64* Cm = wsT<cf64>(c, "rdm:C", (size_t)D * D);
  cf64* R = wsT<cf64>(c, "rdm:R", (size_t)D * D);
  const int np_ = 64;
  cf64* parts = wsT<cf64>(c, "rdm:P", (size_t)np_ * D * D);
  HIPCHK(launch_set_one(Ea, PREC_FP64, st));
  double nrm = 1.0;
  std::vector<cf64> host((size_t)D * D);
  auto batch = [&](int ta, int tb, const std::vector<GemmJob>& jobs, const std::vector<GemmSeg>& segs, int mm, int nn) {
    const size_t bj = ((jobs.size() * sizeof(GemmJob)) + 255) & ~size_t(255);
    char* dsc = (char*)ws_get(c, "rdm:d", bj + segs.size() * sizeof(GemmSeg));
    HIPCHK(hipMemcpyAsync(dsc, jobs.data(), jobs.size() * sizeof(GemmJob), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dsc + bj, segs.data(), segs.size() * sizeof(GemmSeg), hipMemcpyHostToDevice, st));
    HIPCHK(launch_cgemm(PREC_FP64, ta, tb, (GemmJob*)dsc, (int)jobs.size(), (GemmSeg*)(dsc + bj), mm, nn, 0, st));
    HIPCHK(hipStreamSynchronize(st));
  };
  for (int s = 0; s < n_modes; ++s) {
    const int cl = m->dims[s], cr = m->dims[s + 1];
    {  // F = W_s A_s
      std::vector<GemmJob> jobs;
      std::vector<GemmSeg> segs;
      for (int a = 0; a < cl; ++a) {
        segs.push_back({mpo->fock_iso() + (size_t)s * D * d, m->A[s] + (size_t)a * d * cr, d, cr, d, 0});
        jobs.push_back({F + (size_t)a * D * cr, cr, D, cr, a, 1});
      }
      batch(0, 0, jobs, segs, D, cr);
    }
    batch(0, 0, {{Y, (int64_t)D * cr, cl, D * cr, 0, 1}}, {{Ea, F, cl, (int64_t)D * cr, cl, 0}}, cl, D * cr);
    {  // C[n'][n] = sum_a sum_b Y[a][n'][b] conj(F[a][n][b]), split over a
      const int np = std::max(1, std::min(cl, np_));
      std::vector<GemmJob> jobs;
      std::vector<GemmSeg> segs;
      for (int a = 0; a < cl; ++a) segs.push_back({Y + (size_t)a * D * cr, F + (size_t)a * D * cr, cr, cr, cr, 0});
      for (int g = 0; g < np; ++g) {
        const int a0 = (int)((int64_t)cl * g / np), a1 = (int)((int64_t)cl * (g + 1) / np);
        jobs.push_back({parts + (size_t)g * D * D, D, D, D, a0, a1 - a0});
      }
      batch(0, 1, jobs, segs, D, D);
      HIPCHK(launch_reduce_partials(Cm, PREC_FP64, parts, np, (int64_t)D * D, st));
    }
    if (s == 0) {
      std::vector<cf64> tmp((size_t)D * D);
      download(c, tmp.data(), Cm, tmp.size() * sizeof(cf64));
      nrm = 0.0;
      for (int n = 0; n < D; ++n) nrm += tmp[(size_t)n * D + n].x;
      if (!(nrm > 0.0)) TN_THROW(TN_ENUMERIC, "zero norm");
    }
    hipLaunchKernelGGL(rho_scale_kernel, dim3((D * D + 255) / 256), dim3(256), 0, st, Cm, D, 1.0 / nrm, R);
    HIPCHK(hipGetLastError());
    download(c, host.data(), R, host.size() * sizeof(cf64));
    for (size_t i = 0; i < host.size(); ++i) {
      out[2 * ((size_t)s * D * D + i)] = host[i].x;
      out[2 * ((size_t)s * D * D + i) + 1] = host[i].y;
    }
    // E <- sum_n F[n]^dag E F[n] = (F as (cl D) x cr)^dag (Y as (cl D) x cr)
    batch(1, 0, {{Eb, cr, cr, cr, 0, 1}}, {{F, Y, cr, cr, cl * D, 0}}, cr, cr);
    std::swap(Ea, Eb);
  }
  TN_GUARD_END(c)
}

// ------------------------------------------------------------------ warm-start host helpers
// Network input of output mode j: [j/N, N/64] then, for the 16 largest |U_jk|
// (ties by k), (r_k, |U_jk|, cos 2 arg U_jk, sin 2 arg U_jk), zero-padded.  The
// reduced state of mode j of a squeezed Gaussian state depends on U_jk only
// through |U_jk| and U_jk^2 (a squeezed vacuum is even under a_k -> -a_k).
static constexpr int WS_KTOP = 16;
static constexpr int WS_IN = 2 + 4 * WS_KTOP;

extern "C" tn_status tn_ws_features(int32_t N, const double* r, const double* U, float* out) {
  if (N < 1 || N > 4096 || !r || !U || !out) return TN_EINVAL;
  std::vector<int> idx(N);
  for (int j = 0; j < N; ++j) {
    const double* row = U + (size_t)2 * N * j;
    for (int k = 0; k < N; ++k) idx[k] = k;
    auto mag = [&](int k) { return std::hypot(row[2 * k], row[2 * k + 1]); };
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return mag(a) > mag(b); });
    float* f = out + (size_t)WS_IN * j;
    for (int q = 0; q < WS_IN; ++q) f[q] = 0.f;
    f[0] = (float)((double)j / N);
    f[1] = (float)(N / 64.0);
    for (int q = 0; q < std::min(N, WS_KTOP); ++q) {
      const int k = idx[q];
      const double a = mag(k);
      if (!std::isfinite(a) || !std::isfinite(r[k])) return TN_EINVAL;
      f[2 + 4 * q] = (float)r[k];
      f[3 + 4 * q] = (float)a;
      // cos 2t = (re^2 - im^2) / a^2, sin 2t = 2 re im / a^2
      const double re = row[2 * k], im = row[2 * k + 1];
      f[4 + 4 * q] = (float)(a > 0 ? (re * re - im * im) / (a * a) : 1.0);
      f[5 + 4 * q] = (float)(a > 0 ? 2.0 * re * im / (a * a) : 0.0);
    }
  }
  return TN_OK;
}

// Targets from a single-mode state rho[n][n'] = <n|rho|n'>: with n = <a^dag a>
// and m = <a^2>, a squeezed thermal state S(zeta) tau S(zeta)^dag has
// (2 nbar + 1)^2 = (2n + 1)^2 - 4|m|^2, tanh(2|zeta|) = 2|m| / (2n + 1) and
// zeta / |zeta| = -m / |m|.  out[j] = (Re zeta, Im zeta, log(1 + nbar)).
static void moments_to_params(double n, cd m, float* out) {
  const double s = 2 * n + 1, am = std::abs(m);
  const double nu2 = std::max(s * s - 4 * am * am, 1.0);
  const double nbar = 0.5 * (std::sqrt(nu2) - 1.0);
  const double rr = am > 0 ? 0.5 * std::atanh(std::min(2 * am / s, 1 - 1e-15)) : 0.0;
  const cd ph = am > 0 ? -m / am : cd(1.0, 0.0);
  out[0] = (float)(rr * ph.real());
  out[1] = (float)(rr * ph.imag());
  out[2] = (float)std::log1p(std::max(nbar, 0.0));
}

extern "C" tn_status tn_ws_targets(int32_t n_modes, int32_t D, const double* rho, float* out) {
  if (n_modes < 1 || D < 1 || !rho || !out) return TN_EINVAL;
  for (int j = 0; j < n_modes; ++j) {
    const double* R = rho + (size_t)2 * D * D * j;
    double n = 0.0;
    cd m = 0.0;
    for (int k = 0; k < D; ++k) n += k * R[2 * ((size_t)k * D + k)];
    for (int k = 2; k < D; ++k) {
      const size_t e = (size_t)k * D + (k - 2);
      m += cd(R[2 * e], R[2 * e + 1]) * std::sqrt((double)k * (k - 1));
    }
    if (!std::isfinite(n) || !std::isfinite(std::abs(m))) return TN_ENUMERIC;
    moments_to_params(n, m, out + 3 * j);
  }
  return TN_OK;
}

// Analytic parameters of each output mode's reduced Gaussian state: the 2 x 2
// block of V = 1/2 O D^2 O^T (Sec. II.C.1) for mode j,
//   Vxx = 1/2 sum_k (Re U_jk^2 e^{-2 r_k} + Im U_jk^2 e^{2 r_k}),
//   Vpp = 1/2 sum_k (Im U_jk^2 e^{-2 r_k} + Re U_jk^2 e^{2 r_k}),
//   Vxp = 1/2 sum_k Re U_jk Im U_jk (e^{-2 r_k} - e^{2 r_k}),
// gives <a^dag a> = (Vxx + Vpp)/2 - 1/2 and <a^2> = (Vxx - Vpp)/2 + i Vxp; the
// reduced state is exactly the squeezed thermal state with these moments, so
// its squeezed basis is the optimal local basis (eq. OLB).
static bool reduced_covariance(int N, const double* r, const double* U, int j, double& vxx, double& vpp,
                               double& vxp) {
  vxx = vpp = vxp = 0.0;
  for (int k = 0; k < N; ++k) {
    const double re = U[2 * ((size_t)j * N + k)], im = U[2 * ((size_t)j * N + k) + 1];
    if (!std::isfinite(re) || !std::isfinite(im) || !std::isfinite(r[k])) return false;
    const double em = std::exp(-2.0 * r[k]), ep = std::exp(2.0 * r[k]);
    vxx += 0.5 * (re * re * em + im * im * ep);
    vpp += 0.5 * (im * im * em + re * re * ep);
    vxp += 0.5 * re * im * (em - ep);
  }
  return std::isfinite(vxx) && std::isfinite(vpp) && std::isfinite(vxp);
}

extern "C" tn_status tn_ws_gaussian_params(int32_t N, const double* r, const double* U, float* out) {
  if (N < 1 || N > 4096 || !r || !U || !out) return TN_EINVAL;
  for (int j = 0; j < N; ++j) {
    double vxx, vpp, vxp;
    if (!reduced_covariance(N, r, U, j, vxx, vpp, vxp)) return TN_EINVAL;
    moments_to_params(0.5 * (vxx + vpp) - 0.5, cd(0.5 * (vxx - vpp), vxp), out + 3 * j);
  }
  return TN_OK;
}

// Cutoff errors of the Gaussian optimal basis with d kept states per mode.
// nbar_j = sqrt(det V_j) - 1/2 (eq. WilliamsonDecomposition); the thermal
// spectrum nbar^k / (nbar + 1)^(k+1) (eq. diagReducedGaussianDM) discards
// (nbar / (nbar + 1))^d beyond the first d states; eps is the mean of those and
// eps <= eps_D <= N eps (eq. SpecWfromSDsums).  The effective cutoff (eq.
// Effectivecutoff) scans D upward, adding row D - 1 of the first d squeezed
// basis vectors to their Gram matrix, until max |G - 1| <= tol.
extern "C" tn_status tn_cutoff_report(int32_t N, const double* r, const double* U, int32_t d, int32_t D_max, double tol,
                                      double* eps_mode, int32_t* D_eff, double* bounds) {
  if (N < 1 || N > 4096 || d < 1 || D_max < d || D_max > 4096 || !(tol > 0) || !r || !U || !eps_mode || !D_eff ||
      !bounds)
    return TN_EINVAL;
  double sum = 0.0;
  for (int j = 0; j < N; ++j) {
    double vxx, vpp, vxp;
    if (!reduced_covariance(N, r, U, j, vxx, vpp, vxp)) return TN_EINVAL;
    const double nbar = std::max(std::sqrt(std::max(vxx * vpp - vxp * vxp, 0.0)) - 0.5, 0.0);
    eps_mode[j] = std::pow(nbar / (nbar + 1.0), d);
    sum += eps_mode[j];
    // |zeta_j| of the squeezed basis; its phase does not change |V^dag V - 1|
    const double s2 = vxx + vpp, am = 0.5 * std::hypot(vxx - vpp, 2.0 * vxp);
    const double rj = am > 0 ? 0.5 * std::atanh(std::min(2.0 * am / s2, 1.0 - 1e-15)) : 0.0;
    if (rj > 20.0) return TN_EINVAL;
    const auto cols = squeezed_columns(cd(rj, 0.0), D_max + d, d);
    std::vector<cd> G((size_t)d * d, 0.0);
    D_eff[j] = -1;
    for (int D = 1; D <= D_max; ++D) {
      const int i = D - 1;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) G[(size_t)a * d + b] += std::conj(cols[a][i]) * cols[b][i];
      if (D < d) continue;
      double dev = 0.0;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) dev = std::max(dev, std::abs(G[(size_t)a * d + b] - (a == b ? 1.0 : 0.0)));
      if (dev <= tol) {
        D_eff[j] = D;
        break;
      }
    }
  }
  bounds[0] = sum / N;
  bounds[1] = sum;
  return TN_OK;
}

// Warm-start state from network outputs y[j] = (Re zeta, Im zeta, log(1 + nbar)):
// iso[j] = squeezed basis of zeta_j (D x d), and a product MPS whose site j
// holds the thermal amplitudes sqrt(lambda_m), lambda_m ~ nbar^m / (nbar + 1)^(m + 1)
// (normalised over m < d), in bond channel (0, 0), plus complex Gaussian noise of
// scale `noise` on every entry (splitmix64 + Box-Muller, seeded).  Bond
// dimensions min(chi, d^s, d^(N-s)) go to dims (N + 1); tensors (chi_s, d,
// chi_s+1) are written back to back, complex interleaved; when tensors is NULL
// only *need (doubles) is set.
extern "C" tn_status tn_ws_initial_state(int32_t N, int32_t D, int32_t d, int32_t chi, const float* y, uint64_t seed,
                                         double noise, double* iso, int32_t* dims, double* tensors, size_t cap,
                                         size_t* need) {
  if (N < 1 || D < 1 || d < 1 || d > D || chi < 1 || !y || !dims || !need || !(noise >= 0)) return TN_EINVAL;
  for (int s = 0; s <= N; ++s) {
    double l = std::pow((double)d, std::min(s, 40)), rr = std::pow((double)d, std::min(N - s, 40));
    dims[s] = (int32_t)std::min({(double)chi, l, rr});
  }
  size_t tot = 0;
  for (int s = 0; s < N; ++s) tot += (size_t)dims[s] * d * dims[s + 1] * 2;
  *need = tot;
  if (!tensors) return TN_OK;
  if (cap < tot || !iso) return TN_EINVAL;
  uint64_t st = seed;
  auto normal = [&]() {
    const double u1 = ((splitmix(st) >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
  };
  size_t off = 0;
  for (int s = 0; s < N; ++s) {
    const double zr = y[3 * s], zi = y[3 * s + 1], ln = y[3 * s + 2];
    if (!std::isfinite(zr) || !std::isfinite(zi) || !std::isfinite(ln)) return TN_ENUMERIC;
    const tn_status b = tn_squeezed_basis(zr, zi, D, d, 64, iso + (size_t)2 * D * d * s);
    if (b != TN_OK) return b;
    const double nbar = std::max(std::expm1((double)ln), 0.0);
    std::vector<double> lam(d);
    double tl = 0.0;
    for (int m = 0; m < d; ++m) {
      lam[m] = std::pow(nbar / (nbar + 1.0), m) / (nbar + 1.0);
      tl += lam[m];
    }
    const int cl = dims[s], cr = dims[s + 1];
    for (int a = 0; a < cl; ++a)
      for (int m = 0; m < d; ++m)
        for (int q = 0; q < cr; ++q) {
          double re = noise * normal(), im = noise * normal();
          if (a == 0 && q == 0) re += std::sqrt(lam[m] / tl);
          const size_t e = off + 2 * (((size_t)a * d + m) * cr + q);
          tensors[e] = re;
          tensors[e + 1] = im;
        }
    off += (size_t)cl * d * cr * 2;
  }
  return TN_OK;
}
