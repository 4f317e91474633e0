// C ABI: contexts, device memory, problem -> MPO (host FP64 set-up), MPS handles.
#include <cmath>
#include <cstring>
#include <algorithm>
#include "internal.h"

static const char* kVersion = "tn-gfx950 0.1";

// ------------------------------------------------------------------ memory
void* dev_alloc(tn_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (c->has_alloc) {
    p = c->alloc.alloc(bytes, c->alloc.user);
    if (!p) TN_THROW(TN_ENOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      TN_THROW(TN_ENOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
    }
  }
  return p;
}
void dev_free(tn_ctx* c, void* p) {
  if (!p) return;
  if (c->has_alloc) c->alloc.free(p, c->alloc.user);
  else (void)hipFree(p);
}
void* ws_get(tn_ctx* c, const std::string& name, size_t bytes) {
  auto it = c->ws.find(name);
  if (it != c->ws.end() && it->second.second >= bytes) return it->second.first;
  if (it != c->ws.end()) {
    HIPCHK(hipStreamSynchronize(c->stream));
    dev_free(c, it->second.first);
    c->ws.erase(it);
  }
  size_t cap = std::max<size_t>(bytes + bytes / 8, 4096);
  void* p = dev_alloc(c, cap);
  c->ws[name] = {p, cap};
  return p;
}
void upload(tn_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
}
void download(tn_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
}
size_t elem_bytes(int prec) { return prec == PREC_FP64 ? sizeof(cf64) : sizeof(cf32); }

// ------------------------------------------------------------------ ABI helpers
#define TN_GUARD_BEGIN try {
#define TN_GUARD_END(ctx)                                         \
  }                                                               \
  catch (const TnError& e) {                                      \
    if (ctx) (ctx)->err = e.what();                               \
    return e.code;                                                \
  }                                                               \
  catch (const std::bad_alloc&) {                                 \
    if (ctx) (ctx)->err = "host allocation failed";               \
    return TN_ENOMEM;                                             \
  }                                                               \
  catch (const std::exception& e) {                               \
    if (ctx) (ctx)->err = e.what();                               \
    return TN_EINVAL;                                             \
  }                                                               \
  if (ctx) (ctx)->err.clear();                                    \
  return TN_OK;

extern "C" const char* tn_version(void) { return kVersion; }

extern "C" tn_status tn_ctx_create(int device, void* hip_stream, const tn_allocator* alloc, tn_ctx** out) {
  if (!out) return TN_EINVAL;
  *out = nullptr;
  if (alloc && (!alloc->alloc || !alloc->free)) return TN_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return TN_EINVAL;
  }
  if (hipSetDevice(device) != hipSuccess) return TN_EHIP;
  if (sample_scratch_setup(device) != TN_OK) return TN_EHIP;
  tn_ctx* c = new tn_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (alloc) { c->alloc = *alloc; c->has_alloc = true; }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->pinned), 4096 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return TN_ENOMEM;
  }
  bool ok = true;
  for (int i = 0; i < 8; ++i) ok = ok && (hipEventCreate(&c->ev[i]) == hipSuccess);
  for (auto& ps : c->pslot)
    for (int i = 0; i < 6; ++i) ok = ok && (hipEventCreate(&ps.e[i]) == hipSuccess);
  c->ev_ok = ok;
  *out = c;
  return TN_OK;
}

static void ctx_free(tn_ctx* c) {
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->ev_ok) {
    for (int i = 0; i < 8; ++i) (void)hipEventDestroy(c->ev[i]);
    for (auto& ps : c->pslot)
      for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ps.e[i]);
    for (auto e : c->tri_ev) (void)hipEventDestroy(e);
  }
  delete c;
}
void ctx_retain(tn_ctx* c) { ++c->refs; }
void ctx_release(tn_ctx* c) {
  if (--c->refs == 0) ctx_free(c);
}

// Closes the context: its stream is drained and its workspaces freed now; the
// host object lives on until the last MPO, MPS or network made on it is
// destroyed, so those handles may be destroyed in any order.
extern "C" void tn_ctx_destroy(tn_ctx* c) {
  if (!c || c->closed) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& kv : c->ws) dev_free(c, kv.second.first);
  c->ws.clear();
  c->closed = true;
  ctx_release(c);
}

extern "C" const char* tn_last_error(const tn_ctx* c) { return c ? c->err.c_str() : "null context"; }

void prof_harvest(tn_ctx* c, tn_ctx::ProfSlot& ps) {
  HIPCHK(hipEventSynchronize(ps.e[5]));
  for (int i = 0; i < 5; ++i) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ps.e[i], ps.e[i + 1]));
    c->prof_ms[i] += ms;
  }
  for (int i = 0; i < 3; ++i) c->prof_flops[i] += ps.fl[i];
  c->prof_bytes[0] += ps.by[0];
  c->prof_bytes[1] += ps.by[1];
  c->prof_n += 1;
  ps.pending = false;
}

extern "C" tn_status tn_profile(tn_ctx* c, int32_t mode, double* out) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  // collect the slots still outstanding, oldest first
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int64_t k = std::max<int64_t>(0, c->pseq - tn_ctx::PROF_RING); k < c->pseq; ++k) {
    auto& ps = c->pslot[k % tn_ctx::PROF_RING];
    if (ps.pending) prof_harvest(c, ps);
  }
  if (out) {
    for (int i = 0; i < 5; ++i) out[i] = c->prof_ms[i];
    out[5] = (double)c->prof_n;
    for (int i = 0; i < 3; ++i) out[6 + i] = c->prof_flops[i];
    out[9] = c->prof_bytes[0];
    out[10] = c->prof_bytes[1];
    out[11] = c->prof_tri_ms;
    out[12] = (double)c->prof_tri_n;
    out[13] = c->prof_tri_bytes;
    out[14] = (double)c->lz_iters;
    out[15] = (double)c->lz_full;
  }
  if (mode >= 0) {
    c->prof = mode > 0;
    for (int i = 0; i < 5; ++i) c->prof_ms[i] = 0.0;
    for (int i = 0; i < 3; ++i) c->prof_flops[i] = 0.0;
    c->prof_bytes[0] = c->prof_bytes[1] = 0.0;
    c->prof_n = 0;
    c->prof_tri_ms = c->prof_tri_bytes = 0.0;
    c->prof_tri_n = 0;
    c->lz_iters = c->lz_full = 0;
  }
  TN_GUARD_END(c)
  return TN_OK;
}

// ------------------------------------------------------------------ problem set-up (host FP64)
// Bond channel layout of the middle-site MPO (SM Sec. 8), 1-based sites, m = ceil(N/2).
//   bond 0: [S]; bond N: [F]
//   left bonds t < m:  X_k at 2(t-k), P_k at 2(t-k)+1 (k = t..1), S at 2t, F at 2t+1
//   right bonds t >= m: Xw_j at 2(j-t-1), Pw_j at 2(j-t-1)+1 (j = t+1..N), F at 2(N-t), S at 2(N-t)+1
enum ChanType { CH_S, CH_F, CH_X, CH_P, CH_XW, CH_PW };
static int bond_dim(int N, int t) {
  const int m = (N + 1) / 2;
  if (t == 0 || t == N) return 1;
  if (t < m) return 2 * t + 2;
  return 2 * (N - t) + 2;
}
static int chan(int N, int t, ChanType ty, int k = 0) {
  const int m = (N + 1) / 2;
  if (t == 0) return ty == CH_S ? 0 : -1;
  if (t == N) return ty == CH_F ? 0 : -1;
  if (t < m) {
    switch (ty) {
      case CH_X: return (k >= 1 && k <= t) ? 2 * (t - k) : -1;
      case CH_P: return (k >= 1 && k <= t) ? 2 * (t - k) + 1 : -1;
      case CH_S: return 2 * t;
      case CH_F: return 2 * t + 1;
      default: return -1;
    }
  }
  switch (ty) {
    case CH_XW: return (k > t && k <= N) ? 2 * (k - t - 1) : -1;
    case CH_PW: return (k > t && k <= N) ? 2 * (k - t - 1) + 1 : -1;
    case CH_F: return 2 * (N - t);
    case CH_S: return 2 * (N - t) + 1;
    default: return -1;
  }
}

// kind codes: 1 I, 2 X, 3 P, 4 S, 5 c1 X + c2 P, 6 c1 I, 7 X^2, 8 XP + PX, 9 c1 X^2 + c2 (XP + PX)
static CoreEntry make_entry(int r, int c, int kind, double c1, double c2) {
  CoreEntry e{r, c, kind, {0, 0, 0, 0, 0, 0}};
  switch (kind) {
    case 1: e.c[0] = 1.0; break;
    case 2: e.c[1] = 1.0; break;
    case 3: e.c[2] = 1.0; break;
    case 4: e.c[3] = 1.0; break;
    case 5: e.c[1] = c1; e.c[2] = c2; break;
    case 6: e.c[0] = c1; break;
    case 7: e.c[4] = 1.0; break;
    case 8: e.c[5] = 1.0; break;
    case 9: e.c[4] = c1; e.c[5] = c2; break;
  }
  return e;
}

// bond dimension with the global-CZ blocks: the Gaussian channels, then
// [A0, AF, (AX2 i, APt i, AI i) for i <= t] and [B0, BF, (BX i) for i <= t]
static int bond_dim_cz(int N, int t) {
  if (t == 0 || t == N) return 1;
  return bond_dim(N, t) + 4 + 4 * t;
}

// The global-CZ terms kappa H_1 + kappa^2 H_2 (Sec. II.C.2, eq. nonGBSHamiltonian;
// the purple, blue and magenta MPOs of SM Sec. 8) as two left-to-right
// automata appended to the Gaussian channels of each bond:
//   H_1 = Tr(gamma) prod X + sum_i beta_ii P_i prod' X
//         + sum_{i != j} (gamma_ij X_i^2 + beta_ij/2 (XP + PX)_i) prod'' X,
//   H_2 = 1/2 sum_i beta_ii prod' X^2 + sum_{i < j} beta_ij X_i X_j prod'' X^2.
// A0 / B0: background only so far; AF / BF: term complete; AX2 i / APt i: X^2 or
// XP + PX placed at site i, identity partner to come; AI i: identity placed at
// site i, partner to come; BX i: X placed at site i, X partner to come.
static void cz_entries(int N, int s, const std::vector<double>& be, const std::vector<double>& ga, double kappa,
                       std::vector<CoreEntry>& E) {
  auto B = [&](int i, int j) { return be[(i - 1) * N + (j - 1)]; };
  auto G = [&](int i, int j) { return ga[(i - 1) * N + (j - 1)]; };
  const int tl = s - 1, tr = s;
  const bool last = s == N;
  // channel index at bond t of a block label (-1 if the bond lacks it)
  auto a_base = [&](int t) { return bond_dim(N, t); };
  auto b_base = [&](int t) { return bond_dim(N, t) + 2 + 3 * t; };
  auto A0 = [&](int t) { return (t == 0) ? 0 : (t == N ? -1 : a_base(t)); };
  auto AF = [&](int t) { return (t == N) ? 0 : (t == 0 ? -1 : a_base(t) + 1); };
  auto AX2 = [&](int t, int i) { return (t > 0 && t < N && i >= 1 && i <= t) ? a_base(t) + 2 + 3 * (i - 1) : -1; };
  auto APt = [&](int t, int i) { return (t > 0 && t < N && i >= 1 && i <= t) ? a_base(t) + 3 + 3 * (i - 1) : -1; };
  auto AI = [&](int t, int i) { return (t > 0 && t < N && i >= 1 && i <= t) ? a_base(t) + 4 + 3 * (i - 1) : -1; };
  auto B0 = [&](int t) { return (t == 0) ? 0 : (t == N ? -1 : b_base(t)); };
  auto BF = [&](int t) { return (t == N) ? 0 : (t == 0 ? -1 : b_base(t) + 1); };
  auto BX = [&](int t, int i) { return (t > 0 && t < N && i >= 1 && i <= t) ? b_base(t) + 2 + (i - 1) : -1; };
  auto put = [&](int r, int c, int kind, double c1 = 0.0, double c2 = 0.0) {
    if (r < 0 || c < 0) return;
    E.push_back(make_entry(r, c, kind, c1, c2));
  };
  const double k = kappa;
  double trg = 0.0;
  for (int i = 1; i <= N; ++i) trg += G(i, i);
  // H_1 block
  if (!last) {
    put(A0(tl), A0(tr), 2);
    put(A0(tl), AX2(tr, s), 7);
    put(A0(tl), APt(tr, s), 8);
    put(A0(tl), AI(tr, s), 1);
  }
  put(A0(tl), AF(tr), 5, s == 1 ? k * trg : 0.0, k * B(s, s));
  if (s > 1) put(AF(tl), AF(tr), 2);
  for (int i = 1; i < s; ++i) {
    if (!last) {
      put(AX2(tl, i), AX2(tr, i), 2);
      put(APt(tl, i), APt(tr, i), 2);
      put(AI(tl, i), AI(tr, i), 2);
    }
    put(AX2(tl, i), AF(tr), 6, k * G(i, s));
    put(APt(tl, i), AF(tr), 6, 0.5 * k * B(i, s));
    put(AI(tl, i), AF(tr), 9, k * G(s, i), 0.5 * k * B(s, i));
  }
  // H_2 block
  if (!last) {
    put(B0(tl), B0(tr), 7);
    put(B0(tl), BX(tr, s), 2);
  }
  put(B0(tl), BF(tr), 6, 0.5 * k * k * B(s, s));
  if (s > 1) put(BF(tl), BF(tr), 7);
  for (int i = 1; i < s; ++i) {
    if (!last) put(BX(tl, i), BX(tr, i), 7);
    put(BX(tl, i), BF(tr), 5, k * k * B(i, s), 0.0);
  }
}

// entries of core s (1-based) following the paper's L_s / M_{N_m} / R_s construction
static std::vector<CoreEntry> core_entries(int N, int s, const std::vector<double>& al, const std::vector<double>& be,
                                           const std::vector<double>& ga) {
  const int m = (N + 1) / 2;
  auto A = [&](int i, int j) { return al[(i - 1) * N + (j - 1)]; };
  auto B = [&](int i, int j) { return be[(i - 1) * N + (j - 1)]; };
  auto G = [&](int i, int j) { return ga[(i - 1) * N + (j - 1)]; };
  std::vector<CoreEntry> E;
  auto put = [&](int r, int c, int kind, double cx = 0.0, double cp = 0.0) {
    if (r < 0 || c < 0) return;
    E.push_back(make_entry(r, c, kind, cx, cp));
  };
  const int tl = s - 1, tr = s;  // row bond, column bond
  put(chan(N, tl, CH_S), chan(N, tr, CH_S), 1);
  put(chan(N, tl, CH_F), chan(N, tr, CH_F), 1);
  put(chan(N, tl, CH_S), chan(N, tr, CH_F), 4);
  if (s < m) {
    put(chan(N, tl, CH_S), chan(N, tr, CH_X, s), 2);
    put(chan(N, tl, CH_S), chan(N, tr, CH_P, s), 3);
    for (int k = 1; k < s; ++k) {
      put(chan(N, tl, CH_X, k), chan(N, tr, CH_X, k), 1);
      put(chan(N, tl, CH_P, k), chan(N, tr, CH_P, k), 1);
      put(chan(N, tl, CH_X, k), chan(N, tr, CH_F), 5, A(k, s), G(k, s));
      put(chan(N, tl, CH_P, k), chan(N, tr, CH_F), 5, G(s, k), B(k, s));
    }
  } else if (s == m) {
    for (int k = 1; k < s; ++k) {
      put(chan(N, tl, CH_X, k), chan(N, tr, CH_F), 5, A(k, s), G(k, s));
      put(chan(N, tl, CH_P, k), chan(N, tr, CH_F), 5, G(s, k), B(k, s));
    }
    for (int j = s + 1; j <= N; ++j) {
      put(chan(N, tl, CH_S), chan(N, tr, CH_XW, j), 5, A(s, j), G(j, s));
      put(chan(N, tl, CH_S), chan(N, tr, CH_PW, j), 5, G(s, j), B(s, j));
      for (int k = 1; k < s; ++k) {
        put(chan(N, tl, CH_X, k), chan(N, tr, CH_XW, j), 6, A(k, j));
        put(chan(N, tl, CH_X, k), chan(N, tr, CH_PW, j), 6, G(k, j));
        put(chan(N, tl, CH_P, k), chan(N, tr, CH_XW, j), 6, G(j, k));
        put(chan(N, tl, CH_P, k), chan(N, tr, CH_PW, j), 6, B(k, j));
      }
    }
  } else {
    put(chan(N, tl, CH_XW, s), chan(N, tr, CH_F), 2);
    put(chan(N, tl, CH_PW, s), chan(N, tr, CH_F), 3);
    for (int j = s + 1; j <= N; ++j) {
      put(chan(N, tl, CH_XW, j), chan(N, tr, CH_XW, j), 1);
      put(chan(N, tl, CH_PW, j), chan(N, tr, CH_PW, j), 1);
      put(chan(N, tl, CH_S), chan(N, tr, CH_XW, j), 5, A(s, j), G(j, s));
      put(chan(N, tl, CH_S), chan(N, tr, CH_PW, j), 5, G(s, j), B(s, j));
    }
  }
  return E;
}

// Inverse of a symmetric positive-definite matrix by Cholesky (n x n, row-major).
static std::vector<double> spd_inverse(const std::vector<double>& V, int n) {
  std::vector<double> L(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = V[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) TN_THROW(TN_EINVAL, "covariance matrix is not positive definite");
    const double d = std::sqrt(s);
    L[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = V[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / d;
    }
  }
  // inverse of L (lower), then V^{-1} = L^{-T} L^{-1}
  std::vector<double> Li(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    Li[j * n + j] = 1.0 / L[j * n + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[i * n + k] * Li[k * n + j];
      Li[i * n + j] = -s / L[i * n + i];
    }
  }
  std::vector<double> Vi(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = std::max(i, j); k < n; ++k) s += Li[k * n + i] * Li[k * n + j];
      Vi[i * n + j] = s;
    }
  return Vi;
}

static std::vector<cd> matmul(const std::vector<cd>& A, const std::vector<cd>& B, int n, int k, int m) {
  std::vector<cd> C((size_t)n * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < k; ++l) {
      const cd a = A[(size_t)i * k + l];
      if (a == 0.0) continue;
      for (int j = 0; j < m; ++j) C[(size_t)i * m + j] += a * B[(size_t)l * m + j];
    }
  return C;
}

// X, P, S, X^2, XP + PX at dimension D, products formed at D+4 (SM Sec. 5)
static void build_raw_ops(int D, double a_ss, double b_ss, double g_ss, std::vector<cd>& out) {
  const int Db = D + 4;
  std::vector<cd> X(Db * Db, 0.0), P(Db * Db, 0.0);
  const double r2 = std::sqrt(2.0);
  for (int n = 1; n < Db; ++n) {
    const double s = std::sqrt((double)n);
    // a[n-1][n] = sqrt(n); X = (a + a^dag)/sqrt2; P = -i (a - a^dag)/sqrt2
    X[(n - 1) * Db + n] += s / r2;
    X[n * Db + (n - 1)] += s / r2;
    P[(n - 1) * Db + n] += cd(0.0, -1.0) * s / r2;
    P[n * Db + (n - 1)] += cd(0.0, 1.0) * s / r2;
  }
  auto XX = matmul(X, X, Db, Db, Db), PP = matmul(P, P, Db, Db, Db);
  auto XP = matmul(X, P, Db, Db, Db), PX = matmul(P, X, Db, Db, Db);
  out.assign((size_t)NOPS * D * D, 0.0);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      const size_t b = (size_t)i * Db + j;
      out[0 * D * D + i * D + j] = X[b];
      out[1 * D * D + i * D + j] = P[b];
      cd s = 0.5 * (a_ss * XX[b] + b_ss * PP[b] + g_ss * (XP[b] + PX[b]));
      if (i == j) s -= 0.5;
      out[2 * D * D + i * D + j] = s;
      out[3 * D * D + i * D + j] = XX[b];
      out[4 * D * D + i * D + j] = XP[b] + PX[b];
    }
}

static void project_ops(const std::vector<cd>& raw, const std::vector<cd>& W, int D, int d, std::vector<cd>& out) {
  out.assign((size_t)NOPS * d * d, 0.0);
  std::vector<cd> Wh(d * D);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < d; ++j) Wh[j * D + i] = std::conj(W[i * d + j]);
  for (int o = 0; o < NOPS; ++o) {
    std::vector<cd> op(raw.begin() + o * D * D, raw.begin() + (o + 1) * D * D);
    auto t = matmul(op, W, D, D, d);
    auto r = matmul(Wh, t, d, D, d);
    std::copy(r.begin(), r.end(), out.begin() + o * d * d);
  }
}

void tn_mpo::upload_site(int s) {
  const size_t dd = (size_t)d * d, DD = (size_t)D_raw * D_raw;
  std::vector<cf64> h64(NOPS * dd);
  std::vector<cf32> h32(NOPS * dd);
  for (size_t i = 0; i < NOPS * dd; ++i) {
    h64[i] = make_double2(loc_ops[s][i].real(), loc_ops[s][i].imag());
    h32[i] = make_float2((float)loc_ops[s][i].real(), (float)loc_ops[s][i].imag());
  }
  HIPCHK(hipMemcpy(d_ops64 + (size_t)s * NOPS * dd, h64.data(), NOPS * dd * sizeof(cf64), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_ops32 + (size_t)s * NOPS * dd, h32.data(), NOPS * dd * sizeof(cf32), hipMemcpyHostToDevice));
  std::vector<cf64> r64(NOPS * DD);
  std::vector<cf32> r32(NOPS * DD);
  for (size_t i = 0; i < NOPS * DD; ++i) {
    r64[i] = make_double2(raw_ops[s][i].real(), raw_ops[s][i].imag());
    r32[i] = make_float2((float)raw_ops[s][i].real(), (float)raw_ops[s][i].imag());
  }
  HIPCHK(hipMemcpy(d_raw64 + (size_t)s * NOPS * DD, r64.data(), NOPS * DD * sizeof(cf64), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_raw32 + (size_t)s * NOPS * DD, r32.data(), NOPS * DD * sizeof(cf32), hipMemcpyHostToDevice));
  std::vector<cf64> w64((size_t)D_raw * d);
  for (size_t i = 0; i < w64.size(); ++i) w64[i] = make_double2(iso[s][i].real(), iso[s][i].imag());
  HIPCHK(hipMemcpy(d_iso + (size_t)s * D_raw * d, w64.data(), w64.size() * sizeof(cf64), hipMemcpyHostToDevice));
}

const void* tn_mpo::op_ptr(int prec, int site, int k, bool raw) const {
  if (k < 1 || k > NOPS) return nullptr;
  if (raw) {
    const size_t DD = (size_t)D_raw * D_raw;
    return prec == PREC_FP64 ? (const void*)(d_raw64 + ((size_t)site * NOPS + (k - 1)) * DD)
                             : (const void*)(d_raw32 + ((size_t)site * NOPS + (k - 1)) * DD);
  }
  const size_t dd = (size_t)d * d;
  return prec == PREC_FP64 ? (const void*)(d_ops64 + ((size_t)site * NOPS + (k - 1)) * dd)
                           : (const void*)(d_ops32 + ((size_t)site * NOPS + (k - 1)) * dd);
}

static void mpo_free(tn_mpo* m) {
  if (!m) return;
  tn_ctx* c = m->ctx;
  if (c) {
    if (!c->closed) (void)hipStreamSynchronize(c->stream);
    dev_free(c, m->d_ops64);
    dev_free(c, m->d_ops32);
    dev_free(c, m->d_raw64);
    dev_free(c, m->d_raw32);
    dev_free(c, m->d_iso);
    dev_free(c, m->d_fock);
  }
  delete m;
  if (c) ctx_release(c);
}

extern "C" tn_status tn_mpo_build(tn_ctx* ctx, const tn_problem* prob, tn_mpo** out) {
  if (!ctx) return TN_EINVAL;
  TN_CTX_OPEN(ctx);
  tn_mpo* m = nullptr;
  TN_GUARD_BEGIN
  // a handle left half built by a failure is freed while the error unwinds
  struct Free { tn_mpo*& h; ~Free() { if (h) mpo_free(h); } } free_on_error{m};
  if (!prob || !out) TN_THROW(TN_EINVAL, "null argument");
  *out = nullptr;
  const int N = prob->N, D = prob->D_raw, d = prob->d;
  if (N < 1 || N > 4096) TN_THROW(TN_EINVAL, "N must be in [1, 4096]");
  if (D < 1 || D > 64) TN_THROW(TN_EINVAL, "D_raw must be in [1, 64]");
  if (d < 1 || d > D) TN_THROW(TN_EINVAL, "d must satisfy 1 <= d <= D_raw");
  if (!prob->r || !prob->U) TN_THROW(TN_EINVAL, "r and U are required");
  if (!std::isfinite(prob->kappa)) TN_THROW(TN_EINVAL, "non-finite kappa");
  if (prob->kappa != 0.0 && N < 2) TN_THROW(TN_EINVAL, "the global CZ Hamiltonian needs N >= 2");
  for (int j = 0; j < N; ++j)
    if (!std::isfinite(prob->r[j])) TN_THROW(TN_EINVAL, "non-finite squeezing parameter");
  std::vector<cd> U(N * N);
  for (int i = 0; i < N * N; ++i) {
    U[i] = cd(prob->U[2 * i], prob->U[2 * i + 1]);
    if (!std::isfinite(U[i].real()) || !std::isfinite(U[i].imag())) TN_THROW(TN_EINVAL, "non-finite U");
  }
  double uerr = 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      cd s = 0.0;
      for (int k = 0; k < N; ++k) s += std::conj(U[k * N + i]) * U[k * N + j];
      uerr = std::max(uerr, std::abs(s - (i == j ? 1.0 : 0.0)));
    }
  if (uerr > 1e-10) TN_THROW(TN_EINVAL, "U is not unitary to 1e-10");
  // isometries
  std::vector<std::vector<cd>> iso(N, std::vector<cd>((size_t)D * d, 0.0));
  if (prob->iso) {
    for (int s = 0; s < N; ++s) {
      for (int i = 0; i < D * d; ++i)
        iso[s][i] = cd(prob->iso[2 * ((size_t)s * D * d + i)], prob->iso[2 * ((size_t)s * D * d + i) + 1]);
      double e = 0.0;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          cd t = 0.0;
          for (int n = 0; n < D; ++n) t += std::conj(iso[s][n * d + a]) * iso[s][n * d + b];
          e = std::max(e, std::abs(t - (a == b ? 1.0 : 0.0)));
        }
      if (!(e <= 1e-10)) TN_THROW(TN_EINVAL, "isometry of site " + std::to_string(s) + " not orthonormal to 1e-10");
    }
  } else {
    for (int s = 0; s < N; ++s)
      for (int a = 0; a < d; ++a) iso[s][a * d + a] = 1.0;
  }
  m = new tn_mpo();
  m->ctx = ctx;
  ctx_retain(ctx);
  m->N = N; m->D_raw = D; m->d = d;
  m->r.assign(prob->r, prob->r + N);
  m->U = U;
  // V = 1/2 O D^2 O^T, O = [[Re U, -Im U], [Im U, Re U]] (Sec. II.C.1)
  const int n2 = 2 * N;
  std::vector<double> O(n2 * n2);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      O[i * n2 + j] = U[i * N + j].real();
      O[i * n2 + N + j] = -U[i * N + j].imag();
      O[(N + i) * n2 + j] = U[i * N + j].imag();
      O[(N + i) * n2 + N + j] = U[i * N + j].real();
    }
  std::vector<double> D2(n2);
  for (int j = 0; j < N; ++j) { D2[j] = std::exp(-2.0 * m->r[j]); D2[N + j] = std::exp(2.0 * m->r[j]); }
  std::vector<double> V(n2 * n2, 0.0);
  for (int i = 0; i < n2; ++i)
    for (int j = 0; j < n2; ++j) {
      double s = 0.0;
      for (int k = 0; k < n2; ++k) s += O[i * n2 + k] * D2[k] * O[j * n2 + k];
      V[i * n2 + j] = 0.5 * s;
    }
  for (int i = 0; i < n2; ++i)
    for (int j = 0; j < i; ++j) V[i * n2 + j] = V[j * n2 + i] = 0.5 * (V[i * n2 + j] + V[j * n2 + i]);
  std::vector<double> Vi = spd_inverse(V, n2);
  m->alpha.assign(N * N, 0.0); m->beta.assign(N * N, 0.0); m->gamma.assign(N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      m->alpha[i * N + j] = 0.25 * (Vi[i * n2 + j] + Vi[j * n2 + i]);
      m->beta[i * N + j] = 0.25 * (Vi[(N + i) * n2 + N + j] + Vi[(N + j) * n2 + N + i]);
      m->gamma[i * N + j] = 0.25 * (Vi[i * n2 + N + j] + Vi[(N + j) * n2 + i]);
    }
  // structure and entries
  m->kappa = prob->kappa;
  const bool cz = prob->kappa != 0.0;
  m->w.resize(N + 1);
  for (int t = 0; t <= N; ++t) m->w[t] = cz ? bond_dim_cz(N, t) : bond_dim(N, t);
  m->kinds.resize(N);
  m->entries.resize(N);
  for (int s = 0; s < N; ++s) {
    m->entries[s] = core_entries(N, s + 1, m->alpha, m->beta, m->gamma);
    if (cz) cz_entries(N, s + 1, m->beta, m->gamma, prob->kappa, m->entries[s]);
    m->kinds[s].assign((size_t)m->w[s] * m->w[s + 1], 0);
    for (auto& e : m->entries[s]) m->kinds[s][(size_t)e.row * m->w[s + 1] + e.col] = (int8_t)e.kind;
  }
  // local operators
  m->iso = iso;
  m->raw_ops.resize(N);
  m->loc_ops.resize(N);
  for (int s = 0; s < N; ++s) {
    build_raw_ops(D, m->alpha[s * N + s], m->beta[s * N + s], m->gamma[s * N + s], m->raw_ops[s]);
    project_ops(m->raw_ops[s], m->iso[s], D, d, m->loc_ops[s]);
  }
  m->d_ops64 = (cf64*)dev_alloc(ctx, (size_t)N * NOPS * d * d * sizeof(cf64));
  m->d_ops32 = (cf32*)dev_alloc(ctx, (size_t)N * NOPS * d * d * sizeof(cf32));
  m->d_raw64 = (cf64*)dev_alloc(ctx, (size_t)N * NOPS * D * D * sizeof(cf64));
  m->d_raw32 = (cf32*)dev_alloc(ctx, (size_t)N * NOPS * D * D * sizeof(cf32));
  m->d_iso = (cf64*)dev_alloc(ctx, (size_t)N * D * d * sizeof(cf64));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int s = 0; s < N; ++s) m->upload_site(s);
  *out = m;
  m = nullptr;
  TN_GUARD_END(ctx)
}

extern "C" tn_status tn_mpo_structure(const tn_mpo* mpo, int32_t* w, int8_t* kinds) {
  if (!mpo || !w) return TN_EINVAL;
  for (int t = 0; t <= mpo->N; ++t) w[t] = mpo->w[t];
  if (kinds) {
    size_t off = 0;
    for (int s = 0; s < mpo->N; ++s) {
      std::memcpy(kinds + off, mpo->kinds[s].data(), mpo->kinds[s].size());
      off += mpo->kinds[s].size();
    }
  }
  return TN_OK;
}

extern "C" tn_status tn_mpo_coefficients(const tn_mpo* mpo, double* a, double* b, double* g) {
  if (!mpo) return TN_EINVAL;
  const size_t n = (size_t)mpo->N * mpo->N;
  if (a) std::memcpy(a, mpo->alpha.data(), n * sizeof(double));
  if (b) std::memcpy(b, mpo->beta.data(), n * sizeof(double));
  if (g) std::memcpy(g, mpo->gamma.data(), n * sizeof(double));
  return TN_OK;
}

extern "C" tn_status tn_mpo_isometries(const tn_mpo* mpo, double* iso) {
  if (mpo && mpo->ctx && mpo->ctx->closed) return TN_ESTATE;
  if (!mpo || !iso) return TN_EINVAL;
  try {
    plbo_sync_iso(mpo);
  } catch (const TnError& e) {
    return e.code;
  } catch (const std::exception&) {
    return TN_ENOMEM;
  }
  size_t o = 0;
  const bool lin = mpo->plbo && mpo->plbo_lin;  // the Fock image, not the linear isometry
  for (int s = 0; s < mpo->N; ++s)
    for (auto& z : (lin ? mpo->fock[s] : mpo->iso[s])) { iso[o++] = z.real(); iso[o++] = z.imag(); }
  return TN_OK;
}

extern "C" tn_status tn_mpo_site_ops(const tn_mpo* mpo, int32_t site, double* ops) {
  if (!mpo || !ops || site < 0 || site >= mpo->N) return TN_EINVAL;
  size_t o = 0;
  for (auto& z : mpo->loc_ops[site]) { ops[o++] = z.real(); ops[o++] = z.imag(); }
  return TN_OK;
}

extern "C" void tn_mpo_destroy(tn_mpo* mpo) { mpo_free(mpo); }

// ------------------------------------------------------------------ MPS
// Grows site s to hold elems entries.  The new buffer is taken first and the
// current tensor copied into it, so a failed allocation (TN_ENOMEM) leaves the
// MPS exactly as it was.
void tn_mps::ensure_site(int s, size_t elems) {
  if (cap[s] >= elems && A[s]) return;
  cf64* p = (cf64*)dev_alloc(ctx, elems * sizeof(cf64));
  if (A[s]) {
    const size_t keep = std::min(cap[s], elems);
    HIPCHK(hipMemcpyAsync(p, A[s], keep * sizeof(cf64), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    dev_free(ctx, A[s]);
  }
  A[s] = p;
  cap[s] = elems;
}

static void mps_free(tn_mps* m) {
  if (!m) return;
  tn_ctx* c = m->ctx;
  if (c) {
    if (!c->closed) (void)hipStreamSynchronize(c->stream);
    for (auto p : m->A) dev_free(c, p);
    for (auto p : m->L) dev_free(c, p);
    for (auto p : m->Rt) dev_free(c, p);
  }
  delete m;
  if (c) ctx_release(c);
}

extern "C" tn_status tn_mps_create(tn_ctx* ctx, int32_t N, int32_t d, const int32_t* dims, const double* init,
                                   tn_mps** out) {
  if (!ctx) return TN_EINVAL;
  TN_CTX_OPEN(ctx);
  tn_mps* m = nullptr;
  TN_GUARD_BEGIN
  struct Free { tn_mps*& h; ~Free() { if (h) mps_free(h); } } free_on_error{m};
  if (!out || !dims || !init) TN_THROW(TN_EINVAL, "null argument");
  *out = nullptr;
  if (N < 1 || d < 1) TN_THROW(TN_EINVAL, "N and d must be positive");
  if (dims[0] != 1 || dims[N] != 1) TN_THROW(TN_EINVAL, "boundary bond dimensions must be 1");
  for (int s = 0; s <= N; ++s)
    if (dims[s] < 1 || dims[s] > 4096) TN_THROW(TN_EINVAL, "bond dimension out of range");
  for (int s = 0; s < N; ++s) {
    if ((int64_t)dims[s] > (int64_t)d * dims[s + 1] || (int64_t)dims[s + 1] > (int64_t)d * dims[s])
      TN_THROW(TN_EINVAL, "bond dimensions exceed d times a neighbour");
  }
  m = new tn_mps();
  m->ctx = ctx;
  ctx_retain(ctx);
  m->N = N; m->d = d;
  m->dims.assign(dims, dims + N + 1);
  m->A.assign(N, nullptr);
  m->cap.assign(N, 0);
  size_t off = 0;
  for (int s = 0; s < N; ++s) {
    const size_t n = (size_t)dims[s] * d * dims[s + 1];
    m->ensure_site(s, n);
    for (size_t i = 0; i < 2 * n; ++i)
      if (!std::isfinite(init[2 * off + i])) TN_THROW(TN_EINVAL, "non-finite initial tensor");
    HIPCHK(hipMemcpy(m->A[s], init + 2 * off, n * sizeof(cf64), hipMemcpyHostToDevice));
    off += n;
  }
  m->L.assign(N + 1, nullptr); m->Rt.assign(N + 1, nullptr);
  m->Lcap.assign(N + 1, 0); m->Rcap.assign(N + 1, 0);
  m->Lok.assign(N + 1, false); m->Rok.assign(N + 1, false);
  *out = m;
  m = nullptr;
  TN_GUARD_END(ctx)
}

extern "C" tn_status tn_mps_bond_dims(const tn_mps* mps, int32_t* dims) {
  if (!mps || !dims) return TN_EINVAL;
  for (int s = 0; s <= mps->N; ++s) dims[s] = mps->dims[s];
  return TN_OK;
}

extern "C" tn_status tn_mps_export(tn_ctx* ctx, const tn_mps* mps, double* buf, size_t cap, size_t* needed) {
  if (!ctx || !mps) return TN_EINVAL;
  TN_CTX_OPEN(ctx);
  TN_GUARD_BEGIN
  size_t tot = 0;
  for (int s = 0; s < mps->N; ++s) tot += 2 * (size_t)mps->dims[s] * mps->d * mps->dims[s + 1];
  if (needed) *needed = tot;
  if (!buf) return TN_OK;
  if (cap < tot) TN_THROW(TN_EINVAL, "export buffer too small");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  size_t off = 0;
  for (int s = 0; s < mps->N; ++s) {
    const size_t n = (size_t)mps->dims[s] * mps->d * mps->dims[s + 1];
    HIPCHK(hipMemcpy(buf + off, mps->A[s], n * sizeof(cf64), hipMemcpyDeviceToHost));
    off += 2 * n;
  }
  TN_GUARD_END(ctx)
}

// ------------------------------------------------------------------ checkpoint
// Layout (doubles): [magic, version, N, d, centre, sweeps, D_raw (0: no
// isometries), 0], bond dimensions [N + 1], the site tensors (complex,
// concatenated in site order), then the isometries [N][D_raw][d] complex.
static const double kCkptMagic = 1414415184.0;  // "TNCP" read as a big-endian integer
static const int kCkptHeader = 8;

static size_t ckpt_tensor_doubles(const std::vector<int>& dims, int N, int d) {
  size_t tot = 0;
  for (int s = 0; s < N; ++s) tot += 2 * (size_t)dims[s] * d * dims[s + 1];
  return tot;
}

extern "C" tn_status tn_mps_checkpoint(tn_ctx* ctx, const tn_mps* mps, const tn_mpo* mpo, double* buf, size_t cap,
                                       size_t* needed) {
  if (!ctx || !mps) return TN_EINVAL;
  TN_CTX_OPEN(ctx);
  TN_GUARD_BEGIN
  const int N = mps->N, d = mps->d;
  if (mpo && (mpo->N != N || mpo->d != d)) TN_THROW(TN_EINVAL, "MPO and MPS do not match");
  const int D = mpo ? mpo->D_raw : 0;
  const size_t nt = ckpt_tensor_doubles(mps->dims, N, d);
  const size_t tot = kCkptHeader + (size_t)(N + 1) + nt + 2 * (size_t)N * D * d;
  if (needed) *needed = tot;
  if (!buf) return TN_OK;
  if (cap < tot) TN_THROW(TN_EINVAL, "checkpoint buffer too small");
  std::vector<double> iso;
  if (mpo) {
    iso.resize(2 * (size_t)N * D * d);
    const tn_status st = tn_mpo_isometries(mpo, iso.data());
    if (st != TN_OK) TN_THROW(st, "isometries of the MPO could not be read");
  }
  double* h = buf;
  h[0] = kCkptMagic; h[1] = 1.0; h[2] = N; h[3] = d; h[4] = mps->center; h[5] = (double)mps->sweeps;
  h[6] = D; h[7] = 0.0;
  for (int t = 0; t <= N; ++t) h[kCkptHeader + t] = mps->dims[t];
  HIPCHK(hipStreamSynchronize(ctx->stream));
  size_t off = kCkptHeader + N + 1;
  for (int s = 0; s < N; ++s) {
    const size_t n = (size_t)mps->dims[s] * d * mps->dims[s + 1];
    HIPCHK(hipMemcpy(buf + off, mps->A[s], n * sizeof(cf64), hipMemcpyDeviceToHost));
    off += 2 * n;
  }
  if (mpo) std::memcpy(buf + off, iso.data(), iso.size() * sizeof(double));
  TN_GUARD_END(ctx)
}

extern "C" tn_status tn_mps_import(tn_ctx* ctx, const double* buf, size_t len, tn_mps** out, double* iso,
                                   int32_t* info) {
  if (!ctx) return TN_EINVAL;
  TN_CTX_OPEN(ctx);
  tn_mps* m = nullptr;
  TN_GUARD_BEGIN
  if (!buf || !out) TN_THROW(TN_EINVAL, "null argument");
  *out = nullptr;
  if (len < (size_t)kCkptHeader + 2) TN_THROW(TN_EINVAL, "checkpoint too short");
  if (buf[0] != kCkptMagic || buf[1] != 1.0) TN_THROW(TN_EINVAL, "not a version-1 checkpoint");
  auto as_int = [](double v, double lo, double hi, const char* what) {
    if (!(v >= lo && v <= hi) || v != std::floor(v)) TN_THROW(TN_EINVAL, std::string("bad ") + what + " in checkpoint");
    return (int64_t)v;
  };
  const int N = (int)as_int(buf[2], 1, 4096, "N");
  const int d = (int)as_int(buf[3], 1, 64, "d");
  const int centre = (int)as_int(buf[4], -1, N - 1, "centre");
  const int64_t sweeps = as_int(buf[5], 0, 9.0e15, "sweep count");
  const int D = (int)as_int(buf[6], 0, 64, "D_raw");
  if (D != 0 && D < d) TN_THROW(TN_EINVAL, "D_raw below d in checkpoint");
  if (len < (size_t)kCkptHeader + N + 1) TN_THROW(TN_EINVAL, "checkpoint too short");
  std::vector<int32_t> dims(N + 1);
  for (int t = 0; t <= N; ++t) dims[t] = (int32_t)as_int(buf[kCkptHeader + t], 1, 4096, "bond dimension");
  std::vector<int> dv(dims.begin(), dims.end());
  const size_t nt = ckpt_tensor_doubles(dv, N, d);
  const size_t tot = kCkptHeader + (size_t)(N + 1) + nt + 2 * (size_t)N * D * d;
  if (len != tot) TN_THROW(TN_EINVAL, "checkpoint length does not match its header");
  const double* tens = buf + kCkptHeader + N + 1;
  for (size_t i = 0; i < 2 * (size_t)N * D * d; ++i)
    if (!std::isfinite(tens[nt + i])) TN_THROW(TN_EINVAL, "non-finite isometry in checkpoint");
  const tn_status st = tn_mps_create(ctx, N, d, dims.data(), tens, &m);
  if (st != TN_OK) return st;
  m->center = centre;
  m->sweeps = sweeps;
  if (info) { info[0] = D; info[1] = centre; }
  if (iso && D > 0) std::memcpy(iso, tens + nt, 2 * (size_t)N * D * d * sizeof(double));
  *out = m;
  m = nullptr;
  TN_GUARD_END(ctx)
}

extern "C" tn_status tn_mps_sweeps(const tn_mps* mps, int64_t* sweeps) {
  if (!mps || !sweeps) return TN_EINVAL;
  *sweeps = mps->sweeps;
  return TN_OK;
}

extern "C" void tn_mps_destroy(tn_mps* mps) { mps_free(mps); }
