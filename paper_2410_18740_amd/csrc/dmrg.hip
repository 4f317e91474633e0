// Two-site DMRG driver: Lanczos local solver (FP64 Krylov vectors), FP64
// truncation (Gram matrix + Hermitian eigensolver), environment updates, the
// sweep with optional local basis optimisation, and the FP64 energy.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include "internal.h"

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

static double wall() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ small helpers
static double dev_norm2(tn_ctx* c, const cf64* x, int64_t n) {
  const int nb = multidot_blocks(n);
  cf64* part = wsT<cf64>(c, "nrm:part", nb);
  cf64* out = wsT<cf64>(c, "nrm:out", 1);
  const cf64** ptr = wsT<const cf64*>(c, "nrm:ptr", 1);
  HIPCHK(hipMemcpyAsync(ptr, &x, sizeof(cf64*), hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_multidot(ptr, 1, x, n, part, nb, c->stream));
  HIPCHK(launch_multidot_finish(part, 1, nb, out, c->stream));
  cf64 h;
  download(c, &h, out, sizeof(cf64));
  return h.x;
}

static void gemm1(tn_ctx* c, int prec, int ta, int tb, void* C, int64_t ldc, int M, int N, const void* A, int64_t lda,
                  const void* B, int64_t ldb, int K, int acc, const std::string& tag) {
  GemmJob j{C, ldc, M, N, 0, 1};
  GemmSeg s{A, B, lda, ldb, K, 0};
  char* d = (char*)ws_get(c, tag, 512);
  HIPCHK(hipMemcpyAsync(d, &j, sizeof(j), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(d + 256, &s, sizeof(s), hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_cgemm(prec, ta, tb, (GemmJob*)d, 1, (GemmSeg*)(d + 256), M, N, acc, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

// batched GEMMs from host descriptor vectors (descriptors staged synchronously)
static void gemm_batch(tn_ctx* c, int prec, int ta, int tb, const std::vector<GemmJob>& jobs,
                       const std::vector<GemmSeg>& segs, int maxM, int maxN, const std::string& tag) {
  if (jobs.empty()) return;
  const size_t bj = ((jobs.size() * sizeof(GemmJob)) + 255) & ~size_t(255);
  char* d = (char*)ws_get(c, tag, bj + segs.size() * sizeof(GemmSeg));
  HIPCHK(hipMemcpyAsync(d, jobs.data(), jobs.size() * sizeof(GemmJob), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(d + bj, segs.data(), segs.size() * sizeof(GemmSeg), hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_cgemm(prec, ta, tb, (GemmJob*)d, (int)jobs.size(), (GemmSeg*)(d + bj), maxM, maxN, 0, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

// ------------------------------------------------------------------ Lanczos
struct LzResult {
  double lambda = 0.0;
  int matvecs = 0;
  bool converged = false;
  double t_mv = 0.0;
  int full_passes = 0;  // iterations orthogonalised against the whole basis
};

// Lowest eigenpair by Lanczos with partial reorthogonalisation (Simon, Math.
// Comp. 42, 1984).  Each new vector is orthogonalised (two classical
// Gram-Schmidt passes) against the two latest basis vectors only, while the
// recurrence
//   beta_j w_{j+1,k} = beta_k w_{j,k+1} + (alpha_k - alpha_j) w_{j,k}
//                      + beta_{k-1} w_{j,k-1} - beta_{j-1} w_{j-1,k}
// estimates its overlaps w_{j+1,k} with the older ones, each step adding a
// rounding term of unit u (the matvec's relative accuracy).  When an estimate
// exceeds sqrt(u) the vector is orthogonalised against the whole basis, and so
// is the next one; the basis stays orthogonal to sqrt(u), which keeps the Ritz
// values accurate to O(u ||H||).  Restarts every kmax vectors from the Ritz vector.
// Lowest eigenpair of the symmetric tridiagonal matrix with diagonal a[0..n)
// and off-diagonal b[0..n-1): the eigenvalue by bisection on Sturm counts to
// the rounding level, the eigenvector by three steps of inverse iteration
// with the LU factors (partial pivoting) of T - lambda I, normalised with its
// first component non-negative.  Returns lambda; y receives the vector.
static double tridiag_lowest(const std::vector<double>& a, const std::vector<double>& b, int n,
                             std::vector<double>& y) {
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < n - 1 ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  const double sc = std::max(std::fabs(lo), std::fabs(hi)) + 1e-300;
  lo -= 1e-14 * sc;
  hi += 1e-14 * sc;
  auto below = [&](double x) {  // number of eigenvalues < x
    int cnt = 0;
    double q = a[0] - x;
    if (std::fabs(q) < 1e-300) q = -1e-300;
    cnt += q < 0;
    for (int i = 1; i < n; ++i) {
      q = (a[i] - x) - b[i - 1] * b[i - 1] / q;
      if (std::fabs(q) < 1e-300) q = -1e-300;
      cnt += q < 0;
    }
    return cnt;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi) || hi - lo <= 4.4e-16 * std::max(std::fabs(lo), std::fabs(hi)) + 1e-300) break;
    if (below(mid) >= 1) hi = mid;
    else lo = mid;
  }
  const double lam = 0.5 * (lo + hi);
  const double tiny = std::max(2.2e-16 * sc, 1e-300);
  y.assign(n, 1.0);
  if (n == 1) return lam;
  // LU of T - lam I with partial pivoting: row i of U has dd[i], du[i], du2[i]
  std::vector<double> dd(n), du(n, 0.0), du2(n, 0.0), dl(n, 0.0);
  std::vector<char> piv(n, 0);
  {
    double cdd = a[0] - lam, cdu = b[0];
    for (int i = 0; i < n - 1; ++i) {
      const double l = b[i], ndd = a[i + 1] - lam, ndu = (i + 1 < n - 1) ? b[i + 1] : 0.0;
      if (std::fabs(cdd) >= std::fabs(l)) {
        if (cdd == 0.0) cdd = tiny;
        const double f = l / cdd;
        dd[i] = cdd; dl[i] = f; du[i] = cdu;
        cdd = ndd - f * cdu;
        cdu = ndu;
      } else {
        const double f = cdd / l;
        dd[i] = l; dl[i] = f; du[i] = ndd; piv[i] = 1;
        cdd = cdu - f * ndd;
        if (i < n - 2) { du2[i] = ndu; cdu = -f * ndu; }
        else cdu = ndu;
      }
    }
    dd[n - 1] = cdd;
  }
  for (int i = 0; i < n; ++i)
    if (std::fabs(dd[i]) < tiny) dd[i] = dd[i] >= 0 ? tiny : -tiny;
  for (int it = 0; it < 3; ++it) {
    double cb = y[0];
    for (int i = 0; i < n - 1; ++i) {
      const double nb = y[i + 1], l = dl[i];
      if (piv[i]) { y[i] = nb; cb = cb - l * nb; }
      else { y[i] = cb; cb = nb - l * cb; }
    }
    double x1 = cb / dd[n - 1], x2 = 0.0;
    y[n - 1] = x1;
    for (int i = n - 2; i >= 0; --i) {
      const double x0 = (y[i] - du[i] * x1 - du2[i] * x2) / dd[i];
      y[i] = x0;
      x2 = x1;
      x1 = x0;
    }
    double nr = 0.0;
    for (int i = 0; i < n; ++i) nr += y[i] * y[i];
    nr = 1.0 / std::sqrt(nr);
    for (int i = 0; i < n; ++i) y[i] *= nr;
  }
  if (y[0] < 0.0)
    for (int i = 0; i < n; ++i) y[i] = -y[i];
  return lam;
}

template <class MV>
static LzResult lanczos(tn_ctx* c, MV&& matvec, cf64* x, int64_t n, double tol, int kmax, int max_mv, double u) {
  LzResult R;
  hipStream_t st = c->stream;
  kmax = std::max(2, std::min(kmax, 64));
  const int nb = multidot_blocks(n);
  cf64* V = wsT<cf64>(c, "lz:V", (size_t)(kmax + 1) * n);
  cf64* W = wsT<cf64>(c, "lz:W", (size_t)n);
  // pointer table ptrs = [V_0..V_kmax]
  const cf64** ptrs = wsT<const cf64*>(c, "lz:ptr", kmax + 1);
  cf64* part = wsT<cf64>(c, "lz:part", (size_t)nb * (kmax + 2));
  cf64* h1 = wsT<cf64>(c, "lz:h1", kmax + 2);
  cf64* h2 = wsT<cf64>(c, "lz:h2", kmax + 2);
  double* alpha = wsT<double>(c, "lz:al", kmax + 1);
  double* beta = wsT<double>(c, "lz:be", kmax + 1);
  double* inv = wsT<double>(c, "lz:inv", 1);
  double* sc = wsT<double>(c, "lz:sc", 4);
  double* coefs = wsT<double>(c, "lz:cf", kmax + 1);
  {
    std::vector<const cf64*> hp(kmax + 1);
    for (int i = 0; i <= kmax; ++i) hp[i] = V + (size_t)i * n;
    HIPCHK(hipMemcpyAsync(ptrs, hp.data(), hp.size() * sizeof(cf64*), hipMemcpyHostToDevice, st));
  }
  const double thresh = std::sqrt(u);
  double nx = dev_norm2(c, x, n);
  if (!(nx > 0.0) || !std::isfinite(nx)) TN_THROW(TN_ENUMERIC, "Lanczos start vector is zero or non-finite");
  HIPCHK(launch_scale_host(V, x, 1.0 / std::sqrt(nx), n, st));
  double* hout = c->pinned;
  hipEvent_t e0 = c->ev[0], e1 = c->ev[1];
  // two classical Gram-Schmidt passes of W against V_i0..V_{i0+nv-1}; the second
  // pass also returns <w, w>; h1, h2 receive the two passes' dots at offset i0
  auto cgs2 = [&](int i0, int nv) {
    HIPCHK(launch_multidot(ptrs + i0, nv, W, n, part, nb, st));
    HIPCHK(launch_multidot_finish(part, nv, nb, h1 + i0, st));
    HIPCHK(launch_axpy_dot(W, ptrs + i0, nv, h1 + i0, n, part, nb, st));
    HIPCHK(launch_multidot_finish(part, nv + 1, nb, h2 + i0, st));
  };
  while (true) {
    int jlast = -1;
    bool stop = false;
    double lam = 0.0;
    std::vector<double> al, be, om_prev, om_cur{1.0}, om_next;  // om_cur[k] = w_{j,k}
    std::vector<double> ta, tb, ritz;                             // the Ritz problem, on the host
    double anorm = 0.0;
    bool force_full = false;
    for (int j = 0; j < kmax; ++j) {
      HIPCHK(hipEventRecord(e0, st));
      matvec(V + (size_t)j * n, W);
      HIPCHK(hipEventRecord(e1, st));
      R.matvecs++;
      const bool full = force_full;
      const int i0 = full ? 0 : std::max(0, j - 1);
      if (full) R.full_passes++;
      cgs2(i0, j - i0 + 1);
      HIPCHK(launch_lanczos_ab(h1, h2, j, i0, alpha, beta, inv, sc, st));
      HIPCHK(hipMemcpyAsync(hout, sc, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) R.t_mv += ms * 1e-3;
      const double a = hout[0], b = hout[1];
      if (!std::isfinite(a) || !std::isfinite(b)) TN_THROW(TN_ENUMERIC, "non-finite value in Lanczos recurrence");
      // lowest Ritz pair of the (j + 1) x (j + 1) tridiagonal; the residual
      // estimate is beta_j times the Ritz vector's last component
      ta.push_back(a);
      if (j > 0) tb.push_back(be[j - 1]);
      lam = tridiag_lowest(ta, tb, j + 1, ritz);
      const double res = b * std::fabs(ritz[j]);
      if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(lam))
        TN_THROW(TN_ENUMERIC, "non-finite value in Lanczos recurrence");
      jlast = j;
      const double bscale = std::max(1.0, std::fabs(lam));
      if (res <= tol || b <= 1e-14 * bscale) { R.converged = true; stop = true; break; }
      if (R.matvecs >= max_mv) { stop = true; break; }
      if (j + 1 >= kmax) break;
      al.push_back(a);
      be.push_back(b);
      anorm = std::max(anorm, std::fabs(a) + b + (j > 0 ? be[j - 1] : 0.0));
      // overlap estimates of the new vector with V_0..V_{j-2} (V_{j-1}, V_j were projected out)
      om_next.assign(j + 2, u);
      om_next[j + 1] = 1.0;
      double worst = 0.0;
      if (!full) {
        for (int k = 0; k + 1 < j; ++k) {
          double t = be[k] * om_cur[k + 1] + (al[k] - a) * om_cur[k] + (k > 0 ? be[k - 1] * om_cur[k - 1] : 0.0) -
                     (j > 0 ? be[j - 1] * om_prev[k] : 0.0);
          t += (t >= 0.0 ? 1.0 : -1.0) * u * (anorm + be[k] + b);
          om_next[k] = t / b;
          worst = std::max(worst, std::fabs(om_next[k]));
        }
      }
      if (worst > thresh) {
        // the new vector against the whole basis, and the next one as well
        cgs2(0, j + 1);
        HIPCHK(launch_inv_norm(h2, j + 1, inv, st));
        HIPCHK(launch_axpy_scale(V + (size_t)(j + 1) * n, W, ptrs, j + 1, h2, inv, n, st));
        R.full_passes++;
        for (int k = 0; k <= j; ++k) om_next[k] = u;
        force_full = true;
      } else {
        // second update fused with the normalisation: V_{j+1} = (w - sum h2 V) / beta
        HIPCHK(launch_axpy_scale(V + (size_t)(j + 1) * n, W, ptrs + i0, j - i0 + 1, h2 + i0, inv, n, st));
        force_full = false;
      }
      om_prev.swap(om_cur);
      om_cur.swap(om_next);
    }
    // Ritz vector x = sum_i y_i V_i
    HIPCHK(hipMemcpyAsync(coefs, ritz.data(), (size_t)(jlast + 1) * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(launch_lincomb(x, ptrs, jlast + 1, coefs, n, st));
    const double xn = dev_norm2(c, x, n);
    if (!(xn > 0.0) || !std::isfinite(xn)) TN_THROW(TN_ENUMERIC, "non-finite Ritz vector");
    R.lambda = lam;
    if (stop) {
      HIPCHK(launch_scale_host(x, x, 1.0 / std::sqrt(xn), n, st));
      return R;
    }
    HIPCHK(launch_scale_host(V, x, 1.0 / std::sqrt(xn), n, st));
  }
}

// relative accuracy of a matvec in the given GEMM form (the unit of the
// orthogonality estimates)
static double matvec_unit(int prec) {
  if (prec == PREC_FP64) return 2.2e-16;
  if (prec == PREC_FP32) return 1e-6;
  return 1e-5;
}

// ------------------------------------------------------------------ truncation
struct TruncOut {
  int k = 0;
  double disc = 0.0;
  double flops = 0.0;  // implementation flops of the dense stages (see truncate_dev)
  std::vector<double> sv;
};

// Hermitian eigensolve of the p x p matrix G (device, overwritten): top kk eigenpairs,
// eigenvalues to host (descending), eigenvectors as columns of Z (p x ldz, device).
static void herm_top(tn_ctx* c, cf64* G, int p, int kk, std::vector<double>& evals, cf64*& Z, int& ldz) {
  hipStream_t st = c->stream;
  // Jacobi in LDS for the smallest sizes; from 33 on the tridiagonal route is
  // faster (4.7 ms against about 0.5 ms at 64)
  if (p <= 32) {
    double* ev = wsT<double>(c, "eig:ev", p);
    Z = wsT<cf64>(c, "eig:Z", (size_t)p * p);
    HIPCHK(launch_jacobi(G, 0, p, 1, ev, Z, 0, 1, st));
    evals.resize(p);
    download(c, evals.data(), ev, p * sizeof(double));
    evals.resize(kk);
    ldz = p;
    return;
  }
  if (p > 3200) TN_THROW(TN_EINVAL, "eigensolver size " + std::to_string(p) + " exceeds 3200 (LDS-staged reflectors)");
  TridiagWork tw;
  tw.A = G;
  tw.vs = wsT<cf64>(c, "eig:vs", (size_t)p * p);
  tw.taus = wsT<cf64>(c, "eig:tau", p);
  tw.dg = wsT<double>(c, "eig:dg", p);
  tw.off = wsT<double>(c, "eig:off", p);
  tw.y = wsT<cf64>(c, "eig:y", 2 * (size_t)p);
  tw.w = wsT<cf64>(c, "eig:w", 2 * (size_t)p);
  tw.counter = wsT<unsigned int>(c, "eig:cnt", 1);
  // profiling: one event pair around the whole sequence of column launches
  const bool pf = c->prof;
  if (pf) {
    while (c->tri_ev.size() < 2) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      c->tri_ev.push_back(e);
    }
    HIPCHK(hipEventRecord(c->tri_ev[0], st));
  }
  HIPCHK(launch_tridiag(tw, p, st));
  if (pf) HIPCHK(hipEventRecord(c->tri_ev[1], st));
  double* ev = wsT<double>(c, "eig:ev", kk);
  HIPCHK(launch_bisect_top(tw.dg, tw.off, p, kk, ev, st));
  double* X = wsT<double>(c, "eig:X", (size_t)kk * p);
  double* scr = wsT<double>(c, "eig:scr", (size_t)4 * kk * p);
  HIPCHK(launch_inverse_iter(tw.dg, tw.off, p, kk, ev, X, scr, st));
  // inverse iteration gives orthogonal vectors for separated eigenvalues; restore
  // orthonormality (two-pass Gram-Schmidt) from the first defective column on
  int* bad = wsT<int>(c, "eig:bad", kk);
  HIPCHK(launch_fill_int(bad, 0, kk, st));
  HIPCHK(launch_ortho_check(X, p, kk, 1e-13, bad, st));
  std::vector<int> hb(kk);
  download(c, hb.data(), bad, kk * sizeof(int));
  if (pf) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->tri_ev[0], c->tri_ev[1]) == hipSuccess) {
      c->prof_tri_ms += ms;
      c->prof_tri_n += p;
      for (int j = 0; j < p; ++j) c->prof_tri_bytes += 32.0 * (double)(p - j - 1) * (double)(p - j - 1);
    }
  }
  int j0 = kk;
  for (int j = 0; j < kk; ++j)
    if (hb[j]) { j0 = j; break; }
  HIPCHK(launch_orthonormalize_real(X, p, kk, j0, wsT<double>(c, "eig:H", (size_t)kk * 16), st));
  Z = wsT<cf64>(c, "eig:Z", (size_t)p * kk);
  HIPCHK(launch_backtransform_wy(tw.vs, tw.taus, p, X, kk, Z, wsT<cf64>(c, "eig:T", backtransform_wy_workspace(p)),
                                 st));
  evals.resize(kk);
  download(c, evals.data(), ev, kk * sizeof(double));
  ldz = kk;
}

static TruncOut truncate_dev(tn_ctx* c, int m, int n, const cf64* theta, int chi, double sigma_cut, int dir,
                             cf64* left, cf64* right) {
  hipStream_t st = c->stream;
  TruncOut out;
  const int p = dir > 0 ? m : n;
  const int kk = std::max(1, std::min(chi, std::min(m, n)));
  cf64* G = wsT<cf64>(c, "tr:G", (size_t)p * p);
  if (dir > 0) gemm1(c, PREC_FP64, 0, 1, G, p, m, m, theta, n, theta, n, n, 0, "tr:d0");
  else gemm1(c, PREC_FP64, 1, 0, G, p, n, n, theta, n, theta, n, m, 0, "tr:d0");
  const double total = dev_norm2(c, theta, (int64_t)m * n);
  if (!(total > 0.0) || !std::isfinite(total)) TN_THROW(TN_ENUMERIC, "theta is zero or non-finite");
  std::vector<double> ev;
  cf64* Z = nullptr;
  int ldz = 0;
  herm_top(c, G, p, kk, ev, Z, ldz);
  // implementation flops of the dense stages as this path performs them (real
  // flops, complex multiply-add = 8): the Gram GEMM (8 p^2 q, q the other
  // side), the tridiagonalisation (24 r^2 for the column with r trailing rows:
  // the rank-2 update of the whole trailing block and the product with the
  // reflector), the back-transform (16 r per reflector and eigenvector) and the
  // second factor (8 k p q).  Bisection, inverse iteration and the Jacobi route
  // (p <= 32) are not counted.
  {
    const double pd = p, qd = dir > 0 ? n : m, kd = kk;
    double f = 8.0 * pd * pd * qd + 8.0 * kd * pd * qd;
    if (p > 32) f += 24.0 * (pd - 1.0) * pd * (2.0 * pd - 1.0) / 6.0 + 8.0 * kd * pd * (pd - 1.0);
    out.flops = f;
  }
  int k = kk;
  if (sigma_cut > 0.0) {
    int cnt = 0;
    for (int i = 0; i < kk; ++i) cnt += (ev[i] > sigma_cut * sigma_cut * ev[0]);
    k = std::max(1, std::min(k, cnt));
  }
  double kept = 0.0;
  for (int i = 0; i < k; ++i) kept += std::max(ev[i], 0.0);
  if (!(kept > 0.0)) TN_THROW(TN_ENUMERIC, "no positive singular value kept");
  out.k = k;
  out.disc = std::max(0.0, total - kept) / total;
  out.sv.resize(k);
  for (int i = 0; i < k; ++i) out.sv[i] = std::sqrt(std::max(ev[i], 0.0) / total);
  const double sc = 1.0 / std::sqrt(kept);
  if (dir > 0) {
    HIPCHK(launch_copy2d(left, k, Z, ldz, m, k, 0, st));
    gemm1(c, PREC_FP64, 1, 0, right, n, k, n, Z, ldz, theta, n, m, 0, "tr:d1");
    HIPCHK(launch_scale_host(right, right, sc, (int64_t)k * n, st));
  } else {
    HIPCHK(launch_copy2d(right, n, Z, ldz, n, k, 1, st));
    gemm1(c, PREC_FP64, 0, 0, left, k, m, k, theta, n, Z, ldz, n, 0, "tr:d1");
    HIPCHK(launch_scale_host(left, left, sc, (int64_t)m * k, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return out;
}

// ------------------------------------------------------------------ environment updates
static void mixed_envs(tn_ctx* c, int prec, const std::vector<PlanL>& Ls, const std::vector<const void*>& envs,
                       int64_t elems, std::vector<const void*>& ptr, const std::string& tag) {
  const size_t eb = elem_bytes(prec);
  ptr.resize(Ls.size());
  std::vector<MixJob> jobs;
  std::vector<MixTerm> terms;
  int nm = 0;
  for (auto& L : Ls) nm += !(L.src.size() == 1 && L.src[0].second == 1.0);
  char* buf = (char*)ws_get(c, tag + ":mix", std::max(1, nm) * elems * eb);
  int im = 0;
  for (size_t i = 0; i < Ls.size(); ++i) {
    const auto& L = Ls[i];
    if (L.src.size() == 1 && L.src[0].second == 1.0) { ptr[i] = envs[L.src[0].first]; continue; }
    void* dst = buf + (size_t)im * elems * eb;
    ++im;
    jobs.push_back({dst, (int)terms.size(), (int)L.src.size()});
    for (auto& s : L.src) terms.push_back({envs[s.first], s.second});
    ptr[i] = dst;
  }
  if (jobs.empty()) return;
  const size_t bj = (jobs.size() * sizeof(MixJob) + 255) & ~size_t(255);
  char* d = (char*)ws_get(c, tag + ":mixd", bj + terms.size() * sizeof(MixTerm));
  HIPCHK(hipMemcpyAsync(d, jobs.data(), jobs.size() * sizeof(MixJob), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(d + bj, terms.data(), terms.size() * sizeof(MixTerm), hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_envmix(prec == PREC_FP64 ? PREC_FP64 : PREC_FP32, (MixJob*)d, (int)jobs.size(), (MixTerm*)(d + bj),
                       elems, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

// device operators of one site by index; entry 0 (the identity) is never read
using OpTable = std::vector<const void*>;
static OpTable site_ops(const tn_mpo* mpo, int sprec, int site) {
  OpTable t(NOPS + 1, nullptr);
  for (int k = 1; k <= NOPS; ++k) t[k] = mpo->op_ptr(sprec, site, k, false);
  return t;
}

static void run_ops(tn_ctx* c, int sprec, const OpTable& ops, const Plan& P, char* Y, char* T, size_t nel, int chi_l,
                    int ds, int chi_r, const std::string& tag) {
  if (P.T.empty()) return;
  const size_t eb = elem_bytes(sprec);
  std::vector<OpJob> oj;
  std::vector<OpTerm> ot;
  for (size_t j = 0; j < P.T.size(); ++j) {
    oj.push_back({T + j * nel * eb, (int)ot.size(), (int)P.T[j].terms.size(), 0, 0});
    for (auto& t : P.T[j].terms) ot.push_back({Y + (size_t)t.ych * nel * eb, t.a ? ops.at(t.a) : nullptr, nullptr, t.c});
  }
  const size_t bj = (oj.size() * sizeof(OpJob) + 255) & ~size_t(255);
  char* d = (char*)ws_get(c, tag + ":opd", bj + ot.size() * sizeof(OpTerm));
  HIPCHK(hipMemcpyAsync(d, oj.data(), oj.size() * sizeof(OpJob), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(d + bj, ot.data(), ot.size() * sizeof(OpTerm), hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_opapply(sprec, (OpJob*)d, (int)oj.size(), (OpTerm*)(d + bj), chi_l, ds, 1, chi_r, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

// zero the output channels that receive no term
static void zero_channels(tn_ctx* c, int sprec, void* out, int w, int64_t elems, const std::vector<bool>& covered) {
  std::vector<MixJob> jobs;
  const size_t eb = elem_bytes(sprec);
  for (int i = 0; i < w; ++i)
    if (!covered[i]) jobs.push_back({(char*)out + (size_t)i * elems * eb, 0, 0});
  if (jobs.empty()) return;
  char* d = (char*)ws_get(c, "zero:d", jobs.size() * sizeof(MixJob));
  HIPCHK(hipMemcpyAsync(d, jobs.data(), jobs.size() * sizeof(MixJob), hipMemcpyHostToDevice, c->stream));
  HIPCHK(launch_envmix(sprec, (MixJob*)d, (int)jobs.size(), nullptr, elems, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

// A (FP64, chi_l x d x chi_r) in the GEMM precision's storage form
static const void* stage_A(tn_ctx* c, int prec, const cf64* A, size_t n, const std::string& tag) {
  if (prec == PREC_FP64) return A;
  void* p = ws_get(c, tag, n * sizeof(cf32));
  HIPCHK(launch_convert(PREC_FP32, p, PREC_FP64, A, (int64_t)n, c->stream));
  return p;
}

// left update across one site for a single-site term list: Lout[wo][chi_r][chi_r]
// from Lin[.][chi_l][chi_l]; output channels that no term reaches are zeroed when
// zero_rest, and marked in `covered` (size wo) either way
static void env_left_terms(tn_ctx* c, int prec, const Plan& P, int wo, int d, const OpTable& ops, int chi_l,
                           int chi_r, const std::vector<const void*>& Lin, const cf64* A, void* Lout, bool zero_rest,
                           std::vector<bool>& cov, const std::string& tag) {
  const int sprec = prec == PREC_FP64 ? PREC_FP64 : PREC_FP32;
  const size_t eb = elem_bytes(sprec);
  const size_t nel = (size_t)chi_l * d * chi_r;
  const void* AP = stage_A(c, prec, A, nel, tag + ":A");
  std::vector<const void*> Lp;
  mixed_envs(c, sprec, P.L, Lin, (int64_t)chi_l * chi_l, Lp, tag);
  char* Y = (char*)ws_get(c, tag + ":Y", std::max<size_t>(1, P.L.size()) * nel * eb);
  char* T = (char*)ws_get(c, tag + ":T", std::max<size_t>(1, P.T.size()) * nel * eb);
  std::vector<GemmJob> jobs;
  std::vector<GemmSeg> segs;
  for (size_t i = 0; i < P.L.size(); ++i) {
    segs.push_back({Lp[i], AP, chi_l, (int64_t)d * chi_r, chi_l, 0});
    jobs.push_back({Y + i * nel * eb, (int64_t)d * chi_r, chi_l, d * chi_r, (int)segs.size() - 1, 1});
  }
  gemm_batch(c, prec, 0, 0, jobs, segs, chi_l, d * chi_r, tag + ":g1");
  run_ops(c, sprec, ops, P, Y, T, nel, chi_l, d, chi_r, tag);
  jobs.clear(); segs.clear();
  for (auto& R : P.R) {
    const int ch = R.env[0].first;
    cov[ch] = true;
    const void* src = R.kind == 0 ? (const void*)(Y + (size_t)R.idx * nel * eb) : (const void*)(T + (size_t)R.idx * nel * eb);
    segs.push_back({AP, src, chi_r, chi_r, chi_l * d, 0});
    jobs.push_back({(char*)Lout + (size_t)ch * chi_r * chi_r * eb, chi_r, chi_r, chi_r, (int)segs.size() - 1, 1});
  }
  gemm_batch(c, prec, 1, 0, jobs, segs, chi_r, chi_r, tag + ":g2");
  if (zero_rest) zero_channels(c, sprec, Lout, wo, (int64_t)chi_r * chi_r, cov);
}

// left update across `site`: Lout[w_{s+1}][chi_r][chi_r] from Lin[w_s][chi_l][chi_l]
static void env_left(tn_ctx* c, const tn_mpo* mpo, int site, int prec, int chi_l, int chi_r,
                     const std::vector<const void*>& Lin, const cf64* A, void* Lout) {
  const int sprec = prec == PREC_FP64 ? PREC_FP64 : PREC_FP32;
  const int wo = mpo->w[site + 1];
  const Plan P = build_plan(window_terms(mpo, site, 1), mpo->w[site], wo, false);
  std::vector<bool> cov(wo, false);
  env_left_terms(c, prec, P, wo, mpo->d, site_ops(mpo, sprec, site), chi_l, chi_r, Lin, A, Lout, true, cov, "envL");
}

// right update across `site`: Rout[w_s][chi_l][chi_l] (transposed) from Rin[w_{s+1}][chi_r][chi_r] (transposed)
static void env_right(tn_ctx* c, const tn_mpo* mpo, int site, int prec, int chi_l, int chi_r,
                      const std::vector<const void*>& Rin, const cf64* A, void* Rout) {
  const int sprec = prec == PREC_FP64 ? PREC_FP64 : PREC_FP32;
  const size_t eb = elem_bytes(sprec);
  const int d = mpo->d, wo = mpo->w[site];
  const size_t nel = (size_t)chi_l * d * chi_r;
  const void* AP = stage_A(c, prec, A, nel, "envR:A");
  auto terms = window_terms(mpo, site, 1);
  for (auto& t : terms) std::swap(t.l, t.n);
  Plan P = build_plan(terms, mpo->w[site + 1], wo, false);
  std::vector<const void*> Rp;
  mixed_envs(c, sprec, P.L, Rin, (int64_t)chi_r * chi_r, Rp, "envR");
  char* Z = (char*)ws_get(c, "envR:Z", std::max<size_t>(1, P.L.size()) * nel * eb);
  char* T = (char*)ws_get(c, "envR:T", std::max<size_t>(1, P.T.size()) * nel * eb);
  std::vector<GemmJob> jobs;
  std::vector<GemmSeg> segs;
  for (size_t i = 0; i < P.L.size(); ++i) {
    segs.push_back({AP, Rp[i], chi_r, chi_r, chi_r, 0});
    jobs.push_back({Z + i * nel * eb, chi_r, chi_l * d, chi_r, (int)segs.size() - 1, 1});
  }
  gemm_batch(c, prec, 0, 0, jobs, segs, chi_l * d, chi_r, "envR:g1");
  run_ops(c, sprec, site_ops(mpo, sprec, site), P, Z, T, nel, chi_l, d, chi_r, "envR");
  jobs.clear(); segs.clear();
  std::vector<bool> cov(wo, false);
  for (auto& R : P.R) {
    const int ch = R.env[0].first;
    cov[ch] = true;
    const void* src = R.kind == 0 ? (const void*)(Z + (size_t)R.idx * nel * eb) : (const void*)(T + (size_t)R.idx * nel * eb);
    segs.push_back({src, AP, (int64_t)d * chi_r, (int64_t)d * chi_r, d * chi_r, 0});
    jobs.push_back({(char*)Rout + (size_t)ch * chi_l * chi_l * eb, chi_l, chi_l, chi_l, (int)segs.size() - 1, 1});
  }
  gemm_batch(c, prec, 0, 1, jobs, segs, chi_l, chi_l, "envR:g2");
  zero_channels(c, sprec, Rout, wo, (int64_t)chi_l * chi_l, cov);
}

// ------------------------------------------------------------------ environment cache on the MPS
static void* env_buf(tn_mps* m, bool left, int t, size_t bytes) {
  auto& v = left ? m->L : m->Rt;
  auto& cap = left ? m->Lcap : m->Rcap;
  if (cap[t] >= bytes && v[t]) return v[t];
  if (v[t]) {
    HIPCHK(hipStreamSynchronize(m->ctx->stream));
    dev_free(m->ctx, v[t]);
    v[t] = nullptr;
    (left ? m->Lok : m->Rok)[t] = false;  // a failed reallocation must not leave a valid flag
  }
  v[t] = dev_alloc(m->ctx, bytes);
  cap[t] = bytes;
  return v[t];
}
static std::vector<const void*> env_ptrs(tn_mps* m, const tn_mpo* mpo, bool left, int t, int prec) {
  const size_t eb = elem_bytes(prec == PREC_FP64 ? PREC_FP64 : PREC_FP32);
  const int chi = m->dims[t];
  std::vector<const void*> p(mpo->w[t]);
  char* base = (char*)(left ? m->L[t] : m->Rt[t]);
  for (int i = 0; i < mpo->w[t]; ++i) p[i] = base + (size_t)i * chi * chi * eb;
  return p;
}
static void set_boundary(tn_mps* m, bool left, int t, int prec) {
  void* p = env_buf(m, left, t, 256);
  HIPCHK(launch_set_one(p, prec == PREC_FP64 ? PREC_FP64 : PREC_FP32, m->ctx->stream));
  (left ? m->Lok : m->Rok)[t] = true;
}
static void update_left_env(tn_mps* m, const tn_mpo* mpo, int site, int prec, double* flops) {
  const size_t eb = elem_bytes(prec == PREC_FP64 ? PREC_FP64 : PREC_FP32);
  const int cl = m->dims[site], cr = m->dims[site + 1];
  void* out = env_buf(m, true, site + 1, (size_t)mpo->w[site + 1] * cr * cr * eb);
  env_left(m->ctx, mpo, site, prec, cl, cr, env_ptrs(m, mpo, true, site, prec), m->A[site], out);
  m->Lok[site + 1] = true;
  if (flops) *flops += env_flops_formula(mpo, site, cl, cr);
}
static void update_right_env(tn_mps* m, const tn_mpo* mpo, int site, int prec, double* flops) {
  const size_t eb = elem_bytes(prec == PREC_FP64 ? PREC_FP64 : PREC_FP32);
  const int cl = m->dims[site], cr = m->dims[site + 1];
  void* out = env_buf(m, false, site, (size_t)mpo->w[site] * cl * cl * eb);
  env_right(m->ctx, mpo, site, prec, cl, cr, env_ptrs(m, mpo, false, site + 1, prec), m->A[site], out);
  m->Rok[site] = true;
  if (flops) *flops += env_flops_formula(mpo, site, cl, cr);
}

// ------------------------------------------------------------------ canonical form
static void canonicalize(tn_ctx* c, tn_mps* m) {
  const int N = m->N, d = m->d;
  for (int s = N - 1; s >= 1; --s) {
    const int cl = m->dims[s], cr = m->dims[s + 1];
    const int mm = cl, nn = d * cr;
    cf64* left = wsT<cf64>(c, "can:L", (size_t)mm * std::min(mm, nn));
    cf64* right = wsT<cf64>(c, "can:R", (size_t)std::min(mm, nn) * nn);
    TruncOut t = truncate_dev(c, mm, nn, m->A[s], 1 << 30, 0.0, -1, left, right);
    const int k = t.k;
    m->ensure_site(s, (size_t)k * nn);
    HIPCHK(hipMemcpyAsync(m->A[s], right, (size_t)k * nn * sizeof(cf64), hipMemcpyDeviceToDevice, c->stream));
    // A_{s-1} <- A_{s-1} * left   ((chi_{s-1} d) x cl) * (cl x k)
    const int pl = m->dims[s - 1];
    cf64* tmp = wsT<cf64>(c, "can:T", (size_t)pl * d * k);
    gemm1(c, PREC_FP64, 0, 0, tmp, k, pl * d, k, m->A[s - 1], cl, left, k, cl, 0, "can:g");
    m->ensure_site(s - 1, (size_t)pl * d * k);
    HIPCHK(hipMemcpyAsync(m->A[s - 1], tmp, (size_t)pl * d * k * sizeof(cf64), hipMemcpyDeviceToDevice, c->stream));
    m->dims[s] = k;
  }
  const int n0 = m->dims[0] * d * m->dims[1];
  const double nr = dev_norm2(c, m->A[0], n0);
  if (!(nr > 0.0) || !std::isfinite(nr)) TN_THROW(TN_ENUMERIC, "MPS has zero or non-finite norm");
  HIPCHK(launch_scale_host(m->A[0], m->A[0], 1.0 / std::sqrt(nr), n0, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  m->center = 0;
  for (size_t i = 0; i < m->Lok.size(); ++i) { m->Lok[i] = false; m->Rok[i] = false; }
  m->env_mpo = nullptr;
}

static void ensure_right_envs(tn_mps* m, const tn_mpo* mpo, int prec, double* flops) {
  const bool valid = m->env_mpo == mpo && m->env_prec == prec && m->env_version == mpo->version;
  if (!valid) for (size_t i = 0; i < m->Rok.size(); ++i) { m->Rok[i] = false; m->Lok[i] = false; }
  set_boundary(m, false, m->N, prec);
  set_boundary(m, true, 0, prec);
  for (int s = m->N - 1; s >= 1; --s)
    if (!m->Rok[s]) update_right_env(m, mpo, s, prec, flops);
  m->env_mpo = mpo;
  m->env_prec = prec;
  m->env_version = mpo->version;
}

// ------------------------------------------------------------------ LBO on the centre site
static double lbo_site(tn_ctx* c, tn_mpo* mpo, tn_mps* m, int s, const tn_sweep_opts& o, int prec, int64_t* mv) {
  hipStream_t st = c->stream;
  const int D = mpo->D_raw, d = mpo->d;
  const int cl = m->dims[s], cr = m->dims[s + 1];
  const size_t nraw = (size_t)cl * D * cr;
  cf64* B = wsT<cf64>(c, "lbo:B", nraw);
  // B[a] = W_s * A_s[a]
  {
    std::vector<GemmJob> jobs;
    std::vector<GemmSeg> segs;
    for (int a = 0; a < cl; ++a) {
      segs.push_back({mpo->d_iso + (size_t)s * D * d, m->A[s] + (size_t)a * d * cr, d, cr, d, 0});
      jobs.push_back({B + (size_t)a * D * cr, cr, D, cr, a, 1});
    }
    gemm_batch(c, PREC_FP64, 0, 0, jobs, segs, D, cr, "lbo:g0");
  }
  // raw single-site solve
  WindowOp op;
  op.setup(c, mpo, s, 1, prec, cl, cr, env_ptrs(m, mpo, true, s, prec), env_ptrs(m, mpo, false, s + 1, prec), true,
           "lbo");
  LzResult lz = lanczos(c, [&](const cf64* x, cf64* y) { op.apply(x, y); }, B, (int64_t)nraw, o.tol, o.krylov_max,
                        o.lbo_matvecs > 0 ? o.lbo_matvecs : o.max_matvecs, matvec_unit(prec));
  c->lz_iters += lz.matvecs;
  c->lz_full += lz.full_passes;
  if (mv) *mv += lz.matvecs;
  // rho = sum_a B[a] B[a]^dag (D x D): split over a into partial products,
  // then a fixed-order reduction
  cf64* rho = wsT<cf64>(c, "lbo:rho", (size_t)D * D);
  {
    const int np = std::max(1, std::min(cl, 64));
    cf64* parts = wsT<cf64>(c, "lbo:rhop", (size_t)np * D * D);
    std::vector<GemmJob> jobs;
    std::vector<GemmSeg> segs;
    for (int a = 0; a < cl; ++a) segs.push_back({B + (size_t)a * D * cr, B + (size_t)a * D * cr, cr, cr, cr, 0});
    for (int g = 0; g < np; ++g) {
      const int a0 = (int)((int64_t)cl * g / np), a1 = (int)((int64_t)cl * (g + 1) / np);
      jobs.push_back({parts + (size_t)g * D * D, D, D, D, a0, a1 - a0});
    }
    gemm_batch(c, PREC_FP64, 0, 1, jobs, segs, D, D, "lbo:g1");
    HIPCHK(launch_reduce_partials(rho, PREC_FP64, parts, np, (int64_t)D * D, st));
  }
  double* ev = wsT<double>(c, "lbo:ev", D);
  cf64* Zr = wsT<cf64>(c, "lbo:Z", (size_t)D * D);
  HIPCHK(launch_jacobi(rho, 0, D, 1, ev, Zr, 0, 1, st));
  std::vector<double> evh(D);
  std::vector<cf64> Zh((size_t)D * D);
  download(c, evh.data(), ev, D * sizeof(double));
  download(c, Zh.data(), Zr, Zh.size() * sizeof(cf64));
  double tot = 0.0, kept = 0.0;
  for (int i = 0; i < D; ++i) { tot += std::max(0.0, evh[i]); if (i < d) kept += std::max(0.0, evh[i]); }
  const double disc = tot > 0 ? (tot - kept) / tot : 0.0;
  // new isometry: top-d eigenvectors, phase fixed so the largest-modulus entry is real positive
  std::vector<cd> Wn((size_t)D * d);
  for (int j = 0; j < d; ++j) {
    int im = 0;
    double best = -1;
    for (int i = 0; i < D; ++i) {
      const double a = Zh[(size_t)i * D + j].x * Zh[(size_t)i * D + j].x + Zh[(size_t)i * D + j].y * Zh[(size_t)i * D + j].y;
      if (a > best + 1e-14) { best = a; im = i; }
    }
    const cd z(Zh[(size_t)im * D + j].x, Zh[(size_t)im * D + j].y);
    const cd ph = std::abs(z) > 0 ? std::conj(z) / std::abs(z) : cd(1.0);
    for (int i = 0; i < D; ++i) Wn[(size_t)i * d + j] = cd(Zh[(size_t)i * D + j].x, Zh[(size_t)i * D + j].y) * ph;
  }
  mpo->iso[s] = Wn;
  if (mpo->plbo) mpo->iso_stale[s] = true;  // the Fock image follows the new isometry
  // re-project the local operators and upload (ops, raw ops, isometry)
  {
    const auto& raw = mpo->raw_ops[s];
    std::vector<cd> out((size_t)NOPS * d * d, 0.0);
    for (int o2 = 0; o2 < NOPS; ++o2)
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          cd acc = 0.0;
          for (int i = 0; i < D; ++i) {
            const cd wi = std::conj(Wn[(size_t)i * d + a]);
            if (wi == 0.0) continue;
            cd t = 0.0;
            for (int j = 0; j < D; ++j) t += raw[(size_t)o2 * D * D + (size_t)i * D + j] * Wn[(size_t)j * d + b];
            acc += wi * t;
          }
          out[(size_t)o2 * d * d + (size_t)a * d + b] = acc;
        }
    mpo->loc_ops[s] = out;
    HIPCHK(hipStreamSynchronize(st));
    mpo->upload_site(s);
    mpo->version++;
  }
  // A_s = W^dag B, renormalised
  {
    std::vector<GemmJob> jobs;
    std::vector<GemmSeg> segs;
    for (int a = 0; a < cl; ++a) {
      segs.push_back({mpo->d_iso + (size_t)s * D * d, B + (size_t)a * D * cr, d, cr, D, 0});
      jobs.push_back({m->A[s] + (size_t)a * d * cr, cr, d, cr, a, 1});
    }
    gemm_batch(c, PREC_FP64, 1, 0, jobs, segs, d, cr, "lbo:g2");
    const double nr = dev_norm2(c, m->A[s], (int64_t)cl * d * cr);
    if (!(nr > 0.0) || !std::isfinite(nr)) TN_THROW(TN_ENUMERIC, "LBO projection gave a zero tensor");
    HIPCHK(launch_scale_host(m->A[s], m->A[s], 1.0 / std::sqrt(nr), (int64_t)cl * d * cr, st));
  }
  return disc;
}

// ------------------------------------------------------------------ gate-parameterised basis (Sec. III.B)
// loc_ops[s] = W^dag raw W for every operator slot, W = iso[s] (D_raw x d)
static void project_site(tn_mpo* mpo, int s) {
  const int D = mpo->D_raw, d = mpo->d;
  const auto& raw = mpo->raw_ops[s];
  const auto& W = mpo->iso[s];
  std::vector<cd> out((size_t)NOPS * d * d, 0.0), t((size_t)D * d);
  for (int o = 0; o < NOPS; ++o) {
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < d; ++j) {
        cd a = 0.0;
        for (int k = 0; k < D; ++k) a += raw[(size_t)o * D * D + (size_t)i * D + k] * W[(size_t)k * d + j];
        t[(size_t)i * d + j] = a;
      }
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        cd a = 0.0;
        for (int k = 0; k < D; ++k) a += std::conj(W[(size_t)k * d + i]) * t[(size_t)k * d + j];
        out[(size_t)o * d * d + (size_t)i * d + j] = a;
      }
  }
  mpo->loc_ops[s] = out;
}

static void plbo_set_site(tn_mpo* mpo, int s) {
  const int N = mpo->N;
  const size_t ss = (size_t)s * N + s;
  if (mpo->plbo_lin) {
    plbo_local_ops(mpo->D_raw, mpo->pp[s].data(), mpo->alpha[ss], mpo->beta[ss], mpo->gamma[ss], mpo->raw_ops[s],
                   nullptr);
    project_site(mpo, s);
  } else {
    plbo_local_ops(mpo->d, mpo->pp[s].data(), mpo->alpha[ss], mpo->beta[ss], mpo->gamma[ss], mpo->loc_ops[s],
                   nullptr);
  }
  mpo->iso_stale[s] = true;
  mpo->upload_site(s);
  mpo->version++;
}

// The Fock image U[:D, :d] of every basis changed since the last call (a
// cache of the parameters, recomputed before photon-number observables).
void plbo_sync_iso(const tn_mpo* cmpo) {
  tn_mpo* mpo = const_cast<tn_mpo*>(cmpo);
  if (!mpo->plbo) return;
  const int D = mpo->D_raw, d = mpo->d;
  const int levels = std::max(D, d) + 192;
  for (int s = 0; s < mpo->N; ++s) {
    if (!mpo->iso_stale[s]) continue;
    if (mpo->plbo_lin) {
      // Fock image of the raw basis (D x D) times the linear isometry W
      std::vector<cd> full;
      plbo_fock_isometry(D, D, mpo->pp[s].data(), levels, full);
      auto& F = mpo->fock[s];
      F.assign((size_t)D * d, 0.0);
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < d; ++j) {
          cd a = 0.0;
          for (int k = 0; k < D; ++k) a += full[(size_t)i * D + k] * mpo->iso[s][(size_t)k * d + j];
          F[(size_t)i * d + j] = a;
        }
      std::vector<cf64> h(F.size());
      for (size_t i = 0; i < F.size(); ++i) h[i] = make_double2(F[i].real(), F[i].imag());
      HIPCHK(hipMemcpy(mpo->d_fock + (size_t)s * D * d, h.data(), h.size() * sizeof(cf64), hipMemcpyHostToDevice));
    } else {
      plbo_fock_isometry(D, d, mpo->pp[s].data(), levels, mpo->iso[s]);
      mpo->upload_site(s);
    }
    mpo->iso_stale[s] = false;
  }
}

// G[k][n'][n] = dE/dO_k[n'][n], k = 0..NOPS (slot 0: identity), of the single-
// site window at s for the tensor x (chi_l x d x chi_r): E = <x|H_eff|x> is
// sum_k <G_k, O_k> with O_0 = I.  From the window operator's own plan: each
// right entry r adds src_r R_r with src_r = Y_i (identity) or
// sum_t c_t O_{a_t} Y_{i_t}, so G_{a_t} += c_t sum_{a,b} conj(U_r[a][n'][b]) Y_{i_t}[a][n][b]
// with U_r = x R_r^H.
static void plbo_slot_envs(tn_ctx* c, const tn_mpo* mpo, tn_mps* m, int s, int prec, const cf64* x,
                           std::vector<cd>& G) {
  const int d = mpo->d, cl = m->dims[s], cr = m->dims[s + 1];
  const int sprec = prec == PREC_FP64 ? PREC_FP64 : PREC_FP32;
  const size_t eb = elem_bytes(sprec);
  WindowOp op;
  op.setup(c, mpo, s, 1, prec, cl, cr, env_ptrs(m, mpo, true, s, prec), env_ptrs(m, mpo, false, s + 1, prec), false,
           "pg");
  op.apply_left(x);
  const size_t n = op.n;
  const int nR = (int)op.plan.R.size();
  char* U = (char*)ws_get(c, "pg:U", (size_t)std::max(1, nR) * n * eb);
  std::vector<GemmJob> jobs;
  std::vector<GemmSeg> segs;
  for (int r = 0; r < nR; ++r) {
    segs.push_back({op.xin, op.rptr[r], cr, cr, cr, 0});
    jobs.push_back({U + (size_t)r * n * eb, cr, cl * d, cr, r, 1});
  }
  gemm_batch(c, prec, 0, 1, jobs, segs, cl * d, cr, "pg:g");
  std::vector<SlotJob> sj;
  std::vector<std::pair<int, double>> meta;
  for (int r = 0; r < nR; ++r) {
    const auto& R = op.plan.R[r];
    const char* Ur = U + (size_t)r * n * eb;
    if (R.kind == 0) {
      sj.push_back({Ur, op.ybuf + (size_t)R.idx * n * eb});
      meta.push_back({0, 1.0});
    } else {
      for (const auto& t : op.plan.T[R.idx].terms) {
        if (t.b != 0) TN_THROW(TN_EINVAL, "single-site plan with a second leg");
        sj.push_back({Ur, op.ybuf + (size_t)t.ych * n * eb});
        meta.push_back({t.a, t.c});
      }
    }
  }
  G.assign((size_t)(NOPS + 1) * d * d, 0.0);
  if (sj.empty()) return;
  SlotJob* dj = wsT<SlotJob>(c, "pg:jobs", sj.size());
  cf64* part = wsT<cf64>(c, "pg:part", sj.size() * d * d);
  upload(c, dj, sj.data(), sj.size() * sizeof(SlotJob));
  HIPCHK(launch_slot_gram(sprec, dj, (int)sj.size(), cl, d, cr, part, c->stream));
  std::vector<cf64> h(sj.size() * d * d);
  download(c, h.data(), part, h.size() * sizeof(cf64));
  for (size_t j = 0; j < sj.size(); ++j)
    for (int e = 0; e < d * d; ++e)
      G[(size_t)meta[j].first * d * d + e] += meta[j].second * cd(h[j * d * d + e].x, h[j * d * d + e].y);
}

static PlboSite plbo_site_of(const tn_mpo* mpo, int s, const std::vector<cd>& G) {
  const size_t ss = (size_t)s * mpo->N + s;
  PlboSite S{mpo->d, mpo->alpha[ss], mpo->beta[ss], mpo->gamma[ss], &G};
  if (mpo->plbo_lin) {
    S.D = mpo->D_raw;
    S.W = &mpo->iso[s];
  }
  return S;
}

struct PlboStep {
  double e0 = 0.0, e1 = 0.0;  // site energy before and after the parameter steps
  int64_t mv = 0;
};

// One visit of site s (the orthogonality centre): optional single-site Lanczos
// in the current basis, slot environments, then Adam (Kingma & Ba) steps on
// the site's parameters with the tensor held fixed (Sec. III.B: per-site
// gradient optimisation sweeping like single-site DMRG).
static PlboStep plbo_site(tn_ctx* c, tn_mpo* mpo, tn_mps* m, int s, const tn_sweep_opts& o, const tn_plbo_opts& po) {
  PlboStep R;
  const int d = mpo->d, cl = m->dims[s], cr = m->dims[s + 1];
  const int64_t n = (int64_t)cl * d * cr;
  if (po.matvecs > 0) {
    WindowOp op;
    op.setup(c, mpo, s, 1, o.precision, cl, cr, env_ptrs(m, mpo, true, s, o.precision),
             env_ptrs(m, mpo, false, s + 1, o.precision), false, "plz");
    LzResult lz = lanczos(c, [&](const cf64* x, cf64* y) { op.apply(x, y); }, m->A[s], n, o.tol, o.krylov_max,
                          po.matvecs, matvec_unit(o.precision));
    c->lz_iters += lz.matvecs;
    c->lz_full += lz.full_passes;
    R.mv = lz.matvecs;
  }
  const double nr = dev_norm2(c, m->A[s], n);
  if (!(nr > 0.0) || !std::isfinite(nr)) TN_THROW(TN_ENUMERIC, "zero or non-finite centre tensor");
  HIPCHK(launch_scale_host(m->A[s], m->A[s], 1.0 / std::sqrt(nr), n, c->stream));
  std::vector<cd> G;
  plbo_slot_envs(c, mpo, m, s, o.precision, m->A[s], G);
  auto& p = mpo->pp[s];
  const PlboSite S = plbo_site_of(mpo, s, G);
  R.e0 = plbo_site_energy(S, p.data(), nullptr);
  plbo_optimise(S, po, p.data(), mpo->pm[s].data(), mpo->pv[s].data(), &mpo->pt[s]);
  R.e1 = plbo_site_energy(S, p.data(), nullptr);
  for (int j = 0; j < TN_PLBO_NPARAM; ++j)
    if (!std::isfinite(p[j])) TN_THROW(TN_ENUMERIC, "non-finite basis parameter");
  if (po.steps > 0) plbo_set_site(mpo, s);
  return R;
}

static void check_plbo_opts(const tn_plbo_opts* po) {
  if (!po) TN_THROW(TN_EINVAL, "null pLBO options");
  if (po->steps < 0 || po->matvecs < 0) TN_THROW(TN_EINVAL, "steps and matvecs must be >= 0");
  if (!(po->lr > 0.0) || !std::isfinite(po->lr)) TN_THROW(TN_EINVAL, "lr must be positive");
  if (!(po->beta1 >= 0.0 && po->beta1 < 1.0) || !(po->beta2 >= 0.0 && po->beta2 < 1.0))
    TN_THROW(TN_EINVAL, "beta1 and beta2 must be in [0, 1)");
  if (!(po->eps > 0.0)) TN_THROW(TN_EINVAL, "eps must be positive");
  if (po->optimizer != TN_PLBO_ADAM && po->optimizer != TN_PLBO_LBFGS) TN_THROW(TN_EINVAL, "unknown optimizer");
}

// ------------------------------------------------------------------ one two-site update
struct StepStats {
  double disc = 0, lam = 0, t_heff = 0, t_lz = 0, t_svd = 0, t_env = 0, heff_flops = 0, env_flops = 0, svd_flops = 0;
  int64_t mv = 0;
  bool conv = true;
};

static StepStats two_site(tn_ctx* c, tn_mpo* mpo, tn_mps* m, int s, int dir, const tn_sweep_opts& o) {
  StepStats S;
  hipStream_t st = c->stream;
  const int d = mpo->d, prec = o.precision;
  const int cl = m->dims[s], cm = m->dims[s + 1], cr = m->dims[s + 2];
  const size_t nth = (size_t)cl * d * d * cr;
  cf64* th = wsT<cf64>(c, "ts:theta", nth);
  gemm1(c, PREC_FP64, 0, 0, th, d * cr, cl * d, d * cr, m->A[s], cm, m->A[s + 1], d * cr, cm, 0, "ts:g0");
  const double t0 = wall();
  WindowOp op;
  op.setup(c, mpo, s, 2, prec, cl, cr, env_ptrs(m, mpo, true, s, prec), env_ptrs(m, mpo, false, s + 2, prec), false,
           "heff");
  LzResult lz = lanczos(c, [&](const cf64* x, cf64* y) { op.apply(x, y); }, th, (int64_t)nth, o.tol, o.krylov_max,
                        o.max_matvecs, matvec_unit(prec));
  c->lz_iters += lz.matvecs;
  c->lz_full += lz.full_passes;
  const double t1 = wall();
  S.mv = lz.matvecs;
  S.conv = lz.converged;
  S.lam = lz.lambda;
  S.t_heff = lz.t_mv;
  S.t_lz = (t1 - t0) - lz.t_mv;
  S.heff_flops = matvec_flops_formula(mpo, s, cl, cr) * lz.matvecs;
  // truncation
  const int mm = cl * d, nn = d * cr;
  const int kmax = std::max(1, std::min(o.chi_max, std::min(mm, nn)));
  cf64* left = wsT<cf64>(c, "ts:left", (size_t)mm * kmax);
  cf64* right = wsT<cf64>(c, "ts:right", (size_t)kmax * nn);
  TruncOut t = truncate_dev(c, mm, nn, th, o.chi_max, o.sigma_cut, dir, left, right);
  const double t2 = wall();
  S.t_svd = t2 - t1;
  S.svd_flops = t.flops;
  S.disc = t.disc;
  const int k = t.k;
  m->ensure_site(s, (size_t)mm * k);
  m->ensure_site(s + 1, (size_t)k * nn);
  HIPCHK(hipMemcpyAsync(m->A[s], left, (size_t)mm * k * sizeof(cf64), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(m->A[s + 1], right, (size_t)k * nn * sizeof(cf64), hipMemcpyDeviceToDevice, st));
  m->dims[s + 1] = k;
  // non-finite guard on the new tensors
  int* flag = wsT<int>(c, "ts:flag", 1);
  HIPCHK(launch_fill_int(flag, 0, 1, st));
  HIPCHK(launch_finite_check(m->A[s], (int64_t)mm * k, flag, st));
  HIPCHK(launch_finite_check(m->A[s + 1], (int64_t)k * nn, flag, st));
  int fl = 0;
  download(c, &fl, flag, sizeof(int));
  if (fl) TN_THROW(TN_ENUMERIC, "non-finite tensor after truncation");
  if (dir > 0) update_left_env(m, mpo, s, prec, &S.env_flops);
  else update_right_env(m, mpo, s + 1, prec, &S.env_flops);
  HIPCHK(hipStreamSynchronize(st));
  S.t_env = wall() - t2;
  return S;
}

// ------------------------------------------------------------------ energy (FP64)
static double energy_fp64(tn_ctx* c, const tn_mpo* mpo, const tn_mps* m, double* norm2) {
  const int N = m->N, d = m->d;
  hipStream_t st = c->stream;
  size_t maxw = 1;
  for (int t = 0; t <= N; ++t) maxw = std::max(maxw, (size_t)mpo->w[t] * m->dims[t] * m->dims[t]);
  cf64* La = wsT<cf64>(c, "en:La", maxw);
  cf64* Lb = wsT<cf64>(c, "en:Lb", maxw);
  HIPCHK(launch_set_one(La, PREC_FP64, st));
  for (int s = 0; s < N; ++s) {
    const int cl = m->dims[s], cr = m->dims[s + 1];
    std::vector<const void*> lin(mpo->w[s]);
    for (int i = 0; i < mpo->w[s]; ++i) lin[i] = La + (size_t)i * cl * cl;
    env_left(c, mpo, s, PREC_FP64, cl, cr, lin, m->A[s], Lb);
    std::swap(La, Lb);
  }
  cf64 e;
  download(c, &e, La, sizeof(cf64));
  // norm: E_{s+1} = A_s^dag (E_s A_s)
  cf64* Ea = wsT<cf64>(c, "en:Ea", maxw);
  cf64* Eb = wsT<cf64>(c, "en:Eb", maxw);
  cf64* Y = wsT<cf64>(c, "en:Y", [&] { size_t mx = 1; for (int s = 0; s < N; ++s) mx = std::max(mx, (size_t)m->dims[s] * d * m->dims[s + 1]); return mx; }());
  HIPCHK(launch_set_one(Ea, PREC_FP64, st));
  for (int s = 0; s < N; ++s) {
    const int cl = m->dims[s], cr = m->dims[s + 1];
    gemm1(c, PREC_FP64, 0, 0, Y, d * cr, cl, d * cr, Ea, cl, m->A[s], d * cr, cl, 0, "en:g0");
    gemm1(c, PREC_FP64, 1, 0, Eb, cr, cr, cr, m->A[s], cr, Y, cr, cl * d, 0, "en:g1");
    std::swap(Ea, Eb);
  }
  cf64 nn;
  download(c, &nn, Ea, sizeof(cf64));
  if (norm2) *norm2 = nn.x;
  if (!(nn.x > 0.0) || !std::isfinite(e.x)) TN_THROW(TN_ENUMERIC, "non-finite energy or zero norm");
  return e.x / nn.x;
}

// ------------------------------------------------------------------ <(PHP)^2> (FP64)
// Two-layer left environments L[(u, v)][chi][chi], u and v the bond channels of
// the two copies of the MPO.  Each pair of core entries (u -> u', op_a) and
// (v -> v', op_b) of a site is one single-site term (u, v) -> (u', v') whose
// operator is the product Q_ab = W^dag R_a R_b W of the raw-box operators
// (R_0 = 1): (PHP)^2 is taken in the raw box, so with a local basis the
// projector W W^dag is not inserted between the two copies.  The term lists go
// through the same planner and batched GEMMs as the one-layer update; output
// channels are processed in groups of first-layer channels sized to a
// workspace budget.
static void product_ops(const tn_mpo* mpo, int s, std::vector<cd>& Q) {
  const int D = mpo->D_raw, d = mpo->d;
  if (mpo->plbo && !mpo->plbo_lin) {
    // gate-parameterised basis: O_a O_b of the exact operator blocks at d + 8
    // levels (O_b moves a state below d by at most four levels, so every
    // intermediate state is inside), truncated to d
    const int e = d + 8, N = mpo->N;
    const size_t ss = (size_t)s * N + s, ee = (size_t)e * e;
    std::vector<cd> big;
    plbo_local_ops(e, mpo->pp[s].data(), mpo->alpha[ss], mpo->beta[ss], mpo->gamma[ss], big, nullptr);
    auto B = [&](int a, int i, int j) -> cd {
      if (a == 0) return i == j ? cd(1.0) : cd(0.0);
      return big[(size_t)(a - 1) * ee + (size_t)i * e + j];
    };
    Q.assign((size_t)(NOPS + 1) * (NOPS + 1) * d * d, 0.0);
    for (int a = 0; a <= NOPS; ++a)
      for (int b = 0; b <= NOPS; ++b)
        for (int i = 0; i < d; ++i)
          for (int j = 0; j < d; ++j) {
            cd t = 0.0;
            for (int k = 0; k < e; ++k) t += B(a, i, k) * B(b, k, j);
            Q[((size_t)(a * (NOPS + 1) + b) * d + i) * d + j] = t;
          }
    return;
  }
  const auto& raw = mpo->raw_ops[s];
  const auto& W = mpo->iso[s];
  auto R = [&](int a, int i, int j) -> cd {
    if (a == 0) return i == j ? cd(1.0) : cd(0.0);
    return raw[(size_t)(a - 1) * D * D + (size_t)i * D + j];
  };
  Q.assign((size_t)(NOPS + 1) * (NOPS + 1) * d * d, 0.0);
  std::vector<cd> RW((size_t)D * d), RRW((size_t)D * d);
  for (int b = 0; b <= NOPS; ++b) {
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < d; ++j) {
        cd t = 0.0;
        for (int k = 0; k < D; ++k) t += R(b, i, k) * W[(size_t)k * d + j];
        RW[(size_t)i * d + j] = t;
      }
    for (int a = 0; a <= NOPS; ++a) {
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < d; ++j) {
          cd t = 0.0;
          for (int k = 0; k < D; ++k) t += R(a, i, k) * RW[(size_t)k * d + j];
          RRW[(size_t)i * d + j] = t;
        }
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          cd t = 0.0;
          for (int k = 0; k < D; ++k) t += std::conj(W[(size_t)k * d + i]) * RRW[(size_t)k * d + j];
          Q[((size_t)(a * (NOPS + 1) + b) * d + i) * d + j] = t;
        }
    }
  }
}

static double h2_fp64(tn_ctx* c, const tn_mpo* mpo, const tn_mps* m) {
  const int N = m->N, d = m->d;
  hipStream_t st = c->stream;
  size_t maxw = 1;
  for (int t = 0; t <= N; ++t) maxw = std::max(maxw, (size_t)mpo->w[t] * mpo->w[t] * m->dims[t] * m->dims[t]);
  cf64* La = wsT<cf64>(c, "h2:La", maxw);
  cf64* Lb = wsT<cf64>(c, "h2:Lb", maxw);
  cf64* Qd = wsT<cf64>(c, "h2:Q", (size_t)(NOPS + 1) * (NOPS + 1) * d * d);
  HIPCHK(launch_set_one(La, PREC_FP64, st));
  const size_t budget = (size_t)8 << 30;  // Y + T buffers per group
  std::vector<cd> Q;
  std::vector<cf64> Qh((size_t)(NOPS + 1) * (NOPS + 1) * d * d);
  for (int s = 0; s < N; ++s) {
    const int cl = m->dims[s], cr = m->dims[s + 1];
    const int wi = mpo->w[s], wo = mpo->w[s + 1];
    product_ops(mpo, s, Q);
    for (size_t i = 0; i < Q.size(); ++i) Qh[i] = make_double2(Q[i].real(), Q[i].imag());
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(Qd, Qh.data(), Qh.size() * sizeof(cf64), hipMemcpyHostToDevice));
    OpTable ops((NOPS + 1) * (NOPS + 1), nullptr);
    for (int k = 1; k < (NOPS + 1) * (NOPS + 1); ++k) ops[k] = Qd + (size_t)k * d * d;
    // terms grouped by the first layer's output channel
    std::vector<std::vector<Term2>> by_u(wo);
    for (const auto& e1 : mpo->entries[s])
      for (const auto& e2 : mpo->entries[s])
        for (int a = 0; a <= NOPS; ++a) {
          if (e1.c[a] == 0.0) continue;
          for (int b = 0; b <= NOPS; ++b) {
            if (e2.c[b] == 0.0) continue;
            by_u[e1.col].push_back({e1.row * wi + e2.row, e1.col * wo + e2.col, a * (NOPS + 1) + b, 0, e1.c[a] * e2.c[b]});
          }
        }
    std::vector<const void*> lin((size_t)wi * wi);
    for (size_t i = 0; i < lin.size(); ++i) lin[i] = La + i * cl * cl;
    std::vector<bool> cov((size_t)wo * wo, false);
    const size_t nel_b = (size_t)cl * d * cr * sizeof(cf64);
    // first-layer output channels [u0, u1) in one plan, halved while its buffers exceed the budget
    std::function<void(int, int)> run = [&](int u0, int u1) {
      std::vector<Term2> terms;
      for (int u = u0; u < u1; ++u) terms.insert(terms.end(), by_u[u].begin(), by_u[u].end());
      if (terms.empty()) return;
      Plan P = build_plan(terms, wi * wi, wo * wo, false);
      if (u1 - u0 > 1 && (P.L.size() + P.T.size()) * nel_b > budget) {
        run(u0, (u0 + u1) / 2);
        run((u0 + u1) / 2, u1);
        return;
      }
      env_left_terms(c, PREC_FP64, P, wo * wo, d, ops, cl, cr, lin, m->A[s], Lb, false, cov, "h2");
    };
    run(0, wo);
    zero_channels(c, PREC_FP64, Lb, wo * wo, (int64_t)cr * cr, cov);
    std::swap(La, Lb);
  }
  cf64 h;
  download(c, &h, La, sizeof(cf64));
  if (!std::isfinite(h.x)) TN_THROW(TN_ENUMERIC, "non-finite <H^2>");
  return h.x;
}

// ------------------------------------------------------------------ ABI
static void check_opts(const tn_sweep_opts* o) {
  if (!o) TN_THROW(TN_EINVAL, "null options");
  if (o->chi_max < 1) TN_THROW(TN_EINVAL, "chi_max must be >= 1");
  if (!(o->tol > 0.0)) TN_THROW(TN_EINVAL, "tol must be positive");
  if (o->krylov_max < 2 || o->krylov_max > 64) TN_THROW(TN_EINVAL, "krylov_max must be in [2, 64]");
  if (o->max_matvecs < 1) TN_THROW(TN_EINVAL, "max_matvecs must be >= 1");
  if (o->lbo_matvecs < 0) TN_THROW(TN_EINVAL, "lbo_matvecs must be >= 0");
  if (o->precision < 0 || o->precision > 2) TN_THROW(TN_EINVAL, "unknown precision");
  if (!(o->sigma_cut >= 0.0) || o->sigma_cut >= 1.0) TN_THROW(TN_EINVAL, "sigma_cut must be in [0, 1)");
}

static void check_pair(const tn_mpo* mpo, const tn_mps* m) {
  if (mpo->N != m->N) TN_THROW(TN_EINVAL, "MPO and MPS have different N");
  if (mpo->d != m->d) TN_THROW(TN_EINVAL, "MPO and MPS have different local dimension");
}

static void sweep_impl(tn_ctx* c, tn_mpo* mpo, tn_mps* m, const tn_sweep_opts& o, tn_sweep_stats* out,
                       const tn_plbo_opts* po = nullptr, double* plbo_gain = nullptr) {
  const double tstart = wall();
  tn_sweep_stats S{};
  S.energy = NAN;
  if (m->N < 2) TN_THROW(TN_EINVAL, "a sweep needs N >= 2");
  if (o.lbo && mpo->plbo && !mpo->plbo_lin)
    TN_THROW(TN_ESTATE, "linear LBO on a gate-parameterised basis needs tn_plbo_linear first");
  if (m->center != 0) canonicalize(c, m);
  ensure_right_envs(m, mpo, o.precision, &S.env_flops);
  const int N = m->N;
  auto acc = [&](const StepStats& t) {
    S.max_discarded = std::max(S.max_discarded, t.disc);
    S.sum_discarded += t.disc;
    S.matvecs += t.mv;
    S.unconverged_steps += t.conv ? 0 : 1;
    S.heff_flops += t.heff_flops;
    S.env_flops += t.env_flops;
    S.t_heff += t.t_heff;
    S.t_lanczos += t.t_lz;
    S.t_svd += t.t_svd;
    S.svd_flops += t.svd_flops;
    S.t_env += t.t_env;
    S.last_eigenvalue = t.lam;
  };
  auto plbo_visit = [&](int site) {
    const double t0 = wall();
    const PlboStep P = plbo_site(c, mpo, m, site, o, *po);
    S.matvecs += P.mv;
    if (plbo_gain) *plbo_gain += P.e0 - P.e1;
    S.t_lbo += wall() - t0;
  };
  for (int s = 0; s <= N - 2; ++s) {
    if (po) plbo_visit(s);
    if (o.lbo) { const double t0 = wall(); S.lbo_discarded += lbo_site(c, mpo, m, s, o, o.precision, &S.matvecs); S.t_lbo += wall() - t0; }
    acc(two_site(c, mpo, m, s, +1, o));
    m->center = s + 1;
  }
  for (int s = N - 2; s >= 0; --s) {
    if (po) plbo_visit(s + 1);
    if (o.lbo) { const double t0 = wall(); S.lbo_discarded += lbo_site(c, mpo, m, s + 1, o, o.precision, &S.matvecs); S.t_lbo += wall() - t0; }
    acc(two_site(c, mpo, m, s, -1, o));
    m->center = s;
  }
  m->env_mpo = mpo;
  m->env_prec = o.precision;
  m->env_version = mpo->version;
  for (int t = 1; t <= N; ++t) m->Lok[t] = false;
  m->sweeps++;
  if (o.compute_energy) {
    const double t0 = wall();
    S.energy = energy_fp64(c, mpo, m, nullptr);
    S.t_energy = wall() - t0;
  }
  S.t_total = wall() - tstart;
  if (out) *out = S;
}

extern "C" tn_status tn_dmrg_sweep(tn_ctx* c, tn_mpo* mpo, tn_mps* m, const tn_sweep_opts* o, tn_sweep_stats* out) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!mpo || !m) TN_THROW(TN_EINVAL, "null handle");
  check_opts(o);
  check_pair(mpo, m);
  sweep_impl(c, mpo, m, *o, out);
  TN_GUARD_END(c)
}

extern "C" tn_status tn_dmrg_solve(tn_ctx* c, tn_mpo* mpo, tn_mps* m, const tn_solve_opts* so, tn_solve_result* out,
                                   double* etrace, double* ttrace) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!mpo || !m || !so) TN_THROW(TN_EINVAL, "null argument");
  if (so->max_sweeps < 1) TN_THROW(TN_EINVAL, "max_sweeps must be >= 1");
  if (so->bulk_precision < 0 || so->bulk_precision > 2) TN_THROW(TN_EINVAL, "unknown bulk precision");
  if (so->max_refine < 0) TN_THROW(TN_EINVAL, "max_refine must be >= 0");
  check_pair(mpo, m);
  tn_sweep_opts base = so->sweep;
  base.precision = so->bulk_precision;
  base.tol = so->bulk_tol;
  base.compute_energy = 1;
  check_opts(&base);
  if (!(so->refine_tol > 0.0)) TN_THROW(TN_EINVAL, "refine_tol must be positive");
  const double t0 = wall();
  tn_solve_result R{};
  R.t_target = NAN;
  R.energy = NAN;
  bool refining = so->bulk_precision == PREC_FP64;
  int rises = 0, refine_done = 0;
  double prev = NAN;
  for (int sw = 0; sw < so->max_sweeps; ++sw) {
    tn_sweep_opts o = base;
    const bool fp64 = refining || so->bulk_precision == PREC_FP64;
    o.precision = fp64 ? PREC_FP64 : so->bulk_precision;
    o.tol = (refining && so->bulk_precision != PREC_FP64) ? so->refine_tol : so->bulk_tol;
    o.lbo = (refining && so->bulk_precision != PREC_FP64) ? so->lbo_refine : so->lbo_bulk;
    tn_sweep_stats S{};
    sweep_impl(c, mpo, m, o, &S);
    R.sweeps++;
    if (refining && so->bulk_precision != PREC_FP64) { R.refine_sweeps++; refine_done++; }
    R.heff_flops += S.heff_flops;
    R.t_heff += S.t_heff;
    const double E = S.energy;
    const double el = wall() - t0;
    if (etrace) etrace[sw] = E;
    if (ttrace) ttrace[sw] = el;
    R.energy = E;
    if (E <= so->target) {
      if (std::isnan(R.t_target)) R.t_target = el;
      R.reached = 1;
      break;
    }
    const double dE = std::isnan(prev) ? INFINITY : E - prev;
    prev = E;
    if (fp64 && std::fabs(dE) < so->conv_tol * std::max(1.0, std::fabs(E))) break;
    if (!refining) {
      if (dE > 0) ++rises;
      if (std::fabs(dE) < so->switch_tol * std::max(1.0, std::fabs(E)) || rises >= 2) {
        refining = true;
        if (so->max_refine == 0) break;  // the bulk form has stagnated and no refinement is allowed
      }
    } else if (so->bulk_precision != PREC_FP64 && refine_done >= so->max_refine) {
      break;
    }
  }
  R.seconds = wall() - t0;
  if (out) *out = R;
  TN_GUARD_END(c)
}

extern "C" tn_status tn_mps_canonicalize(tn_ctx* c, tn_mps* m) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!m) TN_THROW(TN_EINVAL, "null handle");
  canonicalize(c, m);
  TN_GUARD_END(c)
}

extern "C" tn_status tn_energy(tn_ctx* c, const tn_mpo* mpo, const tn_mps* m, double* energy, double* norm2) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!mpo || !m || !energy) TN_THROW(TN_EINVAL, "null argument");
  check_pair(mpo, m);
  *energy = energy_fp64(c, mpo, m, norm2);
  TN_GUARD_END(c)
}

extern "C" tn_status tn_energy_variance(tn_ctx* c, const tn_mpo* mpo, const tn_mps* m, double* energy,
                                        double* h2, double* variance) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!mpo || !m || !energy || !variance) TN_THROW(TN_EINVAL, "null argument");
  check_pair(mpo, m);
  double n2 = 0.0;
  const double e = energy_fp64(c, mpo, m, &n2);
  const double q = h2_fp64(c, mpo, m) / n2;
  *energy = e;
  if (h2) *h2 = q;
  *variance = q - e * e;
  TN_GUARD_END(c)
}

extern "C" tn_status tn_lbo_step(tn_ctx* c, tn_mpo* mpo, tn_mps* m, int32_t site, const tn_sweep_opts* o,
                                 double* discarded) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!mpo || !m) TN_THROW(TN_EINVAL, "null handle");
  check_opts(o);
  check_pair(mpo, m);
  if (site < -1 || site >= m->N) TN_THROW(TN_EINVAL, "site out of range");
  if (site == -1) {
    tn_sweep_opts oo = *o;
    oo.lbo = 1;
    tn_sweep_stats S{};
    sweep_impl(c, mpo, m, oo, &S);
    if (discarded) *discarded = S.lbo_discarded;
  } else {
    if (m->center != site) TN_THROW(TN_ESTATE, "the orthogonality centre is not at the requested site");
    // environments around the site
    ensure_right_envs(m, mpo, o->precision, nullptr);
    for (int t = 0; t < site; ++t)
      if (!m->Lok[t + 1]) update_left_env(m, mpo, t, o->precision, nullptr);
    const double dsc = lbo_site(c, mpo, m, site, *o, o->precision, nullptr);
    // tensors right of the site are untouched; environments right of the site stay valid
    m->env_version = mpo->version;
    for (int t = site + 1; t <= m->N; ++t) m->Lok[t] = false;
    for (int t = 0; t <= site; ++t) m->Rok[t] = false;
    if (discarded) *discarded = dsc;
  }
  TN_GUARD_END(c)
}

// ------------------------------------------------------------------ step entry points
extern "C" tn_status tn_heff_apply(tn_ctx* c, const tn_mpo* mpo, int32_t site, int32_t chi_l, int32_t chi_r,
                                   const double* L, const double* R, const double* xin, double* yout, int32_t prec) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!mpo || !L || !R || !xin || !yout) TN_THROW(TN_EINVAL, "null argument");
  if (site < 0 || site + 1 >= mpo->N) TN_THROW(TN_EINVAL, "window out of range");
  if (chi_l < 1 || chi_r < 1) TN_THROW(TN_EINVAL, "bond dimensions must be positive");
  if (prec < 0 || prec > 2) TN_THROW(TN_EINVAL, "unknown precision");
  const int sprec = prec == PREC_FP64 ? PREC_FP64 : PREC_FP32;
  const size_t eb = elem_bytes(sprec);
  const int wl = mpo->w[site], wr = mpo->w[site + 2];
  char* Lc = (char*)ws_get(c, "api:L", (size_t)wl * chi_l * chi_l * eb);
  char* Rc = (char*)ws_get(c, "api:R", (size_t)wr * chi_r * chi_r * eb);
  HIPCHK(launch_convert(sprec, Lc, PREC_FP64, L, (int64_t)wl * chi_l * chi_l, c->stream));
  HIPCHK(launch_transpose_from64(sprec, Rc, (const cf64*)R, wr, chi_r, chi_r, c->stream));
  std::vector<const void*> lp(wl), rp(wr);
  for (int i = 0; i < wl; ++i) lp[i] = Lc + (size_t)i * chi_l * chi_l * eb;
  for (int i = 0; i < wr; ++i) rp[i] = Rc + (size_t)i * chi_r * chi_r * eb;
  WindowOp op;
  op.setup(c, mpo, site, 2, prec, chi_l, chi_r, lp, rp, false, "heff");
  op.apply((const cf64*)xin, (cf64*)yout);
  HIPCHK(hipStreamSynchronize(c->stream));
  TN_GUARD_END(c)
}

extern "C" tn_status tn_env_update(tn_ctx* c, const tn_mpo* mpo, int32_t site, int32_t dir, int32_t chi_l,
                                   int32_t chi_r, const double* env_in, const double* A, double* env_out,
                                   int32_t prec) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!mpo || !env_in || !A || !env_out) TN_THROW(TN_EINVAL, "null argument");
  if (site < 0 || site >= mpo->N) TN_THROW(TN_EINVAL, "site out of range");
  if (dir != 1 && dir != -1) TN_THROW(TN_EINVAL, "direction must be +1 or -1");
  if (chi_l < 1 || chi_r < 1) TN_THROW(TN_EINVAL, "bond dimensions must be positive");
  if (prec < 0 || prec > 2) TN_THROW(TN_EINVAL, "unknown precision");
  const int sprec = prec == PREC_FP64 ? PREC_FP64 : PREC_FP32;
  const size_t eb = elem_bytes(sprec);
  if (dir > 0) {
    const int wi = mpo->w[site], wo = mpo->w[site + 1];
    char* in = (char*)ws_get(c, "api:Ein", (size_t)wi * chi_l * chi_l * eb);
    char* out = (char*)ws_get(c, "api:Eout", (size_t)wo * chi_r * chi_r * eb);
    HIPCHK(launch_convert(sprec, in, PREC_FP64, env_in, (int64_t)wi * chi_l * chi_l, c->stream));
    std::vector<const void*> p(wi);
    for (int i = 0; i < wi; ++i) p[i] = in + (size_t)i * chi_l * chi_l * eb;
    env_left(c, mpo, site, prec, chi_l, chi_r, p, (const cf64*)A, out);
    HIPCHK(launch_convert(PREC_FP64, env_out, sprec, out, (int64_t)wo * chi_r * chi_r, c->stream));
  } else {
    const int wi = mpo->w[site + 1], wo = mpo->w[site];
    char* in = (char*)ws_get(c, "api:Ein", (size_t)wi * chi_r * chi_r * eb);
    char* out = (char*)ws_get(c, "api:Eout", (size_t)wo * chi_l * chi_l * eb);
    HIPCHK(launch_transpose_from64(sprec, in, (const cf64*)env_in, wi, chi_r, chi_r, c->stream));
    std::vector<const void*> p(wi);
    for (int i = 0; i < wi; ++i) p[i] = in + (size_t)i * chi_r * chi_r * eb;
    env_right(c, mpo, site, prec, chi_l, chi_r, p, (const cf64*)A, out);
    HIPCHK(launch_transpose_to64(sprec, (cf64*)env_out, out, wo, chi_l, chi_l, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  TN_GUARD_END(c)
}

extern "C" tn_status tn_truncate(tn_ctx* c, int32_t m, int32_t n, const double* theta, int32_t chi, double sigma_cut,
                                 int32_t dir, double* left, double* right, int32_t* k_out, double* sv,
                                 double* discarded) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!theta || !left || !right || !k_out) TN_THROW(TN_EINVAL, "null argument");
  if (m < 1 || n < 1 || chi < 1) TN_THROW(TN_EINVAL, "sizes must be positive");
  if (dir != 1 && dir != -1) TN_THROW(TN_EINVAL, "direction must be +1 or -1");
  if (!(sigma_cut >= 0.0) || sigma_cut >= 1.0) TN_THROW(TN_EINVAL, "sigma_cut must be in [0, 1)");
  TruncOut t = truncate_dev(c, m, n, (const cf64*)theta, chi, sigma_cut, dir, (cf64*)left, (cf64*)right);
  *k_out = t.k;
  if (sv) std::memcpy(sv, t.sv.data(), t.sv.size() * sizeof(double));
  if (discarded) *discarded = t.disc;
  TN_GUARD_END(c)
}

extern "C" double tn_matvec_flops(const tn_mpo* mpo, int32_t site, int32_t chi_l, int32_t chi_r) {
  if (!mpo || site < 0 || site + 1 >= mpo->N) return -1.0;
  return matvec_flops_formula(mpo, site, chi_l, chi_r);
}
extern "C" double tn_env_flops(const tn_mpo* mpo, int32_t site, int32_t chi_l, int32_t chi_r) {
  if (!mpo || site < 0 || site >= mpo->N) return -1.0;
  return env_flops_formula(mpo, site, chi_l, chi_r);
}

extern "C" tn_status tn_cgemm(tn_ctx* c, int32_t prec, int32_t ta, int32_t tb, int32_t M, int32_t N, int32_t K,
                              const void* A, int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!A || !B || !C) TN_THROW(TN_EINVAL, "null argument");
  if (M < 1 || N < 1 || K < 1) TN_THROW(TN_EINVAL, "sizes must be positive");
  if (prec < 0 || prec > 2) TN_THROW(TN_EINVAL, "unknown precision");
  if (lda < (ta ? M : K) || ldb < (tb ? K : N) || ldc < N) TN_THROW(TN_EINVAL, "leading dimension too small");
  gemm1(c, prec, ta ? 1 : 0, tb ? 1 : 0, C, ldc, M, N, A, lda, B, ldb, K, 0, "api:gemm");
  TN_GUARD_END(c)
}

// ------------------------------------------------------------------ gate-parameterised basis entry points
extern "C" tn_status tn_plbo_enable(tn_mpo* mpo, const double* params) {
  if (mpo && mpo->ctx && mpo->ctx->closed) return TN_ESTATE;
  if (!mpo) return TN_EINVAL;
  tn_ctx* c = mpo->ctx;
  TN_GUARD_BEGIN
  const int N = mpo->N;
  if (params)
    for (size_t i = 0; i < (size_t)N * TN_PLBO_NPARAM; ++i)
      if (!std::isfinite(params[i])) TN_THROW(TN_EINVAL, "non-finite basis parameter");
  mpo->plbo = true;
  mpo->pp.assign(N, {});
  mpo->pm.assign(N, {});
  mpo->pv.assign(N, {});
  mpo->pt.assign(N, 0);
  mpo->iso_stale.assign(N, true);
  for (int s = 0; s < N; ++s) {
    for (int j = 0; j < TN_PLBO_NPARAM; ++j) mpo->pp[s][j] = params ? params[(size_t)s * TN_PLBO_NPARAM + j] : 0.0;
    plbo_set_site(mpo, s);
  }
  TN_GUARD_END(c)
}

extern "C" tn_status tn_plbo_params(const tn_mpo* mpo, double* params) {
  if (!mpo || !params) return TN_EINVAL;
  if (!mpo->plbo) return TN_ESTATE;
  for (int s = 0; s < mpo->N; ++s)
    for (int j = 0; j < TN_PLBO_NPARAM; ++j) params[(size_t)s * TN_PLBO_NPARAM + j] = mpo->pp[s][j];
  return TN_OK;
}

extern "C" tn_status tn_plbo_site_gradient(tn_ctx* c, tn_mpo* mpo, tn_mps* m, int32_t site, int32_t precision,
                                           double* G, double* energy, double* grad) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!mpo || !m || !energy) TN_THROW(TN_EINVAL, "null argument");
  check_pair(mpo, m);
  if (!mpo->plbo) TN_THROW(TN_ESTATE, "the MPO has no gate-parameterised basis");
  if (precision < 0 || precision > 2) TN_THROW(TN_EINVAL, "unknown precision");
  if (site < 0 || site >= m->N) TN_THROW(TN_EINVAL, "site out of range");
  ensure_right_envs(m, mpo, precision, nullptr);
  for (int t = 0; t < site; ++t)
    if (!m->Lok[t + 1]) update_left_env(m, mpo, t, precision, nullptr);
  const int d = mpo->d;
  const int64_t n = (int64_t)m->dims[site] * d * m->dims[site + 1];
  cf64* x = wsT<cf64>(c, "pgrad:x", n);
  const double nr = dev_norm2(c, m->A[site], n);
  if (!(nr > 0.0) || !std::isfinite(nr)) TN_THROW(TN_ENUMERIC, "zero or non-finite centre tensor");
  HIPCHK(launch_scale_host(x, m->A[site], 1.0 / std::sqrt(nr), n, c->stream));
  std::vector<cd> Gh;
  plbo_slot_envs(c, mpo, m, site, precision, x, Gh);
  *energy = plbo_site_energy(plbo_site_of(mpo, site, Gh), mpo->pp[site].data(), grad);
  if (G) std::memcpy(G, Gh.data(), Gh.size() * sizeof(cd));
  TN_GUARD_END(c)
}

extern "C" tn_status tn_plbo_sweep(tn_ctx* c, tn_mpo* mpo, tn_mps* m, const tn_sweep_opts* o,
                                   const tn_plbo_opts* po, tn_sweep_stats* out, double* gain) {
  if (!c) return TN_EINVAL;
  TN_CTX_OPEN(c);
  TN_GUARD_BEGIN
  if (!mpo || !m) TN_THROW(TN_EINVAL, "null handle");
  check_opts(o);
  check_plbo_opts(po);
  check_pair(mpo, m);
  if (!mpo->plbo) TN_THROW(TN_ESTATE, "the MPO has no gate-parameterised basis");
  double g = 0.0;
  sweep_impl(c, mpo, m, *o, out, po, &g);
  if (gain) *gain = g;
  TN_GUARD_END(c)
}

extern "C" tn_status tn_plbo_linear(tn_mpo* mpo) {
  if (mpo && mpo->ctx && mpo->ctx->closed) return TN_ESTATE;
  if (!mpo) return TN_EINVAL;
  tn_ctx* c = mpo->ctx;
  TN_GUARD_BEGIN
  if (!mpo->plbo) TN_THROW(TN_ESTATE, "the MPO has no gate-parameterised basis");
  if (mpo->plbo_lin) TN_THROW(TN_ESTATE, "the linear isometry is already on");
  const int N = mpo->N, D = mpo->D_raw, d = mpo->d;
  if (!mpo->d_fock) mpo->d_fock = (cf64*)dev_alloc(c, (size_t)N * D * d * sizeof(cf64));
  mpo->plbo_lin = true;
  mpo->fock.assign(N, {});
  for (int s = 0; s < N; ++s) {
    mpo->iso[s].assign((size_t)D * d, 0.0);
    for (int a = 0; a < d; ++a) mpo->iso[s][(size_t)a * d + a] = 1.0;  // the first d pLBO states
    plbo_set_site(mpo, s);
  }
  TN_GUARD_END(c)
}

extern "C" tn_status tn_plbo_linear_isometries(const tn_mpo* mpo, double* W) {
  if (!mpo || !W) return TN_EINVAL;
  if (!mpo->plbo || !mpo->plbo_lin) return TN_ESTATE;
  size_t o = 0;
  for (int s = 0; s < mpo->N; ++s)
    for (auto& z : mpo->iso[s]) { W[o++] = z.real(); W[o++] = z.imag(); }
  return TN_OK;
}
