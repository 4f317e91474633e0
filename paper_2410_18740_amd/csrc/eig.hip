// Dense Hermitian eigensolvers in FP64 for the truncation step and the Krylov
// projected problem.
//  * n <= 64: cyclic two-sided Jacobi with round-robin (tournament) ordering,
//    one workgroup per matrix, matrix and eigenvectors resident in LDS.
//  * larger n: Householder reduction to real symmetric tridiagonal form
//    (two launches per column: a one-workgroup reflector step and a
//    multi-workgroup row update + matrix-vector product), Sturm-count
//    bisection for the wanted eigenvalues, inverse iteration for their
//    eigenvectors, two-pass Gram-Schmidt to restore orthonormality inside
//    clusters, and back-transformation through the reflectors.
#include "common.h"

#define JAC_N 64
#define HIPCHK_DEV(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

static __device__ __forceinline__ double wave_sum_d(double v) { return wave_reduce_sum(v); }

// round-robin pairing (circle method) over n2 (even) indices; r, k < n2 - 1
static __device__ __forceinline__ void rr_pair(int r, int k, int n2, int& p, int& q) {
  const int m = n2 - 1;
  if (k == 0) { p = r; q = m; }
  else {
    p = r + k;
    if (p >= m) p -= m;
    q = r - k;
    if (q < 0) q += m;
  }
  if (p > q) { int t = p; p = q; q = t; }
}

// RS: power-of-two row span >= n2 of the update loops, so that the (pair,
// row) index of a work item comes from a shift and a mask; IPT work items
// per thread cover (RS / 2) pairs x RS rows
template <int JT, int RS, int IPT = (RS / 2) * RS / JT>
__global__ __launch_bounds__(JT) void jacobi_kernel(const cf64* __restrict__ Ain, int64_t strideA, int n,
                                                      double* __restrict__ evals, cf64* __restrict__ Vout,
                                                      int64_t strideV, int descending) {
  // one padding column: the column updates walk down a column, and rows one
  // element apart in stride fall on different LDS banks
  __shared__ cf64 A[JAC_N][JAC_N + 1];
  __shared__ cf64 V[JAC_N][JAC_N + 1];
  __shared__ double red[2][JT / 64];
  __shared__ int done;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const cf64* a_in = Ain + (int64_t)blockIdx.x * strideA;
  const int n2 = n + (n & 1);
  for (int e = tid; e < n2 * n2; e += JT) {
    const int i = e / n2, j = e % n2;
    A[i][j] = (i < n && j < n) ? a_in[(int64_t)i * n + j] : czero<cf64>();
    V[i][j] = (i == j) ? make_double2(1.0, 0.0) : czero<cf64>();
  }
  if (tid == 0) done = 0;
  __syncthreads();
  // symmetrise (Hermitian part) for robustness
  for (int e = tid; e < n * n; e += JT) {
    const int i = e / n, j = e % n;
    if (i < j) {
      cf64 x = A[i][j], y = A[j][i];
      cf64 h = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
      A[i][j] = h;
      A[j][i] = cconj(h);
    } else if (i == j) {
      A[i][i].y = 0.0;
    }
  }
  __syncthreads();
  const int npairs = n2 / 2;
  double off_prev = INFINITY;  // thread 0 only
  for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
    for (int r = 0; r < n2 - 1; ++r) {
      // every work item (pair k, row or column index) computes its pair's
      // rotation from the pivots into registers, so the rotation parameters
      // make no LDS round trip; one barrier separates the pivot reads from
      // the column update
      int pp[IPT], qq[IPT], ix[IPT];
      double cs[IPT], sn[IPT], cph[IPT], sph[IPT];
#pragma unroll
      for (int t = 0; t < IPT; ++t) {
        const int e = tid + JT * t;
        const int k = e / RS;
        ix[t] = e & (RS - 1);
        cs[t] = 1.0; sn[t] = 0.0; cph[t] = 1.0; sph[t] = 0.0;
        pp[t] = 0; qq[t] = 0;
        if (k < npairs && ix[t] < n2) {
          int p, q;
          rr_pair(r, k, n2, p, q);
          pp[t] = p; qq[t] = q;
          if (q < n) {
            const double app = A[p][p].x, aqq = A[q][q].x;
            const cf64 apq = A[p][q];
            const double b = sqrt(cabs2(apq));
            if (b > 1e-300 && b * b > 1e-34 * (app * app + aqq * aqq)) {
              const double zeta = (aqq - app) / (2.0 * b);
              const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
              cs[t] = 1.0 / sqrt(1.0 + tt * tt);
              sn[t] = tt * cs[t];
              cph[t] = apq.x / b;
              sph[t] = apq.y / b;
            }
          }
        }
      }
      __syncthreads();
      // column update: A <- A J, V <- V J with J = [[cs, sn], [-sn e^{-i phi}, cs e^{-i phi}]]
#pragma unroll
      for (int t = 0; t < IPT; ++t) {
        if (sn[t] == 0.0) continue;
        const int p = pp[t], q = qq[t], row = ix[t];
        const cf64 em = make_double2(cph[t], -sph[t]);  // e^{-i phi}
        cf64 xp = A[row][p], xq = A[row][q];
        cf64 xqe = cmul(xq, em);
        A[row][p] = make_double2(cs[t] * xp.x - sn[t] * xqe.x, cs[t] * xp.y - sn[t] * xqe.y);
        A[row][q] = make_double2(sn[t] * xp.x + cs[t] * xqe.x, sn[t] * xp.y + cs[t] * xqe.y);
        xp = V[row][p]; xq = V[row][q];
        xqe = cmul(xq, em);
        V[row][p] = make_double2(cs[t] * xp.x - sn[t] * xqe.x, cs[t] * xp.y - sn[t] * xqe.y);
        V[row][q] = make_double2(sn[t] * xp.x + cs[t] * xqe.x, sn[t] * xp.y + cs[t] * xqe.y);
      }
      __syncthreads();
      // row update: A <- J^H A, J^H = [[cs, -sn e^{i phi}], [sn, cs e^{i phi}]]; the
      // rotated pair's off-diagonal entries are set to zero and its diagonal made real
#pragma unroll
      for (int t = 0; t < IPT; ++t) {
        if (sn[t] == 0.0) continue;
        const int p = pp[t], q = qq[t], col = ix[t];
        const cf64 ep = make_double2(cph[t], sph[t]);  // e^{i phi}
        const cf64 xp = A[p][col], xq = A[q][col];
        const cf64 xqe = cmul(xq, ep);
        cf64 np_ = make_double2(cs[t] * xp.x - sn[t] * xqe.x, cs[t] * xp.y - sn[t] * xqe.y);
        cf64 nq_ = make_double2(sn[t] * xp.x + cs[t] * xqe.x, sn[t] * xp.y + cs[t] * xqe.y);
        if (col == p) { np_.y = 0.0; nq_ = czero<cf64>(); }
        if (col == q) { np_ = czero<cf64>(); nq_.y = 0.0; }
        A[p][col] = np_;
        A[q][col] = nq_;
      }
      __syncthreads();
    }
    // convergence test
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < n * n; e += JT) {
      const int i = e / n, j = e % n;
      const double v = cabs2(A[i][j]);
      if (i == j) dia += v; else off += v;
    }
    off = wave_sum_d(off);
    dia = wave_sum_d(dia);
    if (lane == 0) { red[0][wave] = off; red[1][wave] = dia; }
    __syncthreads();
    if (tid == 0) {
      double o = 0.0, d = 0.0;
      for (int w = 0; w < JT / 64; ++w) {
        o += red[0][w];
        d += red[1][w];
      }
      // converged, or at the rounding floor: the off-diagonal mass has stopped
      // falling quadratically although it is already at the 1e-12 level
      done = (o <= 1e-31 * d) || (o < 1e-300) || (o <= 1e-24 * d && o > 0.25 * off_prev);
      off_prev = o;
    }
    __syncthreads();
    if (done) break;
  }
  // sort (rank by value, ties by index) and write
  double* ev = evals + (int64_t)blockIdx.x * n;
  cf64* vo = Vout + (int64_t)blockIdx.x * strideV;
  for (int p = tid; p < n; p += JT) {
    const double lp = A[p][p].x;
    int rank = 0;
    for (int q = 0; q < n; ++q) {
      const double lq = A[q][q].x;
      const bool before = descending ? (lq > lp || (lq == lp && q < p)) : (lq < lp || (lq == lp && q < p));
      rank += before;
    }
    ev[rank] = lp;
    for (int i = 0; i < n; ++i) vo[(int64_t)i * n + rank] = V[i][p];
  }
}

hipError_t launch_jacobi(const cf64* A, int64_t strideA, int n, int batch, double* evals, cf64* V, int64_t strideV,
                         int descending, hipStream_t st) {
  if (n < 1 || n > JAC_N || batch <= 0) return hipErrorInvalidValue;
  if (n <= 32)
    hipLaunchKernelGGL((jacobi_kernel<512, 32>), dim3(batch), dim3(512), 0, st, A, strideA, n, evals, V, strideV,
                       descending);
  else
    hipLaunchKernelGGL((jacobi_kernel<512, 64>), dim3(batch), dim3(512), 0, st, A, strideA, n, evals, V, strideV,
                       descending);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Householder tridiagonalisation
// One launch per column j.  Every workgroup recomputes (redundantly, from data
// finalised by the previous launch) w_{j-1} = y_{j-1} - 1/2 tau_{j-1}
// (y_{j-1}^H v_{j-1}) v_{j-1} and the reflector of column j into LDS, then
// updates its own rows i in [j+1, p) with the pending rank-2 term
// (v_{j-1}, w_{j-1}) and forms y_j[i] = tau_j sum_k A[i][k] v_j[k].  A
// workgroup owns TRI_ROWS rows; each row is split over two wavefronts.  The
// step is bound by latency, not bandwidth, so every global load the step needs
// is issued in one round at the start: the first TRI_UNROLL row elements of
// each lane, and y_{j-1}, v_{j-1} and row j (staged in LDS).  Workgroup 0 also
// publishes v_j, tau_j and the diagonal and off-diagonal entries.
static constexpr int TRI_UNROLL = 8;  // row loads in flight per lane

// TRI_ROWS rows per workgroup, two wavefronts each.  Two rows up to p = 1024
// (three workgroups fit a CU's LDS there); beyond, the three LDS vectors take
// up to 150 KiB and one workgroup fills the LDS, so it carries eight rows
// (sixteen wavefronts) to keep the CU busy.
template <int TRI_ROWS>
__global__ __launch_bounds__(128 * TRI_ROWS) void tridiag_col(cf64* __restrict__ A, cf64* __restrict__ vs,
                                                    cf64* __restrict__ taus, double* __restrict__ dg,
                                                    double* __restrict__ off, cf64* __restrict__ y, int p, int j) {
  extern __shared__ unsigned char sm_raw[];
  cf64* vS = reinterpret_cast<cf64*>(sm_raw);  // row j, then v_j
  cf64* wS = vS + p;                           // y_{j-1}, then w_{j-1}
  cf64* pS = wS + p;                           // v_{j-1}
  constexpr int TRI_WAVES = 2 * TRI_ROWS, TRI_THREADS = 64 * TRI_WAVES;
  constexpr int TRI_FILL = TRI_THREADS >= 1024 ? 1 : 1024 / TRI_THREADS;  // vector loads grouped per thread
  __shared__ double red[2][TRI_WAVES];
  __shared__ double red2[TRI_WAVES];
  __shared__ double part[TRI_ROWS][2][2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const cf64* vprev = (j > 0) ? vs + (int64_t)(j - 1) * p : nullptr;
  cf64* ycur = y + (int64_t)(j & 1) * p;            // y_j (written here)
  const cf64* yprev = y + (int64_t)((j + 1) & 1) * p;  // y_{j-1}
  const cf64* rowj = A + (int64_t)j * p;
  // ---- one round of global loads
  // rows are dealt to workgroups so that row i always lands on the same XCD
  // (workgroup b runs on XCD b % 8): XCD x owns the rows i = x (mod 8), in
  // groups of TRI_ROWS, and keeps them in its L2 from one column to the next
  const int rl = wave >> 1, half = wave & 1, tl = half * 64 + lane;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int i0 = j + 1 + ((xcd - (j + 1)) % 8 + 8) % 8;  // first row >= j+1 with i = xcd (mod 8)
  const int i = i0 + 8 * (slot * TRI_ROWS + rl);
  const bool own = (j < p - 1) && (i < p);
  cf64* row = A + (int64_t)(own ? i : 0) * p;
  cf64 a0[TRI_UNROLL];
#pragma unroll
  for (int u = 0; u < TRI_UNROLL; ++u) {
    const int k = j + 1 + tl + 128 * u;
    a0[u] = (own && k < p) ? row[k] : czero<cf64>();
  }
  const cf64 tprev = (j > 0) ? taus[j - 1] : czero<cf64>();
  // entries j of y_{j-1} and v_{j-1}: every thread forms w_{j-1}[j] itself
  const cf64 yj = (j > 0) ? yprev[j] : czero<cf64>();
  const cf64 pj = (j > 0) ? vprev[j] : czero<cf64>();
  double re = 0.0, im = 0.0;
  // each thread owns the entries q = j + tid (mod TRI_THREADS) of the LDS vectors up to
  // the reflector, so only the two reductions need workgroup barriers
  // loads of TRI_FILL entries at a time are issued together (clamped addresses,
  // masked use) so that they share one round trip; the first group is outside
  // any loop, so its loads are in flight together with the row loads above
  auto fill = [&](int q0) {
    cf64 rr[TRI_FILL], yy[TRI_FILL], vv[TRI_FILL];
#pragma unroll
    for (int t = 0; t < TRI_FILL; ++t) {
      const int qc = min(q0 + TRI_THREADS * t, p - 1);
      rr[t] = rowj[qc];
      if (j > 0) {
        yy[t] = yprev[qc];
        vv[t] = vprev[qc];
      }
    }
#pragma unroll
    for (int t = 0; t < TRI_FILL; ++t) {
      const int q = q0 + TRI_THREADS * t;
      if (q < p) {
        vS[q] = cconj(rr[t]);
        if (j > 0) {
          wS[q] = yy[t];
          pS[q] = vv[t];
          re += yy[t].x * vv[t].x + yy[t].y * vv[t].y;
          im += yy[t].x * vv[t].y - yy[t].y * vv[t].x;
        }
      }
    }
  };
  fill(j + tid);
  for (int q0 = j + tid + TRI_THREADS * TRI_FILL; q0 < p; q0 += TRI_THREADS * TRI_FILL) fill(q0);
  // ---- w_{j-1} = y_{j-1} - 1/2 tau_{j-1} (y_{j-1}^H v_{j-1}) v_{j-1}
  cf64 c = czero<cf64>();
  if (j > 0) {
    re = wave_sum_d(re);
    im = wave_sum_d(im);
    if (lane == 0) { red[0][wave] = re; red[1][wave] = im; }
    __syncthreads();
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int w = 0; w < TRI_WAVES; ++w) { sr += red[0][w]; si += red[1][w]; }
    const cf64 k = cmul(tprev, make_double2(sr, si));
    c = make_double2(-0.5 * k.x, -0.5 * k.y);
    for (int q = j + tid; q < p; q += TRI_THREADS) wS[q] = cadd(wS[q], cmul(c, pS[q]));
  }
  // ---- column j (rows >= j) with the pending update; reflector
  const cf64 wj = (j > 0) ? cadd(yj, cmul(c, pj)) : czero<cf64>();
  const cf64 vj = pj;
  // diagonal entry j (stored at the end: a store here would stall the row loads)
  double dj = vS[j].x;
  if (j > 0) dj -= 2.0 * (vj.x * wj.x + vj.y * wj.y);
  if (j == p - 1) {
    if (blockIdx.x == 0 && tid == 0) dg[j] = dj;
    return;
  }
  double nrm = 0.0;
  for (int q = j + tid; q < p; q += TRI_THREADS) {
    if (q == j) continue;
    cf64 x = vS[q];
    if (j > 0) x = csub(x, cadd(cmulc(pS[q], wj), cmulc(wS[q], vj)));
    vS[q] = x;  // the column; the reflector is v = (q == j + 1 ? 1 : x scale)
    if (q > j + 1) nrm += cabs2(x);
  }
  nrm = wave_sum_d(nrm);
  if (lane == 0) red2[wave] = nrm;
  __syncthreads();
  cf64 tau, scale;
  double offj;
  {
    double xn2 = 0.0;
#pragma unroll
    for (int w = 0; w < TRI_WAVES; ++w) xn2 += red2[w];
    const cf64 alpha = vS[j + 1];
    double beta;
    if (xn2 == 0.0 && alpha.y == 0.0) {
      tau = czero<cf64>();
      beta = alpha.x;
      scale = czero<cf64>();
    } else {
      const double nr = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
      beta = (alpha.x >= 0.0) ? -nr : nr;
      tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
      const cf64 den = make_double2(alpha.x - beta, alpha.y);
      const double dd = den.x * den.x + den.y * den.y;
      scale = make_double2(den.x / dd, -den.y / dd);
    }
    offj = beta;
  }
  // ---- own rows: wavefronts (2r, 2r+1) share row i, interleaved by 128 columns
  re = 0.0;
  im = 0.0;
  // the last chunk's updated entries are stored after the final barrier: a
  // barrier waits for the wave's outstanding stores
  cf64 xs[TRI_UNROLL];
  int klast = -1;
  if (own) {
    cf64 vi = czero<cf64>(), wi = czero<cf64>();
    if (j > 0) { vi = pS[i]; wi = wS[i]; }
    for (int k0 = j + 1; k0 < p; k0 += 128 * TRI_UNROLL) {
      cf64 a[TRI_UNROLL];
      if (k0 == j + 1) {
#pragma unroll
        for (int u = 0; u < TRI_UNROLL; ++u) a[u] = a0[u];
      } else {
#pragma unroll
        for (int u = 0; u < TRI_UNROLL; ++u) {
          const int k = k0 + tl + 128 * u;
          a[u] = (k < p) ? row[k] : czero<cf64>();
        }
      }
      // every update first, then all the stores: a store between two uses of
      // loaded data would make the wave wait for the store's completion
      // (loads and stores share one completion counter)
#pragma unroll
      for (int u = 0; u < TRI_UNROLL; ++u) {
        const int k = k0 + tl + 128 * u;
        xs[u] = czero<cf64>();
        if (k < p) {
          cf64 x = a[u];
          if (j > 0) x = csub(x, cadd(cmulc(vi, wS[k]), cmulc(wi, pS[k])));
          xs[u] = x;
          const cf64 vk = (k == j + 1) ? make_double2(1.0, 0.0) : cmul(vS[k], scale);
          re += x.x * vk.x - x.y * vk.y;
          im += x.x * vk.y + x.y * vk.x;
        }
      }
      if (k0 + 128 * TRI_UNROLL >= p) {
        klast = k0;
      } else if (j > 0) {
#pragma unroll
        for (int u = 0; u < TRI_UNROLL; ++u) {
          const int k = k0 + tl + 128 * u;
          if (k < p) row[k] = xs[u];
        }
      }
    }
  }
  re = wave_sum_d(re);
  im = wave_sum_d(im);
  if (lane == 0) { part[rl][half][0] = re; part[rl][half][1] = im; }
  __syncthreads();
  // every store from here on
  if (tid < TRI_ROWS) {
    const int ii = i0 + 8 * (slot * TRI_ROWS + tid);
    if (j < p - 1 && ii < p)
      ycur[ii] = cmul(tau, make_double2(part[tid][0][0] + part[tid][1][0], part[tid][0][1] + part[tid][1][1]));
  }
  if (klast >= 0 && j > 0) {
#pragma unroll
    for (int u = 0; u < TRI_UNROLL; ++u) {
      const int k = klast + tl + 128 * u;
      if (k < p) row[k] = xs[u];
    }
  }
  // workgroup 0 stores the reflector, tau, and the tridiagonal entries j
  if (blockIdx.x == 0) {
    cf64* vout = vs + (int64_t)j * p;
    for (int q = tid; q < p; q += TRI_THREADS) {
      cf64 v = czero<cf64>();
      if (q == j + 1) v = make_double2(1.0, 0.0);
      else if (q > j + 1) v = cmul(vS[q], scale);
      vout[q] = v;
    }
    if (tid == 0) {
      taus[j] = tau;
      off[j] = offj;
      dg[j] = dj;
    }
  }
}

hipError_t launch_tridiag(TridiagWork& tw, int p, hipStream_t st) {
  const size_t shm = (size_t)3 * p * sizeof(cf64);
  if (shm > 150 * 1024) return hipErrorInvalidValue;
  const int R = p <= 1024 ? 2 : 8;  // rows per workgroup
  for (int j = 0; j < p; ++j) {
    const int rows = p - j - 1;
    // 8 XCDs x enough slots of R rows for the largest residue class
    const int per_xcd = (rows + 7) / 8;
    const int slots = std::max(1, (per_xcd + R - 1) / R);
    if (R == 2)
      hipLaunchKernelGGL(tridiag_col<2>, dim3(8 * slots), dim3(256), shm, st, tw.A, tw.vs, tw.taus, tw.dg, tw.off,
                         tw.y, p, j);
    else
      hipLaunchKernelGGL(tridiag_col<8>, dim3(8 * slots), dim3(1024), shm, st, tw.A, tw.vs, tw.taus, tw.dg, tw.off,
                         tw.y, p, j);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ bisection (top-k)
static __device__ int sturm_count(const double* dS, const double* e2S, int p, double x, double pivmin) {
  // number of eigenvalues < x; dS, e2S: diagonal and squared off-diagonal in LDS
  int cnt = 0;
  double q = dS[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++cnt;
#pragma unroll 4
  for (int i = 1; i < p; ++i) {
    q = (dS[i] - x) - e2S[i - 1] * recip_nr(q);
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// One workgroup of BIS_T threads per wanted eigenvalue: each round every thread
// counts the eigenvalues below one of BIS_T equispaced probes of the current
// interval, and the interval shrinks to the probe gap that holds the target
// (BIS_T-way multisection; seven or eight rounds reach full double precision).
constexpr int BIS_T = 256;
__global__ __launch_bounds__(BIS_T) void bisect_kernel(const double* dg, const double* off, int p, int k,
                                                       double* evals) {
  extern __shared__ unsigned char sm_raw[];
  double* dS = reinterpret_cast<double*>(sm_raw);
  double* e2S = dS + p;
  __shared__ double rlo[BIS_T / 64], rhi[BIS_T / 64], rem[BIS_T / 64];
  __shared__ int nle_w[BIS_T / 64];
  const int t = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (t >= k) return;
  double lo = 1e300, hi = -1e300, emax = 0.0;
  for (int i = tid; i < p; i += BIS_T) {
    const double di = dg[i], oi = (i < p - 1) ? off[i] : 0.0, om = (i > 0) ? off[i - 1] : 0.0;
    dS[i] = di;
    e2S[i] = oi * oi;
    const double r = fabs(om) + fabs(oi);
    lo = fmin(lo, di - r);
    hi = fmax(hi, di + r);
    emax = fmax(emax, oi * oi);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
    emax = fmax(emax, __shfl_xor(emax, o, 64));
  }
  if (lane == 0) { rlo[wv] = lo; rhi[wv] = hi; rem[wv] = emax; }
  __syncthreads();
  lo = rlo[0]; hi = rhi[0]; emax = rem[0];
#pragma unroll
  for (int q = 1; q < BIS_T / 64; ++q) {
    lo = fmin(lo, rlo[q]);
    hi = fmax(hi, rhi[q]);
    emax = fmax(emax, rem[q]);
  }
  const double scale = fmax(fabs(lo), fabs(hi));
  const double pivmin = fmax(1e-300, 2.3e-308 * fmax(1.0, emax));
  lo -= 1e-14 * scale + 1e-300;
  hi += 1e-14 * scale + 1e-300;
  const int target = p - 1 - t;  // ascending index of the t-th largest
  for (int it = 0; it < 40; ++it) {
    if (hi - lo <= 4.4e-16 * fmax(fabs(lo), fabs(hi)) + 1e-300) break;
    const double w = (hi - lo) / (double)(BIS_T + 1);
    const double x = lo + w * (double)(tid + 1);
    const int c = sturm_count(dS, e2S, p, x, pivmin);
    // probes with count <= target lie left of the eigenvalue; probes increase
    // with the thread index, so those are threads 0 .. nle - 1
    const unsigned long long le = __ballot(c <= target);
    __syncthreads();  // the previous round's nle_w has been read
    if (lane == 0) nle_w[wv] = __popcll(le);
    __syncthreads();
    int nle = 0;
#pragma unroll
    for (int q = 0; q < BIS_T / 64; ++q) nle += nle_w[q];
    const double nlo = (nle == 0) ? lo : lo + w * (double)nle;
    const double nhi = (nle == BIS_T) ? hi : lo + w * (double)(nle + 1);
    if (!(nhi - nlo < hi - lo)) break;
    lo = nlo;
    hi = nhi;
  }
  if (tid == 0) evals[t] = 0.5 * (lo + hi);
}
hipError_t launch_bisect_top(const double* dg, const double* off, int p, int k, double* evals, hipStream_t st) {
  const size_t shm = (size_t)2 * p * sizeof(double);
  if (shm > 150 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bisect_kernel, dim3(k), dim3(BIS_T), shm, st, dg, off, p, k, evals);
  return hipGetLastError();
}

// ------------------------------------------------------------------ inverse iteration
// One workgroup per eigenvalue; the LU factors of (T - lambda I) with partial
// pivoting live in LDS (5 p doubles), the recurrences run on one lane.
__global__ __launch_bounds__(64) void inverse_iter_kernel(const double* __restrict__ dg, const double* __restrict__ off,
                                                          int p, int k, const double* __restrict__ evals,
                                                          double* __restrict__ X) {
  extern __shared__ unsigned char sm_raw[];
  double* dd = reinterpret_cast<double*>(sm_raw);
  double* du = dd + p;
  double* du2 = du + p;
  double* dl = du2 + p;
  double* b = dl + p;
  unsigned char* piv = reinterpret_cast<unsigned char*>(b + p);
  __shared__ double red[1];
  const int t = blockIdx.x;
  const int lane = threadIdx.x;
  if (t >= k) return;
  double tn = 0.0;
  for (int i = lane; i < p; i += 64) {
    tn = fmax(tn, fabs(dg[i]) + (i > 0 ? fabs(off[i - 1]) : 0.0) + (i < p - 1 ? fabs(off[i]) : 0.0));
    dd[i] = dg[i] - evals[t];
    du[i] = (i < p - 1) ? off[i] : 0.0;
    dl[i] = (i < p - 1) ? off[i] : 0.0;
    du2[i] = 0.0;
    piv[i] = 0;
    b[i] = 1.0 + 0.37 * sin(1.3 * (double)(i + 1) * (double)(t + 1));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) tn = fmax(tn, __shfl_xor(tn, o, 64));
  __syncthreads();
  const double tiny = fmax(2.2e-16 * tn, 1e-300);
  if (lane == 0) {
    // LU with partial pivoting of the tridiagonal T - lambda I; the running
    // diagonal and super-diagonal entries are carried in registers
    double cdd = dd[0], cdu = du[0];
    for (int i = 0; i < p - 1; ++i) {
      const double l = dl[i], ndd = dd[i + 1], ndu = du[i + 1];
      if (fabs(cdd) >= fabs(l)) {
        if (cdd == 0.0) cdd = tiny;
        const double f = l * recip_nr(cdd);
        dd[i] = cdd;
        dl[i] = f;
        du[i] = cdu;
        cdd = ndd - f * cdu;
        cdu = ndu;
      } else {
        const double f = cdd * recip_nr(l);
        dd[i] = l;
        dl[i] = f;
        du[i] = ndd;
        piv[i] = 1;
        cdd = cdu - f * ndd;
        if (i < p - 2) { du2[i] = ndu; cdu = -f * ndu; }
        else cdu = ndu;
      }
    }
    dd[p - 1] = cdd;
  }
  __syncthreads();
  // the pivots are used only through their reciprocals (no division on the
  // solves' dependent chains)
  for (int i = lane; i < p; i += 64) {
    double v = dd[i];
    if (fabs(v) < tiny) v = v >= 0 ? tiny : -tiny;
    dd[i] = 1.0 / v;
  }
  __syncthreads();
  for (int it = 0; it < 2; ++it) {
    if (lane == 0) {
      double cb = b[0];
      for (int i = 0; i < p - 1; ++i) {
        const double nb = b[i + 1], l = dl[i];
        if (piv[i]) { b[i] = nb; cb = cb - l * nb; }
        else { b[i] = cb; cb = nb - l * cb; }
      }
      double x1 = cb * dd[p - 1];
      b[p - 1] = x1;
      double x2 = 0.0;
      if (p >= 2) {
        const double x0 = (b[p - 2] - du[p - 2] * x1) * dd[p - 2];
        b[p - 2] = x0;
        x2 = x1;
        x1 = x0;
      }
      for (int i = p - 3; i >= 0; --i) {
        const double x0 = (b[i] - du[i] * x1 - du2[i] * x2) * dd[i];
        b[i] = x0;
        x2 = x1;
        x1 = x0;
      }
    }
    __syncthreads();
    if (it == 0) {
      double mx = 0.0;
      for (int i = lane; i < p; i += 64) mx = fmax(mx, fabs(b[i]));
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
      const double sc = (mx > 0.0 && isfinite(mx)) ? 1.0 / mx : 0.0;
      for (int i = lane; i < p; i += 64) b[i] *= sc;
      __syncthreads();
    }
  }
  __syncthreads();
  double nr = 0.0;
  for (int i = lane; i < p; i += 64) nr += b[i] * b[i];
  nr = wave_sum_d(nr);
  if (lane == 0) red[0] = nr;
  __syncthreads();
  const double s = (red[0] > 0.0 && isfinite(red[0])) ? 1.0 / sqrt(red[0]) : 0.0;
  double* x = X + (int64_t)t * p;
  for (int i = lane; i < p; i += 64) x[i] = (s > 0.0) ? b[i] * s : (i == (t % p) ? 1.0 : 0.0);
}
hipError_t launch_inverse_iter(const double* dg, const double* off, int p, int k, const double* evals, double* X,
                               double* scratch, hipStream_t st) {
  (void)scratch;
  const size_t shm = (size_t)5 * p * sizeof(double) + (size_t)p;
  if (shm > 160 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(inverse_iter_kernel, dim3(k), dim3(64), shm, st, dg, off, p, k, evals, X);
  return hipGetLastError();
}

// ------------------------------------------------------------------ orthonormalisation of X (k columns of length p)
// Columns [j0, k) are re-orthonormalised in blocks of OB columns, in column
// order (the result is that of classical Gram-Schmidt done twice):
//   1. the block is projected twice against all earlier columns (dot products
//      one wavefront per pair, update one thread per entry: many workgroups);
//   2. one workgroup orthonormalises the block's columns among themselves
//      (two passes); a column that loses more than 1 - 1e-8 of its norm
//      (numerically dependent, e.g. inside a cluster of equal eigenvalues) is
//      replaced by a unit vector and re-orthogonalised against every earlier
//      column.
static constexpr int OB = 16;

__global__ __launch_bounds__(256) void ortho_dot_kernel(const double* __restrict__ X, int p, int c0, int nb,
                                                        double* __restrict__ H) {
  const int lane = threadIdx.x & 63;
  const int pair = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (pair >= c0 * nb) return;
  const int l = pair / nb, c = pair % nb;
  const double* xl = X + (int64_t)l * p;
  const double* xc = X + (int64_t)(c0 + c) * p;
  double s = 0.0;
  for (int i = lane; i < p; i += 64) s += xl[i] * xc[i];
  s = wave_sum_d(s);
  if (lane == 0) H[l * OB + c] = s;
}
__global__ __launch_bounds__(256) void ortho_upd_kernel(double* __restrict__ X, int p, int c0, int nb,
                                                        const double* __restrict__ H) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= p || c >= nb) return;
  double v = X[(int64_t)(c0 + c) * p + i];
  for (int l = 0; l < c0; ++l) v -= H[l * OB + c] * X[(int64_t)l * p + i];
  X[(int64_t)(c0 + c) * p + i] = v;
}
__global__ __launch_bounds__(1024) void ortho_block_kernel(double* __restrict__ X, int p, int c0, int c1) {
  __shared__ double h[1024];
  __shared__ double red[16];
  __shared__ double sc[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = c0; j < c1; ++j) {
    double* xj = X + (int64_t)j * p;
    int trial = 0;
    int lo = c0;  // earlier columns to project against: the block's, or all after a replacement
    while (true) {
      double nb = 0.0;
      for (int i = tid; i < p; i += 1024) nb += xj[i] * xj[i];
      nb = wave_sum_d(nb);
      if (lane == 0) red[wave] = nb;
      __syncthreads();
      if (tid == 0) { double s = 0; for (int w = 0; w < 16; ++w) s += red[w]; sc[0] = s; }
      __syncthreads();
      const double norm0 = sqrt(sc[0]);
      for (int pass = 0; pass < 2; ++pass) {
        for (int l = lo + wave; l < j; l += 16) {
          const double* xl = X + (int64_t)l * p;
          double s = 0.0;
          for (int i = lane; i < p; i += 64) s += xl[i] * xj[i];
          s = wave_sum_d(s);
          if (lane == 0) h[l] = s;
        }
        __syncthreads();
        for (int i = tid; i < p; i += 1024) {
          double v = xj[i];
          for (int l = lo; l < j; ++l) v -= h[l] * X[(int64_t)l * p + i];
          xj[i] = v;
        }
        __syncthreads();
      }
      double na = 0.0;
      for (int i = tid; i < p; i += 1024) na += xj[i] * xj[i];
      na = wave_sum_d(na);
      if (lane == 0) red[wave] = na;
      __syncthreads();
      if (tid == 0) { double s = 0; for (int w = 0; w < 16; ++w) s += red[w]; sc[1] = s; }
      __syncthreads();
      const double norm1 = sqrt(sc[1]);
      if (norm1 > 1e-8 * norm0 && norm1 > 1e-250) {
        const double inv = 1.0 / norm1;
        for (int i = tid; i < p; i += 1024) xj[i] *= inv;
        __syncthreads();
        break;
      }
      // replace by a unit vector and orthogonalise it against every earlier column
      const int pos = (j + 7 * trial) % p;
      for (int i = tid; i < p; i += 1024) xj[i] = (i == pos) ? 1.0 : 0.0;
      __syncthreads();
      lo = 0;
      ++trial;
      if (trial > p + 2) break;
    }
  }
}
hipError_t launch_orthonormalize_real(double* X, int p, int k, int j0, double* H, hipStream_t st) {
  if (k > 1024) return hipErrorInvalidValue;
  for (int c0 = j0; c0 < k; c0 += OB) {
    const int nb = std::min(OB, k - c0);
    if (c0 > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(ortho_dot_kernel, dim3((c0 * nb + 3) / 4), dim3(256), 0, st, X, p, c0, nb, H);
        hipLaunchKernelGGL(ortho_upd_kernel, dim3((p + 255) / 256, nb), dim3(256), 0, st, X, p, c0, nb, H);
      }
    }
    hipLaunchKernelGGL(ortho_block_kernel, dim3(1), dim3(1024), 0, st, X, p, c0, c0 + nb);
  }
  return hipGetLastError();
}

// Orthonormality defect of the columns of X: bad[j] = 1 if column j deviates
// from unit norm or from orthogonality to an earlier column by more than tol.
// One wavefront per pair (a <= b).
__global__ __launch_bounds__(256) void ortho_check_kernel(const double* __restrict__ X, int p, int k, double tol,
                                                          int* __restrict__ bad) {
  const int lane = threadIdx.x & 63;
  const int64_t pair = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t npairs = (int64_t)k * (k + 1) / 2;
  if (pair >= npairs) return;
  // decode pair -> (a, b) with a <= b, row-major over b
  int b = (int)((sqrt(8.0 * (double)pair + 1.0) - 1.0) * 0.5);
  while ((int64_t)b * (b + 1) / 2 > pair) --b;
  while ((int64_t)(b + 1) * (b + 2) / 2 <= pair) ++b;
  const int a = (int)(pair - (int64_t)b * (b + 1) / 2);
  const double* xa = X + (int64_t)a * p;
  const double* xb = X + (int64_t)b * p;
  double s = 0.0;
  for (int i = lane; i < p; i += 64) s += xa[i] * xb[i];
  s = wave_sum_d(s);
  if (lane == 0) {
    const double dev = (a == b) ? fabs(s - 1.0) : fabs(s);
    if (!(dev <= tol)) bad[b] = 1;
  }
}
hipError_t launch_ortho_check(const double* X, int p, int k, double tol, int* bad, hipStream_t st) {
  const int64_t npairs = (int64_t)k * (k + 1) / 2;
  hipLaunchKernelGGL(ortho_check_kernel, dim3((unsigned)((npairs + 3) / 4)), dim3(256), 0, st, X, p, k, tol, bad);
  return hipGetLastError();
}

// ------------------------------------------------------------------ back-transformation U = Q X
// Q = H_0 H_1 ... H_{p-2}, applied in reverse order to each column.  One
// wavefront per column; lane l keeps entries l, l+64, ... of the column in
// registers, and the next DEPTH reflectors are loaded while the current ones
// are applied (DEPTH = 1 measured fastest: the chain of p dependent steps is
// bound by the reduction of each step, not by the loads).
template <int MAXE, int DEPTH>
__global__ __launch_bounds__(64) void backtransform_reg_kernel(const cf64* __restrict__ vs,
                                                               const cf64* __restrict__ taus, int p,
                                                               const double* __restrict__ X, int k,
                                                               cf64* __restrict__ U) {
  const int lane = threadIdx.x;
  const int col = blockIdx.x;
  if (col >= k) return;
  cf64 x[MAXE];
#pragma unroll
  for (int e = 0; e < MAXE; ++e) {
    const int i = lane + 64 * e;
    x[e] = make_double2(i < p ? X[(int64_t)col * p + i] : 0.0, 0.0);
  }
  // reflector j (zero for j < 0, so that applying it is the identity)
  auto load = [&](int j, cf64 (&r)[MAXE], cf64& t) {
    t = (j >= 0) ? taus[j] : czero<cf64>();
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {
      const int i = lane + 64 * e;
      r[e] = (j >= 0 && i < p && i > j) ? vs[(int64_t)j * p + i] : czero<cf64>();
    }
  };
  auto apply = [&](const cf64 (&v)[MAXE], cf64 tau) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {  // v is zero outside (j, p)
      re += v[e].x * x[e].x + v[e].y * x[e].y;
      im += v[e].x * x[e].y - v[e].y * x[e].x;
    }
    re = wave_sum_d(re);
    im = wave_sum_d(im);
    const cf64 c = cmul(tau, make_double2(re, im));
#pragma unroll
    for (int e = 0; e < MAXE; ++e) x[e] = csub(x[e], cmul(c, v[e]));
  };
  cf64 r[DEPTH][MAXE];
  cf64 t[DEPTH];
#pragma unroll
  for (int d = 0; d < DEPTH; ++d) load(p - 2 - d, r[d], t[d]);
  for (int j = p - 2; j >= 0; j -= DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      apply(r[d], t[d]);
      load(j - DEPTH - d, r[d], t[d]);
    }
  }
#pragma unroll
  for (int e = 0; e < MAXE; ++e) {
    const int i = lane + 64 * e;
    if (i < p) U[(int64_t)i * k + col] = x[e];
  }
}

// general fallback: the column in LDS
__global__ __launch_bounds__(64) void backtransform_kernel(const cf64* __restrict__ vs, const cf64* __restrict__ taus,
                                                            int p, const double* __restrict__ X, int k,
                                                            cf64* __restrict__ U) {
  extern __shared__ unsigned char sm_raw[];
  const int lane = threadIdx.x;
  const int col = blockIdx.x;
  cf64* x = reinterpret_cast<cf64*>(sm_raw);
  if (col >= k) return;
  for (int i = lane; i < p; i += 64) x[i] = make_double2(X[(int64_t)col * p + i], 0.0);
  for (int j = p - 2; j >= 0; --j) {
    const cf64 tau = taus[j];
    if (tau.x == 0.0 && tau.y == 0.0) continue;
    const cf64* v = vs + (int64_t)j * p;
    double re = 0.0, im = 0.0;
    for (int i = j + 1 + lane; i < p; i += 64) {
      const cf64 a = v[i], b = x[i];
      re += a.x * b.x + a.y * b.y;
      im += a.x * b.y - a.y * b.x;
    }
    re = wave_sum_d(re);
    im = wave_sum_d(im);
    const cf64 c = cmul(tau, make_double2(re, im));
    for (int i = j + 1 + lane; i < p; i += 64) x[i] = csub(x[i], cmul(c, v[i]));
  }
  for (int i = lane; i < p; i += 64) U[(int64_t)i * k + col] = x[i];
}
// ------------------------------------------------------------------ blocked back-transform
// The reflectors H_j = 1 - tau_j v_j v_j^H in blocks of WY_NB consecutive ones:
// H_j0 ... H_{j0+m-1} = 1 - V T V^H with T upper triangular (the compact WY form
// of Schreiber and Van Loan, SIAM J. Sci. Stat. Comput. 10, 1989): T_ii = tau_i,
// T[0:i, i] = -tau_i T[0:i, 0:i] S[0:i, i], S = V^H V.  One workgroup per block
// builds T; the apply kernel then costs two passes over a block's reflectors and
// one batch of reductions per block instead of a dependent chain per reflector.
constexpr int WY_NB = 16;

__global__ __launch_bounds__(256) void wy_factor_kernel(const cf64* __restrict__ vs, const cf64* __restrict__ taus,
                                                         int p, cf64* __restrict__ Tout) {
  __shared__ cf64 S[WY_NB][WY_NB];
  __shared__ cf64 T[WY_NB][WY_NB];
  const int b = blockIdx.x, j0 = b * WY_NB;
  const int m = min(WY_NB, p - 1 - j0);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // S[l][i] = v_l^H v_i for l < i, over rows r > j0 + i (v_i is zero above)
  for (int q = wv; q < WY_NB * WY_NB; q += 4) {
    const int l = q / WY_NB, i = q % WY_NB;
    if (l >= i || i >= m) continue;
    const cf64* vl = vs + (int64_t)(j0 + l) * p;
    const cf64* vi = vs + (int64_t)(j0 + i) * p;
    double re = 0.0, im = 0.0;
    for (int r = j0 + i + 1 + lane; r < p; r += 64) {
      const cf64 a = vl[r], c = vi[r];
      re += a.x * c.x + a.y * c.y;
      im += a.x * c.y - a.y * c.x;
    }
    re = wave_sum_d(re);
    im = wave_sum_d(im);
    if (lane == 0) S[l][i] = make_double2(re, im);
  }
  for (int q = tid; q < WY_NB * WY_NB; q += 256) T[q / WY_NB][q % WY_NB] = czero<cf64>();
  __syncthreads();
  for (int i = 0; i < m; ++i) {
    const cf64 ti = taus[j0 + i];
    cf64 v = czero<cf64>();
    if (tid < i) {
      for (int q = tid; q < i; ++q) v = cadd(v, cmul(T[tid][q], S[q][i]));
    }
    __syncthreads();
    if (tid < i) T[tid][i] = cmul(make_double2(-ti.x, -ti.y), v);
    if (tid == i) T[i][i] = ti;
    __syncthreads();
  }
  cf64* out = Tout + (int64_t)b * WY_NB * WY_NB;
  for (int q = tid; q < WY_NB * WY_NB; q += 256) out[q] = T[q / WY_NB][q % WY_NB];
}

constexpr int WY_RT = 512;
// Sizes up to 1024: one workgroup of WY_RT threads per eigenvector column;
// thread t keeps rows t + WY_RT e (e < MAXE) in registers.
// Blocks are applied last to first: U = Q_0 Q_1 ... X with Q_b = 1 - V_b T_b V_b^H.
template <int MAXE>
__global__ __launch_bounds__(WY_RT) void wy_apply_reg_kernel(const cf64* __restrict__ vs, const cf64* __restrict__ Tw,
                                                        int p, const double* __restrict__ X, int k,
                                                        cf64* __restrict__ U) {
  __shared__ double red[WY_RT / 64][2 * WY_NB];
  __shared__ cf64 w[WY_NB], w2[WY_NB];
  __shared__ cf64 Ts[WY_NB * WY_NB];
  const int col = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  cf64 x[MAXE];
#pragma unroll
  for (int e = 0; e < MAXE; ++e) {
    const int r = tid + WY_RT * e;
    x[e] = make_double2(r < p ? X[(int64_t)col * p + r] : 0.0, 0.0);
  }
  const int nblk = (p - 1 + WY_NB - 1) / WY_NB;
  for (int b = nblk - 1; b >= 0; --b) {
    const int j0 = b * WY_NB;
    const int m = min(WY_NB, p - 1 - j0);
    // T_b to LDS (one entry per thread), in flight while the dots are formed
    for (int q = tid; q < WY_NB * WY_NB; q += WY_RT) Ts[q] = Tw[(int64_t)b * WY_NB * WY_NB + q];
    // partial dots v_i^H x over this thread's rows (v_i is zero for r <= j0 + i)
    double pr[WY_NB], pi[WY_NB];
#pragma unroll
    for (int i = 0; i < WY_NB; ++i) {
      pr[i] = 0.0;
      pi[i] = 0.0;
      // the stored reflectors carry explicit zeros above their support, so the
      // loads need no mask; rows past p are clamped and weighted by zero, and
      // i >= m reads the block's last reflector (its dot is not used)
      const cf64* vi = vs + (int64_t)(j0 + min(i, m - 1)) * p;
#pragma unroll
      for (int e = 0; e < MAXE; ++e) {
        const int r = tid + WY_RT * e;
        const cf64 a = vi[min(r, p - 1)];
        const double f = (r < p) ? 1.0 : 0.0;
        pr[i] += f * (a.x * x[e].x + a.y * x[e].y);
        pi[i] += f * (a.x * x[e].y - a.y * x[e].x);
      }
    }
#pragma unroll
    for (int i = 0; i < WY_NB; ++i) {
      const double sr = wave_sum_d(pr[i]);
      const double si = wave_sum_d(pi[i]);
      if (lane == 0) {
        red[wv][2 * i] = sr;
        red[wv][2 * i + 1] = si;
      }
    }
    __syncthreads();
    if (tid < WY_NB) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < WY_RT / 64; ++q) {
        sr += red[q][2 * tid];
        si += red[q][2 * tid + 1];
      }
      w[tid] = make_double2(sr, si);
    }
    __syncthreads();
    if (tid < m) {
      cf64 v = czero<cf64>();
#pragma unroll
      for (int l = 0; l < WY_NB; ++l)
        if (l >= tid && l < m) v = cadd(v, cmul(Ts[tid * WY_NB + l], w[l]));
      w2[tid] = v;
    }
    __syncthreads();
    // x -= V_b w2
#pragma unroll
    for (int i = 0; i < WY_NB; ++i) {
      const cf64* vi = vs + (int64_t)(j0 + min(i, m - 1)) * p;
      const cf64 c = (i < m) ? w2[i] : czero<cf64>();
#pragma unroll
      for (int e = 0; e < MAXE; ++e) {
        const int r = tid + WY_RT * e;
        const cf64 a = vi[min(r, p - 1)];  // rows past p are never stored
        x[e] = csub(x[e], cmul(c, a));
      }
    }
    __syncthreads();  // w, w2 and red are rewritten by the next block
  }
#pragma unroll
  for (int e = 0; e < MAXE; ++e) {
    const int r = tid + WY_RT * e;
    if (r < p) U[(int64_t)r * k + col] = x[e];
  }
}

// Larger sizes: one workgroup of WY_T threads per eigenvector column; the
// column lives in LDS and thread t owns its rows t + WY_T e.  Blocks are
// applied last to first, as above.  Each block is a chain of dots, one
// reduction, T w and the update, bound by latency; the rows loop at run time
// with the block's 16 reflector loads per row in flight, so the registers do
// not grow with p (the register form spills to scratch beyond p = 1024; up to
// there it is the faster one).
constexpr int WY_T = 1024;
__global__ __launch_bounds__(WY_T) void wy_apply_lds_kernel(const cf64* __restrict__ vs,
                                                            const cf64* __restrict__ Tw, int p,
                                                            const double* __restrict__ X, int k,
                                                            cf64* __restrict__ U) {
  extern __shared__ unsigned char wy_sm[];
  cf64* xS = reinterpret_cast<cf64*>(wy_sm);  // the column, p entries
  __shared__ double red[WY_T / 64][2 * WY_NB];
  __shared__ cf64 w[WY_NB], w2[WY_NB];
  __shared__ cf64 Ts[WY_NB * WY_NB];
  const int col = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int r = tid; r < p; r += WY_T) xS[r] = make_double2(X[(int64_t)col * p + r], 0.0);
  const int nblk = (p - 1 + WY_NB - 1) / WY_NB;
  for (int b = nblk - 1; b >= 0; --b) {
    const int j0 = b * WY_NB;
    const int m = min(WY_NB, p - 1 - j0);
    // T_b to LDS, in flight while the dots are formed
    for (int q = tid; q < WY_NB * WY_NB; q += WY_T) Ts[q] = Tw[(int64_t)b * WY_NB * WY_NB + q];
    // partial dots v_i^H x over this thread's rows.  The stored reflectors
    // carry explicit zeros above their support; i >= m reads the block's last
    // reflector (its dot is not used)
    double pr[WY_NB], pi[WY_NB];
#pragma unroll
    for (int i = 0; i < WY_NB; ++i) { pr[i] = 0.0; pi[i] = 0.0; }
    for (int r = tid; r < p; r += WY_T) {
      const cf64 xr = xS[r];
#pragma unroll
      for (int i = 0; i < WY_NB; ++i) {
        const cf64 a = vs[(int64_t)(j0 + min(i, m - 1)) * p + r];
        pr[i] += a.x * xr.x + a.y * xr.y;
        pi[i] += a.x * xr.y - a.y * xr.x;
      }
    }
#pragma unroll
    for (int i = 0; i < WY_NB; ++i) {
      const double sr = wave_sum_d(pr[i]);
      const double si = wave_sum_d(pi[i]);
      if (lane == 0) {
        red[wv][2 * i] = sr;
        red[wv][2 * i + 1] = si;
      }
    }
    __syncthreads();
    if (tid < WY_NB) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < WY_T / 64; ++q) {
        sr += red[q][2 * tid];
        si += red[q][2 * tid + 1];
      }
      w[tid] = make_double2(sr, si);
    }
    __syncthreads();
    if (tid < m) {
      cf64 v = czero<cf64>();
#pragma unroll
      for (int l = 0; l < WY_NB; ++l)
        if (l >= tid && l < m) v = cadd(v, cmul(Ts[tid * WY_NB + l], w[l]));
      w2[tid] = v;
    }
    __syncthreads();
    // x -= V_b w2 on this thread's rows
    for (int r = tid; r < p; r += WY_T) {
      cf64 xr = xS[r];
#pragma unroll
      for (int i = 0; i < WY_NB; ++i) {
        const cf64 c = (i < m) ? w2[i] : czero<cf64>();
        const cf64 a = vs[(int64_t)(j0 + min(i, m - 1)) * p + r];
        xr = csub(xr, cmul(c, a));
      }
      xS[r] = xr;
    }
    __syncthreads();  // w, w2, Ts and red are rewritten by the next block
  }
  for (int r = tid; r < p; r += WY_T) U[(int64_t)r * k + col] = xS[r];
}

size_t backtransform_wy_workspace(int p) { return (size_t)((p - 1 + WY_NB - 1) / WY_NB) * WY_NB * WY_NB; }

hipError_t launch_backtransform_wy(const cf64* vs, const cf64* taus, int p, const double* X, int k, cf64* U,
                                   cf64* Tws, hipStream_t st) {
  if (p < 2 || k < 1) return hipErrorInvalidValue;
  if (p > 3072) return launch_backtransform(vs, taus, p, X, k, U, st);
  const int nblk = (p - 1 + WY_NB - 1) / WY_NB;
  hipLaunchKernelGGL(wy_factor_kernel, dim3(nblk), dim3(256), 0, st, vs, taus, p, Tws);
  if (p <= WY_RT * 2)
    hipLaunchKernelGGL((wy_apply_reg_kernel<2>), dim3(k), dim3(WY_RT), 0, st, vs, Tws, p, X, k, U);
  else
    hipLaunchKernelGGL(wy_apply_lds_kernel, dim3(k), dim3(WY_T), (size_t)p * sizeof(cf64), st, vs, Tws, p, X, k,
                       U);
  return hipGetLastError();
}

hipError_t launch_backtransform(const cf64* vs, const cf64* taus, int p, const double* X, int k, cf64* U,
                                hipStream_t st) {
  if (p <= 64 * 8)
    hipLaunchKernelGGL((backtransform_reg_kernel<8, 1>), dim3(k), dim3(64), 0, st, vs, taus, p, X, k, U);
  else if (p <= 64 * 16)
    hipLaunchKernelGGL((backtransform_reg_kernel<16, 1>), dim3(k), dim3(64), 0, st, vs, taus, p, X, k, U);
  else if (p <= 64 * 24)
    hipLaunchKernelGGL((backtransform_reg_kernel<24, 1>), dim3(k), dim3(64), 0, st, vs, taus, p, X, k, U);
  else {
    const size_t shm = (size_t)p * sizeof(cf64);
    if (shm > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(backtransform_kernel, dim3(k), dim3(64), shm, st, vs, taus, p, X, k, U);
  }
  return hipGetLastError();
}
