// Complex GEMM on CDNA4 matrix cores (gfx950), three arithmetic forms:
//   FP64   : v_mfma_f64_16x16x4f64,  real-block complex product (4 real MFMAs)
//   FP32   : v_mfma_f32_32x32x2f32,  three real products per complex block
//            (P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); Re = P1 - P2,
//            Im = P3 - P1 - P2: the 3M method, 3 MFMAs instead of 4)
//   BF16x3 : v_mfma_f32_32x32x16_bf16, each FP32 operand split into bf16 hi + lo,
//            product ~ hi*hi + hi*lo + lo*hi with FP32 accumulation (12 MFMAs
//            per complex block product).
// Complex data are interleaved (re, im).  One workgroup = 4 waves (2 x 2),
// each wave owns a WM x WN output tile; K is staged through LDS in BK slices,
// stored k-major so that a half-wave reads 32 consecutive complex entries.
// A job may chain several K segments (sum_j A_j B_j): this is how the right
// environment contraction of the two-site matvec runs over all MPO channels.
#include "common.h"

typedef float v16f __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int PREC> struct GemmCfg;
template <> struct GemmCfg<PREC_FP32> {
  typedef cf32 CT;
  // 128 x 64 tiles at three workgroups per CU (168 VGPRs): measured faster
  // than 128 x 128 at one, since other waves' MFMAs cover each wave's LDS
  // reads, barriers and epilogue
  static constexpr int BM = 128, BN = 64, BK = 16, WM = 64, WN = 32, MB = 32, KSTEP = 2, MINB = 3;
};
template <> struct GemmCfg<PREC_BF16X3> {
  typedef cf32 CT;
  static constexpr int BM = 128, BN = 64, BK = 16, WM = 64, WN = 32, MB = 32, KSTEP = 16, MINB = 2;
};
template <> struct GemmCfg<PREC_FP64> {
  typedef cf64 CT;
  static constexpr int BM = 64, BN = 64, BK = 16, WM = 32, WN = 32, MB = 16, KSTEP = 4, MINB = 1;
};

static __device__ __forceinline__ __bf16 bf_from_bits(uint32_t b) {
  return __builtin_bit_cast(__bf16, (unsigned short)(b & 0xffffu));
}
// x ~ hi + lo with hi = RNE(x) to bf16, lo = RNE(x - hi) to bf16.
static __device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  uint32_t u = __float_as_uint(x);
  uint32_t hb = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
  float rem = x - __uint_as_float(hb);
  uint32_t v = __float_as_uint(rem);
  uint32_t lb = (v + 0x7fffu + ((v >> 16) & 1u)) >> 16;
  hi = bf_from_bits(hb >> 16);
  lo = bf_from_bits(lb);
}

// Operand loads through global-address-space pointers: the operand pointers
// come from the job tables, so without the cast they would be generic (flat)
// loads, which also count against the LDS wait counter and so would make every
// wait for the current tile's LDS reads wait for the next tile's prefetch too.
template <typename CT> struct RawOf;
template <> struct RawOf<cf32> { typedef float __attribute__((ext_vector_type(2))) T; };
template <> struct RawOf<cf64> { typedef double __attribute__((ext_vector_type(2))) T; };

template <typename CT, bool CONJ>
static __device__ __forceinline__ CT ld_g(const void* base, int64_t idx) {
  using R = typename RawOf<CT>::T;
  const __attribute__((address_space(1))) R* p = (const __attribute__((address_space(1))) R*)base;
  CT v = __builtin_bit_cast(CT, p[idx]);
  if (CONJ) v.y = -v.y;
  return v;
}

// Tile order.  Workgroup b runs on XCD b mod 8, and each XCD has its own L2.
// With the natural order (x = N tile fastest) the tiles of one row of a job
// share their A panel but sit on different XCDs whenever the row has few N
// tiles (the right contraction: N = chi_r, two tiles), so each XCD fetches the
// panel separately.  With xcd_rows set, XCD k instead takes the k-th
// contiguous eighth of the tiles in natural order, so the N tiles of a row run
// on one XCD one after the other and the panel is fetched once.  The map from
// workgroup id to tile is a bijection for any tile count.
static __device__ __forceinline__ void tile_of(int xcd_rows, int& bx, int& by, int& bz) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int id = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  int logical = id;
  if (xcd_rows) {
    const int T = gx * gy * gridDim.z;
    const int q = T >> 3, r = T & 7;
    const int xcd = id & 7, slot = id >> 3;
    logical = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + slot;
  }
  bx = logical % gx;
  by = (logical / gx) % gy;
  bz = logical / (gx * gy);
}

template <int PREC, bool TA, bool TB>
__global__ __launch_bounds__(256, GemmCfg<PREC>::MINB) void cgemm_kernel(const GemmJob* __restrict__ jobs,
                                                    const GemmSeg* __restrict__ segs, int accumulate, int xcd_rows) {
  using Cfg = GemmCfg<PREC>;
  using CT = typename Cfg::CT;
  constexpr int BM = Cfg::BM, BN = Cfg::BN, BK = Cfg::BK, WM = Cfg::WM, WN = Cfg::WN, MB = Cfg::MB;
  constexpr int NI = WM / MB, NJ = WN / MB;
  constexpr int NT = 256;
  constexpr int NA = BM * BK / NT, NB = BK * BN / NT;
  // double-buffered LDS tiles, k-major; one barrier per K tile, the next
  // tile's global loads are in flight (in registers) while the current one
  // feeds the matrix cores.  BF16x3 keeps its tiles already split: four bf16
  // planes (hi and lo of the real and imaginary parts), each laid out as
  // [k / 8][row][k % 8] so that a lane reads its eight k values of one row
  // for v_mfma_f32_32x32x16_bf16 with one 16-byte load, and each element is
  // split once per workgroup instead of once per wave that reads it.
  constexpr bool HSPLIT = PREC == PREC_BF16X3;
  constexpr int SMB = HSPLIT ? 2 * 4 * BK * (BM + BN) * 2 : 2 * BK * ((BM + 1) + (BN + 1)) * (int)sizeof(CT);
  __shared__ __align__(16) unsigned char smraw[SMB];
  auto As = reinterpret_cast<CT(*)[BK][BM + 1]>(smraw);
  auto Bs = reinterpret_cast<CT(*)[BK][BN + 1]>(smraw + 2 * BK * (BM + 1) * sizeof(CT));
  auto Ah = reinterpret_cast<__bf16(*)[4][BK / 8][BM][8]>(smraw);
  auto Bh = reinterpret_cast<__bf16(*)[4][BK / 8][BN][8]>(smraw + 2 * 4 * BK * BM * 2);

  int bx, by, bz;
  tile_of(xcd_rows, bx, by, bz);
  const GemmJob job = jobs[bz];
  const int m0 = by * BM, n0 = bx * BN;
  if (m0 >= job.M || n0 >= job.N) return;
  const int M = job.M, N = job.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;

  typedef typename std::conditional<PREC == PREC_FP64, v4d, v16f>::type AccT;
  // FP32 (3M): accR = P1, accX = P2, accI = P3; other forms: accR = Re, accI = Im
  AccT accR[NI][NJ], accI[NI][NJ], accX[NI][NJ];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      accR[i][j] = AccT{};
      accI[i][j] = AccT{};
      accX[i][j] = AccT{};
    }

  // flattened K-tile sequence over the job's segments
  int ld_seg = 0, ld_k0 = 0;  // next tile to load
  GemmSeg sg = segs[job.seg0];
  CT ra[NA], rb[NB];
  auto load_tile = [&]() {
    const int K = sg.K;
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int idx = tid + t * NT;
      int mm, kk;
      if (!TA) { mm = idx / BK; kk = idx % BK; }
      else     { kk = idx / BM; mm = idx % BM; }
      const int gm = m0 + mm, gk = ld_k0 + kk;
      CT v = czero<CT>();
      if (gm < M && gk < K)
        v = TA ? ld_g<CT, true>(sg.A, (int64_t)gk * sg.lda + gm) : ld_g<CT, false>(sg.A, (int64_t)gm * sg.lda + gk);
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int idx = tid + t * NT;
      int kk, nn;
      if (!TB) { kk = idx / BN; nn = idx % BN; }
      else     { nn = idx / BK; kk = idx % BK; }
      const int gn = n0 + nn, gk = ld_k0 + kk;
      CT v = czero<CT>();
      if (gn < N && gk < K)
        v = TB ? ld_g<CT, true>(sg.B, (int64_t)gn * sg.ldb + gk) : ld_g<CT, false>(sg.B, (int64_t)gk * sg.ldb + gn);
      rb[t] = v;
    }
    // advance to the next tile
    ld_k0 += BK;
    if (ld_k0 >= sg.K && ld_seg + 1 < job.nseg) {
      ++ld_seg;
      ld_k0 = 0;
      sg = segs[job.seg0 + ld_seg];
    } else if (ld_k0 >= sg.K) {
      ld_seg = job.nseg;  // exhausted
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int idx = tid + t * NT;
      int mm, kk;
      if (!TA) { mm = idx / BK; kk = idx % BK; }
      else     { kk = idx / BM; mm = idx % BM; }
      if constexpr (HSPLIT) {
        __bf16 h, l;
        split_bf16(ra[t].x, h, l);
        Ah[buf][0][kk >> 3][mm][kk & 7] = h;
        Ah[buf][1][kk >> 3][mm][kk & 7] = l;
        split_bf16(ra[t].y, h, l);
        Ah[buf][2][kk >> 3][mm][kk & 7] = h;
        Ah[buf][3][kk >> 3][mm][kk & 7] = l;
      } else {
        As[buf][kk][mm] = ra[t];
      }
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int idx = tid + t * NT;
      int kk, nn;
      if (!TB) { kk = idx / BN; nn = idx % BN; }
      else     { nn = idx / BK; kk = idx % BK; }
      if constexpr (HSPLIT) {
        __bf16 h, l;
        split_bf16(rb[t].x, h, l);
        Bh[buf][0][kk >> 3][nn][kk & 7] = h;
        Bh[buf][1][kk >> 3][nn][kk & 7] = l;
        split_bf16(rb[t].y, h, l);
        Bh[buf][2][kk >> 3][nn][kk & 7] = h;
        Bh[buf][3][kk >> 3][nn][kk & 7] = l;
      } else {
        Bs[buf][kk][nn] = rb[t];
      }
    }
  };

  load_tile();
  store_tile(0);
  __syncthreads();
  int buf = 0;
  while (true) {
    const bool more = ld_seg < job.nseg;
    if (more) load_tile();

    if constexpr (PREC == PREC_FP32) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        float ar[NI], ai[NI], sa[NI], br[NJ], bi[NJ], sb[NJ];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          CT v = As[buf][kk + (lane >> 5)][wm0 + 32 * i + (lane & 31)];
          ar[i] = v.x; ai[i] = v.y; sa[i] = v.x + v.y;
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          CT v = Bs[buf][kk + (lane >> 5)][wn0 + 32 * j + (lane & 31)];
          br[j] = v.x; bi[j] = v.y; sb[j] = v.x + v.y;
        }
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            accR[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i], br[j], accR[i][j], 0, 0, 0);
            accX[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[i], bi[j], accX[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[i], sb[j], accI[i][j], 0, 0, 0);
          }
      }
    } else if constexpr (PREC == PREC_FP64) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double ar[NI], ai[NI], br[NJ], bi[NJ];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          CT v = As[buf][kk + (lane >> 4)][wm0 + 16 * i + (lane & 15)];
          ar[i] = v.x; ai[i] = v.y;
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          CT v = Bs[buf][kk + (lane >> 4)][wn0 + 16 * j + (lane & 15)];
          br[j] = v.x; bi[j] = v.y;
        }
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], accR[i][j], 0, 0, 0);
            accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bi[j], accR[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], accI[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], accI[i][j], 0, 0, 0);
          }
      }
    } else {  // BF16x3
#pragma unroll
      for (int kk = 0; kk < BK; kk += 16) {
        v8bf arh[NI], arl[NI], aih[NI], ail[NI], naih[NI], nail[NI];
        v8bf brh[NJ], brl[NJ], bih[NJ], bil[NJ];
        // lane l holds row l % 32 and k = kk + 8 (l / 32) + t, t < 8
        const int kg = (kk >> 3) + (lane >> 5);
        auto ld8 = [](const __bf16* q) { return *reinterpret_cast<const v8bf*>(q); };
        auto neg8 = [](v8bf x) {  // flip the sign bit of each bf16
          typedef unsigned int u4 __attribute__((ext_vector_type(4)));
          return __builtin_bit_cast(v8bf, __builtin_bit_cast(u4, x) ^ (u4)0x80008000u);
        };
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          const int m = wm0 + 32 * i + (lane & 31);
          arh[i] = ld8(Ah[buf][0][kg][m]);
          arl[i] = ld8(Ah[buf][1][kg][m]);
          aih[i] = ld8(Ah[buf][2][kg][m]);
          ail[i] = ld8(Ah[buf][3][kg][m]);
          naih[i] = neg8(aih[i]);
          nail[i] = neg8(ail[i]);
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int nn = wn0 + 32 * j + (lane & 31);
          brh[j] = ld8(Bh[buf][0][kg][nn]);
          brl[j] = ld8(Bh[buf][1][kg][nn]);
          bih[j] = ld8(Bh[buf][2][kg][nn]);
          bil[j] = ld8(Bh[buf][3][kg][nn]);
        }
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            v16f r = accR[i][j], m = accI[i][j];
            r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh[i], brh[j], r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh[i], brl[j], r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl[i], brh[j], r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(naih[i], bih[j], r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(naih[i], bil[j], r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nail[i], bih[j], r, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh[i], bih[j], m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh[i], bil[j], m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl[i], bih[j], m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih[i], brh[j], m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih[i], brl[j], m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail[i], brh[j], m, 0, 0, 0);
            accR[i][j] = r; accI[i][j] = m;
          }
      }
    }
    if (!more) break;
    store_tile(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // ---- epilogue
  CT* __restrict__ C = reinterpret_cast<CT*>(job.C);
  const int64_t ldc = job.ldc;
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if constexpr (PREC == PREC_FP64) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // v_mfma_f64_16x16x4f64: accumulator r of lane l holds D[l/16 + 4r][l%16]
          const int row = m0 + wm0 + 16 * i + (lane >> 4) + 4 * r;
          const int col = n0 + wn0 + 16 * j + (lane & 15);
          if (row < M && col < N) {
            CT v = cmk(accR[i][j][r], accI[i][j][r]);
            CT* p = C + (int64_t)row * ldc + col;
            if (accumulate) v = cadd(v, *p);
            *p = v;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          // 32x32 outputs: accumulator r of lane l holds D[8(r/4) + 4(l/32) + r%4][l%32]
          const int row = m0 + wm0 + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int col = n0 + wn0 + 32 * j + (lane & 31);
          if (row < M && col < N) {
            CT v;
            if constexpr (PREC == PREC_FP32) {
              const float p1 = accR[i][j][r], p2 = accX[i][j][r];
              v = cmk(p1 - p2, accI[i][j][r] - p1 - p2);
            } else {
              v = cmk(accR[i][j][r], accI[i][j][r]);
            }
            CT* p = C + (int64_t)row * ldc + col;
            if (accumulate) v = cadd(v, *p);
            *p = v;
          }
        }
      }
    }
}

template <int PREC>
static hipError_t launch_prec(int ta, int tb, const GemmJob* jobs, int njobs, const GemmSeg* segs, int maxM,
                              int maxN, int acc, hipStream_t st) {
  using Cfg = GemmCfg<PREC>;
  if (njobs <= 0 || maxM <= 0 || maxN <= 0) return hipSuccess;
  dim3 grid((maxN + Cfg::BN - 1) / Cfg::BN, (maxM + Cfg::BM - 1) / Cfg::BM, njobs);
  dim3 block(256);
  // rows of at most 8 N tiles keep their tiles on one XCD (see tile_of); wide
  // rows keep the natural order, which already keeps each B column panel on
  // one XCD across jobs
  const int xr = (grid.x >= 2 && grid.x <= 8) ? 1 : 0;
  if (!ta && !tb) hipLaunchKernelGGL((cgemm_kernel<PREC, false, false>), grid, block, 0, st, jobs, segs, acc, xr);
  else if (ta && !tb) hipLaunchKernelGGL((cgemm_kernel<PREC, true, false>), grid, block, 0, st, jobs, segs, acc, xr);
  else if (!ta && tb) hipLaunchKernelGGL((cgemm_kernel<PREC, false, true>), grid, block, 0, st, jobs, segs, acc, xr);
  else hipLaunchKernelGGL((cgemm_kernel<PREC, true, true>), grid, block, 0, st, jobs, segs, acc, xr);
  return hipGetLastError();
}

hipError_t launch_cgemm(int prec, int trans_a, int trans_b, const GemmJob* d_jobs, int njobs, const GemmSeg* d_segs,
                        int maxM, int maxN, int accumulate, hipStream_t st) {
  switch (prec) {
    case PREC_FP64: return launch_prec<PREC_FP64>(trans_a, trans_b, d_jobs, njobs, d_segs, maxM, maxN, accumulate, st);
    case PREC_FP32: return launch_prec<PREC_FP32>(trans_a, trans_b, d_jobs, njobs, d_segs, maxM, maxN, accumulate, st);
    case PREC_BF16X3:
      return launch_prec<PREC_BF16X3>(trans_a, trans_b, d_jobs, njobs, d_segs, maxM, maxN, accumulate, st);
  }
  return hipErrorInvalidValue;
}
