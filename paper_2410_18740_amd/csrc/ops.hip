// Memory-bound helper kernels: local-operator application on the physical legs
// of a (chi_l, ds, dt, chi_r) tensor, linear combinations of environment
// channels, precision conversion, split-K reduction, and the FP64 Krylov
// vector kernels (multi-dot with fixed-order two-stage reduction, multi-axpy,
// scaling, linear combination).  All reductions are deterministic: block
// partials are combined in a fixed order, never with atomics.
#include <algorithm>
#include "common.h"

// ------------------------------------------------------------------ op apply
// Workgroup = one (job, a, b-chunk).  LDS holds the source slice src[s'][t'][b],
// a temporary after the t-leg operator, and the accumulator.
template <typename CT>
__global__ __launch_bounds__(256) void opapply_kernel(const OpJob* __restrict__ jobs, const OpTerm* __restrict__ terms,
                                                       int chi_l, int ds, int dt, int chi_r, int bw) {
  extern __shared__ unsigned char smem_raw[];
  CT* sm = reinterpret_cast<CT*>(smem_raw);
  const int dsdt = ds * dt;
  const int nb_chunks = (chi_r + bw - 1) / bw;
  const int job_id = blockIdx.y;
  const int a = blockIdx.x / nb_chunks;
  const int b0 = (blockIdx.x % nb_chunks) * bw;
  const int bcnt = min(bw, chi_r - b0);
  const int slice = dsdt * bw;
  CT* src = sm;
  CT* tmp = sm + slice;
  CT* acc = sm + 2 * slice;
  CT* opsm = sm + 3 * slice;  // ds*ds + dt*dt
  const OpJob job = jobs[job_id];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)a * dsdt * chi_r;  // element offset of [a][0][0][0]
  CT* dst = reinterpret_cast<CT*>(job.dst);

  for (int e = tid; e < dsdt * bcnt; e += 256) {
    const int st = e / bcnt, bb = e % bcnt;
    acc[st * bw + bb] = job.accumulate ? dst[base + (int64_t)st * chi_r + b0 + bb] : czero<CT>();
  }
  for (int t = 0; t < job.nterms; ++t) {
    const OpTerm term = terms[job.t0 + t];
    const CT* s = reinterpret_cast<const CT*>(term.src);
    const CT* oA = reinterpret_cast<const CT*>(term.opA);
    const CT* oB = reinterpret_cast<const CT*>(term.opB);
    __syncthreads();
    for (int e = tid; e < dsdt * bcnt; e += 256) {
      const int st = e / bcnt, bb = e % bcnt;
      src[st * bw + bb] = s[base + (int64_t)st * chi_r + b0 + bb];
    }
    for (int e = tid; e < ds * ds; e += 256) opsm[e] = oA ? oA[e] : czero<CT>();
    for (int e = tid; e < dt * dt; e += 256) opsm[ds * ds + e] = oB ? oB[e] : czero<CT>();
    __syncthreads();
    // stage 1: tmp[s'][t][b] = sum_t' opB[t][t'] src[s'][t'][b]
    const CT* in1 = src;
    if (oB) {
      for (int e = tid; e < dsdt * bcnt; e += 256) {
        const int st = e / bcnt, bb = e % bcnt;
        const int sp = st / dt, tt = st % dt;
        CT v = czero<CT>();
        for (int tp = 0; tp < dt; ++tp) v = cadd(v, cmul(opsm[ds * ds + tt * dt + tp], src[(sp * dt + tp) * bw + bb]));
        tmp[st * bw + bb] = v;
      }
      __syncthreads();
      in1 = tmp;
    }
    // stage 2: acc[s][t][b] += coef * sum_s' opA[s][s'] in1[s'][t][b]
    const typename real_of<CT>::type c = (typename real_of<CT>::type)term.coef;
    for (int e = tid; e < dsdt * bcnt; e += 256) {
      const int st = e / bcnt, bb = e % bcnt;
      const int ss = st / dt, tt = st % dt;
      CT v;
      if (oA) {
        v = czero<CT>();
        for (int sp = 0; sp < ds; ++sp) v = cadd(v, cmul(opsm[ss * ds + sp], in1[(sp * dt + tt) * bw + bb]));
      } else {
        v = in1[st * bw + bb];
      }
      acc[st * bw + bb] = cadd(acc[st * bw + bb], cscale(v, c));
    }
  }
  __syncthreads();
  for (int e = tid; e < dsdt * bcnt; e += 256) {
    const int st = e / bcnt, bb = e % bcnt;
    dst[base + (int64_t)st * chi_r + b0 + bb] = acc[st * bw + bb];
  }
}

// Register-blocked form for legs of at most MD states.  One-leg tensors (dt = 1):
// thread (a, bb) owns dst[a][0..ds)[b0 + bb] in registers, loads its column
// src[a][0..ds)[b] per term and applies the s-leg operator in registers.  Two
// legs (ds = dt): block = one (a, b-chunk), thread (t, bb) owns
// dst[a][0..ds)[t][b] in registers; a t-leg operator is applied first with
// thread (s, bb) owning src[a][s][0..dt)[b], and its result crosses to the
// (t, bb) owner through LDS.  Operators are staged in LDS and read as
// wave-uniform broadcasts, so LDS carries one write and one read per element
// and term instead of one read per multiply.
template <typename CT, int MD, bool TWO>
__global__ __launch_bounds__(256) void opapply_reg_kernel(const OpJob* __restrict__ jobs,
                                                           const OpTerm* __restrict__ terms, int chi_l, int ds,
                                                           int dt, int chi_r, int bw) {
  using RT = typename real_of<CT>::type;
  extern __shared__ unsigned char smem_raw[];
  __shared__ int bandS[2];  // one-leg form: bandwidth of the s-leg operator, slots alternate per term
  CT* opa = reinterpret_cast<CT*>(smem_raw);  // ds * ds
  CT* opb = opa + MD * MD;                    // dt * dt
  CT* tmp = opb + MD * MD;                    // [ds][dt][bw] (two legs)
  const int nb = (chi_r + bw - 1) / bw;
  const int tid = threadIdx.x;
  const int bb = tid % bw, row = tid / bw;
  const int b0 = (blockIdx.x % nb) * bw;
  const int b = b0 + bb;
  int a, t;
  if (TWO) {
    a = blockIdx.x / nb;
    t = row;  // < dt: the block has dt * bw threads
  } else {
    a = (blockIdx.x / nb) * (blockDim.x / bw) + row;
    t = 0;
  }
  const bool live = b < chi_r && a < chi_l;
  const OpJob job = jobs[blockIdx.y];
  CT* dst = reinterpret_cast<CT*>(job.dst);
  const int64_t sstride = (int64_t)dt * chi_r;                 // s -> s + 1
  const int64_t col = ((int64_t)a * ds * dt + t) * chi_r + b;  // [a][0][t][b]
  CT acc[MD];
#pragma unroll
  for (int s = 0; s < MD; ++s) acc[s] = czero<CT>();
  if (job.accumulate && live) {
#pragma unroll
    for (int s = 0; s < MD; ++s)
      if (s < ds) acc[s] = dst[col + s * sstride];
  }
  if (!TWO && tid == 0) { bandS[0] = 0; bandS[1] = 0; }
  for (int k = 0; k < job.nterms; ++k) {
    const OpTerm term = terms[job.t0 + k];
    const CT* src = reinterpret_cast<const CT*>(term.src);
    const CT* oA = reinterpret_cast<const CT*>(term.opA);
    const CT* oB = reinterpret_cast<const CT*>(term.opB);
    __syncthreads();  // the previous term is done with opa, opb, tmp and its band slot
    if (TWO) {
      for (int e = tid; e < ds * ds; e += blockDim.x) opa[e] = oA ? oA[e] : czero<CT>();
    } else {
      // stage the operator and record how far its nonzeros reach from the
      // diagonal (the Fock-basis operators are banded: |s' - s| <= 2)
      if (tid == 0) bandS[(k + 1) & 1] = 0;
      for (int e = tid; e < ds * ds; e += blockDim.x) {
        const CT o = oA ? oA[e] : czero<CT>();
        opa[e] = o;
        if (o.x != (RT)0 || o.y != (RT)0) atomicMax(&bandS[k & 1], abs(e / ds - e % ds));
      }
    }
    if (TWO)
      for (int e = tid; e < dt * dt; e += blockDim.x) opb[e] = oB ? oB[e] : czero<CT>();
    CT z[MD];
    if (TWO && oB) {
      // thread (s = row, bb): y[t'] = sum_t opB[t'][t] src[a][s][t][b]
      CT x[MD];
      const int sr = row;
      const int64_t c1 = ((int64_t)a * ds + sr) * dt * chi_r + b;
#pragma unroll
      for (int q = 0; q < MD; ++q) x[q] = (live && q < dt) ? src[c1 + q * chi_r] : czero<CT>();
      __syncthreads();  // opb staged
#pragma unroll
      for (int tp = 0; tp < MD; ++tp) {
        if (tp < dt) {
          CT v = czero<CT>();
#pragma unroll
          for (int q = 0; q < MD; ++q)
            if (q < dt) {
              const CT o = opb[tp * dt + q];
              v.x += o.x * x[q].x - o.y * x[q].y;
              v.y += o.x * x[q].y + o.y * x[q].x;
            }
          tmp[(sr * dt + tp) * bw + bb] = v;
        }
      }
      __syncthreads();  // tmp complete
#pragma unroll
      for (int s = 0; s < MD; ++s) z[s] = (s < ds) ? tmp[(s * dt + t) * bw + bb] : czero<CT>();
    } else {
#pragma unroll
      for (int s = 0; s < MD; ++s) z[s] = (live && s < ds) ? src[col + s * sstride] : czero<CT>();
      __syncthreads();  // opa staged
    }
    const RT c = (RT)term.coef;
    if (!TWO && oA) {
      // v[s'] = sum_s op[s'][s] z[s] along the diagonals the operator occupies;
      // for each s' the terms still come in increasing s, and the entries
      // skipped are zeros, so the sums are those of the dense loop
      const int band = __builtin_amdgcn_readfirstlane(bandS[k & 1]);
      CT v[MD];
#pragma unroll
      for (int sp = 0; sp < MD; ++sp) v[sp] = czero<CT>();
#pragma unroll
      for (int off = -(MD - 1); off <= MD - 1; ++off) {
        if (off < -band || off > band) continue;
#pragma unroll
        for (int sp = 0; sp < MD; ++sp) {
          const int sc = sp + off;
          if (sc < 0 || sc >= MD) continue;
          if (sp < ds && sc < ds) {
            const CT o = opa[sp * ds + sc];
            v[sp].x += o.x * z[sc].x - o.y * z[sc].y;
            v[sp].y += o.x * z[sc].y + o.y * z[sc].x;
          }
        }
      }
#pragma unroll
      for (int sp = 0; sp < MD; ++sp)
        if (sp < ds) {
          acc[sp].x += c * v[sp].x;
          acc[sp].y += c * v[sp].y;
        }
    } else if (oA) {
#pragma unroll
      for (int sp = 0; sp < MD; ++sp) {
        if (sp < ds) {
          CT v = czero<CT>();
#pragma unroll
          for (int s = 0; s < MD; ++s)
            if (s < ds) {
              const CT o = opa[sp * ds + s];
              v.x += o.x * z[s].x - o.y * z[s].y;
              v.y += o.x * z[s].y + o.y * z[s].x;
            }
          acc[sp].x += c * v.x;
          acc[sp].y += c * v.y;
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < MD; ++s) {
        acc[s].x += c * z[s].x;
        acc[s].y += c * z[s].y;
      }
    }
  }
  if (live) {
#pragma unroll
    for (int s = 0; s < MD; ++s)
      if (s < ds) dst[col + s * sstride] = acc[s];
  }
}

template <typename CT, int MD>
static void launch_opapply_reg(const OpJob* d_jobs, int njobs, const OpTerm* d_terms, int chi_l, int ds, int dt,
                               int chi_r, hipStream_t st) {
  const bool two = dt > 1;
  int cap = 1;
  while (cap < chi_r) cap <<= 1;
  int bw = 64;
  if (two) {
    while (bw > 1 && dt * bw > 256) bw >>= 1;
  }
  bw = std::min(bw, cap);
  const int nb = (chi_r + bw - 1) / bw;
  const size_t eb = sizeof(CT);
  if (two) {
    const size_t shm = (2 * MD * MD + (size_t)ds * dt * bw) * eb;
    dim3 grid(chi_l * nb, njobs);
    hipLaunchKernelGGL((opapply_reg_kernel<CT, MD, true>), grid, dim3(dt * bw), shm, st, d_jobs, d_terms, chi_l, ds,
                       dt, chi_r, bw);
  } else {
    const int rows = 256 / bw;
    const size_t shm = 2 * MD * MD * eb;
    dim3 grid(((chi_l + rows - 1) / rows) * nb, njobs);
    hipLaunchKernelGGL((opapply_reg_kernel<CT, MD, false>), grid, dim3(rows * bw), shm, st, d_jobs, d_terms, chi_l,
                       ds, dt, chi_r, bw);
  }
}

static int pick_bw(int elem_bytes, int dsdt, int ds, int dt, int chi_r) {
  const int budget = 96 * 1024;
  int bw = 64;
  while (bw > 1 && (3 * dsdt * bw + ds * ds + dt * dt) * elem_bytes > budget) bw >>= 1;
  if (bw > chi_r) {
    bw = 1;
    while (bw < chi_r) bw <<= 1;
  }
  return bw;
}

hipError_t launch_opapply(int prec, const OpJob* d_jobs, int njobs, const OpTerm* d_terms, int chi_l, int ds, int dt,
                          int chi_r, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  if ((dt == 1 || dt == ds) && ds <= 16) {
    const bool f64 = prec == PREC_FP64;
    if (ds <= 8) {
      if (f64) launch_opapply_reg<cf64, 8>(d_jobs, njobs, d_terms, chi_l, ds, dt, chi_r, st);
      else launch_opapply_reg<cf32, 8>(d_jobs, njobs, d_terms, chi_l, ds, dt, chi_r, st);
    } else if (ds <= 12) {  // d = 10, 12: fewer registers than the 16-state form, more waves
      if (f64) launch_opapply_reg<cf64, 12>(d_jobs, njobs, d_terms, chi_l, ds, dt, chi_r, st);
      else launch_opapply_reg<cf32, 12>(d_jobs, njobs, d_terms, chi_l, ds, dt, chi_r, st);
    } else {
      if (f64) launch_opapply_reg<cf64, 16>(d_jobs, njobs, d_terms, chi_l, ds, dt, chi_r, st);
      else launch_opapply_reg<cf32, 16>(d_jobs, njobs, d_terms, chi_l, ds, dt, chi_r, st);
    }
    return hipGetLastError();
  }
  const int eb = (prec == PREC_FP64) ? 16 : 8;
  const int bw = pick_bw(eb, ds * dt, ds, dt, chi_r);
  const int nb_chunks = (chi_r + bw - 1) / bw;
  dim3 grid(chi_l * nb_chunks, njobs);
  const size_t shm = (size_t)(3 * ds * dt * bw + ds * ds + dt * dt) * eb;
  if (prec == PREC_FP64)
    hipLaunchKernelGGL(opapply_kernel<cf64>, grid, dim3(256), shm, st, d_jobs, d_terms, chi_l, ds, dt, chi_r, bw);
  else
    hipLaunchKernelGGL(opapply_kernel<cf32>, grid, dim3(256), shm, st, d_jobs, d_terms, chi_l, ds, dt, chi_r, bw);
  return hipGetLastError();
}

// ------------------------------------------------------------------ env mixing
template <typename CT>
__global__ void envmix_kernel(const MixJob* __restrict__ jobs, const MixTerm* __restrict__ terms, int64_t n) {
  const MixJob job = jobs[blockIdx.y];
  CT* dst = reinterpret_cast<CT*>(job.dst);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    CT v = czero<CT>();
    for (int t = 0; t < job.nterms; ++t) {
      const MixTerm mt = terms[job.t0 + t];
      v = cadd(v, cscale(reinterpret_cast<const CT*>(mt.src)[e], (typename real_of<CT>::type)mt.coef));
    }
    dst[e] = v;
  }
}
hipError_t launch_envmix(int prec, const MixJob* d_jobs, int njobs, const MixTerm* d_terms, int64_t n_elem,
                         hipStream_t st) {
  if (njobs <= 0 || n_elem <= 0) return hipSuccess;
  int gx = (int)std::min<int64_t>((n_elem + 255) / 256, 1024);
  dim3 grid(gx, njobs);
  if (prec == PREC_FP64)
    hipLaunchKernelGGL(envmix_kernel<cf64>, grid, dim3(256), 0, st, d_jobs, d_terms, n_elem);
  else
    hipLaunchKernelGGL(envmix_kernel<cf32>, grid, dim3(256), 0, st, d_jobs, d_terms, n_elem);
  return hipGetLastError();
}

// ------------------------------------------------------------------ conversion
__global__ void cvt_64_32(cf32* dst, const cf64* src, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = make_float2((float)src[e].x, (float)src[e].y);
}
__global__ void cvt_32_64(cf64* dst, const cf32* src, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = make_double2((double)src[e].x, (double)src[e].y);
}
__global__ void cpy_64(cf64* dst, const cf64* src, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}
__global__ void cpy_32(cf32* dst, const cf32* src, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}
static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048)); }

hipError_t launch_convert(int to_prec, void* dst, int from_prec, const void* src, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const bool to64 = to_prec == PREC_FP64, from64 = from_prec == PREC_FP64;
  if (to64 && from64) hipLaunchKernelGGL(cpy_64, dim3(grid_for(n)), dim3(256), 0, st, (cf64*)dst, (const cf64*)src, n);
  else if (!to64 && from64) hipLaunchKernelGGL(cvt_64_32, dim3(grid_for(n)), dim3(256), 0, st, (cf32*)dst, (const cf64*)src, n);
  else if (to64 && !from64) hipLaunchKernelGGL(cvt_32_64, dim3(grid_for(n)), dim3(256), 0, st, (cf64*)dst, (const cf32*)src, n);
  else hipLaunchKernelGGL(cpy_32, dim3(grid_for(n)), dim3(256), 0, st, (cf32*)dst, (const cf32*)src, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ split-K reduction -> FP64
template <typename CT>
__global__ void reduce_partials_kernel(cf64* out, const CT* parts, int nparts, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int p = 0; p < nparts; ++p) {
      CT v = parts[(int64_t)p * n + e];
      re += (double)v.x;
      im += (double)v.y;
    }
    out[e] = make_double2(re, im);
  }
}
hipError_t launch_reduce_partials(cf64* out, int prec, const void* partials, int nparts, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (prec == PREC_FP64)
    hipLaunchKernelGGL(reduce_partials_kernel<cf64>, dim3(grid_for(n)), dim3(256), 0, st, out, (const cf64*)partials, nparts, n);
  else
    hipLaunchKernelGGL(reduce_partials_kernel<cf32>, dim3(grid_for(n)), dim3(256), 0, st, out, (const cf32*)partials, nparts, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Krylov vector kernels (FP64)
// wavefront-level tree reduction (fixed order) followed by a workgroup stage
static __device__ __forceinline__ double wave_sum(double v) { return wave_reduce_sum(v); }

#define MD_MAXV 72
int multidot_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 2047) / 2048, 512)); }

// partials[v][block] = sum_{e in block} conj(vs[v][e]) * w[e]
__global__ __launch_bounds__(256) void multidot_kernel(const cf64* const* __restrict__ vs, int nv,
                                                        const cf64* __restrict__ w, int64_t n, cf64* partials,
                                                        int nblocks) {
  __shared__ double red[2][4][MD_MAXV];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t per = (n + nblocks - 1) / nblocks;
  const int64_t e0 = (int64_t)blockIdx.x * per, e1 = min(n, e0 + per);
  for (int v = 0; v < nv; ++v) {
    const cf64* x = vs[v];
    double re = 0.0, im = 0.0;
    for (int64_t e = e0 + tid; e < e1; e += 256) {
      const cf64 a = x[e], b = w[e];
      re += a.x * b.x + a.y * b.y;
      im += a.x * b.y - a.y * b.x;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) { red[0][wave][v] = re; red[1][wave][v] = im; }
  }
  __syncthreads();
  for (int v = tid; v < nv; v += 256) {
    double re = red[0][0][v] + red[0][1][v] + red[0][2][v] + red[0][3][v];
    double im = red[1][0][v] + red[1][1][v] + red[1][2][v] + red[1][3][v];
    partials[(int64_t)v * nblocks + blockIdx.x] = make_double2(re, im);
  }
}
__global__ void multidot_finish_kernel(const cf64* partials, int nv, int nblocks, cf64* out) {
  const int v = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ double sre[64], sim[64];
  double re = 0.0, im = 0.0;
  for (int b = tid; b < nblocks; b += 64) {
    re += partials[(int64_t)v * nblocks + b].x;
    im += partials[(int64_t)v * nblocks + b].y;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (tid == 0) out[v] = make_double2(re, im);
  (void)sre; (void)sim;
}
hipError_t launch_multidot(const cf64* const* vs, int nv, const cf64* w, int64_t n, cf64* partials, int nblocks,
                           hipStream_t st) {
  if (nv <= 0) return hipSuccess;
  if (nv > MD_MAXV) return hipErrorInvalidValue;
  hipLaunchKernelGGL(multidot_kernel, dim3(nblocks), dim3(256), 0, st, vs, nv, w, n, partials, nblocks);
  return hipGetLastError();
}
hipError_t launch_multidot_finish(const cf64* partials, int nv, int nblocks, cf64* out, hipStream_t st) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(multidot_finish_kernel, dim3(nv), dim3(64), 0, st, partials, nv, nblocks, out);
  return hipGetLastError();
}

// Fused first update and second-pass dot products of classical Gram-Schmidt:
//   w <- w - sum_v coefs[v] vs[v];  partials[v][block] = <vs[v], w> (v < nv),
//   partials[nv][block] = <w, w>.
// Each chunk of 256 elements is updated (one element per thread), staged in
// LDS, and then dotted with every vs[v] by the wavefront that owns v (v = wave
// mod 4): the vs[v] reads of the dot pass hit the cache lines the update just
// brought in, so the basis makes one trip from memory instead of two.
#define AD_MAXV 72
#define AD_PER_WAVE (AD_MAXV / 4)
__global__ __launch_bounds__(256) void axpy_dot_kernel(cf64* __restrict__ w, const cf64* const* __restrict__ vs, int nv,
                                                       const cf64* __restrict__ coefs, int64_t n,
                                                       cf64* __restrict__ partials, int nblocks) {
  __shared__ cf64 cS[AD_MAXV];
  __shared__ cf64 accS[256];
  __shared__ double redw[2][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int v = tid; v < nv; v += 256) cS[v] = coefs[v];
  const int64_t per = (n + nblocks - 1) / nblocks;
  const int64_t e0 = (int64_t)blockIdx.x * per, e1 = min(n, e0 + per);
  double pr[AD_PER_WAVE], pi[AD_PER_WAVE];
#pragma unroll
  for (int q = 0; q < AD_PER_WAVE; ++q) { pr[q] = 0.0; pi[q] = 0.0; }
  double ww = 0.0;
  __syncthreads();
  for (int64_t c0 = e0; c0 < e1; c0 += 256) {
    const int64_t e = c0 + tid;
    cf64 acc = czero<cf64>();
    if (e < e1) {
      acc = w[e];
      for (int v = 0; v < nv; ++v) {
        const cf64 cc = cS[v];
        const cf64 x = vs[v][e];
        acc.x -= cc.x * x.x - cc.y * x.y;
        acc.y -= cc.x * x.y + cc.y * x.x;
      }
      w[e] = acc;
      ww += acc.x * acc.x + acc.y * acc.y;
    }
    accS[tid] = acc;
    __syncthreads();
    const int cnt = (int)min<int64_t>(256, e1 - c0);
#pragma unroll
    for (int q = 0; q < AD_PER_WAVE; ++q) {
      const int v = wave + 4 * q;
      if (v < nv) {
        const cf64* x = vs[v] + c0;
        for (int t = lane; t < cnt; t += 64) {
          const cf64 a = x[t], b = accS[t];
          pr[q] += a.x * b.x + a.y * b.y;
          pi[q] += a.x * b.y - a.y * b.x;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < AD_PER_WAVE; ++q) {
    const int v = wave + 4 * q;
    if (v < nv) {
      const double r = wave_sum(pr[q]), m = wave_sum(pi[q]);
      if (lane == 0) partials[(int64_t)v * nblocks + blockIdx.x] = make_double2(r, m);
    }
  }
  ww = wave_sum(ww);
  if (lane == 0) redw[0][wave] = ww;
  __syncthreads();
  if (tid == 0)
    partials[(int64_t)nv * nblocks + blockIdx.x] = make_double2(redw[0][0] + redw[0][1] + redw[0][2] + redw[0][3], 0.0);
}
hipError_t launch_axpy_dot(cf64* w, const cf64* const* vs, int nv, const cf64* coefs, int64_t n, cf64* partials,
                           int nblocks, hipStream_t st) {
  if (nv < 0 || nv > AD_MAXV || n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(axpy_dot_kernel, dim3(nblocks), dim3(256), 0, st, w, vs, nv, coefs, n, partials, nblocks);
  return hipGetLastError();
}

// dst = (w - sum_v coefs[v] vs[v]) * inv[0]: the second update fused with the
// normalisation into the next Krylov vector
__global__ void axpy_scale_kernel(cf64* __restrict__ dst, const cf64* __restrict__ w,
                                  const cf64* const* __restrict__ vs, int nv, const cf64* __restrict__ coefs,
                                  const double* __restrict__ inv, int64_t n) {
  const double f = inv[0];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    cf64 acc = w[e];
    for (int v = 0; v < nv; ++v) {
      const cf64 c = coefs[v];
      const cf64 x = vs[v][e];
      acc.x -= c.x * x.x - c.y * x.y;
      acc.y -= c.x * x.y + c.y * x.x;
    }
    dst[e] = make_double2(acc.x * f, acc.y * f);
  }
}
hipError_t launch_axpy_scale(cf64* dst, const cf64* w, const cf64* const* vs, int nv, const cf64* coefs,
                             const double* inv, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_scale_kernel, dim3(grid_for(n)), dim3(256), 0, st, dst, w, vs, nv, coefs, inv, n);
  return hipGetLastError();
}

// dst = sum_v coefs[v] * vs[v]  (real coefficients on device)
__global__ void lincomb_kernel(cf64* dst, const cf64* const* __restrict__ vs, int nv, const double* __restrict__ c,
                               int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int v = 0; v < nv; ++v) {
      const cf64 x = vs[v][e];
      re += c[v] * x.x;
      im += c[v] * x.y;
    }
    dst[e] = make_double2(re, im);
  }
}
hipError_t launch_lincomb(cf64* dst, const cf64* const* vs, int nv, const double* coefs_dev, int64_t n,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(n)), dim3(256), 0, st, dst, vs, nv, coefs_dev, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ batched transpose with precision change
// dst[b][j][i] = src[b][i][j]  (src FP64 complex rows x cols -> dst prec cols x rows)
template <typename CT>
__global__ void transpose_kernel(CT* dst, const cf64* src, int batch, int rows, int cols) {
  const int64_t per = (int64_t)rows * cols;
  const int64_t tot = per * batch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / per, r = e % per;
    const int i = (int)(r / cols), j = (int)(r % cols);
    const cf64 v = src[e];
    CT o;
    o.x = v.x; o.y = v.y;
    dst[b * per + (int64_t)j * rows + i] = o;
  }
}
hipError_t launch_transpose_from64(int prec, void* dst, const cf64* src, int batch, int rows, int cols,
                                   hipStream_t st) {
  const int64_t tot = (int64_t)batch * rows * cols;
  if (tot <= 0) return hipSuccess;
  if (prec == PREC_FP64)
    hipLaunchKernelGGL(transpose_kernel<cf64>, dim3(grid_for(tot)), dim3(256), 0, st, (cf64*)dst, src, batch, rows, cols);
  else
    hipLaunchKernelGGL(transpose_kernel<cf32>, dim3(grid_for(tot)), dim3(256), 0, st, (cf32*)dst, src, batch, rows, cols);
  return hipGetLastError();
}
// dst (FP64) [b][j][i] = src(prec)[b][i][j]
template <typename CT>
__global__ void transpose_to64_kernel(cf64* dst, const CT* src, int batch, int rows, int cols) {
  const int64_t per = (int64_t)rows * cols;
  const int64_t tot = per * batch;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / per, r = e % per;
    const int i = (int)(r / cols), j = (int)(r % cols);
    const CT v = src[e];
    dst[b * per + (int64_t)j * rows + i] = make_double2((double)v.x, (double)v.y);
  }
}
hipError_t launch_transpose_to64(int prec, cf64* dst, const void* src, int batch, int rows, int cols, hipStream_t st) {
  const int64_t tot = (int64_t)batch * rows * cols;
  if (tot <= 0) return hipSuccess;
  if (prec == PREC_FP64)
    hipLaunchKernelGGL(transpose_to64_kernel<cf64>, dim3(grid_for(tot)), dim3(256), 0, st, dst, (const cf64*)src, batch, rows, cols);
  else
    hipLaunchKernelGGL(transpose_to64_kernel<cf32>, dim3(grid_for(tot)), dim3(256), 0, st, dst, (const cf32*)src, batch, rows, cols);
  return hipGetLastError();
}
// dst = src * s (host scalar), FP64 complex
__global__ void scale_host_kernel(cf64* dst, const cf64* src, double s, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = make_double2(src[e].x * s, src[e].y * s);
}
hipError_t launch_scale_host(cf64* dst, const cf64* src, double s, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_host_kernel, dim3(grid_for(n)), dim3(256), 0, st, dst, src, s, n);
  return hipGetLastError();
}
// dst[k x n] = conj-transpose of src[n x k]
__global__ void ctranspose_kernel(cf64* dst, const cf64* src, int n, int k) {
  const int64_t tot = (int64_t)n * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);  // src[i][j]
    const cf64 v = src[e];
    dst[(int64_t)j * n + i] = make_double2(v.x, -v.y);
  }
}
hipError_t launch_ctranspose(cf64* dst, const cf64* src, int n, int k, hipStream_t st) {
  const int64_t tot = (int64_t)n * k;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(ctranspose_kernel, dim3(grid_for(tot)), dim3(256), 0, st, dst, src, n, k);
  return hipGetLastError();
}
// The recurrence scalars alone: alpha_j, beta_j (from the two Gram-Schmidt
// passes' dots) and 1/beta_j for the normalisation, with out[0..1] = alpha_j,
// beta_j for the host, which solves the small Ritz problem itself.
__global__ __launch_bounds__(64) void lanczos_ab_kernel(const cf64* h1, const cf64* h2, int j, int i0, double* alpha,
                                                        double* beta, double* inv, double* out) {
  const int lane = threadIdx.x;
  double part = 0.0;
  for (int i = i0 + lane; i <= j; i += 64) part += h2[i].x * h2[i].x + h2[i].y * h2[i].y;
  const double sum = wave_sum(part);
  if (lane == 0) {
    const double a = h1[j].x + h2[j].x;
    const double w2 = h2[j + 1].x - sum;
    const double b = sqrt(fmax(w2, 0.0));
    alpha[j] = a;
    beta[j] = b;
    inv[0] = (b > 0.0) ? 1.0 / b : 0.0;
    out[0] = a;
    out[1] = b;
  }
}
hipError_t launch_lanczos_ab(const cf64* h1, const cf64* h2, int j, int i0, double* alpha, double* beta, double* inv,
                             double* out, hipStream_t st) {
  if (i0 < 0 || i0 > j) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lanczos_ab_kernel, dim3(1), dim3(64), 0, st, h1, h2, j, i0, alpha, beta, inv, out);
  return hipGetLastError();
}

// inv[0] = 1 / sqrt(h[nv] - sum_{i < nv} |h_i|^2): the norm after a Gram-Schmidt
// update whose second-pass dots are h[0..nv) and whose <w, w> before it is h[nv]
__global__ __launch_bounds__(64) void inv_norm_kernel(const cf64* h, int nv, double* inv) {
  const int lane = threadIdx.x;
  double part = 0.0;
  for (int i = lane; i < nv; i += 64) part += h[i].x * h[i].x + h[i].y * h[i].y;
  const double sum = wave_sum(part);
  if (lane == 0) {
    const double w2 = h[nv].x - sum;
    inv[0] = (w2 > 0.0) ? 1.0 / sqrt(w2) : 0.0;
  }
}
hipError_t launch_inv_norm(const cf64* h, int nv, double* inv, hipStream_t st) {
  hipLaunchKernelGGL(inv_norm_kernel, dim3(1), dim3(64), 0, st, h, nv, inv);
  return hipGetLastError();
}
// non-finite check: flag[0] = 1 if any entry is NaN/Inf
__global__ void finite_check_kernel(const cf64* x, int64_t n, int* flag) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const cf64 v = x[e];
    if (!isfinite(v.x) || !isfinite(v.y)) flag[0] = 1;
  }
}
hipError_t launch_finite_check(const cf64* x, int64_t n, int* flag, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(finite_check_kernel, dim3(grid_for(n)), dim3(256), 0, st, x, n, flag);
  return hipGetLastError();
}
__global__ void fill_int_kernel(int* p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st) {
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}
// set boundary environment [[[1]]]
__global__ void set_one_kernel(void* p, int prec) {
  if (threadIdx.x == 0) {
    if (prec == PREC_FP64) ((cf64*)p)[0] = make_double2(1.0, 0.0);
    else ((cf32*)p)[0] = make_float2(1.f, 0.f);
  }
}
hipError_t launch_set_one(void* p, int prec, hipStream_t st) {
  hipLaunchKernelGGL(set_one_kernel, dim3(1), dim3(64), 0, st, p, prec);
  return hipGetLastError();
}
// dst[i*ldd + j] = conj?(src[i*lds + j]) for i < rows, j < cols (FP64 complex)
__global__ void copy2d_kernel(cf64* dst, int64_t ldd, const cf64* src, int64_t lds, int rows, int cols, int conj_t) {
  const int64_t tot = (int64_t)rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / cols), j = (int)(e % cols);
    const cf64 v = src[(int64_t)i * lds + j];
    if (conj_t) dst[(int64_t)j * ldd + i] = make_double2(v.x, -v.y);  // dst is cols x rows
    else dst[(int64_t)i * ldd + j] = v;
  }
}
hipError_t launch_copy2d(cf64* dst, int64_t ldd, const cf64* src, int64_t lds, int rows, int cols, int conj_t,
                         hipStream_t st) {
  const int64_t tot = (int64_t)rows * cols;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for(tot)), dim3(256), 0, st, dst, ldd, src, lds, rows, cols, conj_t);
  return hipGetLastError();
}
