// L2 / NRMSE-bounded mode: the paper's own error control (Sec. 2.4), with
// the local-subspace basis of every block.
//
// The user's target eps_t,v is a relative L2 error (the NRMSE of Sec. 2.4,
// as a fraction).  The global budget is eps_v = eps_t,v ||u_v|| and every
// block receives the equal share e2 = c_v M_b W_b, c_v = eps_v^2 / K_v, of
// the squared budget (Eq. (4) and the text after it).  Per block:
//   rank  r = 0 when the whole energy fits 0.36 e2, else the smallest r >= 1
//         whose eigenvalue tail (its squared projection error, Eckart-Young)
//         is <= 0.36 e2 -- the plain eigensolve gives it when the variable's
//         bound is sqrt(0.36 c_v);
//   basis qV = rint(V_r 2^24); coefficients A = X^T V_r in FP64, step
//         d = 0.4 sqrt(e2 / (r M)), qA = rint(A / d);
//   check the exact error of the decoder's values, sum (x - xhat)^2 with
//         xhat = dtype(sum_k (qV 2^-24)(qA d)) summed over k in order, must
//         be <= e2; a failing block is encoded again at r + 1 (Alg. 1 step 3:
//         candidates are tested until the tolerance holds), and stored
//         verbatim (raw) past the rank cap or when a coefficient overflows.
//
//   k_l2_gram     the slices' Gram partials in FP64 (matrix cores) and the
//                 sums of squares of their finite values
//   k_l2_fsq_part / k_l2_budget   c_v and the eigensolve bound sqrt(0.36 c_v)
//   k_l2_params   per block: budget, rank (first pass), step, payload sizes
//   k_l2_encode   one workgroup per slice: projection, quantization, the
//                 decoder's values and the slice's squared error
//   k_l2_check    per block: the error against the budget; raises the rank
//   k_l2_decode   one workgroup per slice: the decoder
//
// Compiled with -ffp-contract=off: encoder and decoder must round the
// reconstruction identically.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dls_device.h"
#include "dls_kernels.h"

namespace dls {
namespace {

constexpr int64_t kL2LaunchItems = int64_t(1) << 23;
constexpr double kL2TailShare = 0.36;
constexpr double kL2StepShare = 0.4;
constexpr double kL2BasisScale = 16777216.0;       // 2^24
constexpr double kL2BasisUnit = 1.0 / 16777216.0;  // 2^-24

__device__ __forceinline__ uint32_t zz32(int32_t v) { return (uint32_t(v) << 1) ^ uint32_t(v >> 31); }
__device__ __forceinline__ int32_t unzz32(uint32_t z) { return int32_t(z >> 1) ^ -int32_t(z & 1); }

typedef double f64x4 __attribute__((ext_vector_type(4)));

// One slice's four consecutive points of one time row (zero past the
// slice's end, or for a padded row); `cont` when the four are one aligned
// run in memory (a block whose patch rows are 16-byte aligned runs of 4k
// values, and slices that start on a patch row).
template <typename T>
__device__ __forceinline__ void l2_load4(const T* row, int p0, int pb, int np, bool cont, int px, int py,
                                         int64_t nx, int64_t nxy, double x[4]) {
  if (row == nullptr) {
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = 0.0;
    return;
  }
  if (cont && pb + 3 < np) {
    const int64_t off = point_off(p0 + pb, px, py, nx, nxy);
    if constexpr (sizeof(T) == 4) {
      const float4 v = *reinterpret_cast<const float4*>(row + off);
      x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] = double(row[off + j]);
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
    x[j] = pb + j < np ? double(row[point_off(p0 + pb + j, px, py, nx, nxy)]) : 0.0;
}

// The Gram partial of one slice in FP64 (the L2 mode's ranks come from
// eigenvalue tails compared with 0.36 e2, which at tight targets is ~1e-8 of
// the block's energy: an FP32-accumulated Gram cannot resolve it), on the
// FP64 matrix cores: v_mfma_f64_16x16x4f64 takes 16 rows x 4 points, lane l
// holding row l % 16 of point slot l / 16, and the same register feeds both
// operands (G = X X^T).  A lane loads four consecutive points of its row and
// gives one to each of four MFMAs, so a wave covers 16 points per step and
// the four waves of the workgroup interleave.  Also the sum of squares of
// the slice's finite values (the variable's norm, for the budget).
template <int WP, typename T>
__global__ __launch_bounds__(256) void k_l2_gram(const T* __restrict__ F, Dims dims,
                                                 const BlockDesc* __restrict__ desc,
                                                 const Item* __restrict__ items, int64_t nitems,
                                                 double* __restrict__ gpart, double* __restrict__ fsq) {
  constexpr int NT = WP == 16 ? 1 : 3;  // tiles 00 (and 01, 11)
  constexpr int LDR = 68;                // staged row: 64 points + 4 floats of padding
  constexpr size_t kStage = size_t(4) * WP * LDR * sizeof(float);
  constexpr size_t kRed = size_t(4) * NT * 64 * sizeof(f64x4);
  __shared__ __align__(16) char smem[kStage > kRed ? kStage : kRed];
  f64x4 (*red)[NT][64] = reinterpret_cast<f64x4 (*)[NT][64]>(smem);
  __shared__ double fred[4];
  const int64_t i = blockIdx.x;
  if (i >= nitems) return;
  const Item it = items[i];
  const BlockDesc d = desc[it.block];
  const int W = d.w();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = lane & 15, slot = lane >> 4;
  const int64_t nxy = dims.nx * dims.ny, tstride = dims.nz * nxy;
  const T* base = F + fidx(dims, d.var, d.t0, d.z0, d.y0, d.x0);
  const T* row0 = t < W ? base + int64_t(t) * tstride : nullptr;
  const T* row1 = (WP == 32 && t + 16 < W) ? base + int64_t(t + 16) * tstride : nullptr;
  const bool cont = d.vec != 0;
  const int px = d.px(), py = d.py();
  f64x4 acc[NT];
#pragma unroll
  for (int a = 0; a < NT; ++a) acc[a] = f64x4{0.0, 0.0, 0.0, 0.0};
  double fs = 0.0;
  if (sizeof(T) == 4 && cont) {
    // FP32 rows of 4-aligned points: each load instruction covers 4 time
    // rows x 64 consecutive points of a chunk (full cache lines), CPW chunks'
    // loads issued together; a chunk goes through LDS into the MFMA operand
    // layout (lane (slot, t): row t, points 16 j + 4 slot + e of the chunk,
    // MFMA 4 j + e)
    constexpr int CPW = WP == 16 ? 4 : 2;
    float* stage = reinterpret_cast<float*>(smem) + wave * WP * LDR;
    const int lr = lane >> 4, lp = 4 * (lane & 15);
    for (int c0 = wave; c0 * 64 < it.np; c0 += 4 * CPW) {
      float4 raw[CPW][WP / 4];
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        const int ps = (c0 + 4 * u) * 64 + lp;
        const bool okp = ps < it.np;
        const int64_t off = point_off(it.p0 + (okp ? ps : 0), px, py, dims.nx, nxy);
#pragma unroll
        for (int g = 0; g < WP / 4; ++g) {
          const int tt = 4 * g + lr;
          raw[u][g] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (okp && tt < W)
            raw[u][g] = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(base) +
                                                         int64_t(tt) * tstride + off);
        }
      }
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        if ((c0 + 4 * u) * 64 >= it.np) continue;
#pragma unroll
        for (int g = 0; g < WP / 4; ++g)
          *reinterpret_cast<float4*>(stage + (4 * g + lr) * LDR + lp) = raw[u][g];
        wave_sync();
        double v0[16], v1[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float4 a4 = *reinterpret_cast<const float4*>(stage + t * LDR + 16 * j + 4 * slot);
          v0[4 * j] = a4.x; v0[4 * j + 1] = a4.y; v0[4 * j + 2] = a4.z; v0[4 * j + 3] = a4.w;
          if (WP == 32) {
            const float4 b4 = *reinterpret_cast<const float4*>(stage + (16 + t) * LDR + 16 * j + 4 * slot);
            v1[4 * j] = b4.x; v1[4 * j + 1] = b4.y; v1[4 * j + 2] = b4.z; v1[4 * j + 3] = b4.w;
          }
        }
        wave_sync();
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          fs += isfinite(v0[m]) ? v0[m] * v0[m] : 0.0;
          acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(v0[m], v0[m], acc[0], 0, 0, 0);
          if (WP == 32) {
            fs += isfinite(v1[m]) ? v1[m] * v1[m] : 0.0;
            acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(v0[m], v1[m], acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(v1[m], v1[m], acc[2], 0, 0, 0);
          }
        }
      }
    }
  } else {
    for (int c = wave * 16; c < it.np; c += 64) {
      const int pb = c + 4 * slot;
      double x0[4], x1[4];
      l2_load4(row0, it.p0, pb, it.np, cont, px, py, dims.nx, nxy, x0);
      if (WP == 32) l2_load4(row1, it.p0, pb, it.np, cont, px, py, dims.nx, nxy, x1);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        fs += isfinite(x0[j]) ? x0[j] * x0[j] : 0.0;
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[j], x0[j], acc[0], 0, 0, 0);
        if (WP == 32) {
          fs += isfinite(x1[j]) ? x1[j] * x1[j] : 0.0;
          acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[j], x1[j], acc[1], 0, 0, 0);
          acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[j], x1[j], acc[2], 0, 0, 0);
        }
      }
    }
  }
  __syncthreads();  // every wave is done with its staging area before it becomes `red`
#pragma unroll
  for (int a = 0; a < NT; ++a) red[wave][a][lane] = acc[a];
  fs = wave_sum(fs);
  if (lane == 0) fred[wave] = fs;
  __syncthreads();
  // the FP64 accumulator holds D[l / 16 + 4 v][l % 16] in lane l, element v
  // (not the FP32 instruction's D[4 (l / 16) + v][l % 16]); the four waves'
  // partials are summed in wave order
  double* out = gpart + i * WP * WP;
  const int ei = int(threadIdx.x) >> 4, ej = int(threadIdx.x) & 15;
  const int l = ej + 16 * (ei & 3), v = ei >> 2;
#pragma unroll
  for (int a = 0; a < NT; ++a) {
    double g = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) g += red[w][a][l][v];
    if (a == 0) {
      out[ei * WP + ej] = g;
    } else if (a == 1) {
      out[ei * WP + 16 + ej] = g;
      out[(16 + ej) * WP + ei] = g;
    } else {
      out[(16 + ei) * WP + 16 + ej] = g;
    }
  }
  if (threadIdx.x == 0) fsq[i] = ((fred[0] + fred[1]) + fred[2]) + fred[3];
}

// c_v = (eps_t,v)^2 ||u_v||^2 / K_v and the eigensolve's bound sqrt(0.36 c_v);
// ||u_v||^2 is the sum of the variable's slices' finite sums of squares (the
// plan tiles the field, so every value is in exactly one slice).  The
// slices of variable v are the contiguous range [range[2v], range[2v + 1])
// (blocks are variable-major); a fixed grid of partial sums, then the
// partials in order.
constexpr int kL2Parts = 256;

__global__ __launch_bounds__(256) void k_l2_fsq_part(const double* __restrict__ fsq,
                                                     const int64_t* __restrict__ range,
                                                     double* __restrict__ part) {
  __shared__ double red[256];
  const int v = blockIdx.y;
  const int64_t i0 = range[2 * v], i1 = range[2 * v + 1];
  double s = 0.0;
  for (int64_t i = i0 + int64_t(blockIdx.x) * 256 + threadIdx.x; i < i1; i += int64_t(kL2Parts) * 256) s += fsq[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[int64_t(v) * kL2Parts + blockIdx.x] = red[0];
}

__global__ void k_l2_budget(const double* __restrict__ part, const double* __restrict__ target, int64_t per_var,
                            int nvars, double* __restrict__ cv, double* __restrict__ eig_eps) {
  const int v = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= nvars) return;
  double s = 0.0;
  for (int j = 0; j < kL2Parts; ++j) s += part[int64_t(v) * kL2Parts + j];
  const double c = target[v] * target[v] * s / double(per_var);
  cv[v] = c;
  eig_eps[v] = sqrt(kL2TailShare * c);
}

// first: the rank from the eigensolve (0 when the energy fits the tail
// share); later passes keep the rank the check set
__global__ __launch_bounds__(256) void k_l2_params(const BlockDesc* __restrict__ desc, int64_t nblocks,
                                                   const double* __restrict__ lam, int wp,
                                                   const uint8_t* __restrict__ eig_rank,
                                                   const double* __restrict__ cv, int first, int esize,
                                                   uint8_t* __restrict__ l2rank, double* __restrict__ step,
                                                   double* __restrict__ e2, int64_t* __restrict__ qv_size,
                                                   int64_t* __restrict__ qa_size) {
  const int64_t b = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (b >= nblocks) return;
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m;
  const double eb = cv[d.var] * double(M) * double(W);
  int r;
  if (first) {
    if (eig_rank[b] == 0) {
      r = kL2Raw;  // non-finite input
    } else {
      double tr = 0.0;
      for (int k = 0; k < wp; ++k) tr += lam[b * wp + k];
      r = tr <= kL2TailShare * eb ? 0 : int(eig_rank[b]);
      if (r > 0 && !(eb > 0.0)) r = kL2Raw;
    }
    l2rank[b] = uint8_t(r);
  } else {
    r = l2rank[b];
  }
  e2[b] = eb;
  if (r == kL2Raw) {
    step[b] = 0.0;
    qv_size[b] = 0;
    qa_size[b] = pad16(int64_t(W) * M * esize);
  } else if (r == 0) {
    step[b] = 0.0;
    qv_size[b] = 0;
    qa_size[b] = 0;
  } else {
    step[b] = kL2StepShare * sqrt(eb / (double(r) * double(M)));
    qv_size[b] = 4 * pad16(int64_t(W) * r);
    qa_size[b] = 4 * pad16(int64_t(M) * r);
  }
}

// PPT consecutive points of one time row as one aligned vector load (the
// run is contiguous and aligned: a block whose patch rows are 16-byte
// aligned runs of 4k values, the run starting at a multiple of PPT).
template <typename T, int PPT>
__device__ __forceinline__ void l2_load_run(const T* __restrict__ src, T (&v)[PPT]) {
  if constexpr (sizeof(T) == 4 && PPT == 4) {
    const float4 a = *reinterpret_cast<const float4*>(src);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  } else if constexpr (sizeof(T) == 4 && PPT == 2) {
    const float2 a = *reinterpret_cast<const float2*>(src);
    v[0] = a.x; v[1] = a.y;
  } else if constexpr (sizeof(T) == 8 && PPT == 2) {
    const double2 a = *reinterpret_cast<const double2*>(src);
    v[0] = a.x; v[1] = a.y;
  } else {
#pragma unroll
    for (int e = 0; e < PPT; ++e) v[e] = src[e];
  }
}

// One workgroup per slice; each thread takes PPT consecutive points (every
// step's values of all of them loaded before the first use, so a slice is
// one round of loads), then encodes them one after the other.
template <int WP, typename T>
__global__ __launch_bounds__(256) void k_l2_encode(const T* __restrict__ F, Dims dims,
                                                   const BlockDesc* __restrict__ desc,
                                                   const Item* __restrict__ items, int64_t nitems,
                                                   const uint8_t* __restrict__ l2rank,
                                                   const double* __restrict__ step,
                                                   const double* __restrict__ basis,
                                                   const int64_t* __restrict__ qv_off,
                                                   const int64_t* __restrict__ qa_off, uint8_t* __restrict__ qv_buf,
                                                   uint8_t* __restrict__ qa_buf, uint8_t* __restrict__ overflow,
                                                   double* __restrict__ errp) {
  // four points per thread for W = 16 FP32 (16 float4 loads in flight); one
  // otherwise, where more would not fit the registers of W rows
  constexpr int PPT = (WP == 16 && sizeof(T) == 4) ? 4 : 1;
  __shared__ double Vs[WP][WP];   // FP64 basis, [k][t]
  __shared__ double Vq[WP][WP];   // quantized basis qV 2^-24, [k][t]
  __shared__ double red[256];
  const int64_t i = blockIdx.x;
  if (i >= nitems) return;
  const Item it = items[i];
  const int b = it.block;
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m;
  const int r = l2rank[b];
  const int R = r == kL2Raw ? 0 : r;
  for (int idx = threadIdx.x; idx < R * WP; idx += 256) {
    const int k = idx / WP, t = idx % WP;
    const double v = basis[int64_t(b) * WP * WP + idx];
    const double q = rint(v * kL2BasisScale);
    Vs[k][t] = v;
    Vq[k][t] = q * kL2BasisUnit;
    if (it.first && t < W) {
      const uint32_t z = zz32(int32_t(q));
      const int64_t plane = pad16(int64_t(W) * r);
      uint8_t* dst = qv_buf + qv_off[b] + k * W + t;
      for (int j = 0; j < 4; ++j) dst[j * plane] = uint8_t(z >> (8 * j));
    }
  }
  __syncthreads();
  const double dstep = step[b];
  const T* base = F + fidx(dims, d.var, d.t0, d.z0, d.y0, d.x0);
  const int64_t nxy = dims.nx * dims.ny, tstride = dims.nz * nxy;
  double err = 0.0;
  const bool cont = d.vec != 0;
  for (int pb = PPT * int(threadIdx.x); pb < it.np; pb += 256 * PPT) {
    const int valid = (it.np - pb) < PPT ? (it.np - pb) : PPT;
    const bool run = cont && valid == PPT;
    int64_t offs[PPT];
#pragma unroll
    for (int e = 0; e < PPT; ++e)
      offs[e] = point_off(it.p0 + pb + (run ? 0 : (e < valid ? e : 0)), d.px(), d.py(), dims.nx, nxy);
    // the points' W values, every load issued before the first use
    T xv[WP][PPT];
#pragma unroll
    for (int t = 0; t < WP; ++t) {
      if (t < W) {
        const T* row = base + int64_t(t) * tstride;
        if (run) {
          l2_load_run<T, PPT>(row + offs[0], xv[t]);
        } else {
#pragma unroll
          for (int e = 0; e < PPT; ++e) xv[t][e] = e < valid ? row[offs[e]] : T(0);
        }
      } else {
#pragma unroll
        for (int e = 0; e < PPT; ++e) xv[t][e] = T(0);
      }
    }
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      if (e >= valid) continue;
      const int p = it.p0 + pb + e;
      T xs[WP];
#pragma unroll
      for (int t = 0; t < WP; ++t) xs[t] = xv[t][e];
      if (r == kL2Raw) {
        uint8_t* dst = qa_buf + qa_off[b];
#pragma unroll
        for (int t = 0; t < WP; ++t)
          if (t < W) *reinterpret_cast<T*>(dst + (int64_t(t) * M + p) * int64_t(sizeof(T))) = xs[t];
        continue;
      }
      if (r == 0) {
#pragma unroll
        for (int t = 0; t < WP; ++t) {
          const double x = double(xs[t]);
          if (t < W) err += x * x;
        }
        continue;
      }
      // per mode k (in order): the projection, a running FMA over the steps in
      // order; its quantized coefficient; and its term of the decoder's
      // values, which sum the modes in order k = 0, 1, ...  (step indices are
      // compile-time, so xs[] and rec[] stay in registers)
      double rec[WP];
#pragma unroll
      for (int t = 0; t < WP; ++t) rec[t] = 0.0;
      bool ovf = false;
      const int64_t plane = pad16(int64_t(M) * r);
      uint8_t* dst = qa_buf + qa_off[b];
      for (int k = 0; k < R; ++k) {
        double a = 0.0;
#pragma unroll
        for (int t = 0; t < WP; ++t)
          if (t < W) a = fma(double(xs[t]), Vs[k][t], a);
        const double qa = rint(a / dstep);
        const bool ok = fabs(qa) < 2147483648.0;
        ovf = ovf || !ok;
        const int32_t qi = ok ? int32_t(qa) : 0;
        const double c = double(qi) * dstep;
        const uint32_t z = zz32(qi);
        for (int j = 0; j < 4; ++j) dst[j * plane + int64_t(k) * M + p] = uint8_t(z >> (8 * j));
#pragma unroll
        for (int t = 0; t < WP; ++t) rec[t] = rec[t] + Vq[k][t] * c;
      }
      if (ovf) overflow[b] = 1;
#pragma unroll
      for (int t = 0; t < WP; ++t) {
        const double dx = double(xs[t]) - double(T(rec[t]));
        if (t < W) err += dx * dx;
      }
    }
  }
  red[threadIdx.x] = err;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) errp[i] = red[0];
}

// per block: the slices' errors summed in slice order against the budget; a
// failing block takes the next rank, or raw past the cap
__global__ __launch_bounds__(256) void k_l2_check(const BlockDesc* __restrict__ desc,
                                                  const int32_t* __restrict__ item_start, int64_t nblocks,
                                                  const double* __restrict__ errp, const double* __restrict__ e2,
                                                  const uint8_t* __restrict__ overflow, int rcap,
                                                  uint8_t* __restrict__ l2rank, double* __restrict__ berr,
                                                  unsigned int* __restrict__ nfail) {
  const int64_t b = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (b >= nblocks) return;
  const int r = l2rank[b];
  if (r == kL2Raw) {
    berr[b] = 0.0;
    return;
  }
  double s = 0.0;
  for (int i = item_start[b]; i < item_start[b + 1]; ++i) s += errp[i];
  berr[b] = s;
  if (!overflow[b] && s <= e2[b]) return;
  const BlockDesc d = desc[b];
  int cap = rcap < d.w() ? rcap : d.w();
  const int nr = (overflow[b] || r + 1 > cap || !(e2[b] > 0.0)) ? kL2Raw : r + 1;
  l2rank[b] = uint8_t(nr);
  atomicAdd(nfail, 1u);
}

template <int WP, typename T>
__global__ __launch_bounds__(256) void k_l2_decode(T* __restrict__ F, Dims dims, const BlockDesc* __restrict__ desc,
                                                   const Item* __restrict__ items, int64_t nitems,
                                                   const uint8_t* __restrict__ l2rank,
                                                   const double* __restrict__ step,
                                                   const int64_t* __restrict__ qv_off,
                                                   const int64_t* __restrict__ qa_off,
                                                   const uint8_t* __restrict__ qv_buf,
                                                   const uint8_t* __restrict__ qa_buf) {
  __shared__ double Vq[WP][WP];
  const int64_t i = blockIdx.x;
  if (i >= nitems) return;
  const Item it = items[i];
  const int b = it.block;
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m;
  const int r = l2rank[b];
  const int R = r == kL2Raw ? 0 : r;
  const int64_t vplane = pad16(int64_t(W) * R);
  for (int idx = threadIdx.x; idx < R * WP; idx += 256) {
    const int k = idx / WP, t = idx % WP;
    double v = 0.0;
    if (t < W) {
      const uint8_t* src = qv_buf + qv_off[b] + k * W + t;
      uint32_t z = 0;
      for (int j = 0; j < 4; ++j) z |= uint32_t(src[j * vplane]) << (8 * j);
      v = double(unzz32(z)) * kL2BasisUnit;
    }
    Vq[k][t] = v;
  }
  __syncthreads();
  const double dstep = step[b];
  T* base = F + fidx(dims, d.var, d.t0, d.z0, d.y0, d.x0);
  const int64_t nxy = dims.nx * dims.ny, tstride = dims.nz * nxy;
  const int64_t plane = pad16(int64_t(M) * R);
  for (int q = threadIdx.x; q < it.np; q += 256) {
    const int p = it.p0 + q;
    const int64_t off = point_off(p, d.px(), d.py(), dims.nx, nxy);
    if (r == kL2Raw) {
      const uint8_t* src = qa_buf + qa_off[b];
      for (int t = 0; t < W; ++t)
        base[int64_t(t) * tstride + off] = *reinterpret_cast<const T*>(src + (int64_t(t) * M + p) * int64_t(sizeof(T)));
      continue;
    }
    double c[WP];
    const uint8_t* src = qa_buf + qa_off[b];
#pragma unroll
    for (int k = 0; k < WP; ++k) {
      c[k] = 0.0;
      if (k >= R) continue;
      uint32_t z = 0;
      for (int j = 0; j < 4; ++j) z |= uint32_t(src[j * plane + int64_t(k) * M + p]) << (8 * j);
      c[k] = double(unzz32(z)) * dstep;
    }
    for (int t = 0; t < W; ++t) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < WP; ++k)
        if (k < R) acc = acc + Vq[k][t] * c[k];
      base[int64_t(t) * tstride + off] = T(acc);
    }
  }
}

}  // namespace

hipError_t launch_l2_gram(int wp, int dtype, const void* F, const Dims& dims, const BlockDesc* desc,
                          const Item* items, int64_t nitems, double* gpart, double* fsq, hipStream_t s) {
  // one workgroup per slice, in dispatches of at most kL2LaunchItems
  // workgroups (a dispatch holds under 2^32 work-items)
  for (int64_t off = 0; off < nitems; off += kL2LaunchItems) {
    const int64_t n = std::min<int64_t>(nitems - off, kL2LaunchItems);
    const dim3 g{unsigned(n)}, bl{256};
    const Item* it = items + off;
    double* gp = gpart + off * wp * wp;
    double* fs = fsq + off;
#define DLS_L2G(WPV, TV) \
  hipLaunchKernelGGL((k_l2_gram<WPV, TV>), g, bl, 0, s, static_cast<const TV*>(F), dims, desc, it, n, gp, fs)
    if (wp == 16) { if (dtype == 0) DLS_L2G(16, float); else DLS_L2G(16, double); }
    else { if (dtype == 0) DLS_L2G(32, float); else DLS_L2G(32, double); }
#undef DLS_L2G
  }
  return hipGetLastError();
}

hipError_t launch_l2_budget(const double* fsq, const int64_t* range, double* part, const double* target,
                            int64_t per_var, int nvars, double* cv, double* eig_eps, hipStream_t s) {
  if (nvars == 0) return hipSuccess;
  const dim3 g = dim3(unsigned(kL2Parts), unsigned(nvars));
  hipLaunchKernelGGL(k_l2_fsq_part, g, dim3{256}, 0, s, fsq, range, part);
  hipLaunchKernelGGL(k_l2_budget, dim3{unsigned((nvars + 63) / 64)}, dim3{64}, 0, s, part, target, per_var, nvars, cv,
                     eig_eps);
  return hipGetLastError();
}

hipError_t launch_l2_params(const BlockDesc* desc, int64_t nblocks, const double* lam, int wp,
                            const uint8_t* eig_rank, const double* cv, bool first, int esize, uint8_t* l2rank,
                            double* step, double* e2, int64_t* qv_size, int64_t* qa_size, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_l2_params, dim3{unsigned((nblocks + 255) / 256)}, dim3{256}, 0, s, desc, nblocks, lam, wp,
                     eig_rank, cv, first ? 1 : 0, esize, l2rank, step, e2, qv_size, qa_size);
  return hipGetLastError();
}

hipError_t launch_l2_encode(int wp, int dtype, const void* F, const Dims& dims, const BlockDesc* desc,
                            const Item* items, int64_t nitems, const uint8_t* l2rank, const double* step,
                            const double* basis, const int64_t* qv_off, const int64_t* qa_off, uint8_t* qv,
                            uint8_t* qa, uint8_t* overflow, double* errp, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  for (int64_t off = 0; off < nitems; off += kL2LaunchItems) {
    const int64_t n = std::min<int64_t>(nitems - off, kL2LaunchItems);
    const dim3 g{unsigned(n)}, bl{256};
    const Item* it = items + off;
    double* ep = errp + off;
#define DLS_L2E(WPV, TV)                                                                                   \
  hipLaunchKernelGGL((k_l2_encode<WPV, TV>), g, bl, 0, s, static_cast<const TV*>(F), dims, desc, it, n, \
                     l2rank, step, basis, qv_off, qa_off, qv, qa, overflow, ep)
    if (wp == 16) { if (dtype == 0) DLS_L2E(16, float); else DLS_L2E(16, double); }
    else { if (dtype == 0) DLS_L2E(32, float); else DLS_L2E(32, double); }
#undef DLS_L2E
  }
  return hipGetLastError();
}

hipError_t launch_l2_check(const BlockDesc* desc, const int32_t* item_start, int64_t nblocks, const double* errp,
                           const double* e2, const uint8_t* overflow, int rcap, uint8_t* l2rank, double* berr,
                           unsigned int* nfail, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_l2_check, dim3{unsigned((nblocks + 255) / 256)}, dim3{256}, 0, s, desc, item_start, nblocks,
                     errp, e2, overflow, rcap, l2rank, berr, nfail);
  return hipGetLastError();
}

hipError_t launch_l2_decode(int wp, int dtype, void* F, const Dims& dims, const BlockDesc* desc, const Item* items,
                            int64_t nitems, const uint8_t* l2rank, const double* step, const int64_t* qv_off,
                            const int64_t* qa_off, const uint8_t* qv, const uint8_t* qa, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  for (int64_t off = 0; off < nitems; off += kL2LaunchItems) {
    const int64_t n = std::min<int64_t>(nitems - off, kL2LaunchItems);
    const dim3 g{unsigned(n)}, bl{256};
    const Item* it = items + off;
#define DLS_L2D(WPV, TV)                                                                                          \
  hipLaunchKernelGGL((k_l2_decode<WPV, TV>), g, bl, 0, s, static_cast<TV*>(F), dims, desc, it, n, l2rank, step, \
                     qv_off, qa_off, qv, qa)
    if (wp == 16) { if (dtype == 0) DLS_L2D(16, float); else DLS_L2D(16, double); }
    else { if (dtype == 0) DLS_L2D(32, float); else DLS_L2D(32, double); }
#undef DLS_L2D
  }
  return hipGetLastError();
}

}  // namespace dls
