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
//   k_l2_sumsq    sum of squares of the finite values of every variable
//                 (fixed partial grid, fixed summation order)
//   k_l2_budget   c_v and the eigensolve bound sqrt(0.36 c_v)
//   k_l2_gram     the slices' Gram partials in FP64
//   k_l2_params   per block: budget, rank (first pass), step, payload sizes
//   k_l2_encode   one workgroup per slice: projection, quantization, the
//                 decoder's values and the slice's squared error
//   k_l2_check    per block: the error against the budget; raises the rank
//   k_l2_decode   one workgroup per slice: the decoder
//
// Compiled with -ffp-contract=off: encoder and decoder must round the
// reconstruction identically.
#include <hip/hip_runtime.h>

#include "dls_device.h"
#include "dls_kernels.h"

namespace dls {
namespace {

constexpr double kL2TailShare = 0.36;
constexpr double kL2StepShare = 0.4;
constexpr double kL2BasisScale = 16777216.0;       // 2^24
constexpr double kL2BasisUnit = 1.0 / 16777216.0;  // 2^-24

__device__ __forceinline__ uint32_t zz32(int32_t v) { return (uint32_t(v) << 1) ^ uint32_t(v >> 31); }
__device__ __forceinline__ int32_t unzz32(uint32_t z) { return int32_t(z >> 1) ^ -int32_t(z & 1); }

template <typename T>
__global__ __launch_bounds__(256) void k_l2_sumsq(const T* __restrict__ F, int64_t per_var,
                                                  double* __restrict__ part) {
  __shared__ double red[256];
  const int v = blockIdx.y;
  const T* f = F + int64_t(v) * per_var;
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < per_var; i += int64_t(gridDim.x) * 256) {
    const double x = double(f[i]);
    if (isfinite(x)) s += x * x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[int64_t(v) * kL2Parts + blockIdx.x] = red[0];
}

// The Gram partial of one slice in FP64 (the L2 mode's ranks come from
// eigenvalue tails compared with 0.36 e2, which at tight targets is ~1e-8 of
// the block's energy: an FP32-accumulated Gram cannot resolve it).  One
// workgroup per slice; 64-point chunks staged in LDS; thread e owns entries
// e, e + 256, ... of the WP x WP matrix and sums its products over the
// slice's points in order.
template <int WP, typename T>
__global__ __launch_bounds__(256) void k_l2_gram(const T* __restrict__ F, Dims dims,
                                                 const BlockDesc* __restrict__ desc,
                                                 const Item* __restrict__ items, int64_t nitems,
                                                 double* __restrict__ gpart) {
  constexpr int CP = 64, NE = WP * WP / 256;
  __shared__ double sx[WP][CP + 1];
  const int64_t i = blockIdx.x;
  if (i >= nitems) return;
  const Item it = items[i];
  const BlockDesc d = desc[it.block];
  const int W = d.w();
  const T* base = F + fidx(dims, d.var, d.t0, d.z0, d.y0, d.x0);
  const int64_t nxy = dims.nx * dims.ny, tstride = dims.nz * nxy;
  double acc[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) acc[e] = 0.0;
  for (int c0 = 0; c0 < it.np; c0 += CP) {
    const int n = it.np - c0 < CP ? it.np - c0 : CP;
    for (int idx = threadIdx.x; idx < WP * CP; idx += 256) {
      const int t = idx / CP, q = idx % CP;
      double v = 0.0;
      if (t < W && q < n) {
        const int64_t off = point_off(it.p0 + c0 + q, d.px(), d.py(), dims.nx, nxy);
        v = double(base[int64_t(t) * tstride + off]);
      }
      sx[t][q] = v;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int ent = int(threadIdx.x) + 256 * e, r = ent / WP, c = ent % WP;
      double a = acc[e];
      for (int q = 0; q < n; ++q) a = fma(sx[r][q], sx[c][q], a);
      acc[e] = a;
    }
    __syncthreads();
  }
  double* out = gpart + i * WP * WP;
#pragma unroll
  for (int e = 0; e < NE; ++e) out[threadIdx.x + 256 * e] = acc[e];
}

// c_v = (eps_t,v)^2 ||u_v||^2 / K_v and the eigensolve's bound sqrt(0.36 c_v)
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

// One workgroup per slice, one thread per point (256 threads, up to four
// points each).  RMAX: the rank class of the launch.
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
  for (int q = threadIdx.x; q < it.np; q += 256) {
    const int p = it.p0 + q;
    const int64_t off = point_off(p, d.px(), d.py(), dims.nx, nxy);
    if (r == kL2Raw) {
      uint8_t* dst = qa_buf + qa_off[b];
      for (int t = 0; t < W; ++t)
        *reinterpret_cast<T*>(dst + (int64_t(t) * M + p) * int64_t(sizeof(T))) = base[int64_t(t) * tstride + off];
      continue;
    }
    if (r == 0) {
      for (int t = 0; t < W; ++t) {
        const double x = double(base[int64_t(t) * tstride + off]);
        err += x * x;
      }
      continue;
    }
    // projection: per mode a running FMA over the steps in order (the mode
    // index is compile-time, so a[] and c[] stay in registers)
    double a[WP];
#pragma unroll
    for (int k = 0; k < WP; ++k) a[k] = 0.0;
    for (int t = 0; t < W; ++t) {
      const double x = double(base[int64_t(t) * tstride + off]);
#pragma unroll
      for (int k = 0; k < WP; ++k)
        if (k < R) a[k] = fma(x, Vs[k][t], a[k]);
    }
    double c[WP];
    bool ovf = false;
    const int64_t plane = pad16(int64_t(M) * r);
    uint8_t* dst = qa_buf + qa_off[b];
#pragma unroll
    for (int k = 0; k < WP; ++k) {
      c[k] = 0.0;
      if (k >= R) continue;
      const double qa = rint(a[k] / dstep);
      const bool ok = fabs(qa) < 2147483648.0;
      ovf = ovf || !ok;
      const int32_t qi = ok ? int32_t(qa) : 0;
      c[k] = double(qi) * dstep;
      const uint32_t z = zz32(qi);
      for (int j = 0; j < 4; ++j) dst[j * plane + int64_t(k) * M + p] = uint8_t(z >> (8 * j));
    }
    if (ovf) overflow[b] = 1;
    // the decoder's values: per step, the modes summed in order k = 0, 1, ...
    for (int t = 0; t < W; ++t) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < WP; ++k)
        if (k < R) acc = acc + Vq[k][t] * c[k];
      const double e = double(base[int64_t(t) * tstride + off]) - double(T(acc));
      err += e * e;
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

hipError_t launch_l2_budget(int dtype, const void* F, int64_t per_var, int nvars, const double* target,
                            double* part, double* cv, double* eig_eps, hipStream_t s) {
  const dim3 g{unsigned(kL2Parts), unsigned(nvars)};
  if (dtype == 0)
    hipLaunchKernelGGL(k_l2_sumsq<float>, g, dim3{256}, 0, s, static_cast<const float*>(F), per_var, part);
  else
    hipLaunchKernelGGL(k_l2_sumsq<double>, g, dim3{256}, 0, s, static_cast<const double*>(F), per_var, part);
  hipLaunchKernelGGL(k_l2_budget, dim3{unsigned((nvars + 63) / 64)}, dim3{64}, 0, s, part, target, per_var, nvars,
                     cv, eig_eps);
  return hipGetLastError();
}

hipError_t launch_l2_gram(int wp, int dtype, const void* F, const Dims& dims, const BlockDesc* desc,
                          const Item* items, int64_t nitems, double* gpart, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  if (nitems > int64_t(INT32_MAX)) return hipErrorInvalidValue;
  const dim3 g{unsigned(nitems)}, bl{256};
#define DLS_L2G(WPV, TV) \
  hipLaunchKernelGGL((k_l2_gram<WPV, TV>), g, bl, 0, s, static_cast<const TV*>(F), dims, desc, items, nitems, gpart)
  if (wp == 16) { if (dtype == 0) DLS_L2G(16, float); else DLS_L2G(16, double); }
  else { if (dtype == 0) DLS_L2G(32, float); else DLS_L2G(32, double); }
#undef DLS_L2G
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
  if (nitems > int64_t(INT32_MAX)) return hipErrorInvalidValue;
  const dim3 g{unsigned(nitems)}, bl{256};
#define DLS_L2E(WPV, TV)                                                                                           \
  hipLaunchKernelGGL((k_l2_encode<WPV, TV>), g, bl, 0, s, static_cast<const TV*>(F), dims, desc, items, nitems,   \
                     l2rank, step, basis, qv_off, qa_off, qv, qa, overflow, errp)
  if (wp == 16) { if (dtype == 0) DLS_L2E(16, float); else DLS_L2E(16, double); }
  else { if (dtype == 0) DLS_L2E(32, float); else DLS_L2E(32, double); }
#undef DLS_L2E
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
  if (nitems > int64_t(INT32_MAX)) return hipErrorInvalidValue;
  const dim3 g{unsigned(nitems)}, bl{256};
#define DLS_L2D(WPV, TV)                                                                                            \
  hipLaunchKernelGGL((k_l2_decode<WPV, TV>), g, bl, 0, s, static_cast<TV*>(F), dims, desc, items, nitems, l2rank,  \
                     step, qv_off, qa_off, qv, qa)
  if (wp == 16) { if (dtype == 0) DLS_L2D(16, float); else DLS_L2D(16, double); }
  else { if (dtype == 0) DLS_L2D(32, float); else DLS_L2D(32, double); }
#undef DLS_L2D
  return hipGetLastError();
}

}  // namespace dls
