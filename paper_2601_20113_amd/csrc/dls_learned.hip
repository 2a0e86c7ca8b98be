// Learned warm start of the per-block eigensolve (gfx950 kernels).
//
// The plain method eigensolves every block's Gram matrix with Jacobi.  Here
// a small network (80 -> 128 -> 128 -> 272, ReLU; bf16 operands on the
// matrix cores with FP32 accumulation) predicts from per-block statistics a
// rank rhat and a 16 x rhat starting basis; a few steps of subspace
// iteration (Y = G Q, Q = orth(Y), FP64) and a Rayleigh-Ritz step refine it.
// The plain method then judges the result: the rank is the smallest r whose
// discarded energy trace(G) - sum_{k<=r} theta_k, exact for the Ritz basis,
// meets the local tolerance of Sec. 2.4 Eq. (4); a block whose prediction
// cannot meet it falls back to the full Jacobi eigensolve.  The network is
// trained on the GPU by the kernels below (forward, loss, backward, Adam).
#include <hip/hip_runtime.h>

#include "dls_device.h"
#include "dls_kernels.h"

namespace dls {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return short(uint16_t((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16));
}

// ---------------------------------------------------------------------------
// Per-block features: 16 statistics then the 8 x 8 pooled time-mean image
// (normalised by the block mean and standard deviation), FP64 sums.  Blocks
// of more than kWarmMaxPoints points get zeros (they take no warm start).
// Blocks of at most 16 points: 16 lanes each, four per wavefront (sums by
// DPP row reductions).  Other blocks: one wavefront each, points in chunks
// of 64 lanes.  Neighbours in x and y come from other lanes where they hold
// them, else from memory; the central moments take a second pass over the
// values (kept in registers for the last chunk, reloaded for the others).
// The 16 statistics are computed one per lane.
// ---------------------------------------------------------------------------
template <int CTRL, bool MAX>
__device__ __forceinline__ double dpp_minmax(double v) {
  const double o = dpp_f64<CTRL>(v);
  return MAX ? fmax(v, o) : fmin(v, o);
}
template <bool MAX>
__device__ __forceinline__ double row_minmax(double v) {
  v = dpp_minmax<0xB1, MAX>(v);
  v = dpp_minmax<0x4E, MAX>(v);
  v = dpp_minmax<0x141, MAX>(v);
  return dpp_minmax<0x140, MAX>(v);
}
// G = 16: over the lane's DPP row; G = 64: over the wavefront
template <int G>
__device__ __forceinline__ double fsum(double v) {
  v = row_sum(v);
  if constexpr (G == 64) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
  }
  return v;
}
template <int G, bool MAX>
__device__ __forceinline__ double fminmax(double v) {
  v = row_minmax<MAX>(v);
  if constexpr (G == 64) {
    const double a = __shfl_xor(v, 16, 64);
    v = MAX ? fmax(v, a) : fmin(v, a);
    const double b = __shfl_xor(v, 32, 64);
    v = MAX ? fmax(v, b) : fmin(v, b);
  }
  return v;
}

// Block sums of one block's values (first pass) and central sums (second).
struct FeatSums {
  double s1 = 0, s2 = 0, mn = INFINITY, mx = -INFINITY, adt = 0, sdt = 0, sdt2 = 0, adx = 0, ady = 0, tme = 0;
  double cvar = 0, c3 = 0, c4 = 0, l1 = 0, l2 = 0;
};

// first-pass sums of one point: x its W values, xr / xd the values of its
// +x / +y neighbour (used when hr / hd); returns the point's time sum
template <typename T>
__device__ __forceinline__ double feat_point(FeatSums& S, const T* x, const T* xr, const T* xd, int W, bool hr,
                                             bool hd) {
  double ts = 0.0, prev = 0.0;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    if (t < W) {
      const double v = double(x[t]);
      S.s1 += v;
      S.s2 += v * v;
      S.mn = fmin(S.mn, v);
      S.mx = fmax(S.mx, v);
      ts += v;
      if (t > 0) {
        const double dt = v - prev;
        S.adt += fabs(dt);
        S.sdt += dt;
        S.sdt2 += dt * dt;
      }
      if (hr) S.adx += fabs(double(xr[t]) - v);
      if (hd) S.ady += fabs(double(xd[t]) - v);
      prev = v;
    }
  }
  S.tme += ts * ts;
  return ts;
}

template <typename T>
__device__ __forceinline__ void feat_central(FeatSums& S, const T* x, int W, double mu) {
  double ym1 = 0.0, ym2 = 0.0;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    if (t < W) {
      const double y = double(x[t]) - mu;
      const double y2 = y * y;
      S.cvar += y2;
      S.c3 += y2 * y;
      S.c4 += y2 * y2;
      if (t >= 1) S.l1 += y * ym1;
      if (t >= 2) S.l2 += y * ym2;
      ym2 = ym1;
      ym1 = y;
    }
  }
}

// statistic q (0..15) of a block from its reduced sums (same value in every
// lane that asks for the same q): one division, and one log10 for the lanes
// that need it
__device__ __forceinline__ float moment_feature(int q, const FeatSums& S, int W, int M, int px, int py, int pz,
                                                double eps) {
  const double n = double(W) * M, nd = double(W - 1) * M;
  const double mu = S.s1 / n, var = S.cvar / n, sd = sqrt(var);
  const double inv = sd > 0.0 ? 1.0 / sd : 0.0;
  double a = 0.0, b = 1.0, lo = 0.0, scale = 1.0;
  int post = 0;  // 1: -3, 2: std of dt, 3: log10, 4: times inv
  bool on = true;
  switch (q) {
    case 0: a = S.s1; b = n; break;
    case 1: a = sd; break;
    case 2: a = S.mn; break;
    case 3: a = S.mx; break;
    case 4: on = sd > 0.0; a = S.c3; b = n * (sd * sd * sd); break;
    case 5: on = sd > 0.0; a = S.c4; b = n * (var * var); post = 1; break;
    case 6: on = W > 1; a = S.adt; b = nd; post = 4; break;
    case 7: on = W > 1; a = S.sdt2; b = nd; post = 2; break;
    case 8: on = px > 1; a = S.adx; b = double(W) * (px - 1) * py * pz; post = 4; break;
    case 9: on = py > 1; a = S.ady; b = double(W) * px * (py - 1) * pz; post = 4; break;
    case 10: on = W > 1 && sd > 0.0; a = S.l1; b = nd * var; break;
    case 11: on = W > 2 && sd > 0.0; a = S.l2; b = double(W - 2) * M * var; break;
    case 12: a = S.s2; b = n * (eps * eps); post = 3; lo = 1e-30; break;
    case 13: a = sd; b = eps; post = 3; lo = 1e-15; break;
    case 14: on = S.s2 > 0.0; a = S.tme; b = double(W) * S.s2; break;
    default: a = double(M); post = 3; scale = 3.321928094887362; break;  // log2 M = log10 M / log10 2
  }
  if (!on) return 0.f;
  double v = a / b;
  if (post == 1) {
    v -= 3.0;
  } else if (post == 2) {
    const double mdt = S.sdt / nd;
    v = sqrt(fmax(v - mdt * mdt, 0.0)) * inv;
  } else if (post == 3) {
    v = log10(fmax(v, lo)) * scale;
  } else if (post == 4) {
    v *= inv;
  }
  return float(v);
}

// pooled cell c = 8 b + a: mean over t and z of the rows / columns that fall
// in the cell (or the single nearest one), from the per-point time sums ts
__device__ __forceinline__ float pooled_cell(int c, const double* ts, int W, int px, int py, int pz, double mu,
                                             double sd) {
  const int bb = c >> 3, aa = c & 7;
  int j0 = (bb * py + 7) / 8, j1 = ((bb + 1) * py + 7) / 8;
  int i0 = (aa * px + 7) / 8, i1 = ((aa + 1) * px + 7) / 8;
  if (j1 <= j0) { j0 = (bb * py) / 8; j1 = j0 + 1; }
  if (i1 <= i0) { i0 = (aa * px) / 8; i1 = i0 + 1; }
  double s = 0.0;
  for (int kk = 0; kk < pz; ++kk)
    for (int jj = j0; jj < j1; ++jj)
      for (int ii = i0; ii < i1; ++ii) s += ts[(kk * py + jj) * px + ii];
  const double cellv = s / double((i1 - i0) * (j1 - j0) * pz * W);
  return float(sd > 0.0 ? (cellv - mu) / sd : 0.0);
}

// Blocks of at most 16 points: 16 lanes per block (lane = point), four blocks
// per wavefront, sixteen per workgroup.  Every lane of a DPP row takes part in
// the reductions; a lane past the list end computes on a copy of the last
// listed block and writes nothing.
template <typename T>
__global__ __launch_bounds__(256) void k_features_small(const T* __restrict__ F, Dims dims,
                                                       const BlockDesc* __restrict__ desc,
                                                       const int32_t* __restrict__ list, int64_t nlist,
                                                       const double* __restrict__ eps_v, float* __restrict__ feat) {
  __shared__ double sts[16][16];
  const int lane = threadIdx.x & 63, g = lane & 15, grp = threadIdx.x >> 4;
  const int64_t li = int64_t(blockIdx.x) * 16 + grp;
  const bool have = li < nlist;
  const int64_t b = list[have ? li : nlist - 1];
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m, px = d.px(), py = d.py(), pz = d.pz();
  const int64_t nxy = dims.nx * dims.ny, tstride = dims.nz * nxy;
  const int p = g;
  const bool act = p < M;
  const int i = p % px, rho = p / px, j = rho % py, k = rho / py;
  T x[16];
  {
    const T* pt = F + (((int64_t(d.var) * dims.nt + d.t0) * dims.nz + d.z0 + k) * dims.ny + d.y0 + j) * dims.nx +
                  d.x0 + i;
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = (act && t < W) ? pt[int64_t(t) * tstride] : T(0);
  }
  // the +x and +y neighbours of a point of the block are points of the block,
  // so they sit in this lane's 16-lane group
  T xr[16], xd[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    xr[t] = __shfl(x[t], (lane + 1) & 63, 64);
    xd[t] = __shfl(x[t], (lane + px) & 63, 64);
  }
  FeatSums S;
  if (act) sts[grp][p] = feat_point<T>(S, x, xr, xd, W, i + 1 < px, j + 1 < py);
  S.s1 = fsum<16>(S.s1); S.s2 = fsum<16>(S.s2); S.adt = fsum<16>(S.adt); S.sdt = fsum<16>(S.sdt);
  S.sdt2 = fsum<16>(S.sdt2); S.adx = fsum<16>(S.adx); S.ady = fsum<16>(S.ady); S.tme = fsum<16>(S.tme);
  S.mn = fminmax<16, false>(S.mn);
  S.mx = fminmax<16, true>(S.mx);
  const double n = double(W) * M, mu = S.s1 / n;
  if (act) feat_central<T>(S, x, W, mu);
  S.cvar = fsum<16>(S.cvar); S.c3 = fsum<16>(S.c3); S.c4 = fsum<16>(S.c4); S.l1 = fsum<16>(S.l1);
  S.l2 = fsum<16>(S.l2);
  const float fq = moment_feature(g, S, W, M, px, py, pz, eps_v[d.var]);
  const double sd = sqrt(S.cvar / n);
  wave_sync();
  float cells[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) cells[u] = pooled_cell(g + 16 * u, sts[grp], W, px, py, pz, mu, sd);
  if (!have) return;
  float* o = feat + b * 80;
  o[g] = fq;
#pragma unroll
  for (int u = 0; u < 4; ++u) o[16 + g + 16 * u] = cells[u];
}

// Blocks of 17..kWarmMaxPoints points: one wavefront per block, four per
// workgroup; point p = 64 c + lane in chunk c.
template <typename T>
__global__ __launch_bounds__(256) void k_features_wave(const T* __restrict__ F, Dims dims,
                                                      const BlockDesc* __restrict__ desc,
                                                      const int32_t* __restrict__ list, int64_t nlist,
                                                      const double* __restrict__ eps_v, float* __restrict__ feat) {
  __shared__ double sts[4][kWarmMaxPoints];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t li = int64_t(blockIdx.x) * 4 + wv;
  if (li >= nlist) return;
  const int64_t b = list[li];
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m, px = d.px(), py = d.py(), pz = d.pz();
  const int64_t nxy = dims.nx * dims.ny, tstride = dims.nz * nxy;
  const T* base = F + (((int64_t(d.var) * dims.nt + d.t0) * dims.nz + d.z0) * dims.ny + d.y0) * dims.nx + d.x0;
  const int nchunk = (M + 63) >> 6;
  auto point_ptr = [&](int p) {
    const int i = p % px, rho = p / px, j = rho % py, k = rho / py;
    return base + int64_t(k) * nxy + int64_t(j) * dims.nx + i;
  };
  auto load = [&](int p, T* x) {
    const T* pt = point_ptr(p < M ? p : 0);
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = (p < M && t < W) ? pt[int64_t(t) * tstride] : T(0);
  };
  FeatSums S;
  T x[16];
  for (int c = 0; c < nchunk; ++c) {
    const int p = 64 * c + lane;
    load(p, x);
    const bool act = p < M;
    const int i = p % px, j = (p / px) % py;
    const bool hr = act && i + 1 < px, hd = act && j + 1 < py;
    // a neighbour outside this chunk's lanes is read from memory
    const bool mr = hr && lane == 63, md = hd && lane + px >= 64;
    T xr[16], xd[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      xr[t] = __shfl(x[t], (lane + 1) & 63, 64);
      xd[t] = __shfl(x[t], (lane + px) & 63, 64);
    }
    if (mr || md) {
      const T* pt = point_ptr(p);
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        if (t < W) {
          if (mr) xr[t] = pt[int64_t(t) * tstride + 1];
          if (md) xd[t] = pt[int64_t(t) * tstride + dims.nx];
        }
      }
    }
    if (act) sts[wv][p] = feat_point<T>(S, x, xr, xd, W, hr, hd);
  }
  S.s1 = fsum<64>(S.s1); S.s2 = fsum<64>(S.s2); S.adt = fsum<64>(S.adt); S.sdt = fsum<64>(S.sdt);
  S.sdt2 = fsum<64>(S.sdt2); S.adx = fsum<64>(S.adx); S.ady = fsum<64>(S.ady); S.tme = fsum<64>(S.tme);
  S.mn = fminmax<64, false>(S.mn);
  S.mx = fminmax<64, true>(S.mx);
  const double n = double(W) * M, mu = S.s1 / n;
  // second pass, last chunk first: its values are still in registers
  for (int c = nchunk - 1; c >= 0; --c) {
    const int p = 64 * c + lane;
    if (c != nchunk - 1) load(p, x);
    if (p < M) feat_central<T>(S, x, W, mu);
  }
  S.cvar = fsum<64>(S.cvar); S.c3 = fsum<64>(S.c3); S.c4 = fsum<64>(S.c4); S.l1 = fsum<64>(S.l1);
  S.l2 = fsum<64>(S.l2);
  const float fq = moment_feature(lane & 15, S, W, M, px, py, pz, eps_v[d.var]);
  const double sd = sqrt(S.cvar / n);
  wave_sync();
  const float cell = pooled_cell(lane, sts[wv], W, px, py, pz, mu, sd);
  float* o = feat + b * 80;
  if (lane < 16) o[lane] = fq;
  o[16 + lane] = cell;
}

// zero feature rows (blocks that take no warm start)
__global__ __launch_bounds__(256) void k_features_zero(const int32_t* __restrict__ list, int64_t nlist,
                                                       float* __restrict__ feat) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= nlist * 80) return;
  feat[int64_t(list[i / 80]) * 80 + i % 80] = 0.f;
}

// z-score the 16 statistics with the model's training statistics
__global__ __launch_bounds__(256) void k_normalize(const float* __restrict__ raw, int64_t n,
                                                   const float* __restrict__ norm, float* __restrict__ z) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n * 80) return;
  const int f = int(i % 80);
  z[i] = f < 16 ? (raw[i] - norm[f]) / norm[16 + f] : raw[i];
}

// ---------------------------------------------------------------------------
// C (M x N, FP32) = op(A) (M x K) op(B) (K x N) [+ bias] [ReLU].
// op(A)[i][k] = TA ? A[k lda + i] : A[i lda + k]; op(B)[k][j] = TB ? B[j ldb + k]
// : B[k ldb + j].  One wavefront per 16 x 16 output tile; BF16 rounds both
// operands to bfloat16 (v_mfma_f32_16x16x16bf16_1k), otherwise FP32
// products (v_mfma_f32_16x16x4f32).
// ---------------------------------------------------------------------------
template <bool TA, bool TB, bool BF16>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ A, int lda, const float* __restrict__ B,
                                              int ldb, float* __restrict__ C, int ldc, int Mr, int Nc, int K,
                                              const float* __restrict__ bias, int relu) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tiles_n = (Nc + 15) / 16;
  const int64_t tile = int64_t(blockIdx.x) * 4 + wave;
  const int64_t tiles = int64_t((Mr + 15) / 16) * tiles_n;
  if (tile >= tiles) return;
  const int i0 = int(tile / tiles_n) * 16, j0 = int(tile % tiles_n) * 16;
  const int r = lane & 15, q = lane >> 4;
  auto a_at = [&](int i, int k) -> float {
    if (i >= Mr || k >= K) return 0.f;
    return TA ? A[int64_t(k) * lda + i] : A[int64_t(i) * lda + k];
  };
  auto b_at = [&](int k, int j) -> float {
    if (k >= K || j >= Nc) return 0.f;
    return TB ? B[int64_t(j) * ldb + k] : B[int64_t(k) * ldb + j];
  };
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if constexpr (BF16) {
    for (int k0 = 0; k0 < K; k0 += 16) {
      bf16x4 av, bv;
      for (int e = 0; e < 4; ++e) {
        av[e] = to_bf16(a_at(i0 + r, k0 + 4 * q + e));
        bv[e] = to_bf16(b_at(k0 + 4 * q + e, j0 + r));
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += 4)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a_at(i0 + r, k0 + q), b_at(k0 + q, j0 + r), acc, 0, 0, 0);
  }
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + 4 * q + v, j = j0 + r;
    if (i < Mr && j < Nc) {
      float c = acc[v];
      if (bias) c += bias[j];
      if (relu) c = c > 0.f ? c : 0.f;
      C[int64_t(i) * ldc + j] = c;
    }
  }
}

// ---------------------------------------------------------------------------
// Inference forward, three layers fused: 64 rows per workgroup (16 per
// wave).  Each layer's weights are staged in LDS as bf16, transposed to
// [out][in] so a lane's four k values are contiguous; the hidden
// activations pass through LDS (bf16) to change from the MFMA output layout
// (lane = column) to the operand layout (lane = row).  Products, the k order
// of the accumulation and every rounding are those of k_gemm with BF16.
// ---------------------------------------------------------------------------
// bf16 copies of W1, W2, W3, each transposed to [out][in] with leading
// dimension kPackLd (inputs beyond K are zero): the LDS image the fused
// forward stages with plain 16-byte copies.
__global__ __launch_bounds__(256) void k_pack_weights(const float* __restrict__ P, short* __restrict__ packed) {
  const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t rows = kH + kH + kNO;
  if (idx >= rows * kPackLd) return;
  int j = int(idx / kPackLd);
  const int k = int(idx % kPackLd);
  const float* Wg;
  int K, N;
  if (j < kH) {
    Wg = P + kOffW1; K = kNF; N = kH;
  } else if (j < 2 * kH) {
    Wg = P + kOffW2; K = kH; N = kH; j -= kH;
  } else {
    Wg = P + kOffW3; K = kH; N = kNO; j -= 2 * kH;
  }
  packed[idx] = k < K ? to_bf16(Wg[int64_t(k) * N + j]) : short(0);
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ raw, int64_t n,
                                                     const float* __restrict__ norm, const float* __restrict__ P,
                                                     const short* __restrict__ packed, float* __restrict__ out) {
  constexpr int LW = kPackLd;
  // one layer's weights at a time, the output layer in parts of at most kH
  // rows, so that three workgroups fit in a CU's LDS
  __shared__ __align__(16) short sW[kH * LW];
  __shared__ __align__(16) short sH[4][16 * LW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, q = lane >> 4;
  const int64_t row0 = int64_t(blockIdx.x) * 64 + wave * 16;
  const bool row_ok = row0 + r < n;
  short* H = sH[wave];
  // N packed rows (outputs) from row `first` of the packed image (layers 1, 2
  // and 3 start at rows 0, kH and 2 kH) into LDS
  auto stage = [&](int first, int N) {
    const uint4* src = reinterpret_cast<const uint4*>(packed + int64_t(first) * LW);
    uint4* dst = reinterpret_cast<uint4*>(sW);
    const int n16 = N * LW * 2 / 16;
    for (int i = threadIdx.x; i < n16; i += 256) dst[i] = src[i];
  };
  // one layer: A fragments from `afrag(ks)`, K = 16 * KS inputs, N outputs;
  // epilogue(nt, acc) consumes each 16 x 16 output tile
  auto layer = [&](auto afrag, int KS, int N, auto epilogue) {
    for (int nt = 0; nt < N / 16; ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < KS; ++ks) {
        const bf16x4 bv = *reinterpret_cast<const bf16x4*>(&sW[(nt * 16 + r) * LW + ks * 16 + 4 * q]);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(afrag(ks), bv, acc, 0, 0, 0);
      }
      epilogue(nt, acc);
    }
  };
  auto hidden_out = [&](const float* bias) {
    return [=](int nt, f32x4 acc) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float c = acc[v] + bias[nt * 16 + r];
        c = c > 0.f ? c : 0.f;
        H[(4 * q + v) * LW + nt * 16 + r] = to_bf16(c);
      }
    };
  };
  auto from_h = [&](int ks) { return *reinterpret_cast<const bf16x4*>(&H[r * LW + ks * 16 + 4 * q]); };

  // layer 1: z = (raw - mean) / std on the 16 statistics, raw on the rest
  bf16x4 z[5];
#pragma unroll
  for (int ks = 0; ks < 5; ++ks)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = ks * 16 + 4 * q + e;
      float v = row_ok ? raw[(row0 + r) * kNF + k] : 0.f;
      if (row_ok && k < 16) v = (v - norm[k]) / norm[16 + k];
      z[ks][e] = to_bf16(v);
    }
  stage(0, kH);
  __syncthreads();
  layer([&](int ks) { return z[ks]; }, 5, kH, hidden_out(P + kOffb1));
  __syncthreads();
  stage(kH, kH);
  __syncthreads();
  // h1 is read from H and h2 written back into it: read all fragments first
  bf16x4 h[8];
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) h[ks] = from_h(ks);
  __syncthreads();
  layer([&](int ks) { return h[ks]; }, 8, kH, hidden_out(P + kOffb2));
  __syncthreads();
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) h[ks] = from_h(ks);
  const float* b3 = P + kOffb3;
  // output layer in three parts of 96, 96 and 80 outputs
  for (int part = 0; part < 3; ++part) {
    const int c0 = 96 * part, N = part < 2 ? 96 : kNO - 192;
    __syncthreads();  // the previous weights are no longer read
    stage(2 * kH + c0, N);
    __syncthreads();
    layer([&](int ks) { return h[ks]; }, 8, N, [&](int nt, f32x4 acc) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = row0 + 4 * q + v;
        const int c = c0 + nt * 16 + r;
        if (i < n) out[i * kNO + c] = acc[v] + b3[c];
      }
    });
  }
}

// Loss CE(logits, r - 1) + masked MSE of the basis, per sample; gout = dL/dout
// of the batch-mean loss.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ out, const int32_t* __restrict__ rank,
                                              const float* __restrict__ basis, const int32_t* __restrict__ wb,
                                              int64_t n, float* __restrict__ gout, float* __restrict__ loss) {
  const int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (s >= n) return;
  const float* o = out + s * 272;
  float* g = gout + s * 272;
  const int r = rank[s], w = wb[s];
  double mx = o[0];
  for (int k = 1; k < 16; ++k) mx = fmax(mx, double(o[k]));
  double z = 0.0;
  for (int k = 0; k < 16; ++k) z += exp(double(o[k]) - mx);
  const double inv_n = 1.0 / double(n);
  double l = -(double(o[r - 1]) - mx - log(z));
  for (int k = 0; k < 16; ++k) {
    const double pk = exp(double(o[k]) - mx) / z;
    g[k] = float((pk - (k == r - 1 ? 1.0 : 0.0)) * inv_n);
  }
  const int cnt = r * w > 0 ? r * w : 1;
  double mse = 0.0;
  for (int k = 0; k < 16; ++k)
    for (int t = 0; t < 16; ++t) {
      const int idx = 16 + k * 16 + t;
      if (k < r && t < w) {
        const double dlt = double(o[idx]) - double(basis[s * 256 + k * 16 + t]);
        mse += dlt * dlt;
        g[idx] = float(2.0 * dlt / cnt * inv_n);
      } else {
        g[idx] = 0.f;
      }
    }
  loss[s] = float(l + mse / cnt);
}

// column sums, one wavefront per column, lanes stride the rows, fixed-order
// shuffle reduction
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ G, int64_t n, int cols,
                                                float* __restrict__ out) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= cols) return;
  double s = 0.0;
  for (int64_t i = lane; i < n; i += 64) s += G[i * cols + j];
  s = wave_sum(s);
  if (lane == 0) out[j] = float(s);
}

__global__ __launch_bounds__(256) void k_relu_mask(float* __restrict__ dh, const float* __restrict__ h, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n && !(h[i] > 0.f)) dh[i] = 0.f;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                              float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// ---------------------------------------------------------------------------
// Warm-started eigensolve: 16 lanes per block, four blocks per wavefront,
// sixteen per workgroup.  Lane t owns row t of G and of the iterate Q
// (registers); sums over the 16 rows use DPP row operations, so every lane
// of a group holds bitwise the same sum and all lanes take the same
// decisions.  LDS carries the broadcasts of Q and the small Rayleigh-Ritz
// matrix.  A group touches only its own LDS and its own DPP row, and the
// 16 lanes of a group are always active together, so within the group no
// workgroup barrier is needed: wave_sync() only keeps the compiler from
// moving LDS accesses across it (a wavefront's LDS accesses complete in
// issue order).  Predictions of more than kWarmMax columns go to the
// Jacobi fallback.
// ---------------------------------------------------------------------------
constexpr int kWarmMax = 8;      // most columns an attempt iterates
constexpr int kRetryExtra = 4;   // columns the second attempt adds
constexpr int kRetryIters = 2;   // iterations the second attempt adds

// Orthonormalise the first r columns of Q (row t in q[]), classical
// Gram-Schmidt applied twice per column; a column that collapses is
// replaced by the first unit vector e_j (j < W) that stays independent.
__device__ __forceinline__ void orth_rows(double (&q)[kWarmMax], int r, int W, int t) {
#pragma unroll
  for (int k = 0; k < kWarmMax; ++k) {
    if (k < r) {
      auto project_out = [&](double y) {
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
          double c[kWarmMax];
#pragma unroll
          for (int j = 0; j < k; ++j) c[j] = row_sum(q[j] * y);
#pragma unroll
          for (int j = 0; j < k; ++j) y -= c[j] * q[j];
        }
        return y;
      };
      double y = q[k];
      const double n0 = sqrt(row_sum(y * y));
      y = project_out(y);
      double nrm = sqrt(row_sum(y * y));
      if (!(nrm > 1e-12 * n0) || n0 == 0.0) {
        for (int e = 0; e < W; ++e) {
          y = project_out(t == e ? 1.0 : 0.0);
          nrm = sqrt(row_sum(y * y));
          if (nrm > 0.5) break;
        }
      }
      q[k] = (t < W) ? y / nrm : 0.0;
    }
  }
}

// Cyclic Jacobi with the round-robin ordering on the leading n x n block of
// H (LDS, leading dimension kWarmMax + 1), n <= kWarmMax, rotations
// accumulated into U.  The 16 lanes of one group call it together; false
// when kJacobiMaxSweeps sweeps left it unconverged.
__device__ bool jacobi_group(double* H, double* U, double* alpha, double* beta, int* partner, int n, int t) {
  constexpr int LD = kWarmMax + 1;
  if (n <= 1) return true;
  const int ne = n + (n & 1);
  const int nn = ne * ne;
  for (int sweep = 0;; ++sweep) {
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t + 16 * e;
      if (idx < nn) {
        const int i = idx / ne, j = idx % ne;
        const double a = (i < n && j < n) ? H[i * LD + j] : 0.0;
        tot += a * a;
        if (i != j) off += a * a;
      }
    }
    off = row_sum(off);
    tot = row_sum(tot);
    if (!(off > 1e-26 * tot)) return true;
    if (sweep >= kJacobiMaxSweeps) return false;
    for (int step = 0; step < ne - 1; ++step) {
      if (t < ne / 2) {
        int p = rr_player(t, step, ne), q = rr_player(ne - 1 - t, step, ne);
        if (p > q) { const int x = p; p = q; q = x; }
        double c = 1.0, s = 0.0;
        if (q < n) jacobi_rotation(H[p * LD + p], H[q * LD + q], H[p * LD + q], c, s);
        partner[p] = q; partner[q] = p;
        alpha[p] = c; beta[p] = -s;
        alpha[q] = c; beta[q] = s;
      }
      wave_sync();
      double na[4], nu[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = t + 16 * e;
        na[e] = nu[e] = 0.0;
        if (idx < nn) {
          const int i = idx / ne, j = idx % ne;
          if (i < n && j < n) {
            const int mi = partner[i], mj = partner[j];
            const double ai = alpha[i], bi = beta[i], aj = alpha[j], bj = beta[j];
            const double amj = mj < n ? H[i * LD + mj] : 0.0;
            const double ami = mi < n ? H[mi * LD + j] : 0.0;
            const double amm = (mi < n && mj < n) ? H[mi * LD + mj] : 0.0;
            const double ri = fma(aj, H[i * LD + j], bj * amj);
            const double rm = fma(aj, ami, bj * amm);
            na[e] = fma(ai, ri, bi * rm);
            const double umj = mj < n ? U[i * LD + mj] : 0.0;
            nu[e] = fma(aj, U[i * LD + j], bj * umj);
          }
        }
      }
      wave_sync();
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = t + 16 * e;
        if (idx < nn) {
          const int i = idx / ne, j = idx % ne;
          if (i < n && j < n) {
            H[i * LD + j] = na[e];
            U[i * LD + j] = nu[e];
          }
        }
      }
      wave_sync();
    }
  }
}

__global__ __launch_bounds__(256) void k_warmstart(const double* __restrict__ gpart, const int32_t* __restrict__ item_start,
                                                   const BlockDesc* __restrict__ desc, int64_t nblocks,
                                                   const double* __restrict__ eps_v, int r_max,
                                                   const float* __restrict__ mlp_out, int iters, int margin,
                                                   int retry,
                                                   uint8_t* __restrict__ rank_out, double* __restrict__ lam_out,
                                                   double* __restrict__ basis_out, int64_t* __restrict__ qv_size,
                                                   int64_t* __restrict__ qa_size, uint8_t* __restrict__ reject,
                                                   unsigned long long* __restrict__ counters,
                                                   unsigned long long* __restrict__ jstats) {
  constexpr int RH = kWarmMax, LQ = RH, LH = RH + 1;
  __shared__ double sQ[16][16 * LQ];
  __shared__ double sH[16][RH * LH], sU[16][RH * LH];
  __shared__ double sAl[16][RH], sBe[16][RH], sTh[16][RH], sSg[16][RH];
  __shared__ int sPa[16][RH], sPe[16][RH];
  __shared__ unsigned int n_acc, n_rej;
  const int grp = threadIdx.x >> 4, t = threadIdx.x & 15;
  if (threadIdx.x == 0) { n_acc = 0; n_rej = 0; }
  __syncthreads();
  const int64_t b = int64_t(blockIdx.x) * 16 + grp;
  double* Q = sQ[grp];
  double* H = sH[grp];
  double* U = sU[grp];
  int verdict = 0;  // 0: no block, 1: accepted, 2: rejected
  if (retry && b < nblocks && reject[b] == 0) {
    verdict = 1;  // accepted by attempt 1
  } else if (b < nblocks) {
    const BlockDesc d = desc[b];
    const int W = d.w(), M = d.m;
    int rcap = r_max < W ? r_max : W;
    rcap = rcap < M ? rcap : M;
    const float* o = mlp_out + b * 272;
    int rhat = 0;
    float best = o[0];
    for (int k = 1; k < 16; ++k)
      if (o[k] > best) { best = o[k]; rhat = k; }
    rhat = rhat + 1 + margin;
    rhat = rhat < rcap ? rhat : rcap;
    // attempt 1: the predicted rhat columns and `iters` iterations; attempt 2
    // (a second launch, blocks rejected by attempt 1 only): kRetryExtra more
    // columns, kRetryIters more iterations
    int rhat2 = rhat + kRetryExtra;
    rhat2 = rhat2 < RH ? rhat2 : RH;
    rhat2 = rhat2 < rcap ? rhat2 : rcap;
    const int nc = retry ? rhat2 : rhat;
    const int nit = retry ? iters + kRetryIters : iters;
    // a block that takes no attempt here (too large, too many columns, or
    // no wider retry) is left to the Jacobi fallback without reading its Gram
    const bool attempt = M <= kWarmMaxPoints && nc <= RH && (!retry || rhat2 > rhat);
    bool fin = true;
    double g[16], gc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) g[j] = gc[j] = 0.0;
    if (attempt) {
      const int i0 = item_start[b], i1 = item_start[b + 1];
      for (int it = i0; it < i1; ++it) {  // every entry's loads of an item issued together
        const double* gp = gpart + int64_t(it) * 256;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          g[j] += gp[t * 16 + j];
          gc[j] += gp[j * 16 + t];
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        g[j] = 0.5 * (g[j] + gc[j]);
        fin = fin && isfinite(g[j]);
      }
      fin = row_sum(fin ? 0.0 : 1.0) == 0.0;
    }
    int r = 0;
    if (attempt && fin) {
      double q[RH];
#pragma unroll
      for (int k = 0; k < RH; ++k) q[k] = (t < W && k < nc) ? double(o[16 + k * 16 + t]) : 0.0;
      orth_rows(q, nc, W, t);
      double y[RH], z[RH];
      auto times_g = [&]() {  // y = G Q, row t
#pragma unroll
        for (int k = 0; k < RH; ++k) Q[t * LQ + k] = q[k];
        wave_sync();
#pragma unroll
        for (int k = 0; k < RH; ++k) y[k] = 0.0;
#pragma unroll
        for (int j = 0; j < 16; ++j)
#pragma unroll
          for (int k = 0; k < RH; ++k) y[k] = fma(g[j], Q[j * LQ + k], y[k]);
        wave_sync();
      };
      for (int s = 0; s < nit; ++s) {
        times_g();
#pragma unroll
        for (int k = 0; k < RH; ++k) q[k] = y[k];
        orth_rows(q, nc, W, t);
      }
      // Rayleigh-Ritz: H = Q^T G Q (upper triangle, mirrored), U = I
      times_g();
#pragma unroll
      for (int a = 0; a < RH; ++a)
#pragma unroll
        for (int c = a; c < RH; ++c) {
          const double h = row_sum(q[a] * y[c]);
          if (t == 0) {
            H[a * LH + c] = (a < nc && c < nc) ? h : 0.0;
            H[c * LH + a] = (a < nc && c < nc) ? h : 0.0;
            U[a * LH + c] = a == c ? 1.0 : 0.0;
            U[c * LH + a] = a == c ? 1.0 : 0.0;
          }
        }
      wave_sync();
      if (!jacobi_group(H, U, sAl[grp], sBe[grp], sPa[grp], nc, t) && t == 0) atomicAdd(jstats, 1ull);
      // descending order of the Ritz values (stable by index)
      if (t < nc) {
        const double dk = H[t * LH + t];
        int pos = 0;
        for (int j = 0; j < nc; ++j) {
          const double dj = H[j * LH + j];
          pos += (dj > dk || (dj == dk && j < t)) ? 1 : 0;
        }
        sPe[grp][pos] = t;
        sTh[grp][pos] = dk;
      }
      wave_sync();
      // Ritz vectors Z[:, c] = Q U[:, perm[c]], then canonical signs
#pragma unroll
      for (int c = 0; c < RH; ++c) {
        double v = 0.0;
        if (c < nc) {
          const int col = sPe[grp][c];
#pragma unroll
          for (int j = 0; j < RH; ++j) v = fma(q[j], U[j * LH + col], v);
        }
        z[c] = v;
        Q[t * LQ + c] = v;
      }
      wave_sync();
      if (t < nc) {
        double besta = -1.0, sg = 1.0;
        for (int i = 0; i < 16; ++i) {
          const double v = Q[i * LQ + t];
          if (fabs(v) > besta) { besta = fabs(v); sg = v < 0.0 ? -1.0 : 1.0; }
        }
        sSg[grp][t] = sg;
      }
      wave_sync();
#pragma unroll
      for (int c = 0; c < RH; ++c) z[c] = c < nc ? z[c] * sSg[grp][c] : 0.0;
      // acceptance: smallest r <= nc whose discarded energy meets tau
      double diag = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) diag = (j == t) ? g[j] : diag;
      const double tr = row_sum(diag);
      const double eps = eps_v[d.var];
      const double tau = kKappa * eps * eps * double(M) * double(W);
      double cum = 0.0;
      for (int k = 1; k <= nc; ++k) {
        cum += sTh[grp][k - 1];
        if (tr - cum <= tau) { r = k; break; }
      }
      if (r > 0) {
        lam_out[b * 16 + t] = t < r ? fmax(sTh[grp][t < RH ? t : 0], 0.0) : 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) basis_out[b * 256 + k * 16 + t] = (k < r && k < RH) ? z[k < RH ? k : 0] : 0.0;
      }
    }
    if (r == 0) {
      verdict = 2;
      if (t == 0) reject[b] = 1;
    } else {
      verdict = 1;
      if (t == 0) {
        reject[b] = 0;
        rank_out[b] = uint8_t(r);
        qv_size[b] = 4 * pad16(int64_t(W) * r);
        qa_size[b] = 4 * pad16(int64_t(M) * r);
      }
    }
  }
  if (t == 0 && verdict == 1) atomicAdd(&n_acc, 1u);
  if (t == 0 && verdict == 2) atomicAdd(&n_rej, 1u);
  __syncthreads();
  if (threadIdx.x == 0 && retry) {  // final counts after both attempts
    if (n_acc) atomicAdd(counters, (unsigned long long)n_acc);
    if (n_rej) atomicAdd(counters + 1, (unsigned long long)n_rej);
  }
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_features(int dtype, const void* F, const Dims& dims, const BlockDesc* desc,
                           const FeatureLists& L, const double* eps_v, float* feat, hipStream_t s) {
  const dim3 bl{256};
  if (L.nsmall > 0) {
    const dim3 g{unsigned((L.nsmall + 15) / 16)};
    if (dtype == 0)
      hipLaunchKernelGGL(k_features_small<float>, g, bl, 0, s, (const float*)F, dims, desc, L.small, L.nsmall, eps_v,
                         feat);
    else
      hipLaunchKernelGGL(k_features_small<double>, g, bl, 0, s, (const double*)F, dims, desc, L.small, L.nsmall,
                         eps_v, feat);
    if (hipError_t e = hipGetLastError()) return e;
  }
  if (L.nwave > 0) {
    const dim3 g{unsigned((L.nwave + 3) / 4)};
    if (dtype == 0)
      hipLaunchKernelGGL(k_features_wave<float>, g, bl, 0, s, (const float*)F, dims, desc, L.wave, L.nwave, eps_v,
                         feat);
    else
      hipLaunchKernelGGL(k_features_wave<double>, g, bl, 0, s, (const double*)F, dims, desc, L.wave, L.nwave,
                         eps_v, feat);
    if (hipError_t e = hipGetLastError()) return e;
  }
  if (L.nzero > 0) {
    hipLaunchKernelGGL(k_features_zero, dim3{unsigned((L.nzero * 80 + 255) / 256)}, bl, 0, s, L.zero, L.nzero, feat);
    if (hipError_t e = hipGetLastError()) return e;
  }
  return hipSuccess;
}

hipError_t launch_normalize(const float* raw, int64_t n, const float* norm, float* z, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_normalize, dim3{unsigned((n * 80 + 255) / 256)}, dim3{256}, 0, s, raw, n, norm, z);
  return hipGetLastError();
}

hipError_t launch_gemm(bool ta, bool tb, bool bf16, const float* A, int lda, const float* B, int ldb, float* C,
                       int ldc, int M, int N, int K, const float* bias, int relu, hipStream_t s) {
  const int64_t tiles = int64_t((M + 15) / 16) * ((N + 15) / 16);
  if (tiles == 0) return hipSuccess;
  const dim3 g{unsigned((tiles + 3) / 4)}, bl{256};
#define DLS_GEMM(TA, TB, BF)                                                                       \
  hipLaunchKernelGGL((k_gemm<TA, TB, BF>), g, bl, 0, s, A, lda, B, ldb, C, ldc, M, N, K, bias, relu)
  if (!ta && !tb) { if (bf16) DLS_GEMM(false, false, true); else DLS_GEMM(false, false, false); }
  else if (ta && !tb) { if (bf16) DLS_GEMM(true, false, true); else DLS_GEMM(true, false, false); }
  else if (!ta && tb) { if (bf16) DLS_GEMM(false, true, true); else DLS_GEMM(false, true, false); }
  else return hipErrorInvalidValue;
#undef DLS_GEMM
  return hipGetLastError();
}

hipError_t launch_pack_weights(const float* P, short* packed, hipStream_t s) {
  const int64_t total = int64_t(kH + kH + kNO) * kPackLd;
  hipLaunchKernelGGL(k_pack_weights, dim3{unsigned((total + 255) / 256)}, dim3{256}, 0, s, P, packed);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* raw, int64_t n, const float* norm, const float* P, const short* packed,
                              float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3{unsigned((n + 63) / 64)}, dim3{256}, 0, s, raw, n, norm, P, packed, out);
  return hipGetLastError();
}

hipError_t launch_loss(const float* out, const int32_t* rank, const float* basis, const int32_t* wb, int64_t n,
                       float* gout, float* loss, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_loss, dim3{unsigned((n + 255) / 256)}, dim3{256}, 0, s, out, rank, basis, wb, n, gout, loss);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* G, int64_t n, int cols, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3{unsigned((cols + 3) / 4)}, dim3{256}, 0, s, G, n, cols, out);
  return hipGetLastError();
}

hipError_t launch_relu_mask(float* dh, const float* h, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_relu_mask, dim3{unsigned((n + 255) / 256)}, dim3{256}, 0, s, dh, h, n);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float c1, float c2,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3{unsigned((n + 255) / 256)}, dim3{256}, 0, s, p, g, m, v, n, lr, c1, c2);
  return hipGetLastError();
}

hipError_t launch_warmstart(const double* gpart, const int32_t* item_start, const BlockDesc* desc, int64_t nblocks,
                            const double* eps_v, int r_max, const float* mlp_out, int iters, int margin,
                            uint8_t* rank, double* lam, double* basis, int64_t* qv_size, int64_t* qa_size,
                            uint8_t* reject, unsigned long long* counters, unsigned long long* jstats,
                            hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  for (int retry = 0; retry < 2; ++retry)
    hipLaunchKernelGGL(k_warmstart, dim3{unsigned((nblocks + 15) / 16)}, dim3{256}, 0, s, gpart, item_start, desc,
                       nblocks, eps_v, r_max, mlp_out, iters, margin, retry, rank, lam, basis, qv_size, qa_size,
                       reject, counters, jstats);
  return hipGetLastError();
}

}  // namespace dls
