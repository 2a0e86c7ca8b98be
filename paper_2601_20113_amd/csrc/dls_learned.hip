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
// (normalised by the block mean and standard deviation).  One wavefront per
// block (four per workgroup): lanes stride the block's points, FP64 sums are
// reduced with a fixed xor-shuffle tree; lane c computes pooled cell c.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_features(const T* __restrict__ F, Dims dims,
                                                  const BlockDesc* __restrict__ desc, int64_t nblocks,
                                                  const double* __restrict__ eps_v, float* __restrict__ feat) {
  constexpr int kStage = kWarmMaxPoints;  // the block's per-point time sums live in LDS
  __shared__ double sts[4][kStage];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t b = int64_t(blockIdx.x) * 4 + wv;
  if (b >= nblocks) return;
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m, px = d.px(), py = d.py(), pz = d.pz();
  if (M > kWarmMaxPoints) {  // no warm start for this block: no features either
    feat[b * 80 + lane] = 0.f;
    if (lane < 16) feat[b * 80 + 64 + lane] = 0.f;
    return;
  }
  const int64_t nxy = dims.nx * dims.ny, tstride = dims.nz * nxy;
  const T* base = F + (((int64_t(d.var) * dims.nt + d.t0) * dims.nz + d.z0) * dims.ny + d.y0) * dims.nx + d.x0;
  const bool stage = true;  // M <= kWarmMaxPoints = kStage
  // the W values of point p (W <= 16), all loads issued before any use
  auto load_point = [&](int p, int64_t shift, double* x) {
    const int i = p % px, rho = p / px, j = rho % py, k = rho / py;
    const T* pt = base + int64_t(k) * nxy + int64_t(j) * dims.nx + i + shift;
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = (t < W) ? double(pt[int64_t(t) * tstride]) : 0.0;
  };
  double s1 = 0, s2 = 0, mn = INFINITY, mx = -INFINITY, adt = 0, sdt = 0, sdt2 = 0, adx = 0, ady = 0, tme = 0;
  // first-pass sums of point p from its values x and, where they exist, its
  // +x and +y neighbours xr, xd
  auto accumulate = [&](int p, const double* x, const double* xr, const double* xd) {
    const int i = p % px, j = (p / px) % py;
    double ts = 0.0;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      if (t < W) {
        const double v = x[t];
        s1 += v;
        s2 += v * v;
        mn = fmin(mn, v);
        mx = fmax(mx, v);
        ts += v;
        if (t > 0) {
          const double dt = v - x[t - 1];
          adt += fabs(dt);
          sdt += dt;
          sdt2 += dt * dt;
        }
        if (i + 1 < px) adx += fabs(xr[t] - v);
        if (j + 1 < py) ady += fabs(xd[t] - v);
      }
    }
    tme += ts * ts;
    if (stage) sts[wv][p] = ts;
  };
  // second-pass (central) sums of point p
  double c3 = 0, c4 = 0, l1 = 0, l2 = 0, cvar = 0;
  auto central = [&](const double* x, double mu) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      if (t < W) {
        const double y = x[t] - mu;
        const double y2 = y * y;
        cvar += y2;
        c3 += y2 * y;
        c4 += y2 * y2;
        if (t >= 1) l1 += y * (x[t - 1] - mu);
        if (t >= 2) l2 += y * (x[t - 2] - mu);
      }
    }
  };
  const bool one = M <= 64;  // one point per lane: neighbours come from other lanes, values stay in registers
  // FP32 blocks of 65..256 points: four points per lane (p = lane + 64 r),
  // kept in registers as loaded; neighbours come from other lanes
  const bool regs4 = sizeof(T) == 4 && !one;
  double x1[16];
  float xf[4][16];
  if (regs4) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = lane + 64 * r;
      const int i = p % px, rho = p / px, j = rho % py, k = rho / py;
      const T* pt = base + int64_t(k) * nxy + int64_t(j) * dims.nx + i;
#pragma unroll
      for (int t = 0; t < 16; ++t) xf[r][t] = (p < M && t < W) ? float(pt[int64_t(t) * tstride]) : 0.f;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = lane + 64 * r;
      const int i = p % px, j = (p / px) % py;
      const bool hr = i + 1 < px && p < M, hd = j + 1 < py && p < M;
      const int lr = (lane + 1) & 63, ld = (lane + px) & 63;
      const bool rr_next = lane + 1 >= 64, rd_next = lane + px >= 64;
      double ts = 0.0, prev = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        // every lane takes part in the shuffles
        const float ar = __shfl(xf[r][t], lr, 64), ad = __shfl(xf[r][t], ld, 64);
        const float br = r < 3 ? __shfl(xf[r < 3 ? r + 1 : r][t], lr, 64) : 0.f;
        const float bd = r < 3 ? __shfl(xf[r < 3 ? r + 1 : r][t], ld, 64) : 0.f;
        if (p < M && t < W) {
          const double v = xf[r][t];
          s1 += v;
          s2 += v * v;
          mn = fmin(mn, v);
          mx = fmax(mx, v);
          ts += v;
          if (t > 0) {
            const double dt = v - prev;
            adt += fabs(dt);
            sdt += dt;
            sdt2 += dt * dt;
          }
          if (hr) adx += fabs(double(rr_next ? br : ar) - v);
          if (hd) ady += fabs(double(rd_next ? bd : ad) - v);
          prev = v;
        }
      }
      if (p < M) {
        tme += ts * ts;
        sts[wv][p] = ts;
      }
    }
  } else if (one) {
    const bool act = lane < M;
    if (act) {
      load_point(lane, 0, x1);
    } else {
#pragma unroll
      for (int t = 0; t < 16; ++t) x1[t] = 0.0;
    }
    double xr[16], xd[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      xr[t] = __shfl(x1[t], lane + 1, 64);
      xd[t] = __shfl(x1[t], lane + px, 64);
    }
    if (act) accumulate(lane, x1, xr, xd);
  } else {
    for (int p = lane; p < M; p += 64) {
      const int i = p % px, j = (p / px) % py;
      double x[16], xr[16], xd[16];
      load_point(p, 0, x);
      if (i + 1 < px) load_point(p, 1, xr);
      if (j + 1 < py) load_point(p, dims.nx, xd);
      accumulate(p, x, xr, xd);
    }
  }
  s1 = wave_sum(s1); s2 = wave_sum(s2); adt = wave_sum(adt); sdt = wave_sum(sdt); sdt2 = wave_sum(sdt2);
  adx = wave_sum(adx); ady = wave_sum(ady); tme = wave_sum(tme);
  for (int o = 32; o >= 1; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  const double n = double(W) * M;
  const double mu = s1 / n;
  if (regs4) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (lane + 64 * r < M) {
        double x[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) x[t] = xf[r][t];
        central(x, mu);
      }
    }
  } else if (one) {
    if (lane < M) central(x1, mu);
  } else {
    for (int p = lane; p < M; p += 64) {
      double x[16];
      load_point(p, 0, x);
      central(x, mu);
    }
  }
  cvar = wave_sum(cvar); c3 = wave_sum(c3); c4 = wave_sum(c4); l1 = wave_sum(l1); l2 = wave_sum(l2);
  const double var = cvar / n;
  const double sd = sqrt(var);
  const double inv = sd > 0.0 ? 1.0 / sd : 0.0;
  wave_sync();
  // pooled time-mean: lane c owns cell (row group c / 8, column group c % 8)
  double cellv;
  {
    const int bb = lane >> 3, aa = lane & 7;
    int j0 = (bb * py + 7) / 8, j1 = ((bb + 1) * py + 7) / 8;
    int i0 = (aa * px + 7) / 8, i1 = ((aa + 1) * px + 7) / 8;
    if (j1 <= j0) { j0 = (bb * py) / 8; j1 = j0 + 1; }
    if (i1 <= i0) { i0 = (aa * px) / 8; i1 = i0 + 1; }
    double s = 0.0;
    if (stage) {
      for (int kk = 0; kk < pz; ++kk)
        for (int jj = j0; jj < j1; ++jj)
          for (int ii = i0; ii < i1; ++ii) s += sts[wv][(kk * py + jj) * px + ii];
    } else {
      for (int t = 0; t < W; ++t)
        for (int kk = 0; kk < pz; ++kk)
          for (int jj = j0; jj < j1; ++jj)
            for (int ii = i0; ii < i1; ++ii)
              s += double(base[int64_t(t) * tstride + int64_t(kk) * nxy + int64_t(jj) * dims.nx + ii]);
    }
    cellv = s / double((i1 - i0) * (j1 - j0) * pz * W);
  }
  float* o = feat + b * 80;
  o[16 + lane] = float(sd > 0.0 ? (cellv - mu) / sd : 0.0);
  if (lane == 0) {
    const double eps = eps_v[d.var];
    double f[16];
    f[0] = mu;
    f[1] = sd;
    f[2] = mn;
    f[3] = mx;
    f[4] = sd > 0.0 ? (c3 / n) / (sd * sd * sd) : 0.0;
    f[5] = sd > 0.0 ? (c4 / n) / (var * var) - 3.0 : 0.0;
    const double nd = double(W - 1) * M;
    f[6] = W > 1 ? (adt / nd) * inv : 0.0;
    const double mdt = W > 1 ? sdt / nd : 0.0;
    f[7] = W > 1 ? sqrt(fmax(sdt2 / nd - mdt * mdt, 0.0)) * inv : 0.0;
    f[8] = px > 1 ? (adx / (double(W) * (px - 1) * py * pz)) * inv : 0.0;
    f[9] = py > 1 ? (ady / (double(W) * px * (py - 1) * pz)) * inv : 0.0;
    f[10] = (W > 1 && sd > 0.0) ? (l1 / (double(W - 1) * M)) / var : 0.0;
    f[11] = (W > 2 && sd > 0.0) ? (l2 / (double(W - 2) * M)) / var : 0.0;
    f[12] = log10(fmax((s2 / n) / (eps * eps), 1e-30));
    f[13] = log10(fmax(sd / eps, 1e-15));
    f[14] = s2 > 0.0 ? tme / (double(W) * s2) : 0.0;
    f[15] = log2(double(M));
    for (int q = 0; q < 16; ++q) o[q] = float(f[q]);
  }
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
  __shared__ __align__(16) short sW[kNO * LW];
  __shared__ __align__(16) short sH[4][16 * LW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, q = lane >> 4;
  const int64_t row0 = int64_t(blockIdx.x) * 64 + wave * 16;
  const bool row_ok = row0 + r < n;
  short* H = sH[wave];
  // layer `l` (0, 1, 2) of N outputs: copy its packed image into LDS
  auto stage = [&](int l, int N) {
    const uint4* src = reinterpret_cast<const uint4*>(packed + int64_t(l) * kH * LW);
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
  stage(1, kH);
  __syncthreads();
  // h1 is read from H and h2 written back into it: read all fragments first
  bf16x4 h[8];
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) h[ks] = from_h(ks);
  __syncthreads();
  layer([&](int ks) { return h[ks]; }, 8, kH, hidden_out(P + kOffb2));
  __syncthreads();
  stage(2, kNO);
  __syncthreads();
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) h[ks] = from_h(ks);
  const float* b3 = P + kOffb3;
  layer([&](int ks) { return h[ks]; }, 8, kNO, [&](int nt, f32x4 acc) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = row0 + 4 * q + v;
      if (i < n) out[i * kNO + nt * 16 + r] = acc[v] + b3[nt * 16 + r];
    }
  });
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
// accumulated into U.  The 16 lanes of one group call it together.
__device__ void jacobi_group(double* H, double* U, double* alpha, double* beta, int* partner, int n, int t) {
  constexpr int LD = kWarmMax + 1;
  if (n <= 1) return;
  const int ne = n + (n & 1);
  const int nn = ne * ne;
  for (int sweep = 0; sweep < 12; ++sweep) {
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
    if (!(off > 1e-26 * tot)) break;
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
                                                   unsigned long long* __restrict__ counters) {
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
    const int i0 = item_start[b], i1 = item_start[b + 1];
    double g[16], gc[16];
    bool fin = true;
#pragma unroll
    for (int j = 0; j < 16; ++j) g[j] = gc[j] = 0.0;
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
    int r = 0;
    if (fin && M <= kWarmMaxPoints && nc <= RH && (!retry || rhat2 > rhat)) {
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
      jacobi_group(H, U, sAl[grp], sBe[grp], sPa[grp], nc, t);
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
hipError_t launch_features(int dtype, const void* F, const Dims& dims, const BlockDesc* desc, int64_t nblocks,
                           const double* eps_v, float* feat, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  const dim3 g{unsigned((nblocks + 3) / 4)}, bl{256};
  if (dtype == 0) hipLaunchKernelGGL(k_features<float>, g, bl, 0, s, (const float*)F, dims, desc, nblocks, eps_v, feat);
  else hipLaunchKernelGGL(k_features<double>, g, bl, 0, s, (const double*)F, dims, desc, nblocks, eps_v, feat);
  return hipGetLastError();
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
                            uint8_t* reject, unsigned long long* counters, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  for (int retry = 0; retry < 2; ++retry)
    hipLaunchKernelGGL(k_warmstart, dim3{unsigned((nblocks + 15) / 16)}, dim3{256}, 0, s, gpart, item_start, desc,
                       nblocks, eps_v, r_max, mlp_out, iters, margin, retry, rank, lam, basis, qv_size, qa_size,
                       reject, counters);
  return hipGetLastError();
}

}  // namespace dls
