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
  const int lane = threadIdx.x & 63;
  const int64_t b = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (b >= nblocks) return;
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m, px = d.px(), py = d.py(), pz = d.pz();
  const int64_t nxy = dims.nx * dims.ny, tstride = dims.nz * nxy;
  const T* base = F + (((int64_t(d.var) * dims.nt + d.t0) * dims.nz + d.z0) * dims.ny + d.y0) * dims.nx + d.x0;
  auto at = [&](int t, int i, int j, int k) {
    return double(base[int64_t(t) * tstride + int64_t(k) * nxy + int64_t(j) * dims.nx + i]);
  };
  double s1 = 0, s2 = 0, mn = INFINITY, mx = -INFINITY, adt = 0, sdt = 0, sdt2 = 0, adx = 0, ady = 0, tme = 0;
  for (int p = lane; p < M; p += 64) {
    const int i = p % px, rho = p / px, j = rho % py, k = rho / py;
    double prev = 0.0, ts = 0.0;
    for (int t = 0; t < W; ++t) {
      const double x = at(t, i, j, k);
      s1 += x;
      s2 += x * x;
      mn = fmin(mn, x);
      mx = fmax(mx, x);
      ts += x;
      if (t > 0) {
        const double dt = x - prev;
        adt += fabs(dt);
        sdt += dt;
        sdt2 += dt * dt;
      }
      if (i + 1 < px) adx += fabs(at(t, i + 1, j, k) - x);
      if (j + 1 < py) ady += fabs(at(t, i, j + 1, k) - x);
      prev = x;
    }
    tme += ts * ts;
  }
  s1 = wave_sum(s1); s2 = wave_sum(s2); adt = wave_sum(adt); sdt = wave_sum(sdt); sdt2 = wave_sum(sdt2);
  adx = wave_sum(adx); ady = wave_sum(ady); tme = wave_sum(tme);
  for (int o = 32; o >= 1; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  const double n = double(W) * M;
  const double mu = s1 / n;
  double c3 = 0, c4 = 0, l1 = 0, l2 = 0, cvar = 0;
  for (int p = lane; p < M; p += 64) {
    const int i = p % px, rho = p / px, j = rho % py, k = rho / py;
    double x1 = 0, x2 = 0;
    for (int t = 0; t < W; ++t) {
      const double y = at(t, i, j, k) - mu;
      const double y2 = y * y;
      cvar += y2;
      c3 += y2 * y;
      c4 += y2 * y2;
      if (t >= 1) l1 += y * x1;
      if (t >= 2) l2 += y * x2;
      x2 = x1;
      x1 = y;
    }
  }
  cvar = wave_sum(cvar); c3 = wave_sum(c3); c4 = wave_sum(c4); l1 = wave_sum(l1); l2 = wave_sum(l2);
  const double var = cvar / n;
  const double sd = sqrt(var);
  const double inv = sd > 0.0 ? 1.0 / sd : 0.0;
  // pooled time-mean: lane c owns cell (row group c / 8, column group c % 8)
  double cellv;
  {
    const int bb = lane >> 3, aa = lane & 7;
    int j0 = (bb * py + 7) / 8, j1 = ((bb + 1) * py + 7) / 8;
    int i0 = (aa * px + 7) / 8, i1 = ((aa + 1) * px + 7) / 8;
    if (j1 <= j0) { j0 = (bb * py) / 8; j1 = j0 + 1; }
    if (i1 <= i0) { i0 = (aa * px) / 8; i1 = i0 + 1; }
    double s = 0.0;
    for (int t = 0; t < W; ++t)
      for (int kk = 0; kk < pz; ++kk)
        for (int jj = j0; jj < j1; ++jj)
          for (int ii = i0; ii < i1; ++ii) s += at(t, ii, jj, kk);
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
constexpr int kWarmMax = 8;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = uint64_t(__double_as_longlong(v));
  const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(u)), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)((uint64_t(uint32_t(hi)) << 32) | uint64_t(uint32_t(lo))));
}

// Sum over the 16 lanes of a DPP row.  Each step adds a lane's value to its
// partner's (x + y in one lane, y + x in the other: the same bits), so all
// 16 lanes end with the same result.
__device__ __forceinline__ double row_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return v;
}

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
        if (q < n) {
          const double app = H[p * LD + p], aqq = H[q * LD + q], apq = H[p * LD + q];
          if (apq != 0.0) {
            const double theta = (aqq - app) / (2.0 * apq);
            double tt = 1.0 / (fabs(theta) + sqrt(1.0 + theta * theta));
            if (theta < 0.0) tt = -tt;
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
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
  if (b < nblocks) {
    const BlockDesc d = desc[b];
    const int W = d.w(), M = d.m;
    const int i0 = item_start[b], i1 = item_start[b + 1];
    double g[16];
    bool fin = true;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      double s1 = 0.0, s2 = 0.0;
      for (int it = i0; it < i1; ++it) {
        s1 += gpart[int64_t(it) * 256 + t * 16 + j];
        s2 += gpart[int64_t(it) * 256 + j * 16 + t];
      }
      g[j] = 0.5 * (s1 + s2);
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
    int r = 0;
    double z[RH];
    if (fin && rhat <= RH) {
      double q[RH];
#pragma unroll
      for (int k = 0; k < RH; ++k) q[k] = (t < W && k < rhat) ? double(o[16 + k * 16 + t]) : 0.0;
      orth_rows(q, rhat, W, t);
      double y[RH];
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
      for (int s = 0; s < iters; ++s) {
        times_g();
#pragma unroll
        for (int k = 0; k < RH; ++k) q[k] = y[k];
        orth_rows(q, rhat, W, t);
      }
      // Rayleigh-Ritz: H = Q^T G Q (upper triangle, mirrored), U = I
      times_g();
#pragma unroll
      for (int a = 0; a < RH; ++a)
#pragma unroll
        for (int c = a; c < RH; ++c) {
          const double h = row_sum(q[a] * y[c]);
          if (t == 0) {
            H[a * LH + c] = (a < rhat && c < rhat) ? h : 0.0;
            H[c * LH + a] = (a < rhat && c < rhat) ? h : 0.0;
            U[a * LH + c] = a == c ? 1.0 : 0.0;
            U[c * LH + a] = a == c ? 1.0 : 0.0;
          }
        }
      wave_sync();
      jacobi_group(H, U, sAl[grp], sBe[grp], sPa[grp], rhat, t);
      // descending order of the Ritz values (stable by index)
      if (t < rhat) {
        const double dk = H[t * LH + t];
        int pos = 0;
        for (int j = 0; j < rhat; ++j) {
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
        if (c < rhat) {
          const int col = sPe[grp][c];
#pragma unroll
          for (int j = 0; j < RH; ++j) v = fma(q[j], U[j * LH + col], v);
        }
        z[c] = v;
        Q[t * LQ + c] = v;
      }
      wave_sync();
      if (t < rhat) {
        double besta = -1.0, sg = 1.0;
        for (int i = 0; i < 16; ++i) {
          const double v = Q[i * LQ + t];
          if (fabs(v) > besta) { besta = fabs(v); sg = v < 0.0 ? -1.0 : 1.0; }
        }
        sSg[grp][t] = sg;
      }
      wave_sync();
#pragma unroll
      for (int c = 0; c < RH; ++c) z[c] = c < rhat ? z[c] * sSg[grp][c] : 0.0;
      // acceptance: smallest r <= rhat whose discarded energy meets tau
      double diag = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) diag = (j == t) ? g[j] : diag;
      const double tr = row_sum(diag);
      const double eps = eps_v[d.var];
      const double tau = kKappa * eps * eps * double(M) * double(W);
      double cum = 0.0;
      for (int k = 1; k <= rhat; ++k) {
        cum += sTh[grp][k - 1];
        if (tr - cum <= tau) { r = k; break; }
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
      lam_out[b * 16 + t] = t < r ? fmax(sTh[grp][t < RH ? t : 0], 0.0) : 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) basis_out[b * 256 + k * 16 + t] = (k < r && k < RH) ? z[k < RH ? k : 0] : 0.0;
    }
  }
  if (t == 0 && verdict == 1) atomicAdd(&n_acc, 1u);
  if (t == 0 && verdict == 2) atomicAdd(&n_rej, 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
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
  hipLaunchKernelGGL(k_warmstart, dim3{unsigned((nblocks + 15) / 16)}, dim3{256}, 0, s, gpart, item_start, desc,
                     nblocks, eps_v, r_max, mlp_out, iters, margin, rank, lam, basis, qv_size, qa_size, reject,
                     counters);
  return hipGetLastError();
}

}  // namespace dls
