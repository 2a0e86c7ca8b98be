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
// (normalised by the block mean and standard deviation).  One 256-thread
// workgroup per block, FP64 sums reduced in a fixed order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_min(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(256) void k_features(const T* __restrict__ F, Dims dims,
                                                  const BlockDesc* __restrict__ desc,
                                                  const double* __restrict__ eps_v, float* __restrict__ feat) {
  __shared__ double red[256];
  __shared__ double cell[64];
  const int b = blockIdx.x;
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m, px = d.px(), py = d.py(), pz = d.pz();
  const int64_t nxy = dims.nx * dims.ny, tstride = dims.nz * nxy;
  const T* base = F + (((int64_t(d.var) * dims.nt + d.t0) * dims.nz + d.z0) * dims.ny + d.y0) * dims.nx + d.x0;
  auto at = [&](int t, int i, int j, int k) { return double(base[int64_t(t) * tstride + int64_t(k) * nxy + int64_t(j) * dims.nx + i]); };

  double s1 = 0, s2 = 0, mn = INFINITY, mx = -INFINITY, adt = 0, sdt = 0, sdt2 = 0, adx = 0, ady = 0, tme = 0;
  for (int p = threadIdx.x; p < M; p += 256) {
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
  const double n = double(W) * M;
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  mn = block_min(mn, red);
  mx = -block_min(-mx, red);
  adt = block_sum(adt, red);
  sdt = block_sum(sdt, red);
  sdt2 = block_sum(sdt2, red);
  adx = block_sum(adx, red);
  ady = block_sum(ady, red);
  tme = block_sum(tme, red);
  const double mu = s1 / n;

  double c3 = 0, c4 = 0, l1 = 0, l2 = 0, cvar = 0;
  for (int p = threadIdx.x; p < M; p += 256) {
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
  cvar = block_sum(cvar, red);
  c3 = block_sum(c3, red);
  c4 = block_sum(c4, red);
  l1 = block_sum(l1, red);
  l2 = block_sum(l2, red);
  const double var = cvar / n;
  const double sd = sqrt(var);
  const double inv = sd > 0.0 ? 1.0 / sd : 0.0;

  // pooled time-mean: cell c = (row group bb, column group aa), 4 threads per cell
  {
    const int c = threadIdx.x >> 2, sub = threadIdx.x & 3;
    const int bb = c >> 3, aa = c & 7;
    int j0 = (bb * py + 7) / 8, j1 = ((bb + 1) * py + 7) / 8;
    int i0 = (aa * px + 7) / 8, i1 = ((aa + 1) * px + 7) / 8;
    if (j1 <= j0) { j0 = (bb * py) / 8; j1 = j0 + 1; }
    if (i1 <= i0) { i0 = (aa * px) / 8; i1 = i0 + 1; }
    const int ci = i1 - i0, cj = j1 - j0;
    const int npix = ci * cj * pz * W;
    double s = 0.0;
    for (int q = sub; q < npix; q += 4) {
      const int ii = q % ci, r1 = q / ci, jj = r1 % cj, r2 = r1 / cj, kk = r2 % pz, t = r2 / pz;
      s += at(t, i0 + ii, j0 + jj, kk);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (sub == 0) {
      const double tot = ((red[threadIdx.x] + red[threadIdx.x + 1]) + red[threadIdx.x + 2]) + red[threadIdx.x + 3];
      cell[c] = tot / double(npix);
    }
    __syncthreads();
  }

  if (threadIdx.x == 0) {
    const double eps = eps_v[d.var];
    float* o = feat + int64_t(b) * 80;
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
    for (int q = 0; q < 64; ++q) o[16 + q] = float(sd > 0.0 ? (cell[q] - mu) / sd : 0.0);
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

__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ G, int64_t n, int cols,
                                                float* __restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += G[i * cols + j];
  out[j] = float(s);
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
// Warm-started eigensolve of one block (W <= 16): one 64-lane workgroup.
// ---------------------------------------------------------------------------
// Modified Gram-Schmidt (twice) of the first r columns of Q (LDS, [t][k],
// leading dimension 17) over rows t < W; a collapsing column is replaced by
// the first unit vector e_j that stays independent.  Lanes t < 16 own row t.
__device__ void mgs16(double* Q, int r, int W, int tid) {
  const int t = tid & 15;
  const bool own = tid < 16;
  auto dot16 = [&](double v) {
    for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
    return v;
  };
  for (int k = 0; k < r; ++k) {
    double y = (t < W) ? Q[t * 17 + k] : 0.0;
    const double n0 = sqrt(dot16(y * y));
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < k; ++j) {
        const double qj = (t < W) ? Q[t * 17 + j] : 0.0;
        const double c = dot16(qj * y);
        y -= c * qj;
      }
    double nrm = sqrt(dot16(y * y));
    if (!(nrm > 1e-12 * n0) || n0 == 0.0) {
      for (int e = 0; e < W; ++e) {
        y = (t == e) ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass)
          for (int j = 0; j < k; ++j) {
            const double qj = (t < W) ? Q[t * 17 + j] : 0.0;
            const double c = dot16(qj * y);
            y -= c * qj;
          }
        nrm = sqrt(dot16(y * y));
        if (nrm > 0.5) break;
      }
    }
    __syncthreads();
    if (own) Q[t * 17 + k] = (t < W) ? y / nrm : 0.0;
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void k_warmstart(const double* __restrict__ gpart, const int32_t* __restrict__ item_start,
                                                  const BlockDesc* __restrict__ desc, const double* __restrict__ eps_v,
                                                  int r_max, const float* __restrict__ mlp_out, int iters,
                                                  uint8_t* __restrict__ rank_out, double* __restrict__ lam_out,
                                                  double* __restrict__ basis_out, int64_t* __restrict__ qv_size,
                                                  int64_t* __restrict__ qa_size, uint8_t* __restrict__ reject,
                                                  unsigned long long* __restrict__ counters) {
  constexpr int LD = 17;
  __shared__ double G[16 * LD], Q[16 * LD], Y[16 * LD], H[16 * LD], U[16 * LD];
  __shared__ double alpha[16], beta[16], th[16];
  __shared__ int partner[16], perm[16];
  const int b = blockIdx.x, tid = threadIdx.x;
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m;
  const int i0 = item_start[b], i1 = item_start[b + 1];
  bool fin = true;
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 64 * e;
    double s = 0.0;
    for (int it = i0; it < i1; ++it) s += gpart[int64_t(it) * 256 + idx];
    G[(idx >> 4) * LD + (idx & 15)] = s;
  }
  __syncthreads();
  double gs[4];
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 64 * e, i = idx >> 4, j = idx & 15;
    gs[e] = 0.5 * (G[i * LD + j] + G[j * LD + i]);
    fin = fin && isfinite(gs[e]);
  }
  __syncthreads();
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 64 * e;
    G[(idx >> 4) * LD + (idx & 15)] = gs[e];
  }
  fin = __syncthreads_and(fin);
  if (!fin) {  // non-finite block: the plain path makes it a raw block
    if (tid == 0) reject[b] = 1;
    return;
  }
  int rcap = r_max < W ? r_max : W;
  rcap = rcap < M ? rcap : M;
  const float* o = mlp_out + int64_t(b) * 272;
  int rhat = 0;
  float best = o[0];
  for (int k = 1; k < 16; ++k)
    if (o[k] > best) { best = o[k]; rhat = k; }
  rhat = rhat + 1;
  rhat = rhat < rcap ? rhat : rcap;
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 64 * e, t = idx >> 4, k = idx & 15;
    Q[t * LD + k] = (t < W && k < rhat) ? double(o[16 + k * 16 + t]) : 0.0;
  }
  __syncthreads();
  mgs16(Q, rhat, W, tid);
  for (int s = 0; s < iters; ++s) {
    for (int e = 0; e < 4; ++e) {  // Y = G Q
      const int idx = tid + 64 * e, t = idx >> 4, k = idx & 15;
      double y = 0.0;
      if (k < rhat)
        for (int j = 0; j < 16; ++j) y = fma(G[t * LD + j], Q[j * LD + k], y);
      Y[t * LD + k] = y;
    }
    __syncthreads();
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 64 * e, t = idx >> 4, k = idx & 15;
      Q[t * LD + k] = Y[t * LD + k];
    }
    __syncthreads();
    mgs16(Q, rhat, W, tid);
  }
  // Rayleigh-Ritz: H = Q^T (G Q), padded to 16 with zeros; Jacobi; sort
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 64 * e, t = idx >> 4, k = idx & 15;
    double y = 0.0;
    if (k < rhat)
      for (int j = 0; j < 16; ++j) y = fma(G[t * LD + j], Q[j * LD + k], y);
    Y[t * LD + k] = y;
  }
  __syncthreads();
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 64 * e, i = idx >> 4, j = idx & 15;
    double h = 0.0;
    if (i < rhat && j < rhat)
      for (int t = 0; t < 16; ++t) h = fma(Q[t * LD + i], Y[t * LD + j], h);
    H[i * LD + j] = h;
    U[i * LD + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int e = 0; e < 4; ++e) {  // symmetrise
    const int idx = tid + 64 * e, i = idx >> 4, j = idx & 15;
    gs[e] = 0.5 * (H[i * LD + j] + H[j * LD + i]);
  }
  __syncthreads();
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 64 * e;
    H[(idx >> 4) * LD + (idx & 15)] = gs[e];
  }
  __syncthreads();
  jacobi_lds<16>(H, U, alpha, beta, partner, tid);
  if (tid < 16) perm[tid] = tid;
  __syncthreads();
  if (tid < 16) {
    const double dk = tid < rhat ? H[tid * LD + tid] : -INFINITY;
    int pos = 0;
    for (int j = 0; j < 16; ++j) {
      const double dj = j < rhat ? H[j * LD + j] : -INFINITY;
      pos += (dj > dk || (dj == dk && j < tid)) ? 1 : 0;
    }
    perm[pos] = tid;
  }
  __syncthreads();
  // Ritz vectors Z[:, c] = Q U[:, perm[c]], canonical signs
  if (tid < 16) {
    const int c = tid;
    int col = perm[c];
    col = (col >= 0 && col < 16) ? col : c;
    th[c] = c < rhat ? H[col * LD + col] : 0.0;
    double best_a = -1.0, sgn = 1.0;
    for (int t = 0; t < 16; ++t) {
      double z = 0.0;
      if (c < rhat)
        for (int j = 0; j < 16; ++j) z = fma(Q[t * LD + j], U[j * LD + col], z);
      Y[t * LD + c] = z;
      if (fabs(z) > best_a) { best_a = fabs(z); sgn = z < 0.0 ? -1.0 : 1.0; }
    }
    for (int t = 0; t < 16; ++t) Y[t * LD + c] *= sgn;
  }
  __syncthreads();
  __shared__ int acc_r;
  if (tid == 0) {
    double tr = 0.0;
    for (int t = 0; t < 16; ++t) tr += G[t * LD + t];
    const double eps = eps_v[d.var];
    const double tau = kKappa * eps * eps * double(M) * double(W);
    int r = 0;
    double cum = 0.0;
    for (int k = 1; k <= rhat; ++k) {
      cum += th[k - 1];
      if (tr - cum <= tau) { r = k; break; }
    }
    acc_r = r;
    if (r == 0) {
      reject[b] = 1;
      atomicAdd(counters + 1, 1ULL);
    } else {
      reject[b] = 0;
      atomicAdd(counters, 1ULL);
      rank_out[b] = uint8_t(r);
      qv_size[b] = 4 * pad16(int64_t(W) * r);
      qa_size[b] = 4 * pad16(int64_t(M) * r);
    }
  }
  __syncthreads();
  const int r = acc_r;
  if (r == 0) return;
  if (tid < 16) lam_out[int64_t(b) * 16 + tid] = tid < r ? fmax(th[tid], 0.0) : 0.0;
  for (int e = 0; e < 4; ++e) {
    const int idx = tid + 64 * e, k = idx >> 4, t = idx & 15;
    basis_out[int64_t(b) * 256 + idx] = (k < r) ? Y[t * LD + k] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_features(int dtype, const void* F, const Dims& dims, const BlockDesc* desc, int64_t nblocks,
                           const double* eps_v, float* feat, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  const dim3 g{unsigned(nblocks)}, bl{256};
  if (dtype == 0) hipLaunchKernelGGL(k_features<float>, g, bl, 0, s, (const float*)F, dims, desc, eps_v, feat);
  else hipLaunchKernelGGL(k_features<double>, g, bl, 0, s, (const double*)F, dims, desc, eps_v, feat);
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
  hipLaunchKernelGGL(k_colsum, dim3{unsigned((cols + 255) / 256)}, dim3{256}, 0, s, G, n, cols, out);
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
                            const double* eps_v, int r_max, const float* mlp_out, int iters, uint8_t* rank,
                            double* lam, double* basis, int64_t* qv_size, int64_t* qa_size, uint8_t* reject,
                            unsigned long long* counters, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_warmstart, dim3{unsigned(nblocks)}, dim3{64}, 0, s, gpart, item_start, desc, eps_v, r_max,
                     mlp_out, iters, rank, lam, basis, qv_size, qa_size, reject, counters);
  return hipGetLastError();
}

}  // namespace dls
