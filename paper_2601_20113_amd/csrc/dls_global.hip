// Global-basis mode: the paper's own method (Sec. 2.2-2.5, Alg. 1) -- one
// basis per variable, learned once, applied to every patch of every
// snapshot under the L2 target of Sec. 2.4.
//
//   learn   S = 4M patches of M = Px Py Pz points at SplitMix64 positions
//           of the first snapshot form Q (S x M); the full eigenbasis of
//           Q^T Q (the right singular vectors of Q, Eqs. (2)-(3), Sec. 2.7.1)
//           is the compression matrix, eigenvalues descending, canonical
//           signs, stored on the 2^-24 grid.  The basis study of Sec. 4 adds
//           the orthonormal DCT-II tensor basis and the eigenbasis of a
//           uniform random M x M matrix.
//   budget  e2 = c_v M_b, c_v = (eps_t,v ||u_v||)^2 / K_v (Eq. (4)).
//   encode  alpha = Phi^T u per patch and snapshot (u zero-padded at the
//           edges); the fewest coefficients in decreasing |alpha| (ties: the
//           lower index) whose dropped energy is <= 0.36 e2; bit grooming on
//           the grid d = 2^k, k = floor(log2(0.4 sqrt(e2 / n))); the exact
//           squared error of the returned values must be <= e2, else one
//           more coefficient (Alg. 1 step 3, Eq. (6)); raw past n = M, on
//           |q| >= 2^31 or non-finite input.
//
// Kernels:
//   k_gb_sumsq / k_gb_budget   c_v (fixed partial grid, fixed order)
//   k_gb_samples               Q from the counter form of SplitMix64
//   k_gb_gram                  Q^T Q on the FP64 matrix cores
//   k_gb_eye                   V = I
//   k_gb_jacobi_round          one round of the parallel cyclic Jacobi:
//                              M/2 disjoint rotations applied at once
//   k_gb_offnorm / k_gb_sum    the sweep's off-diagonal and total norms
//   k_gb_jacobi_lds            the whole eigensolve of order <= 64 in LDS
//   k_gb_finish                order, signs, 2^-24 grid
//   k_gb_cosine                the DCT-II tensor basis
//   k_gb_project               alpha = U Phi on the FP64 matrix cores
//   k_gb_select                per patch: order, count, grooming, exact check
//   k_gb_patch64               the same with the coefficients, one team of
//                              16, 32 or 64 lanes per patch of at most that
//                              many points
//   k_gb_compact               the per-patch slots into packed arrays
//   k_gb_decode64              the decoder for patches of at most 64 points
//                              (persistent, Phi in LDS, teams as above)
//   k_gb_decode                the decoder, a workgroup per patch above 64
//
// Compiled with -ffp-contract=off: encoder and decoder must round the
// reconstruction identically.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dls_device.h"
#include "dls_kernels.h"

namespace dls {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr double kGbTailShare = 0.36;
constexpr double kGbStepShare = 0.4;
constexpr double kGbGrid = 16777216.0;  // 2^24
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

// SplitMix64 output number d (0-based) of the sequence that starts from
// state s0: the state after d + 1 steps is s0 + (d + 1) gamma.
__device__ __forceinline__ uint64_t splitmix(uint64_t s0, uint64_t d) {
  uint64_t z = s0 + (d + 1) * kGamma;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t zz32(int32_t v) { return (uint32_t(v) << 1) ^ uint32_t(v >> 31); }

template <typename T>
__global__ __launch_bounds__(256) void k_gb_sumsq(const T* __restrict__ F, int64_t per_var,
                                                  double* __restrict__ part) {
  __shared__ double red[256];
  const int v = blockIdx.y;
  const T* f = F + int64_t(v) * per_var;
  double s = 0.0;
  // four loads in flight per thread, added in index order
  const int64_t stride = int64_t(gridDim.x) * 256;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < per_var; i += 4 * stride) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = i + u * stride < per_var ? double(f[i + u * stride]) : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (isfinite(x[u])) s += x[u] * x[u];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[int64_t(v) * gridDim.x + blockIdx.x] = red[0];
}

// One workgroup per variable: each thread adds its strided share of the
// partials in order, then a fixed tree (one thread per variable adding the
// 2048 partials in sequence took ~150 us).
__global__ __launch_bounds__(256) void k_gb_budget(const double* __restrict__ part, int nparts,
                                                   const double* __restrict__ target, int64_t per_var, int nvars,
                                                   double* __restrict__ cv) {
  __shared__ double red[256];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < nparts; j += 256) s += part[int64_t(v) * nparts + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) cv[v] = target[v] * target[v] * red[0] / double(per_var);
}

// Q[s][i] (S x M, FP64): kind 0 -- the patch of snapshot 0 at the sample's
// position (three draws per sample: x0, y0, z0, each modulo its range);
// kind 2 -- uniform [-1, 1) entries, draw s M + i.
template <typename T>
__global__ __launch_bounds__(256) void k_gb_samples(const T* __restrict__ F, Dims dims, int var, int px, int py,
                                                    int pz, int kind, uint64_t s0, int64_t S,
                                                    double* __restrict__ Q) {
  const int M = px * py * pz;
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= S * M) return;
  const int64_t s = e / M;
  const int i = int(e - s * M);
  if (kind == 2) {
    Q[e] = double(splitmix(s0, uint64_t(e)) >> 11) * 0x1p-52 - 1.0;
    return;
  }
  const int64_t x0 = int64_t(splitmix(s0, uint64_t(3 * s)) % uint64_t(dims.nx - px + 1));
  const int64_t y0 = int64_t(splitmix(s0, uint64_t(3 * s + 1)) % uint64_t(dims.ny - py + 1));
  const int64_t z0 = int64_t(splitmix(s0, uint64_t(3 * s + 2)) % uint64_t(dims.nz - pz + 1));
  const int ix = i % px, jy = (i / px) % py, kz = i / (px * py);
  Q[e] = double(F[fidx(dims, var, 0, int(z0 + kz), int(y0 + jy), int(x0 + ix))]);
}

// G = Q^T Q (Mp x Mp, zero beyond M): one wave per 16 x 16 tile, four points
// of the sample dimension per v_mfma_f64_16x16x4f64 (A = Q^T rows of the
// tile, B = Q columns); lane l holds element (l % 16, l / 16) of each operand
// and D[l / 16 + 4 v][l % 16] of the result.
__global__ __launch_bounds__(256) void k_gb_gram(const double* __restrict__ Q, int64_t S, int M, int Mp,
                                                 double* __restrict__ G) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tiles = (Mp + 15) / 16;
  const int tile = int(blockIdx.x) * 4 + wave;
  if (tile >= tiles * tiles) return;
  const int ti = tile / tiles, tj = tile % tiles;
  const int li = lane & 15, lk = lane >> 4;
  const int ra = ti * 16 + li, cb = tj * 16 + li;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t s0 = 0; s0 < S; s0 += 4) {
    const int64_t s = s0 + lk;
    const double a = (s < S && ra < M) ? Q[s * M + ra] : 0.0;
    const double b = (s < S && cb < M) ? Q[s * M + cb] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = ti * 16 + (lane >> 4) + 4 * v, c = tj * 16 + (lane & 15);
    if (r < Mp && c < Mp) G[int64_t(r) * Mp + c] = acc[v];
  }
}

__global__ __launch_bounds__(256) void k_gb_eye(double* __restrict__ V, int Mp) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= int64_t(Mp) * Mp) return;
  V[e] = (e / Mp == e % Mp) ? 1.0 : 0.0;
}

__device__ __forceinline__ int gb_player(int pos, int round, int n) {
  return pos == 0 ? 0 : ((pos - 1 + round) % (n - 1)) + 1;
}

// The symmetric Schur rotation of pair (p, q) (Golub and Van Loan): t is
// the smaller root of t^2 + 2 theta t - 1 = 0, theta = (a_qq - a_pp) / (2 a_pq).
__device__ __forceinline__ void gb_rotation(double app, double aqq, double apq, double& c, double& s, double& t) {
  if (apq == 0.0) {
    c = 1.0; s = 0.0; t = 0.0;
    return;
  }
  const double theta = (aqq - app) / (2.0 * apq);
  t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  c = 1.0 / sqrt(t * t + 1.0);
  s = t * c;
}

// One round of the round-robin ordering: thread (a, b) takes the 2 x 2 block
// of rows (p_a, q_a) and columns (p_b, q_b); A_out = J^T A_in J with J the
// product of the round's disjoint rotations [[c, s], [-s, c]]; V = V J in
// place (thread (a, b) owns rows p_a, q_a of columns p_b, q_b).
__global__ __launch_bounds__(256) void k_gb_jacobi_round(const double* __restrict__ Ain, double* __restrict__ Aout,
                                                         double* __restrict__ V, int Mp, int round) {
  const int P = Mp / 2;
  const int a = int(blockIdx.y) * 16 + int(threadIdx.x >> 4), b = int(blockIdx.x) * 16 + int(threadIdx.x & 15);
  if (a >= P || b >= P) return;
  const int pa = gb_player(a, round, Mp), qa = gb_player(Mp - 1 - a, round, Mp);
  const int pb = gb_player(b, round, Mp), qb = gb_player(Mp - 1 - b, round, Mp);
  const int64_t n = Mp;
  double ca, sa, ta, cb, sb, tb;
  gb_rotation(Ain[pa * n + pa], Ain[qa * n + qa], Ain[pa * n + qa], ca, sa, ta);
  gb_rotation(Ain[pb * n + pb], Ain[qb * n + qb], Ain[pb * n + qb], cb, sb, tb);
  if (a == b) {
    const double apq = Ain[pa * n + qa];
    Aout[pa * n + pa] = Ain[pa * n + pa] - ta * apq;
    Aout[qa * n + qa] = Ain[qa * n + qa] + ta * apq;
    Aout[pa * n + qa] = 0.0;
    Aout[qa * n + pa] = 0.0;
  } else {
    const double b00 = Ain[pa * n + pb], b01 = Ain[pa * n + qb], b10 = Ain[qa * n + pb], b11 = Ain[qa * n + qb];
    const double t00 = cb * b00 - sb * b01, t01 = sb * b00 + cb * b01;
    const double t10 = cb * b10 - sb * b11, t11 = sb * b10 + cb * b11;
    Aout[pa * n + pb] = ca * t00 - sa * t10;
    Aout[pa * n + qb] = ca * t01 - sa * t11;
    Aout[qa * n + pb] = sa * t00 + ca * t10;
    Aout[qa * n + qb] = sa * t01 + ca * t11;
  }
  const double v00 = V[pa * n + pb], v01 = V[pa * n + qb], v10 = V[qa * n + pb], v11 = V[qa * n + qb];
  V[pa * n + pb] = cb * v00 - sb * v01;
  V[pa * n + qb] = sb * v00 + cb * v01;
  V[qa * n + pb] = cb * v10 - sb * v11;
  V[qa * n + qb] = sb * v10 + cb * v11;
}

// The whole eigensolve of a basis of order Mp <= 64 in one workgroup of
// 1024 threads with A (two buffers) and V in LDS: the same rounds and
// rotations as k_gb_jacobi_round, a barrier between rounds, and after each
// sweep the off-diagonal and total sums of squares (fixed tree order) for
// the same stopping rule as the host loop (off <= floor2 * total, or a
// sweep that leaves off above 0.9 of the previous one), at most max_sweeps.
// A (the diagonal carries the eigenvalues) and V go back to global memory;
// info[0] = sweeps, info[1] = 1 when the rule was not met.
__global__ __launch_bounds__(1024) void k_gb_jacobi_lds(const double* __restrict__ G, int Mp, double floor2,
                                                        int max_sweeps, double* __restrict__ Aout,
                                                        double* __restrict__ Vout, int* __restrict__ info) {
  __shared__ double A[2][64 * 64], V[64 * 64];
  __shared__ double r0[1024], r1[1024];
  const int tid = threadIdx.x;
  const int n2 = Mp * Mp;
  for (int e = tid; e < n2; e += 1024) {
    A[0][e] = G[e];
    V[e] = (e / Mp == e % Mp) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int P = Mp / 2;
  const int a = tid >> 5, b = tid & 31;
  const bool act = a < P && b < P;
  int cur = 0, sweep = 0;
  bool conv = false;
  double prev = HUGE_VAL;
  while (!conv && sweep < max_sweeps) {
    for (int round = 0; round < Mp - 1; ++round) {
      const double* Ai = A[cur];
      double* Ao = A[cur ^ 1];
      if (act) {
        const int pa = gb_player(a, round, Mp), qa = gb_player(Mp - 1 - a, round, Mp);
        const int pb = gb_player(b, round, Mp), qb = gb_player(Mp - 1 - b, round, Mp);
        double ca, sa, ta, cb, sb, tb;
        gb_rotation(Ai[pa * Mp + pa], Ai[qa * Mp + qa], Ai[pa * Mp + qa], ca, sa, ta);
        gb_rotation(Ai[pb * Mp + pb], Ai[qb * Mp + qb], Ai[pb * Mp + qb], cb, sb, tb);
        if (a == b) {
          const double apq = Ai[pa * Mp + qa];
          Ao[pa * Mp + pa] = Ai[pa * Mp + pa] - ta * apq;
          Ao[qa * Mp + qa] = Ai[qa * Mp + qa] + ta * apq;
          Ao[pa * Mp + qa] = 0.0;
          Ao[qa * Mp + pa] = 0.0;
        } else {
          const double b00 = Ai[pa * Mp + pb], b01 = Ai[pa * Mp + qb], b10 = Ai[qa * Mp + pb], b11 = Ai[qa * Mp + qb];
          const double t00 = cb * b00 - sb * b01, t01 = sb * b00 + cb * b01;
          const double t10 = cb * b10 - sb * b11, t11 = sb * b10 + cb * b11;
          Ao[pa * Mp + pb] = ca * t00 - sa * t10;
          Ao[pa * Mp + qb] = ca * t01 - sa * t11;
          Ao[qa * Mp + pb] = sa * t00 + ca * t10;
          Ao[qa * Mp + qb] = sa * t01 + ca * t11;
        }
        const double v00 = V[pa * Mp + pb], v01 = V[pa * Mp + qb], v10 = V[qa * Mp + pb], v11 = V[qa * Mp + qb];
        V[pa * Mp + pb] = cb * v00 - sb * v01;
        V[pa * Mp + qb] = sb * v00 + cb * v01;
        V[qa * Mp + pb] = cb * v10 - sb * v11;
        V[qa * Mp + qb] = sb * v10 + cb * v11;
      }
      cur ^= 1;
      __syncthreads();
    }
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n2; e += 1024) {
      const double x = A[cur][e];
      tot += x * x;
      if (e / Mp != e % Mp) off += x * x;
    }
    r0[tid] = off;
    r1[tid] = tot;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
      if (tid < o) {
        r0[tid] += r0[tid + o];
        r1[tid] += r1[tid + o];
      }
      __syncthreads();
    }
    off = r0[0];
    tot = r1[0];
    ++sweep;
    conv = off <= floor2 * tot || off >= 0.9 * prev;
    prev = off;
    __syncthreads();
  }
  for (int e = tid; e < n2; e += 1024) {
    Aout[e] = A[cur][e];
    Vout[e] = V[e];
  }
  if (tid == 0) {
    info[0] = sweep;
    info[1] = conv ? 0 : 1;
  }
}

// Per block of a fixed grid: the sums of squares of the off-diagonal and of
// all entries of A (and A copied to Acopy, so every sweep starts from the
// same buffer).
__global__ __launch_bounds__(256) void k_gb_offnorm(const double* __restrict__ A, double* __restrict__ Acopy,
                                                    int Mp, double* __restrict__ part) {
  __shared__ double r0[256], r1[256];
  const int64_t n2 = int64_t(Mp) * Mp;
  double off = 0.0, tot = 0.0;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < n2; e += int64_t(gridDim.x) * 256) {
    const double x = A[e];
    Acopy[e] = x;
    tot += x * x;
    if (e / Mp != e % Mp) off += x * x;
  }
  r0[threadIdx.x] = off;
  r1[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r0[0];
    part[2 * blockIdx.x + 1] = r1[0];
  }
}

__global__ void k_gb_sum(const double* __restrict__ part, int nparts, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int j = 0; j < nparts; ++j) {
    a += part[2 * j];
    b += part[2 * j + 1];
  }
  out[0] = a;
  out[1] = b;
}

// Column k of V (k < M; the padding column M of an odd M is e_M and takes
// no part) goes to position rank_k of the descending eigenvalue order (ties:
// the lower index first), its largest-|v_i| entry made positive (first index
// on ties), then onto the 2^-24 grid.  Phi[i][s] row-major.
__global__ __launch_bounds__(256) void k_gb_finish(const double* __restrict__ A, const double* __restrict__ V,
                                                   int M, int Mp, double* __restrict__ Phi) {
  const int k = int(blockIdx.x) * 256 + threadIdx.x;
  if (k >= M) return;
  const double lk = A[int64_t(k) * Mp + k];
  int rank = 0;
  for (int j = 0; j < M; ++j) {
    const double lj = A[int64_t(j) * Mp + j];
    rank += (lj > lk || (lj == lk && j < k)) ? 1 : 0;
  }
  int imax = 0;
  double vmax = -1.0;
  for (int i = 0; i < M; ++i) {
    const double a = fabs(V[int64_t(i) * Mp + k]);
    if (a > vmax) {
      vmax = a;
      imax = i;
    }
  }
  const double sg = V[int64_t(imax) * Mp + k] < 0.0 ? -1.0 : 1.0;
  for (int i = 0; i < M; ++i) Phi[int64_t(i) * M + rank] = rint(sg * V[int64_t(i) * Mp + k] * kGbGrid) / kGbGrid;
}

// Orthonormal DCT-II tensor basis on the 2^-24 grid: column (c Py + b) Px + a
// at row (k Py + j) Px + i is C_a(i) C_b(j) C_c(k).
__device__ __forceinline__ double dct2(int a, int i, int n) {
  return sqrt((a == 0 ? 1.0 : 2.0) / double(n)) * cos(M_PI * double(2 * i + 1) * double(a) / double(2 * n));
}

__global__ __launch_bounds__(256) void k_gb_cosine(int px, int py, int pz, double* __restrict__ Phi) {
  const int M = px * py * pz;
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= int64_t(M) * M) return;
  const int row = int(e / M), col = int(e % M);
  const int i = row % px, j = (row / px) % py, k = row / (px * py);
  const int a = col % px, b = (col / px) % py, c = col / (px * py);
  const double v = dct2(a, i, px) * dct2(b, j, py) * dct2(c, k, pz);
  Phi[e] = rint(v * kGbGrid) / kGbGrid;
}

// Value of full-patch point k of block d (0 outside the domain); `in` is set
// when the point lies inside.
template <typename T>
__device__ __forceinline__ double gb_point(const T* __restrict__ F, const Dims& dims, const BlockDesc& d, int px,
                                           int py, int k, bool& in) {
  const int ix = k % px, jy = (k / px) % py, kz = k / (px * py);
  in = ix < d.px() && jy < d.py() && kz < d.pz();
  if (!in) return 0.0;
  return double(F[fidx(dims, d.var, d.t0, d.z0 + kz, d.y0 + jy, d.x0 + ix)]);
}

// alpha[n][s] = sum_i Phi_v[i][s] u_n[i] for 16 patches x 64 columns per
// workgroup: wave w takes columns 16 (4 blockIdx.y + w) .. + 15, four
// points per v_mfma_f64_16x16x4f64.  One launch per variable: the patches
// [nb0, nb1) share its basis phi (lane l supplies B column l % 16, so every
// row of a tile must use the same basis).
template <typename T>
__global__ __launch_bounds__(256) void k_gb_project(const T* __restrict__ F, Dims dims,
                                                    const BlockDesc* __restrict__ desc, int64_t nb0, int64_t nb1,
                                                    const double* __restrict__ phi, int px, int py, int M,
                                                    double* __restrict__ alpha) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t n0 = nb0 + int64_t(blockIdx.x) * 16;
  const int s0 = (int(blockIdx.y) * 4 + wave) * 16;
  if (s0 >= M) return;
  const int64_t n = n0 + li;
  const bool live = n < nb1;
  const BlockDesc d = desc[live ? n : nb0];
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < M; k0 += 4) {
    const int k = k0 + lk;
    bool in = false;
    const double a = (live && k < M) ? gb_point(F, dims, d, px, py, k, in) : 0.0;
    const double b = (k < M && s0 + li < M) ? phi[int64_t(k) * M + s0 + li] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t r = n0 + (lane >> 4) + 4 * v;
    const int c = s0 + (lane & 15);
    if (r < nb1 && c < M) alpha[r * M + c] = acc[v];
  }
}

// One workgroup per patch-snapshot.  Slot layout (8 M bytes): kept indices
// (u16) at 0, their coefficients (int32) at 4 M; or the raw values.
template <typename T>
__global__ __launch_bounds__(256) void k_gb_select(const T* __restrict__ F, Dims dims,
                                                   const BlockDesc* __restrict__ desc, int64_t nblocks,
                                                   const double* __restrict__ phi_all, const double* __restrict__ cv,
                                                   const double* __restrict__ alpha, int px, int py, int M, int Mpow,
                                                   int32_t* __restrict__ count, int32_t* __restrict__ kexp,
                                                   uint8_t* __restrict__ slot, int32_t* __restrict__ n0_out,
                                                   int64_t off) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* key = reinterpret_cast<double*>(smem);          // Mpow: |alpha| (-1 padding)
  int* idx = reinterpret_cast<int*>(key + Mpow);           // Mpow: basis index
  double* xs = reinterpret_cast<double*>(idx + Mpow);      // M: the patch's values (0 outside)
  double* al = xs + M;                                     // M: alpha
  int* flag = reinterpret_cast<int*>(al + M);              // M: kept flag by basis index, then its list position
  int* list = flag + M;                                    // M: kept indices ascending
  double* red = reinterpret_cast<double*>(list + M);       // 256
  __shared__ int sh_n, sh_fin, sh_bad;
  const int64_t b = off + int64_t(blockIdx.x);
  if (b >= nblocks) return;
  const BlockDesc d = desc[b];
  const double* phi = phi_all + int64_t(d.var) * M * M;
  const double e2 = cv[d.var] * double(d.m);
  bool finite = true;
  for (int k = threadIdx.x; k < M; k += 256) {
    bool in;
    const double x = gb_point(F, dims, d, px, py, k, in);
    xs[k] = x;
    if (in && !isfinite(x)) finite = false;
    al[k] = alpha[b * M + k];
  }
  for (int k = threadIdx.x; k < Mpow; k += 256) {
    key[k] = k < M ? fabs(alpha[b * M + k]) : -1.0;
    idx[k] = k;
  }
  if (threadIdx.x == 0) sh_bad = 0;
  __syncthreads();
  if (!finite) sh_bad = 1;
  __syncthreads();
  uint8_t* out = slot + b * int64_t(8) * M;
  if (sh_bad) {
    for (int k = threadIdx.x; k < d.m; k += 256) {
      const int ix = k % d.px(), jy = (k / d.px()) % d.py(), kz = k / (d.px() * d.py());
      reinterpret_cast<T*>(out)[k] = F[fidx(dims, d.var, d.t0, d.z0 + kz, d.y0 + jy, d.x0 + ix)];
    }
    if (threadIdx.x == 0) {
      count[b] = 0xFFFF;
      kexp[b] = 0;
      n0_out[b] = 0;
    }
    return;
  }
  // bitonic sort: |alpha| descending, the lower index first on ties
  for (int size = 2; size <= Mpow; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < Mpow; i += 256) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc_dir = (i & size) == 0;
          const double ki = key[i], kj = key[j];
          const int ii = idx[i], ij = idx[j];
          // "i before j" in the final order: larger key, or equal key and lower index
          const bool i_first = ki > kj || (ki == kj && ii < ij);
          if (desc_dir != i_first) {
            key[i] = kj; key[j] = ki;
            idx[i] = ij; idx[j] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  // the energy rule: the tail summed from the end, as a recurrence
  if (threadIdx.x == 0) {
    const double tau = kGbTailShare * e2;
    double t = 0.0;
    int n = 0;
    for (int j = M - 1; j >= 0; --j) {
      const double a = al[idx[j]];
      const double tn = t + a * a;
      if (tn > tau) {
        n = j + 1;
        break;
      }
      t = tn;
    }
    sh_n = n;
    n0_out[b] = n;
  }
  __syncthreads();
  int n = sh_n;
  for (;;) {
    if (n > M || !(e2 > 0.0) && n > 0) {
      n = -1;  // raw
      break;
    }
    // kept flags by basis index, then the ascending list by a prefix count
    for (int k = threadIdx.x; k < M; k += 256) flag[k] = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += 256) flag[idx[j]] = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
      int c = 0;
      for (int k = 0; k < M; ++k)
        if (flag[k]) list[c++] = k;
      sh_bad = 0;
    }
    __syncthreads();
    double d2 = 1.0;
    int kx = 0;
    if (n > 0) {
      int ex;
      frexp(kGbStepShare * sqrt(e2 / double(n)), &ex);
      kx = ex - 1;
      d2 = ldexp(1.0, kx);
    }
    // quantized coefficients in list order (stored in flag[] as int32)
    for (int j = threadIdx.x; j < n; j += 256) {
      const double qa = rint(al[list[j]] / d2);
      const bool ok = fabs(qa) < 2147483648.0;
      if (!ok) sh_bad = 1;
      flag[j] = ok ? int32_t(qa) : 0;
    }
    __syncthreads();
    if (sh_bad) {
      n = -1;
      break;
    }
    // the decoder's values and the exact squared error of the in-domain points
    double err = 0.0;
    for (int k = threadIdx.x; k < M; k += 256) {
      const int ix = k % px, jy = (k / px) % py, kz = k / (px * py);
      if (ix >= d.px() || jy >= d.py() || kz >= d.pz()) continue;
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc = acc + phi[int64_t(k) * M + list[j]] * (double(flag[j]) * d2);
      const double e = xs[k] - double(T(acc));
      err += e * e;
    }
    red[threadIdx.x] = err;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    const double tot = red[0];
    __syncthreads();
    if (tot <= e2) {
      // the kept indices and coefficients into the slot
      for (int j = threadIdx.x; j < n; j += 256) {
        reinterpret_cast<uint16_t*>(out)[j] = uint16_t(list[j]);
        reinterpret_cast<int32_t*>(out + 4 * int64_t(M))[j] = flag[j];
      }
      if (threadIdx.x == 0) {
        count[b] = n;
        kexp[b] = n > 0 ? kx : 0;
      }
      return;
    }
    ++n;
  }
  for (int k = threadIdx.x; k < d.m; k += 256) {
    const int ix = k % d.px(), jy = (k / d.px()) % d.py(), kz = k / (d.px() * d.py());
    reinterpret_cast<T*>(out)[k] = F[fidx(dims, d.var, d.t0, d.z0 + kz, d.y0 + jy, d.x0 + ix)];
  }
  if (threadIdx.x == 0) {
    count[b] = 0xFFFF;
    kexp[b] = 0;
  }
}

// Patches of at most S points (S = 64, 32 or 16): one team of S lanes per
// patch-snapshot, 64 / S teams per wave, no barriers after the basis is
// staged.  One launch per variable: the workgroup copies the variable's Phi
// into LDS once (rows padded to M + 1, so both the row reads of the
// coefficients and the column reads of the decoder are conflict-free) and
// its teams walk the patches [nb0, nb1) with a grid stride.  Team lane i
// holds point i (zero-padded), then coefficient alpha_i = sum_k Phi[k][i]
// u_k (points broadcast from LDS in order, FP64 FMA), then its position in
// the magnitude order (|alpha| descending, index ascending: the number of
// keys before its own), where it writes its coefficient; the energy rule
// comes from a suffix scan of the sorted values' squares over the team,
// checked against the sequential recurrence's rounding (which runs when the
// check fails); the kept set is a ballot over basis indices, its ascending list
// positions come from the lanes below; the decoder's values are summed over
// the kept indices in ascending order.  Every cross-lane step is confined
// to the team (ballots masked to its lanes, sums over its lanes), and every
// branch that leaves a loop is taken by a whole team.  Same slot layout as
// k_gb_select.  Registers are capped for six waves per SIMD (LDS holds
// seven workgroups per compute unit).
template <typename T, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_gb_patch64(const T* __restrict__ F, Dims dims,
                                                    const BlockDesc* __restrict__ desc, int64_t nb0, int64_t nb1,
                                                    const double* __restrict__ phi_g, const double* __restrict__ cv,
                                                    int px, int py, int M, int32_t* __restrict__ count,
                                                    int32_t* __restrict__ kexp, uint8_t* __restrict__ slot,
                                                    int32_t* __restrict__ n0_out) {
  constexpr int NTM = 64 / S;  // teams per wave
  // the basis values are k 2^-24 with |k| <= 2^24, exact in FP32
  __shared__ float phi[S * (S + 1)];
  __shared__ double xs[4][64], sa[4][64], tq[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tb = S == 64 ? 0 : lane & ~(S - 1), tl = lane - tb;  // team's first lane, lane in the team
  const unsigned long long tmask = (S == 64 ? ~0ull : ((1ull << S) - 1ull)) << tb;
  const int ld = M + 1;
  for (int e = threadIdx.x; e < M * M; e += 256) phi[(e / M) * ld + e % M] = float(phi_g[e]);
  __syncthreads();
  for (int64_t b0 = nb0 + (int64_t(blockIdx.x) * 4 + wave) * NTM; b0 < nb1; b0 += int64_t(gridDim.x) * 4 * NTM) {
    const int64_t b = b0 + tb / S;
    if (b >= nb1) continue;  // a whole team (the wave's last teams)
    const BlockDesc d = desc[b];
    const double e2 = cv[d.var] * double(d.m);
    bool in = false;
    const double x = tl < M ? gb_point(F, dims, d, px, py, tl, in) : 0.0;
    uint8_t* out = slot + b * int64_t(8) * M;
    if ((__ballot(in && !isfinite(x)) & tmask) != 0) {
      if (tl < d.m) {
        const int ix = tl % d.px(), jy = (tl / d.px()) % d.py(), kz = tl / (d.px() * d.py());
        reinterpret_cast<T*>(out)[tl] = F[fidx(dims, d.var, d.t0, d.z0 + kz, d.y0 + jy, d.x0 + ix)];
      }
      if (tl == 0) {
        count[b] = kGbRaw;
        kexp[b] = 0;
        n0_out[b] = 0;
      }
      continue;
    }
    xs[wave][lane] = x;
    wave_sync();
    // coefficients
    double a = 0.0;
    if (tl < M)
      for (int k = 0; k < M; ++k) a = fma(double(phi[k * ld + tl]), xs[wave][tb + k], a);
    // magnitude order (|alpha| desc, index asc; lanes >= M last): every
    // lane counts the keys that precede its own, which is its position in
    // that total order, and places its coefficient there
    const double key = tl < M ? fabs(a) : -1.0;
    // The high word of a key's bit pattern, read as a signed integer, never
    // orders two keys against their order (all are >= 0 but the padding's
    // -1).  While the points' high words are distinct, the count of larger
    // ones is the position: each point claims its slot, and a slot claimed
    // twice (equal high words) or a NaN key sends the team to the count on
    // the full keys with the index rule.  Words and claims live in xs, free
    // once the coefficients are formed.
    int* xw = reinterpret_cast<int*>(&xs[wave][0]);
    const int hk = __double2hiint(key);
    xw[64 + lane] = hk;
    wave_sync();
    int mypos = 0;
#pragma unroll 16
    for (int j = 0; j < S; ++j) mypos += xw[64 + tb + j] > hk ? 1 : 0;
    if (tl < M) xw[tb + mypos] = tl;
    wave_sync();
    if ((__ballot(tl < M && (xw[tb + mypos] != tl || isnan(key))) & tmask) != 0) {
      tq[wave][lane] = key;
      wave_sync();
      mypos = 0;
#pragma unroll 8
      for (int j = 0; j < S; ++j) {
        const double kj = tq[wave][tb + j];
        mypos += (kj > key || (kj == key && j < tl)) ? 1 : 0;
      }
    }
    sa[wave][tb + mypos] = a;
    wave_sync();
    // the energy rule: n is one more than the last sorted position whose tail
    // (the squares from it to the end, added from the end one by one)
    // exceeds tau.  A suffix scan over the team gives every tail at once in
    // another summation order.  Over the same rounded squares (at most 64)
    // the two orders differ by at most (63 + 6) u of the total (u = 2^-53),
    // so a margin of 2^-44 (total + tau) also covers the rounding of
    // tau +- margin: when no scanned tail lies within it of tau, both orders
    // put the same positions above tau, and the sequential tails, never
    // decreasing towards the front, make that set the first n positions.
    // Otherwise (and for a non-finite total) the recurrence runs as written.
    const double tau = kGbTailShare * e2;
    const double sv = tl < M ? sa[wave][lane] : 0.0;
    double tail = sv * sv;
#pragma unroll
    for (int o = 1; o < S; o <<= 1) {
      const double y = __shfl_down(tail, o, S);
      if (tl + o < S) tail += y;
    }
    const double total = __shfl(tail, tb, 64);
    const double margin = 0x1p-44 * (total + tau);
    const unsigned long long above = __ballot(tail > tau + margin) & tmask;
    const bool fast = isfinite(total) && above == (__ballot(tail > tau - margin) & tmask);
    int n = fast ? __popcll(above) : 0;
    double t = 0.0;
    bool found = fast;
    for (int j0 = M - 1; j0 >= 0 && !found; j0 -= 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = j0 - u >= 0 ? sa[wave][tb + j0 - u] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (found || j0 - u < 0) continue;
        const double tn = t + v[u] * v[u];
        if (tn > tau) {
          n = j0 - u + 1;
          found = true;
        } else {
          t = tn;
        }
      }
    }
    if (tl == 0) n0_out[b] = n;
    if (tl >= M) mypos = 64;
    bool done = false;
    for (;;) {
      if (n > M || (!(e2 > 0.0) && n > 0)) break;
      const bool kept = tl < M && mypos < n;
      const unsigned long long mask = __ballot(kept) & tmask;
      double dd = 1.0;
      int kx = 0;
      if (n > 0) {
        int ex;
        frexp(kGbStepShare * sqrt(e2 / double(n)), &ex);
        kx = ex - 1;
        dd = ldexp(1.0, kx);
      }
      const double qa = rint(a / dd);
      if ((__ballot(kept && !(fabs(qa) < 2147483648.0)) & tmask) != 0) break;
      const int32_t qi = kept ? int32_t(qa) : 0;
      tq[wave][lane] = double(qi) * dd;
      wave_sync();
      // the decoder's values at this lane's point
      double acc = 0.0;
      unsigned long long m = mask;
      const int row = tl < M ? tl : 0;
      while (m) {
        const int sl = __ffsll((long long)m) - 1;
        m &= m - 1;
        acc = acc + double(phi[row * ld + (sl - tb)]) * tq[wave][sl];
      }
      double e = in ? x - double(T(acc)) : 0.0;
      double err = e * e;
#pragma unroll
      for (int o = S / 2; o >= 1; o >>= 1) err += __shfl_xor(err, o, 64);
      wave_sync();
      if (err <= e2) {
        if (kept) {
          const int j = __popcll(mask & ((1ull << lane) - 1ull));
          reinterpret_cast<uint16_t*>(out)[j] = uint16_t(tl);
          reinterpret_cast<int32_t*>(out + 4 * int64_t(M))[j] = qi;
        }
        if (tl == 0) {
          count[b] = n;
          kexp[b] = n > 0 ? kx : 0;
        }
        done = true;
        break;
      }
      ++n;
    }
    if (!done) {
      if (tl < d.m) {
        const int ix = tl % d.px(), jy = (tl / d.px()) % d.py(), kz = tl / (d.px() * d.py());
        reinterpret_cast<T*>(out)[tl] = F[fidx(dims, d.var, d.t0, d.z0 + kz, d.y0 + jy, d.x0 + ix)];
      }
      if (tl == 0) {
        count[b] = kGbRaw;
        kexp[b] = 0;
      }
    }
  }
}

// sizes per patch: kept indices (2 n B), coefficients (4 n B), raw values
__global__ __launch_bounds__(256) void k_gb_sizes(const BlockDesc* __restrict__ desc, int64_t nblocks,
                                                  const int32_t* __restrict__ count, int esize,
                                                  int64_t* __restrict__ nidx, int64_t* __restrict__ nraw,
                                                  unsigned long long* __restrict__ raw_patches) {
  const int64_t b = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const bool raw = b < nblocks && count[b] == kGbRaw;
  const unsigned long long m = __ballot(raw);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(raw_patches, (unsigned long long)__popcll(m));
  if (b >= nblocks) return;
  const int c = count[b];
  nidx[b] = raw ? 0 : c;
  nraw[b] = raw ? int64_t(desc[b].m) * esize : 0;
}

// One team of S lanes per patch-snapshot (launched with S = 8), 256 / S
// per workgroup; the kept entries and raw bytes in strides of S.
template <int S>
__global__ __launch_bounds__(256) void k_gb_compact(const BlockDesc* __restrict__ desc, int64_t nblocks, int M,
                                                    const int32_t* __restrict__ count,
                                                    const uint8_t* __restrict__ slot,
                                                    const int64_t* __restrict__ idx_off,
                                                    const int64_t* __restrict__ raw_off, int esize,
                                                    uint16_t* __restrict__ idx_out, int32_t* __restrict__ q_out,
                                                    uint8_t* __restrict__ raw_out, int64_t off) {
  const int lane = int(threadIdx.x) % S;
  const int64_t b = off + int64_t(blockIdx.x) * (256 / S) + int(threadIdx.x) / S;
  if (b >= nblocks) return;
  const int c = count[b];
  const uint8_t* s = slot + b * int64_t(8) * M;
  if (c == kGbRaw) {
    const int64_t nb = int64_t(desc[b].m) * esize;
    for (int64_t j = lane; j < nb; j += S) raw_out[raw_off[b] + j] = s[j];
    return;
  }
  for (int j = lane; j < c; j += S) {
    idx_out[idx_off[b] + j] = reinterpret_cast<const uint16_t*>(s)[j];
    q_out[idx_off[b] + j] = reinterpret_cast<const int32_t*>(s + 4 * int64_t(M))[j];
  }
}

// Workgroups per launch of the one-patch-per-team kernels: a dispatch's
// work-item count (workgroups x 256) must stay below 2^32.
constexpr int64_t kGbLaunchGroups = int64_t(1) << 23;

// The decoder: one team of S lanes per patch-snapshot, 256 / S per
// workgroup (launched with S = 256 for patches above 64 points).
template <typename T, int S>
__global__ __launch_bounds__(256) void k_gb_decode(T* __restrict__ F, Dims dims, const BlockDesc* __restrict__ desc,
                                                   int64_t nblocks, const double* __restrict__ phi_all, int px, int py,
                                                   int M, const int32_t* __restrict__ count,
                                                   const int32_t* __restrict__ kexp,
                                                   const int64_t* __restrict__ idx_off,
                                                   const int64_t* __restrict__ raw_off,
                                                   const uint16_t* __restrict__ idx,
                                                   const int32_t* __restrict__ q, const uint8_t* __restrict__ raw,
                                                   int64_t off) {
  const int tl = int(threadIdx.x) % S;
  const int64_t b = off + int64_t(blockIdx.x) * (256 / S) + int(threadIdx.x) / S;
  if (b >= nblocks) return;
  const BlockDesc d = desc[b];
  const int c = count[b];
  if (c == 0xFFFF) {
    const T* src = reinterpret_cast<const T*>(raw + raw_off[b]);
    for (int k = tl; k < d.m; k += S) {
      const int ix = k % d.px(), jy = (k / d.px()) % d.py(), kz = k / (d.px() * d.py());
      F[fidx(dims, d.var, d.t0, d.z0 + kz, d.y0 + jy, d.x0 + ix)] = src[k];
    }
    return;
  }
  const double* phi = phi_all + int64_t(d.var) * M * M;
  const double dd = ldexp(1.0, kexp[b]);
  const uint16_t* li = idx + idx_off[b];
  const int32_t* lq = q + idx_off[b];
  for (int k = tl; k < M; k += S) {
    const int ix = k % px, jy = (k / px) % py, kz = k / (px * py);
    if (ix >= d.px() || jy >= d.py() || kz >= d.pz()) continue;
    double acc = 0.0;
    for (int j = 0; j < c; ++j) acc = acc + phi[int64_t(k) * M + li[j]] * (double(lq[j]) * dd);
    F[fidx(dims, d.var, d.t0, d.z0 + kz, d.y0 + jy, d.x0 + ix)] = T(acc);
  }
}

// The decoder for patches of at most 64 points: persistent like
// k_gb_patch64, one launch per variable with its Phi staged once per
// workgroup of 16 wavefronts in LDS (FP64, rows padded to M + 1: two
// workgroups fill a compute unit's 32 wavefront slots), one team of S lanes
// per patch-snapshot.  The team's lanes load the kept list (indices, and the
// quantised coefficients times the grid step) into LDS, then team lane k
// sums its point's terms over the list in order, the arithmetic of
// k_gb_decode.
template <typename T, int S>
__global__ __launch_bounds__(1024) void k_gb_decode64(T* __restrict__ F, Dims dims, const BlockDesc* __restrict__ desc,
                                                     int64_t nb0, int64_t nb1, const double* __restrict__ phi_g,
                                                     int px, int py, int M, const int32_t* __restrict__ count,
                                                     const int32_t* __restrict__ kexp,
                                                     const int64_t* __restrict__ idx_off,
                                                     const int64_t* __restrict__ raw_off,
                                                     const uint16_t* __restrict__ idx, const int32_t* __restrict__ q,
                                                     const uint8_t* __restrict__ raw) {
  constexpr int NTM = 64 / S;  // teams per wave
  __shared__ double phi[S * (S + 1)];
  __shared__ double kv[16][64];
  __shared__ int kc[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tb = S == 64 ? 0 : lane & ~(S - 1), tl = lane - tb;
  const int ld = M + 1;
  for (int e = threadIdx.x; e < M * M; e += 1024) phi[(e / M) * ld + e % M] = phi_g[e];
  __syncthreads();
  const int ix = tl % px, jy = (tl / px) % py, kz = tl / (px * py);
  for (int64_t b0 = nb0 + (int64_t(blockIdx.x) * 16 + wave) * NTM; b0 < nb1; b0 += int64_t(gridDim.x) * 16 * NTM) {
    const int64_t b = b0 + tb / S;
    if (b >= nb1) continue;  // a whole team (the wave's last teams)
    const BlockDesc d = desc[b];
    const int c = count[b];
    if (c == kGbRaw) {
      if (tl < d.m) {
        const int rx = tl % d.px(), ry = (tl / d.px()) % d.py(), rz = tl / (d.px() * d.py());
        F[fidx(dims, d.var, d.t0, d.z0 + rz, d.y0 + ry, d.x0 + rx)] =
            reinterpret_cast<const T*>(raw + raw_off[b])[tl];
      }
      continue;
    }
    const double dd = ldexp(1.0, kexp[b]);
    if (tl < c) {
      const int64_t o = idx_off[b];
      kc[wave][lane] = idx[o + tl];
      kv[wave][lane] = double(q[o + tl]) * dd;
    }
    wave_sync();
    if (tl < M && ix < d.px() && jy < d.py() && kz < d.pz()) {
      double acc = 0.0;
      for (int j = 0; j < c; ++j) acc = acc + phi[tl * ld + kc[wave][tb + j]] * kv[wave][tb + j];
      F[fidx(dims, d.var, d.t0, d.z0 + kz, d.y0 + jy, d.x0 + ix)] = T(acc);
    }
    wave_sync();  // the list is read before the team's next patch writes it
  }
}

}  // namespace

hipError_t launch_gb_budget(int dtype, const void* F, int64_t per_var, int nvars, const double* target,
                            double* part, double* cv, hipStream_t s) {
  const dim3 g{unsigned(kGbSumParts), unsigned(nvars)};
  if (dtype == 0)
    hipLaunchKernelGGL(k_gb_sumsq<float>, g, dim3{256}, 0, s, static_cast<const float*>(F), per_var, part);
  else
    hipLaunchKernelGGL(k_gb_sumsq<double>, g, dim3{256}, 0, s, static_cast<const double*>(F), per_var, part);
  hipLaunchKernelGGL(k_gb_budget, dim3{unsigned(nvars)}, dim3{256}, 0, s, part, int(kGbSumParts), target, per_var,
                     nvars, cv);
  return hipGetLastError();
}

hipError_t launch_gb_samples(int dtype, const void* F, const Dims& dims, int var, int px, int py, int pz, int kind,
                             uint64_t s0, int64_t S, double* Q, hipStream_t s) {
  const int64_t n = S * px * py * pz;
  if (n == 0) return hipSuccess;
  const dim3 g{unsigned((n + 255) / 256)};
  if (dtype == 0)
    hipLaunchKernelGGL(k_gb_samples<float>, g, dim3{256}, 0, s, static_cast<const float*>(F), dims, var, px, py, pz,
                       kind, s0, S, Q);
  else
    hipLaunchKernelGGL(k_gb_samples<double>, g, dim3{256}, 0, s, static_cast<const double*>(F), dims, var, px, py,
                       pz, kind, s0, S, Q);
  return hipGetLastError();
}

hipError_t launch_gb_gram(const double* Q, int64_t S, int M, int Mp, double* G, hipStream_t s) {
  const int tiles = (Mp + 15) / 16;
  hipLaunchKernelGGL(k_gb_gram, dim3{unsigned((tiles * tiles + 3) / 4)}, dim3{256}, 0, s, Q, S, M, Mp, G);
  return hipGetLastError();
}

hipError_t launch_gb_eye(double* V, int Mp, hipStream_t s) {
  const int64_t n = int64_t(Mp) * Mp;
  hipLaunchKernelGGL(k_gb_eye, dim3{unsigned((n + 255) / 256)}, dim3{256}, 0, s, V, Mp);
  return hipGetLastError();
}

hipError_t launch_gb_jacobi_round(const double* Ain, double* Aout, double* V, int Mp, int round, hipStream_t s) {
  const int P = Mp / 2, g = (P + 15) / 16;
  const dim3 grid = dim3(unsigned(g), unsigned(g));
  hipLaunchKernelGGL(k_gb_jacobi_round, grid, dim3{256}, 0, s, Ain, Aout, V, Mp, round);
  return hipGetLastError();
}

hipError_t launch_gb_jacobi_lds(const double* G, int Mp, double floor2, int max_sweeps, double* A, double* V,
                                int* info, hipStream_t s) {
  if (Mp > 64 || (Mp & 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gb_jacobi_lds, dim3{1}, dim3{1024}, 0, s, G, Mp, floor2, max_sweeps, A, V, info);
  return hipGetLastError();
}

hipError_t launch_gb_offnorm(const double* A, double* Acopy, int Mp, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gb_offnorm, dim3{unsigned(kGbParts)}, dim3{256}, 0, s, A, Acopy, Mp, part);
  hipLaunchKernelGGL(k_gb_sum, dim3{1}, dim3{64}, 0, s, part, int(kGbParts), out);
  return hipGetLastError();
}

hipError_t launch_gb_finish(const double* A, const double* V, int M, int Mp, double* Phi, hipStream_t s) {
  hipLaunchKernelGGL(k_gb_finish, dim3{unsigned((M + 255) / 256)}, dim3{256}, 0, s, A, V, M, Mp, Phi);
  return hipGetLastError();
}

hipError_t launch_gb_cosine(int px, int py, int pz, double* Phi, hipStream_t s) {
  const int64_t n = int64_t(px) * py * pz * px * py * pz;
  hipLaunchKernelGGL(k_gb_cosine, dim3{unsigned((n + 255) / 256)}, dim3{256}, 0, s, px, py, pz, Phi);
  return hipGetLastError();
}

hipError_t launch_gb_project(int dtype, const void* F, const Dims& dims, const BlockDesc* desc, int64_t nb0,
                             int64_t nb1, const double* phi, int px, int py, int M, double* alpha, hipStream_t s) {
  if (nb1 <= nb0) return hipSuccess;
  if ((nb1 - nb0 + 15) / 16 > int64_t(INT32_MAX)) return hipErrorInvalidValue;
  const dim3 g{unsigned((nb1 - nb0 + 15) / 16), unsigned((M + 63) / 64)};
  if (dtype == 0)
    hipLaunchKernelGGL(k_gb_project<float>, g, dim3{256}, 0, s, static_cast<const float*>(F), dims, desc, nb0, nb1,
                       phi, px, py, M, alpha);
  else
    hipLaunchKernelGGL(k_gb_project<double>, g, dim3{256}, 0, s, static_cast<const double*>(F), dims, desc, nb0, nb1,
                       phi, px, py, M, alpha);
  return hipGetLastError();
}

size_t gb_select_lds(int M, int Mpow) {
  return size_t(Mpow) * (8 + 4) + size_t(M) * (8 + 8 + 4 + 4) + 256 * 8;
}

hipError_t launch_gb_select(int dtype, const void* F, const Dims& dims, const BlockDesc* desc, int64_t nblocks,
                            const double* phi, const double* cv, const double* alpha, int px, int py, int M,
                            int32_t* count, int32_t* kexp, uint8_t* slot, int32_t* n0, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  int Mpow = 1;
  while (Mpow < M) Mpow <<= 1;
  const size_t lds = gb_select_lds(M, Mpow);
  // launches of at most kGbLaunchGroups workgroups (a dispatch holds under
  // 2^32 work-items)
  for (int64_t off = 0; off < nblocks; off += kGbLaunchGroups) {
    const dim3 g{unsigned(std::min<int64_t>(nblocks - off, kGbLaunchGroups))};
    if (dtype == 0)
      hipLaunchKernelGGL(k_gb_select<float>, g, dim3{256}, lds, s, static_cast<const float*>(F), dims, desc, nblocks,
                         phi, cv, alpha, px, py, M, Mpow, count, kexp, slot, n0, off);
    else
      hipLaunchKernelGGL(k_gb_select<double>, g, dim3{256}, lds, s, static_cast<const double*>(F), dims, desc,
                         nblocks, phi, cv, alpha, px, py, M, Mpow, count, kexp, slot, n0, off);
  }
  return hipGetLastError();
}

hipError_t launch_gb_patch64(int dtype, const void* F, const Dims& dims, const BlockDesc* desc, int64_t nb0,
                             int64_t nb1, const double* phi, const double* cv, int px, int py, int M, int32_t* count,
                             int32_t* kexp, uint8_t* slot, int32_t* n0, hipStream_t s) {
  if (nb1 <= nb0) return hipSuccess;
  if (M > 64) return hipErrorInvalidValue;
  // teams of S lanes, S the smallest of 16, 32, 64 that holds the patch;
  // enough workgroups to fill the chip several times (each stages Phi once)
  const int S = M <= 16 ? 16 : (M <= 32 ? 32 : 64);
  const int64_t per_wg = 4 * (64 / S);
  const int64_t want = (nb1 - nb0 + per_wg - 1) / per_wg;
  const dim3 g{unsigned(std::min<int64_t>(want, 8192))};
#define DLS_GBP(TV, SV)                                                                                       \
  hipLaunchKernelGGL((k_gb_patch64<TV, SV>), g, dim3{256}, 0, s, static_cast<const TV*>(F), dims, desc, nb0, \
                     nb1, phi, cv, px, py, M, count, kexp, slot, n0)
  if (dtype == 0) {
    if (S == 16) DLS_GBP(float, 16); else if (S == 32) DLS_GBP(float, 32); else DLS_GBP(float, 64);
  } else {
    if (S == 16) DLS_GBP(double, 16); else if (S == 32) DLS_GBP(double, 32); else DLS_GBP(double, 64);
  }
#undef DLS_GBP
  return hipGetLastError();
}

hipError_t launch_gb_sizes(const BlockDesc* desc, int64_t nblocks, const int32_t* count, int esize, int64_t* nidx,
                           int64_t* nraw, unsigned long long* raw_patches, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gb_sizes, dim3{unsigned((nblocks + 255) / 256)}, dim3{256}, 0, s, desc, nblocks, count, esize,
                     nidx, nraw, raw_patches);
  return hipGetLastError();
}

hipError_t launch_gb_compact(const BlockDesc* desc, int64_t nblocks, int M, const int32_t* count, const uint8_t* slot,
                             const int64_t* idx_off, const int64_t* raw_off, int esize, uint16_t* idx_out,
                             int32_t* q_out, uint8_t* raw_out, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  // teams of 8 lanes whatever the patch size: a patch keeps ~10
  // coefficients on average, and 32 patches per workgroup take an eighth of
  // the workgroups of one patch per wave (8 x 8 patches: 2.9 -> 0.8 ms)
  constexpr int S = 8;
  const int64_t per_wg = 256 / S, per_launch = kGbLaunchGroups * per_wg;
  for (int64_t off = 0; off < nblocks; off += per_launch) {
    const int64_t n = std::min<int64_t>(nblocks - off, per_launch);
    const dim3 g{unsigned((n + per_wg - 1) / per_wg)};
    hipLaunchKernelGGL((k_gb_compact<S>), g, dim3{256}, 0, s, desc, nblocks, M, count, slot, idx_off, raw_off, esize,
                       idx_out, q_out, raw_out, off);
  }
  return hipGetLastError();
}

hipError_t launch_gb_decode(int dtype, void* F, const Dims& dims, const BlockDesc* desc, int64_t nblocks,
                            int nvars, const double* phi, int px, int py, int M, const int32_t* count,
                            const int32_t* kexp, const int64_t* idx_off, const int64_t* raw_off,
                            const uint16_t* idx, const int32_t* q, const uint8_t* raw, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (M <= 64) {
    // blocks are variable-major (the plan's order), nblocks / nvars each
    if (nvars <= 0 || nblocks % nvars != 0) return hipErrorInvalidValue;
    const int64_t nbv = nblocks / nvars;
    const int S = M <= 16 ? 16 : (M <= 32 ? 32 : 64);
    const int64_t per_wg = 16 * (64 / S);
    const dim3 g{unsigned(std::min<int64_t>((nbv + per_wg - 1) / per_wg, 2048))};
    for (int v = 0; v < nvars; ++v) {
      const double* pv = phi + int64_t(v) * M * M;
#define DLS_GBD(TV, SV)                                                                                         \
  hipLaunchKernelGGL((k_gb_decode64<TV, SV>), g, dim3{1024}, 0, s, static_cast<TV*>(F), dims, desc, v * nbv,    \
                     (v + 1) * nbv, pv, px, py, M, count, kexp, idx_off, raw_off, idx, q, raw)
      if (dtype == 0) {
        if (S == 16) DLS_GBD(float, 16); else if (S == 32) DLS_GBD(float, 32); else DLS_GBD(float, 64);
      } else {
        if (S == 16) DLS_GBD(double, 16); else if (S == 32) DLS_GBD(double, 32); else DLS_GBD(double, 64);
      }
#undef DLS_GBD
    }
    return hipGetLastError();
  }
  const int64_t per_wg = 1, per_launch = kGbLaunchGroups * per_wg;
  for (int64_t off = 0; off < nblocks; off += per_launch) {
    const int64_t n = std::min<int64_t>(nblocks - off, per_launch);
    const dim3 g{unsigned((n + per_wg - 1) / per_wg)};
    if (dtype == 0)
      hipLaunchKernelGGL((k_gb_decode<float, 256>), g, dim3{256}, 0, s, static_cast<float*>(F), dims, desc, nblocks,
                         phi, px, py, M, count, kexp, idx_off, raw_off, idx, q, raw, off);
    else
      hipLaunchKernelGGL((k_gb_decode<double, 256>), g, dim3{256}, 0, s, static_cast<double*>(F), dims, desc,
                         nblocks, phi, px, py, M, count, kexp, idx_off, raw_off, idx, q, raw, off);
  }
  return hipGetLastError();
}

}  // namespace dls
