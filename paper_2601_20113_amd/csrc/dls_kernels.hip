// gfx950 kernels of the DLS block encoder / decoder.
//
//   k_gram    Gram product G = X X^T of every block slice on the matrix cores
//             (v_mfma_f32_16x16x4f32, FP32 products; every 64-point chunk is
//             flushed into FP64 accumulators), Sec. 2.7.1 cross-product SVD.
//   k_eigen   W lanes per block: sum of the slice Grams in FP64, cyclic
//             Jacobi in FP64 with a parallel (round-robin) ordering,
//             descending sort, canonical signs, and the rank rule of
//             Sec. 2.4 Eq. (4) / Alg. 1 step 3.
//   k_scan_*  exclusive scan of the per-block payload sizes (the offset scan
//             the paper does with MPI_Scan, Sec. 2.7.2).
//   k_encode, k_decode live in dls_codec.hip (compiled once per padded
//             window, element type and part); this file holds their
//             dispatchers.
//
// The file is compiled with -ffp-contract=off: the lattice arithmetic must
// round exactly as written so that the decoder reproduces the encoder bit
// for bit.  Fused multiply-adds are written explicitly where wanted.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "dls_device.h"
#include "dls_kernels.h"

// steps of a Jacobi sweep unrolled per loop iteration: the position
// rotation after each step is a register permutation, which unrolling turns
// into renaming.  With the partner row read pair by pair and four waves per
// SIMD (128 registers), one step per iteration is as fast as three or five
// at three waves (W = 16, 247 583 quadtree blocks: 3.11 / 3.17 / 3.15 ms);
// the kernel is bound by its LDS traffic and per-step latency, not by the
// few register moves.
#ifndef DLS_JACOBI_UNROLL
#define DLS_JACOBI_UNROLL 1
#endif

namespace dls {


template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ row, int64_t off, float* v);

template <>
__device__ __forceinline__ void load4<float>(const float* __restrict__ row, int64_t off, float* v) {
  float4 a = *reinterpret_cast<const float4*>(row + off);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

template <>
__device__ __forceinline__ void load4<double>(const double* __restrict__ row, int64_t off, float* v) {
  double2 a = *reinterpret_cast<const double2*>(row + off);
  double2 b = *reinterpret_cast<const double2*>(row + off + 2);
  v[0] = float(a.x); v[1] = float(a.y); v[2] = float(b.x); v[3] = float(b.y);
}

// Load the 16 values one lane feeds to 16 MFMA steps of a 64-point chunk:
// lane quarter q holds points 16 j + 4 q + e (j, e < 4) of time row `row`.
template <typename T>
__device__ __forceinline__ void load_chunk(const T* __restrict__ row, const Item& it, const BlockDesc& d,
                                           int chunk, int q, int64_t nx, int64_t nxy, float* v) {
#pragma unroll
  for (int s = 0; s < 16; ++s) v[s] = 0.f;
  if (row == nullptr) return;
  const int px = d.px(), py = d.py();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int ps = chunk * 64 + 16 * j + 4 * q;
    if (d.vec) {
      if (ps < it.np) load4<T>(row, point_off(it.p0 + ps, px, py, nx, nxy), v + 4 * j);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (ps + e < it.np) v[4 * j + e] = float(row[point_off(it.p0 + ps + e, px, py, nx, nxy)]);
    }
  }
}

// ---------------------------------------------------------------------------
// Gram: one workgroup (4 waves) per item; output gpart[item][WP][WP] (FP64).
// ---------------------------------------------------------------------------

// BF: bfloat16 operands (v_mfma_f32_16x16x16bf16_1k, one instruction per 16
// points); otherwise FP32 operands (v_mfma_f32_16x16x4f32, one per 4 points).
// Either way the lane feeds the same points, so the products are those of
// X X^T with the operands rounded as the instruction takes them.
template <int WP, typename T, bool BF>
__global__ __launch_bounds__(256) void k_gram(const T* __restrict__ F, Dims dims,
                                              const BlockDesc* __restrict__ desc,
                                              const Item* __restrict__ items,
                                              const int32_t* __restrict__ list,
                                              double* __restrict__ gpart) {
  constexpr int NT = (WP == 16) ? 1 : 3;  // 16x16 tiles: 00 (and 01, 11 when WP = 32)
  constexpr int LDR = 68;                 // staged row: 64 points + 4 floats of padding
  constexpr size_t kStage = size_t(4) * WP * LDR * sizeof(float);
  constexpr size_t kRed = size_t(4) * NT * 4 * 64 * sizeof(double);
  __shared__ __align__(16) char smem[kStage > kRed ? kStage : kRed];
  const int64_t item = list ? int64_t(list[blockIdx.x]) : int64_t(blockIdx.x);
  const Item it = items[item];
  const BlockDesc d = desc[it.block];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tl = lane & 15, q = lane >> 4;
  const int W = d.w();
  const int64_t nxy = dims.nx * dims.ny;
  const T* row0 = (tl < W) ? F + fidx(dims, d.var, d.t0 + tl, d.z0, d.y0, d.x0) : nullptr;
  const T* row1 = (WP == 32 && tl + 16 < W) ? F + fidx(dims, d.var, d.t0 + tl + 16, d.z0, d.y0, d.x0) : nullptr;

  double acc[NT][4];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[a][v] = 0.0;

  // G += X X^T of one 64-point chunk held as the MFMA operands v0 (rows
  // 0..15) and v1 (rows 16..31): lane (t, q) holds points 16 j + 4 q + e
  auto mfma_chunk = [&](const float* v0, const float* v1) {
    f32x4 a00 = {0.f, 0.f, 0.f, 0.f}, a01 = a00, a11 = a00;
    if constexpr (BF) {
      // MFMA j takes points 16 j + 4 q + e (e < 4) as its k index 4 q + e
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bf16x4 b0 = to_bf16x4(v0 + 4 * j);
        bf16x4 b1 = b0;
        if (WP == 32) b1 = to_bf16x4(v1 + 4 * j);
        a00 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b0, b0, a00, 0, 0, 0);
        if (WP == 32) {
          a01 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b0, b1, a01, 0, 0, 0);
          a11 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b1, b1, a11, 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        a00 = __builtin_amdgcn_mfma_f32_16x16x4f32(v0[s], v0[s], a00, 0, 0, 0);
        if (WP == 32) {
          a01 = __builtin_amdgcn_mfma_f32_16x16x4f32(v0[s], v1[s], a01, 0, 0, 0);
          a11 = __builtin_amdgcn_mfma_f32_16x16x4f32(v1[s], v1[s], a11, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      acc[0][v] += double(a00[v]);
      if (WP == 32) {
        acc[1][v] += double(a01[v]);
        acc[2][v] += double(a11[v]);
      }
    }
  };

  // the wave's chunks c = wave, wave + 4, ... are taken CPW at a time, with
  // every load of the group issued before the first MFMA
  constexpr int CPW = (WP == 16) ? 4 : 2;
  bool staged = false;
  if constexpr (sizeof(T) == 4) staged = d.vec != 0;
  if (staged) {
    // FP32 rows of 4-aligned points: each load instruction covers 4 time rows
    // x 64 consecutive chunk points (full cache lines); the chunk goes through
    // LDS into the MFMA operand layout
    float* stage = reinterpret_cast<float*>(smem) + wave * WP * LDR;
    const int lr = lane >> 4, lp = 4 * (lane & 15);
    const int px = d.px(), py = d.py();
    for (int c0 = wave; c0 * 64 < it.np; c0 += 4 * CPW) {
      float4 raw[CPW][WP / 4];
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        const int ps = (c0 + 4 * u) * 64 + lp;
        const bool okp = ps < it.np;
        const int64_t off = point_off(it.p0 + (okp ? ps : 0), px, py, dims.nx, nxy);
#pragma unroll
        for (int i = 0; i < WP / 4; ++i) {
          const int t = 4 * i + lr;
          raw[u][i] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (okp && t < W)
            raw[u][i] = *reinterpret_cast<const float4*>(
                reinterpret_cast<const float*>(F) + fidx(dims, d.var, d.t0 + t, d.z0, d.y0, d.x0) + off);
        }
      }
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        if ((c0 + 4 * u) * 64 >= it.np) continue;
#pragma unroll
        for (int i = 0; i < WP / 4; ++i)
          *reinterpret_cast<float4*>(stage + (4 * i + lr) * LDR + lp) = raw[u][i];
        wave_sync();
        float v0[16], v1[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float4 a = *reinterpret_cast<const float4*>(stage + tl * LDR + 16 * j + 4 * q);
          v0[4 * j] = a.x; v0[4 * j + 1] = a.y; v0[4 * j + 2] = a.z; v0[4 * j + 3] = a.w;
          if (WP == 32) {
            const float4 b = *reinterpret_cast<const float4*>(stage + (16 + tl) * LDR + 16 * j + 4 * q);
            v1[4 * j] = b.x; v1[4 * j + 1] = b.y; v1[4 * j + 2] = b.z; v1[4 * j + 3] = b.w;
          }
        }
        wave_sync();
        mfma_chunk(v0, v1);
      }
    }
  } else {
    for (int c0 = wave; c0 * 64 < it.np; c0 += 4 * CPW) {
      float vv0[CPW][16], vv1[CPW][16];
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        load_chunk<T>(row0, it, d, c0 + 4 * u, q, dims.nx, nxy, vv0[u]);
        if (WP == 32) load_chunk<T>(row1, it, d, c0 + 4 * u, q, dims.nx, nxy, vv1[u]);
      }
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        if ((c0 + 4 * u) * 64 >= it.np) continue;
        mfma_chunk(vv0[u], vv1[u]);
      }
    }
  }

  __syncthreads();  // every wave is done with its staging area before it becomes `red`
  double (*red)[NT * 4][64] = reinterpret_cast<double (*)[NT * 4][64]>(smem);
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][a * 4 + v][lane] = acc[a][v];
  __syncthreads();
  if (wave != 0) return;
  double* out = gpart + item * WP * WP;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = a * 4 + v;
      double g = ((red[0][s][lane] + red[1][s][lane]) + red[2][s][lane]) + red[3][s][lane];
      // MFMA 16x16 output: lane l, register v holds row 4 (l / 16) + v, column l % 16
      const int i = 4 * q + v, j = tl;
      if (a == 0) {
        out[i * WP + j] = g;
      } else if (a == 1) {
        out[i * WP + 16 + j] = g;
        out[(16 + j) * WP + i] = g;
      } else {
        out[(16 + i) * WP + 16 + j] = g;
      }
    }
}

// Gram of small slices (<= 256 points): one wavefront per slice, four
// slices per workgroup, no cross-wave reduction.  The chunk order and the
// FP64 flush per chunk are those of k_gram's wave 0 over the same slice, so
// the partial Gram is bitwise the same.
template <int WP, typename T, bool BF>
__global__ __launch_bounds__(256) void k_gram_wave(const T* __restrict__ F, Dims dims,
                                                   const BlockDesc* __restrict__ desc,
                                                   const Item* __restrict__ items,
                                                   const int32_t* __restrict__ list, int64_t nlist,
                                                   double* __restrict__ gpart) {
  constexpr int NT = (WP == 16) ? 1 : 3;
  const int lane = threadIdx.x & 63;
  const int64_t li = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (li >= nlist) return;
  const int64_t item = list[li];
  const Item it = items[item];
  const BlockDesc d = desc[it.block];
  const int tl = lane & 15, q = lane >> 4;
  const int W = d.w();
  const int64_t nxy = dims.nx * dims.ny;
  const T* row0 = (tl < W) ? F + fidx(dims, d.var, d.t0 + tl, d.z0, d.y0, d.x0) : nullptr;
  const T* row1 = (WP == 32 && tl + 16 < W) ? F + fidx(dims, d.var, d.t0 + tl + 16, d.z0, d.y0, d.x0) : nullptr;
  double acc[NT][4];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[a][v] = 0.0;
  float vv0[4][16], vv1[4][16];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    load_chunk<T>(row0, it, d, c, q, dims.nx, nxy, vv0[c]);
    if (WP == 32) load_chunk<T>(row1, it, d, c, q, dims.nx, nxy, vv1[c]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c * 64 >= it.np) continue;
    const float* v0 = vv0[c];
    const float* v1 = vv1[c];
    f32x4 a00 = {0.f, 0.f, 0.f, 0.f}, a01 = a00, a11 = a00;
    if constexpr (BF) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bf16x4 b0 = to_bf16x4(v0 + 4 * j);
        bf16x4 b1 = b0;
        if (WP == 32) b1 = to_bf16x4(v1 + 4 * j);
        a00 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b0, b0, a00, 0, 0, 0);
        if (WP == 32) {
          a01 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b0, b1, a01, 0, 0, 0);
          a11 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b1, b1, a11, 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        a00 = __builtin_amdgcn_mfma_f32_16x16x4f32(v0[s], v0[s], a00, 0, 0, 0);
        if (WP == 32) {
          a01 = __builtin_amdgcn_mfma_f32_16x16x4f32(v0[s], v1[s], a01, 0, 0, 0);
          a11 = __builtin_amdgcn_mfma_f32_16x16x4f32(v1[s], v1[s], a11, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      acc[0][v] += double(a00[v]);
      if (WP == 32) {
        acc[1][v] += double(a01[v]);
        acc[2][v] += double(a11[v]);
      }
    }
  }
  double* out = gpart + item * WP * WP;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double g = acc[a][v];
      const int i = 4 * q + v, j = tl;
      if (a == 0) {
        out[i * WP + j] = g;
      } else if (a == 1) {
        out[i * WP + 16 + j] = g;
        out[(16 + j) * WP + i] = g;
      } else {
        out[(16 + i) * WP + 16 + j] = g;
      }
    }
}

// ---------------------------------------------------------------------------
// Eigensolve + rank.  WP lanes per block (lane i owns row i of the Gram
// matrix A and row i of the accumulated rotations V, in registers), 256 / WP
// blocks per workgroup.  Cyclic Jacobi in FP64 with the parallel round-robin
// ordering: at each step the WP / 2 disjoint pairs sit at positions
// (k, WP-1-k); the columns are held in position order and rotated by one
// position after every step, so the partner of register k is always register
// WP-1-k.  Each step: every lane publishes its row in LDS, the lower lane of
// each pair computes the rotation, then every lane forms its new row from
// its own row and its partner's.  A group only touches its own LDS and its
// lanes are active together, so no workgroup barrier is used.
// ---------------------------------------------------------------------------
// off(A) <= 1e-13 ||A|| (squared: 1e-26), A's rows held one per lane of a
// WP-lane group, positions in natural order
template <int WP>
__device__ __forceinline__ bool jacobi_converged(const double (&a)[WP], int i) {
  double off = 0.0, tot = 0.0;
#pragma unroll
  for (int j = 0; j < WP; ++j) {
    const double x = a[j] * a[j];
    tot += x;
    off += (j == i) ? 0.0 : x;
  }
  off = group_sum<WP>(off);
  tot = group_sum<WP>(tot);
  return !(off > 1e-26 * tot);
}

template <int WP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WP == 16 ? 4 : 1, 8))) void k_eigen(const double* __restrict__ gpart,
                                               const int32_t* __restrict__ item_start,
                                               const BlockDesc* __restrict__ desc, int64_t nblocks,
                                               const double* __restrict__ eps_v, int r_max,
                                               uint8_t* __restrict__ rank_out,
                                               double* __restrict__ lam_out,
                                               double* __restrict__ basis_out,
                                               int64_t* __restrict__ qv_size,
                                               int64_t* __restrict__ qa_size,
                                               unsigned long long* __restrict__ nraw,
                                               const int32_t* __restrict__ list,
                                               const unsigned int* __restrict__ list_count,
                                               unsigned long long* __restrict__ jstats, int max_sweeps) {
  constexpr int GPW = 256 / WP;
  constexpr int LD = WP + 1;
  __shared__ double sA[GPW][WP * LD];
  // one (c, s) per position pair, kept at its lower position k < WP / 2
  __shared__ double2 sCS[GPW][WP / 2];
  __shared__ double sLam[GPW][WP];
  const int grp = threadIdx.x / WP, i = threadIdx.x % WP;
  // every block, or (list != NULL) the blocks of the device-written list
  const int64_t li = int64_t(blockIdx.x) * GPW + grp;
  if (li >= (list ? int64_t(*list_count) : nblocks)) return;
  const int64_t b = list ? int64_t(list[li]) : li;
  double* A = sA[grp];
  double2* CS = sCS[grp];
  // after the sweeps: the sort permutation in the rotation slots (WP ints
  // in WP / 2 double2) and the column signs in the pad column of A, so that
  // four workgroups of W = 16 fit in one compute unit's LDS
  int* Perm = reinterpret_cast<int*>(CS);
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m;
  const int i0 = item_start[b], i1 = item_start[b + 1];

  // Gram row i = sum of the slice Grams, symmetrised through LDS
  double a[WP], v[WP];
#pragma unroll
  for (int j = 0; j < WP; ++j) a[j] = 0.0;
  for (int it = i0; it < i1; ++it) {  // every entry's loads of an item issued together
    const double* gp = gpart + int64_t(it) * WP * WP + i * WP;
#pragma unroll
    for (int j = 0; j < WP; ++j) a[j] += gp[j];
  }
#pragma unroll
  for (int j = 0; j < WP; ++j) A[i * LD + j] = a[j];
  wave_sync();
  bool fin = true;
#pragma unroll
  for (int j = 0; j < WP; ++j) {
    a[j] = 0.5 * (a[j] + A[j * LD + i]);
    fin = fin && isfinite(a[j]);
    v[j] = (j == i) ? 1.0 : 0.0;
  }
  wave_sync();
  if (group_sum<WP>(fin ? 0.0 : 1.0) != 0.0) {  // non-finite input: raw block
    if (i == 0) {
      rank_out[b] = 0;
      qv_size[b] = 0;
      qa_size[b] = 0;
      atomicAdd(nraw, 1ULL);
    }
    lam_out[b * WP + i] = 0.0;
#pragma unroll
    for (int k = 0; k < WP; ++k) basis_out[(b * WP + k) * WP + i] = (k == i) ? 1.0 : 0.0;
    return;
  }

  // the convergence test runs before every sweep; a block that uses every
  // sweep of the cap is counted as unconverged (its last sweep unchecked: a
  // test after the loop costs W = 32 a wave of occupancy)
  int sweep = 0;
  bool converged = false;
  // round-robin state of this lane, advanced step by step (it returns to
  // its start after the WP - 1 steps of a sweep): its position, and mm with
  // partner m = mm + 1 (player 0 when the lane sits at position WP - 1)
  int pos = rr_slot(i, 0, WP);
  const int inc = i == 0 ? 1 : 2;
  int mm = i == 0 ? WP - 2 : (WP - 2 - i) % (WP - 1);
  for (; sweep < max_sweeps; ++sweep) {
    if (jacobi_converged<WP>(a, i)) {
      converged = true;
      break;
    }
    // W = 32 keeps one step per iteration: unrolled, its rows need all 256
    // registers (one wave per SIMD)
    constexpr int kUnroll = WP == 16 ? DLS_JACOBI_UNROLL : 1;
#pragma unroll kUnroll
    for (int step = 0; step < WP - 1; ++step) {
#pragma unroll
      for (int k = 0; k < WP; ++k) A[i * LD + k] = a[k];
      wave_sync();
      const int mpos = WP - 1 - pos;
      const int m = pos == WP - 1 ? 0 : mm + 1;  // rr_player(mpos, step, WP)
      if (i < m) {
        double c, s;
        jacobi_rotation(A[i * LD + pos], A[m * LD + mpos], A[i * LD + mpos], c, s);
        // seen from position pos the pair rotates by (c, -s), from mpos by (c, s)
        if (pos < mpos) CS[pos] = make_double2(c, -s);
        else CS[mpos] = make_double2(c, s);
      }
      wave_sync();
      double2 ci = CS[pos < mpos ? pos : mpos];
      if (pos > mpos) ci.y = -ci.y;
#pragma unroll
      for (int k = 0; k < WP / 2; ++k) {
        const int mk = WP - 1 - k;
        const double pk = A[m * LD + k], pmk = A[m * LD + mk];  // the partner's row, pair by pair
        const double2 ck = CS[k], cm = make_double2(ck.x, -ck.y);
        // row rotation (own row with the partner's), then column rotation
        const double rk = fma(ci.x, a[k], ci.y * pk);
        const double rm = fma(ci.x, a[mk], ci.y * pmk);
        a[k] = fma(ck.x, rk, ck.y * rm);
        a[mk] = fma(cm.x, rm, cm.y * rk);
        const double vk = fma(ck.x, v[k], ck.y * v[mk]);
        const double vm = fma(cm.x, v[mk], cm.y * v[k]);
        v[k] = vk;
        v[mk] = vm;
      }
      // next step: position k takes the column of position k + 1, the last
      // position takes the column of position 1, position 0 stays
      const double a1 = a[1], v1 = v[1];
#pragma unroll
      for (int k = 1; k < WP - 1; ++k) {
        a[k] = a[k + 1];
        v[k] = v[k + 1];
      }
      a[WP - 1] = a1;
      v[WP - 1] = v1;
      pos = i == 0 ? 0 : (pos == 1 ? WP - 1 : pos - 1);
      mm += inc;
      mm -= mm >= WP - 1 ? WP - 1 : 0;
      wave_sync();
    }
  }

  // V rows and the diagonal to LDS; descending order of the eigenvalue
  // estimates diag(A) (stable by index).  Padded indices i >= W_b have zero
  // Gram rows, are never rotated, and sort last.
  double di = 0.0;
#pragma unroll
  for (int j = 0; j < WP; ++j) {
    A[i * LD + j] = v[j];
    di = (j == i) ? a[j] : di;
  }
  sLam[grp][i] = i < W ? di : -INFINITY;
  wave_sync();
  {
    const double dk = sLam[grp][i];
    int pos = 0;
    for (int j = 0; j < WP; ++j) {
      const double dj = sLam[grp][j];
      pos += (dj > dk || (dj == dk && j < i)) ? 1 : 0;
    }
    Perm[pos] = i;
  }
  wave_sync();
  // sorted column i: its eigenvalue and canonical sign (largest |component|
  // positive, lowest row on a tie)
  const int col = Perm[i];
  const double lam = fmax(i < W ? sLam[grp][col] : 0.0, 0.0);
  {
    double best = -1.0, sg = 1.0;
    for (int t = 0; t < WP; ++t) {
      const double x = A[t * LD + col];
      if (fabs(x) > best) { best = fabs(x); sg = x < 0.0 ? -1.0 : 1.0; }
    }
    A[i * LD + WP] = sg;  // the sign of sorted column i, in row i's pad entry
  }
  wave_sync();
  sLam[grp][i] = lam;
  lam_out[b * WP + i] = lam;
#pragma unroll 4
  for (int k = 0; k < WP; ++k) basis_out[(b * WP + k) * WP + i] = A[k * LD + WP] * A[i * LD + Perm[k]];
  wave_sync();
  if (i == 0) {
    const double eps = eps_v[d.var];
    const double tau = kKappa * eps * eps * double(M) * double(W);
    int rcap = r_max < W ? r_max : W;
    rcap = rcap < M ? rcap : M;
    // suffix sums tail_k = sum_{j >= k} lambda_j; r = the smallest k <= rcap
    // with tail_k <= tau, else rcap
    double tail = 0.0;
    int r = rcap;
    for (int k = WP - 1; k >= 1; --k) {
      tail += sLam[grp][k];
      if (k <= rcap && tail <= tau) r = k;
    }
    rank_out[b] = uint8_t(r);
    qv_size[b] = 4 * pad16(int64_t(W) * r);
    qa_size[b] = 4 * pad16(int64_t(M) * r);
    if (sweep) atomicAdd(jstats + 1 + blockIdx.x % kJacobiSlots, (unsigned long long)sweep);
    if (!converged) atomicAdd(jstats, 1ull);
  }
}

// ---------------------------------------------------------------------------
// Exclusive scan of int64 sizes (n <= 1024 * 1024 * 4 per level).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scan_local(const int64_t* __restrict__ in, int64_t n,
                                                    int64_t* __restrict__ out, int64_t* __restrict__ tops) {
  __shared__ int64_t s[256];
  const int64_t base = int64_t(blockIdx.x) * 1024;
  int64_t v[4], sum = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = base + threadIdx.x * 4 + e;
    v[e] = i < n ? in[i] : 0;
    sum += v[e];
  }
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int64_t add = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = s[threadIdx.x] - sum;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = base + threadIdx.x * 4 + e;
    if (i < n) out[i] = run;
    run += v[e];
  }
  if (threadIdx.x == 255) tops[blockIdx.x] = s[255];
}

__global__ __launch_bounds__(256) void k_scan_add(int64_t* __restrict__ out, int64_t n,
                                                  const int64_t* __restrict__ tops_scanned) {
  const int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  const int64_t add = tops_scanned[blockIdx.x];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (i + 256 * e < n) out[i + 256 * e] += add;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter(T* __restrict__ F, const int64_t* __restrict__ idx,
                                                 const uint64_t* __restrict__ bits, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  if (sizeof(T) == 4) {
    reinterpret_cast<uint32_t*>(F)[idx[i]] = uint32_t(bits[i]);
  } else {
    reinterpret_cast<uint64_t*>(F)[idx[i]] = bits[i];
  }
}

// ---------------------------------------------------------------------------
// Per-variable value range (min, max) in FP64: grid-stride partials, then one
// workgroup folds the partials.  Non-finite values are skipped.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_range_partial(const T* __restrict__ F, int64_t n_per_var,
                                                       double* __restrict__ part) {
  const int v = blockIdx.y;
  const T* base = F + int64_t(v) * n_per_var;
  double lo = INFINITY, hi = -INFINITY;
  // four loads in flight per thread, 16-byte loads where the variable is
  // 16-byte aligned FP32 (min and max do not depend on the order)
  const int64_t stride = int64_t(gridDim.x) * 256;
  const int64_t i0 = int64_t(blockIdx.x) * 256 + threadIdx.x;
  auto take = [&](double x) {
    if (isfinite(x)) {
      lo = fmin(lo, x);
      hi = fmax(hi, x);
    }
  };
  if (sizeof(T) == 4 && (n_per_var & 3) == 0 && (reinterpret_cast<uintptr_t>(base) & 15) == 0) {
    const float4* b4 = reinterpret_cast<const float4*>(base);
    const int64_t n4 = n_per_var / 4;
    for (int64_t i = i0; i < n4; i += 4 * stride) {
      float4 x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = i + u * stride < n4 ? b4[i + u * stride] : make_float4(NAN, NAN, NAN, NAN);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        take(double(x[u].x));
        take(double(x[u].y));
        take(double(x[u].z));
        take(double(x[u].w));
      }
    }
  } else {
    for (int64_t i = i0; i < n_per_var; i += 4 * stride) {
      double x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = i + u * stride < n_per_var ? double(base[i + u * stride]) : NAN;
#pragma unroll
      for (int u = 0; u < 4; ++u) take(x[u]);
    }
  }
  __shared__ double slo[256], shi[256];
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + o]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * (int64_t(v) * gridDim.x + blockIdx.x)] = slo[0];
    part[2 * (int64_t(v) * gridDim.x + blockIdx.x) + 1] = shi[0];
  }
}

__global__ __launch_bounds__(256) void k_range_final(const double* __restrict__ part, int nparts,
                                                     double* __restrict__ out) {
  const int v = blockIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  for (int i = threadIdx.x; i < nparts; i += 256) {
    lo = fmin(lo, part[2 * (int64_t(v) * nparts + i)]);
    hi = fmax(hi, part[2 * (int64_t(v) * nparts + i) + 1]);
  }
  __shared__ double slo[256], shi[256];
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + o]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * v] = slo[0];
    out[2 * v + 1] = shi[0];
  }
}

hipError_t launch_range(int dtype, const void* F, int nvars, int64_t n_per_var, double* part, int nparts,
                        double* out, hipStream_t s) {
  const dim3 g{unsigned(nparts), unsigned(nvars)}, bl{256};
  if (dtype == 0) hipLaunchKernelGGL(k_range_partial<float>, g, bl, 0, s, (const float*)F, n_per_var, part);
  else hipLaunchKernelGGL(k_range_partial<double>, g, bl, 0, s, (const double*)F, n_per_var, part);
  hipLaunchKernelGGL(k_range_final, dim3{unsigned(nvars)}, bl, 0, s, (const double*)part, nparts, out);
  return hipGetLastError();
}

// Fixed device scratch of the allocation-free range (dls_range_noalloc):
// the per-variable partial minima / maxima (kRangeParts per variable) and
// the folded results, for at most kRangeNoAllocVars variables.  One copy per
// GPU, kept for the life of the process; every launch writes every slot it
// later reads, so nothing needs clearing.  Host code uses the address
// returned by range_scratch(), never this name.
static __device__ __align__(256) double scratch[kRangeNoAllocVars * (2 * kRangeParts + 2)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t range_scratch(int device, double** ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    void* p = nullptr;
    // the caller has made `device` current: this is its copy of the array
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_range_noalloc(double* scratch_ptr, int dtype, const void* F, int nvars, int64_t n_per_var,
                                hipStream_t s) {
  const int nparts = int(std::min<int64_t>(kRangeParts, (n_per_var + 255) / 256));
  double* part = scratch_ptr;
  double* out = scratch_ptr + int64_t(nvars) * 2 * kRangeParts;
  return launch_range(dtype, F, nvars, n_per_var, part, nparts, out, s);
}

// Bucket the work items by the rank class of their block (one list per class,
// order within a list is irrelevant: items write disjoint outputs).
__device__ __forceinline__ int rank_class(int r) {
  return r <= 1 ? 0 : r <= 2 ? 1 : r <= 4 ? 2 : r <= 8 ? 3 : r <= 16 ? 4 : 5;
}

// Rank class of every slice (and, when small_limit > 0, slices of at most
// small_limit points go to the small-slice classes kRankClasses + c).
__global__ __launch_bounds__(256) void k_classify(const Item* __restrict__ items, int64_t nitems,
                                                  const uint8_t* __restrict__ rank, int small_limit,
                                                  unsigned int* __restrict__ counts,
                                                  int32_t* __restrict__ lists,
                                                  const unsigned int* __restrict__ skip) {
  // counts are aggregated per workgroup in LDS: one global atomic per class
  constexpr int NC = 2 * kRankClasses;
  __shared__ unsigned int lcount[NC], lbase[NC];
  if (threadIdx.x < NC) lcount[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  int c = -1;
  unsigned int lpos = 0;
  if (i < nitems) {
    const Item it = items[i];
    if (skip == nullptr || skip[it.block] != 1u) {
      c = rank_class(rank[it.block]) + (it.np <= small_limit ? kRankClasses : 0);
      lpos = atomicAdd(&lcount[c], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x < NC && lcount[threadIdx.x] > 0)
    lbase[threadIdx.x] = atomicAdd(counts + threadIdx.x, lcount[threadIdx.x]);
  __syncthreads();
  if (c >= 0) lists[int64_t(c) * nitems + lbase[c] + lpos] = int32_t(i);
}

// Escapes straight from the encoder's list: key = block << 32 | (t M_b + p)
template <typename T>
__global__ __launch_bounds__(256) void k_scatter_keys(T* __restrict__ F, Dims dims,
                                                      const BlockDesc* __restrict__ desc,
                                                      const uint64_t* __restrict__ key,
                                                      const uint64_t* __restrict__ bits, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t kk = key[i];
  if (kk == ~uint64_t(0)) return;  // an escape the single pass dropped
  const BlockDesc d = desc[kk >> 32];
  const uint32_t tp = uint32_t(kk);
  const int t = int(tp / uint32_t(d.m)), p = int(tp % uint32_t(d.m));
  const int64_t at = fidx(dims, d.var, d.t0 + t, d.z0, d.y0, d.x0) +
                     point_off(p, d.px(), d.py(), dims.nx, dims.nx * dims.ny);
  if (sizeof(T) == 4) {
    reinterpret_cast<uint32_t*>(F)[at] = uint32_t(bits[i]);
  } else {
    reinterpret_cast<uint64_t*>(F)[at] = bits[i];
  }
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_zero(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_totals(const int64_t* __restrict__ qv_off, const int64_t* __restrict__ qv_size,
                         const int64_t* __restrict__ qa_off, const int64_t* __restrict__ qa_size, int64_t n,
                         int64_t* __restrict__ totals) {
  if (threadIdx.x == 0) {
    totals[0] = n ? qv_off[n - 1] + qv_size[n - 1] : 0;
    totals[1] = n ? qa_off[n - 1] + qa_size[n - 1] : 0;
  }
}

// wave-aggregated compaction: one atomic per wavefront
__global__ __launch_bounds__(256) void k_compact_flags(const uint8_t* __restrict__ flag, int64_t n,
                                                       int32_t* __restrict__ list, unsigned int* __restrict__ count) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const bool on = i < n && flag[i] != 0;
  const uint64_t m = __ballot(on);
  const int lane = threadIdx.x & 63;
  unsigned int base = 0;
  if (lane == 0 && m) base = atomicAdd(count, unsigned(__popcll(m)));
  base = __shfl(base, 0, 64);
  if (on) list[base + __popcll(m & ((1ULL << lane) - 1ULL))] = int32_t(i);
}

hipError_t launch_compact_flags(const uint8_t* flag, int64_t n, int32_t* list, unsigned int* count, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact_flags, dim3{unsigned((n + 255) / 256)}, dim3{256}, 0, s, flag, n, list, count);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t n = int64_t(bytes / 4);  // whole words; every user passes a multiple of 4
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3{unsigned((n + 255) / 256)}, dim3{256}, 0, s, static_cast<uint32_t*>(p), n);
  return hipGetLastError();
}

hipError_t launch_totals(const int64_t* qv_off, const int64_t* qv_size, const int64_t* qa_off,
                         const int64_t* qa_size, int64_t n, int64_t* totals, hipStream_t s) {
  hipLaunchKernelGGL(k_totals, dim3{1}, dim3{64}, 0, s, qv_off, qv_size, qa_off, qa_size, n, totals);
  return hipGetLastError();
}

// Workgroups per dispatch of the one-team-per-slice launches: a dispatch's
// work-items (workgroups x threads) must stay below 2^32.
constexpr int64_t kDecodeLaunchItems = int64_t(1) << 23;

hipError_t launch_gram(int wp, int dtype, bool bf16, const void* F, const Dims& dims, const BlockDesc* desc,
                       const Item* items, int64_t nitems, const GramSplit* split, double* gpart, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  const dim3 bl{256};
  // without a split every slice takes a 4-wave workgroup; with one, the large
  // slices do and the small ones share workgroups, one wave each
  const int32_t* list = split ? split->large : nullptr;
  const int64_t nlarge = split ? split->nlarge : nitems;
  const int64_t nsmall = split ? split->nsmall : 0;
  // launches of at most kDecodeLaunchItems workgroups (a dispatch holds
  // under 2^32 work-items) over consecutive ranges of the lists; without a
  // list the items (and their Gram partials) are shifted instead
  for (int64_t off = 0; off < nlarge; off += kDecodeLaunchItems) {
    const dim3 g{unsigned(std::min<int64_t>(nlarge - off, kDecodeLaunchItems))};
    const Item* it = list ? items : items + off;
    const int32_t* li = list ? list + off : nullptr;
    double* gp = list ? gpart : gpart + off * wp * wp;
#define DLS_GRAM(WPV, TV, BFV) hipLaunchKernelGGL((k_gram<WPV, TV, BFV>), g, bl, 0, s, (const TV*)F, dims, desc, it, li, gp)
    if (wp == 16) {
      if (dtype == 0) { if (bf16) DLS_GRAM(16, float, true); else DLS_GRAM(16, float, false); }
      else { if (bf16) DLS_GRAM(16, double, true); else DLS_GRAM(16, double, false); }
    } else {
      if (dtype == 0) { if (bf16) DLS_GRAM(32, float, true); else DLS_GRAM(32, float, false); }
      else { if (bf16) DLS_GRAM(32, double, true); else DLS_GRAM(32, double, false); }
    }
#undef DLS_GRAM
  }
  for (int64_t off = 0; off < nsmall; off += 4 * kDecodeLaunchItems) {
    const int64_t n = std::min<int64_t>(nsmall - off, 4 * kDecodeLaunchItems);
    const dim3 gs{unsigned((n + 3) / 4)};
    const int32_t* li = split->small + off;
#define DLS_GRAMW(WPV, TV, BFV) \
  hipLaunchKernelGGL((k_gram_wave<WPV, TV, BFV>), gs, bl, 0, s, (const TV*)F, dims, desc, items, li, n, gpart)
    if (wp == 16) {
      if (dtype == 0) { if (bf16) DLS_GRAMW(16, float, true); else DLS_GRAMW(16, float, false); }
      else { if (bf16) DLS_GRAMW(16, double, true); else DLS_GRAMW(16, double, false); }
    } else {
      if (dtype == 0) { if (bf16) DLS_GRAMW(32, float, true); else DLS_GRAMW(32, float, false); }
      else { if (bf16) DLS_GRAMW(32, double, true); else DLS_GRAMW(32, double, false); }
    }
#undef DLS_GRAMW
  }
  return hipGetLastError();
}

hipError_t launch_eigen(int wp, const double* gpart, const int32_t* item_start, const BlockDesc* desc,
                        int64_t nblocks, const double* eps_v, int r_max, uint8_t* rank, double* lam,
                        double* basis, int64_t* qv_size, int64_t* qa_size, unsigned long long* nraw,
                        const int32_t* list, const unsigned int* list_count, unsigned long long* jstats,
                        int max_sweeps, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  const dim3 bl{256};
  if (wp == 16)
    hipLaunchKernelGGL(k_eigen<16>, dim3{unsigned((nblocks + 15) / 16)}, bl, 0, s, gpart, item_start, desc, nblocks,
                       eps_v, r_max, rank, lam, basis, qv_size, qa_size, nraw, list, list_count, jstats, max_sweeps);
  else
    hipLaunchKernelGGL(k_eigen<32>, dim3{unsigned((nblocks + 7) / 8)}, bl, 0, s, gpart, item_start, desc, nblocks,
                       eps_v, r_max, rank, lam, basis, qv_size, qa_size, nraw, list, list_count, jstats, max_sweeps);
  return hipGetLastError();
}

hipError_t launch_scan(const int64_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s) {
  // tmp holds 2 * ceil(n / 1024) + 2 * ceil(n / 2^20) + 2 entries
  if (n == 0) return hipSuccess;
  const int64_t nb = (n + 1023) / 1024;
  int64_t* tops = tmp;
  int64_t* tops_scan = tmp + nb;
  hipLaunchKernelGGL(k_scan_local, dim3(unsigned(nb)), dim3(256), 0, s, in, n, out, tops);
  if (nb > 1) {
    hipError_t e = launch_scan(tops, nb, tops_scan, tmp + 2 * nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3(unsigned(nb)), dim3(256), 0, s, out, n, (const int64_t*)tops_scan);
  }
  return hipGetLastError();
}

hipError_t launch_classify(const Item* items, int64_t nitems, const uint8_t* rank, int small_limit,
                           unsigned int* counts, int32_t* lists, hipStream_t s, const unsigned int* skip) {
  if (nitems == 0) return hipSuccess;
  const dim3 g{unsigned((nitems + 255) / 256)}, bl{256};
  hipLaunchKernelGGL(k_classify, g, bl, 0, s, items, nitems, rank, small_limit, counts, lists, skip);
  return hipGetLastError();
}

// Payload regions of the blocks the fused kernel deferred, taken from the
// same bump cursors (any order: the stream is written block by block from
// the offsets, so the layout of the device payload does not matter).
__global__ __launch_bounds__(256) void k_alloc_deferred(const int32_t* __restrict__ list,
                                                        const unsigned int* __restrict__ count,
                                                        const int64_t* __restrict__ qv_size,
                                                        const int64_t* __restrict__ qa_size,
                                                        unsigned long long* __restrict__ counters,
                                                        int64_t qv_base, int64_t qa_base,
                                                        int64_t* __restrict__ qv_off, int64_t* __restrict__ qa_off) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= int64_t(*count)) return;
  const int b = list[i];
  qv_off[b] = qv_base + int64_t(atomicAdd(counters + kFusedQvCursor, (unsigned long long)qv_size[b]));
  qa_off[b] = qa_base + int64_t(atomicAdd(counters + kFusedQaCursor, (unsigned long long)qa_size[b]));
}

hipError_t launch_alloc_deferred(const int32_t* list, const unsigned int* count, int64_t nmax, const int64_t* qv_size,
                                 const int64_t* qa_size, unsigned long long* counters, int64_t qv_base,
                                 int64_t qa_base, int64_t* qv_off, int64_t* qa_off, hipStream_t s) {
  if (nmax == 0) return hipSuccess;
  hipLaunchKernelGGL(k_alloc_deferred, dim3{unsigned((nmax + 255) / 256)}, dim3{256}, 0, s, list, count, qv_size,
                     qa_size, counters, qv_base, qa_base, qv_off, qa_off);
  return hipGetLastError();
}

int encode_small_limit(int wp, int dtype) { return (wp == 16 && dtype == 0) ? 16 * 4 : 64 * 2; }

hipError_t launch_encode(int wp, int dtype, int cls, const void* F, const Dims& dims, const BlockDesc* desc,
                         const Item* items, const int32_t* list, const EncodeWork& work, const uint8_t* rank,
                         const double* basis, const int64_t* qv_off, const int64_t* qa_off,
                         const int64_t* code_off, const VarConst* vc, uint8_t* qv, uint8_t* qa,
                         uint8_t* codes, float* coef, EscOut esc, hipStream_t s) {
  // classes kRankClasses.. hold small slices: 16 per workgroup (FP32, W <= 16)
  // or 4.  Host-driven: one team per slice; device-driven: a grid that fills
  // the chip a few times over and walks the list
  const bool small = cls >= kRankClasses;
  const int rc = cls % kRankClasses;
  const int64_t per = small ? ((wp == 16 && dtype == 0) ? 16 : 4) : 1;
#define DLS_ENC_PART(TAG, G, L, W)                                                                                \
  (small ? encode_small_##TAG : encode_large_##TAG)(rc, G, s, F, dims, desc, items, L, rank, basis, qv_off, qa_off, \
                                                    code_off, vc, qv, qa, codes, coef, esc, W)
#define DLS_ENC_ANY(G, L, W)                                       \
  ((wp == 16 && dtype == 0) ? DLS_ENC_PART(w16_f32, G, L, W)      \
   : (wp == 16)             ? DLS_ENC_PART(w16_f64, G, L, W)      \
   : (dtype == 0)           ? DLS_ENC_PART(w32_f32, G, L, W)      \
                            : DLS_ENC_PART(w32_f64, G, L, W))
  if (work.dcount) {
    const int64_t grid = std::min<int64_t>((work.count + per - 1) / per, 4096);
    if (grid == 0) return hipSuccess;
    return DLS_ENC_ANY(dim3{unsigned(grid)}, list, work);
  }
  // host-driven: one team per slice, in dispatches of at most
  // kDecodeLaunchItems workgroups (a dispatch holds under 2^32 work-items)
  const int64_t per_launch = kDecodeLaunchItems * per;
  for (int64_t off = 0; off < work.count; off += per_launch) {
    EncodeWork w = work;
    w.count = std::min<int64_t>(work.count - off, per_launch);
    const hipError_t e = DLS_ENC_ANY(dim3{unsigned((w.count + per - 1) / per)}, list + off, w);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
#undef DLS_ENC_ANY
#undef DLS_ENC_PART
}

static hipError_t decode_dispatch(int wp, int dtype, int rc, const dim3& g, const dim3& bl, hipStream_t s, void* F,
                                  const Dims& dims, const BlockDesc* desc, const Item* items, const int32_t* list,
                                  const uint8_t* rank, const int64_t* qv_off, const int64_t* qa_off,
                                  const int64_t* code_off, const VarConst* vc, const uint8_t* qv, const uint8_t* qa,
                                  const uint8_t* codes, int64_t count = 0, bool team = false) {
#define DLS_DEC_PART(TAG)                                                                                        \
  decode_part_##TAG(rc, g, bl, s, F, dims, desc, items, list, rank, qv_off, qa_off, code_off, vc, qv, qa, codes, \
                    count, team)
  if (wp == 16 && dtype == 0) return DLS_DEC_PART(w16_f32);
  if (wp == 16) return DLS_DEC_PART(w16_f64);
  if (dtype == 0) return DLS_DEC_PART(w32_f32);
  return DLS_DEC_PART(w32_f64);
#undef DLS_DEC_PART
}

hipError_t launch_decode(int wp, int dtype, void* F, const Dims& dims, const BlockDesc* desc,
                         const Item* items, int64_t nitems, const uint8_t* rank, const int64_t* qv_off,
                         const int64_t* qa_off, const int64_t* code_off, const VarConst* vc,
                         const uint8_t* qv, const uint8_t* qa, const uint8_t* codes, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  // one workgroup per slice, in dispatches of at most kDecodeLaunchItems
  // workgroups (a dispatch holds under 2^32 work-items)
  for (int64_t off = 0; off < nitems; off += kDecodeLaunchItems) {
    const int64_t n = std::min<int64_t>(nitems - off, kDecodeLaunchItems);
    const hipError_t e = decode_dispatch(wp, dtype, -1, dim3{unsigned(n)}, dim3{256}, s, F, dims, desc, items + off,
                                         nullptr, rank, qv_off, qa_off, code_off, vc, qv, qa, codes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_decode_class(int wp, int dtype, int rc, bool small, const int32_t* list, int64_t count, void* F,
                               const Dims& dims, const BlockDesc* desc, const Item* items, const uint8_t* rank,
                               const int64_t* qv_off, const int64_t* qa_off, const int64_t* code_off,
                               const VarConst* vc, const uint8_t* qv, const uint8_t* qa, const uint8_t* codes,
                               hipStream_t s) {
  if (count == 0) return hipSuccess;
  // small slices: 16-lane teams, sixteen slices per workgroup, where a team
  // covers the class's slices in one pass (FP32 at W <= 16: 64 points), as
  // the encode does; otherwise one wave per small slice
  const bool team = small && wp == 16 && dtype == 0;
  for (int64_t off = 0; off < count; off += kDecodeLaunchItems) {
    const int64_t n = std::min<int64_t>(count - off, kDecodeLaunchItems);
    const hipError_t e = decode_dispatch(wp, dtype, rc, dim3{unsigned(n)}, dim3{small ? 64u : 256u}, s, F, dims,
                                         desc, items, list + off, rank, qv_off, qa_off, code_off, vc, qv, qa, codes,
                                         n, team);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_scatter_keys(int dtype, void* F, const Dims& dims, const BlockDesc* desc, const uint64_t* key,
                              const uint64_t* bits, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 g{unsigned((n + 255) / 256)}, bl{256};
  if (dtype == 0) hipLaunchKernelGGL(k_scatter_keys<float>, g, bl, 0, s, (float*)F, dims, desc, key, bits, n);
  else hipLaunchKernelGGL(k_scatter_keys<double>, g, bl, 0, s, (double*)F, dims, desc, key, bits, n);
  return hipGetLastError();
}

hipError_t launch_scatter(int dtype, void* F, const int64_t* idx, const uint64_t* bits, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 g{unsigned((n + 255) / 256)}, bl{256};
  if (dtype == 0) hipLaunchKernelGGL(k_scatter<float>, g, bl, 0, s, (float*)F, idx, bits, n);
  else hipLaunchKernelGGL(k_scatter<double>, g, bl, 0, s, (double*)F, idx, bits, n);
  return hipGetLastError();
}

}  // namespace dls
