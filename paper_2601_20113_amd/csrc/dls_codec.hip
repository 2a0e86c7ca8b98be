// Encode and decode kernels of one (padded window, element type) pair.
//
// The build compiles this file once per pair and part, with
//   DLS_CODEC_WP    16 or 32 (padded window)
//   DLS_CODEC_T     float or double
//   DLS_CODEC_PPT   points per thread of the large-slice encode
//   DLS_CODEC_TAG   w16_f32, w16_f64, w32_f32 or w32_f64 (entry point names)
//   DLS_CODEC_PART  0: large-slice encode, 1: small-slice encode, 2: decode,
//                   3: the fused single-pass encode (W <= 16, FP32 only)
// so that the rank-class instantiations compile in parallel.
//
//   k_encode  projection A = X^T V_r (Eq. (5)), coefficient and basis
//             quantization, exact integer-lattice reconstruction in FP64 and
//             the residual codes that enforce the absolute bound, with escapes.
//   k_decode  Alg. 2: lattice values from (qV, qA, codes) and scatter, Eq. (7).
//   k_fused   one pass over the field for plans of large blocks: every
//             slice is read once into registers, its Gram formed on the
//             matrix cores, the block's eigenproblem solved by the slice that
//             completes it (rank-1 power iteration with the exact acceptance
//             test of the rank rule), and the slice encoded from registers.
//
// Compiled with -ffp-contract=off: the lattice arithmetic must round exactly
// as written so that the decoder reproduces the encoder bit for bit.
#ifndef DLS_CODEC_TAG
#define DLS_CODEC_WP 16
#define DLS_CODEC_T float
#define DLS_CODEC_PPT 4
#define DLS_CODEC_TAG w16_f32
#define DLS_CODEC_PART 0
#endif
#define DLS_CODEC_CAT2(a, b) a##_##b
#define DLS_CODEC_CAT(a, b) DLS_CODEC_CAT2(a, b)
#define DLS_CODEC_FN(name) DLS_CODEC_CAT(name, DLS_CODEC_TAG)

#include <hip/hip_runtime.h>

#include <algorithm>

#include "dls_device.h"
#include "dls_kernels.h"

namespace dls {
namespace {

// ---------------------------------------------------------------------------
// Encode: projection, quantization, lattice reconstruction, residual codes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t zigzag32(int32_t v) {
  return (uint32_t(v) << 1) ^ uint32_t(v >> 31);
}
__device__ __forceinline__ int32_t unzigzag32(uint32_t z) {
  return int32_t(z >> 1) ^ -int32_t(z & 1);
}

template <typename T>
__device__ __forceinline__ uint64_t bits_of(T v);
template <>
__device__ __forceinline__ uint64_t bits_of<float>(float v) { return uint64_t(__float_as_uint(v)); }
template <>
__device__ __forceinline__ uint64_t bits_of<double>(double v) { return uint64_t(__double_as_longlong(v)); }

template <int PPT>
__device__ __forceinline__ void store_bytes(uint8_t* __restrict__ dst, const uint32_t* bytes, int valid, bool vec) {
  if (vec && valid == PPT) {
    if (PPT == 4) {
      *reinterpret_cast<uint32_t*>(dst) = bytes[0] | (bytes[1] << 8) | (bytes[2] << 16) | (bytes[3] << 24);
    } else if (PPT == 2) {
      *reinterpret_cast<uint16_t*>(dst) = uint16_t(bytes[0] | (bytes[1] << 8));
    } else {
      dst[0] = uint8_t(bytes[0]);
    }
  } else {
    for (int e = 0; e < valid; ++e) dst[e] = uint8_t(bytes[e]);
  }
}

// RMAX is the rank class of the launch (every block in it has r <= RMAX), so
// the per-point coefficient registers are sized for the class, not for W.
// One slice, encoded by a team of TEAM threads (the workgroup, 256, or, for
// small slices, part of one wavefront: SmallTeam lanes, at most
// SmallTeam * PPT points); `tid` < TEAM.
template <int WP, typename T>
constexpr int SmallTeam = (WP == 16 && sizeof(T) == 4) ? 16 : 64;

template <int TEAM>
__device__ __forceinline__ void team_sync() {
  if constexpr (TEAM <= 64) wave_sync();  // the team's lanes are in one wavefront
  else __syncthreads();
}

// Loads the values of PPT consecutive slice points (slice-relative first
// point ps0, `valid` of them in the slice) for every step of the window:
// x[t][e], zero for t >= W_b and for invalid points.
template <int WP, typename T, int PPT>
__device__ __forceinline__ void load_slice_values(const T* __restrict__ F, const Dims& dims, const BlockDesc& d,
                                                  const Item& it, int ps0, int valid, T (&x)[WP][PPT]) {
  const int W = d.w();
  const int p = it.p0 + ps0;
  const int px = d.px(), py = d.py();
  const int64_t nxy = dims.nx * dims.ny;
  const T* base = F + fidx(dims, d.var, d.t0, d.z0, d.y0, d.x0);
  const int64_t tstride = dims.nz * nxy;
  int64_t poff[PPT];
#pragma unroll
  for (int e = 0; e < PPT; ++e) poff[e] = point_off(p + (e < valid ? e : 0), px, py, dims.nx, nxy);
  const bool vec = d.vec != 0;
#pragma unroll
  for (int t = 0; t < WP; ++t) {
    if (t < W) {
      const T* row = base + int64_t(t) * tstride;
      if (vec && valid == PPT) {
        if constexpr (sizeof(T) == 4 && PPT == 4) {
          float4 a = *reinterpret_cast<const float4*>(row + poff[0]);
          x[t][0] = a.x; x[t][1] = a.y; x[t][2] = a.z; x[t][3] = a.w;
        } else if constexpr (sizeof(T) == 4 && PPT == 2) {
          float2 a = *reinterpret_cast<const float2*>(row + poff[0]);
          x[t][0] = a.x; x[t][1] = a.y;
        } else {
#pragma unroll
          for (int e = 0; e < PPT; e += 2) {
            double2 a = *reinterpret_cast<const double2*>(row + poff[0] + e);
            x[t][e] = T(a.x); x[t][e + 1] = T(a.y);
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < PPT; ++e) x[t][e] = (e < valid) ? row[poff[e]] : T(0);
      }
    } else {
#pragma unroll
      for (int e = 0; e < PPT; ++e) x[t][e] = T(0);
    }
  }
}

// Stages block b's basis (its first RMAX columns, rank r) in LDS for a team
// of TEAM threads: FP32 values for the projection, the quantized codes
// qV = rint(V 2^16) for the lattice; the block's first slice also writes the
// qV codes to the payload.  A team barrier must follow before the values
// are used.
template <int WP, int RMAX, int TEAM>
__device__ __forceinline__ void stage_basis(int tid, const Item& it, int b, const BlockDesc& d, int r,
                                            float (&Vf)[RMAX][WP], double (&Qv)[WP][RMAX],
                                            const double* __restrict__ basis, const int64_t* __restrict__ qv_off,
                                            uint8_t* __restrict__ qv_buf) {
  const int W = d.w();
  for (int idx = tid; idx < RMAX * WP; idx += TEAM) {
    const int k = idx / WP, t = idx % WP;
    const double v = basis[int64_t(b) * WP * WP + idx];
    const double qv = rint(v * 65536.0);
    Vf[k][t] = float(v);
    Qv[t][k] = qv;
    if (it.first && k < r && t < W) {
      const uint32_t z = zigzag32(int32_t(qv));
      const int64_t plane = pad16(int64_t(W) * r);
      uint8_t* dst = qv_buf + qv_off[b] + k * W + t;
#pragma unroll
      for (int j = 0; j < 4; ++j) dst[j * plane] = uint8_t(z >> (8 * j));
    }
  }
}

// Everything after the loads, for the PPT points of one thread of a team of
// TEAM threads (`tid` < TEAM) encoding block b's slice `it` at rank r: the
// basis is staged in LDS (and its quantized codes written by the block's
// first slice), then projection, quantization, lattice reconstruction and
// residual codes of x.
template <int WP, typename T, int PPT, int RMAX, int TEAM, bool STAGED = false>
__device__ __forceinline__ void encode_values(int tid, const Item& it, int b, const BlockDesc& d, int r,
                                              const VarConst& K, int ps0, int valid, const T (&x)[WP][PPT],
                                              float (&Vf)[RMAX][WP], double (&Qv)[WP][RMAX],
                                              const double* __restrict__ basis,
                                              const int64_t* __restrict__ qv_off,
                                              const int64_t* __restrict__ qa_off,
                                              const int64_t* __restrict__ code_off,
                                              uint8_t* __restrict__ qv_buf,
                                              uint8_t* __restrict__ qa_buf,
                                              uint8_t* __restrict__ codes,
                                              float* __restrict__ coef,
                                              const EscOut& esc, uint64_t key_mark = 0) {
  const int W = d.w(), M = d.m;
  const int p = it.p0 + ps0;
  const bool vec = d.vec != 0;
  if constexpr (!STAGED) {
    stage_basis<WP, RMAX, TEAM>(tid, it, b, d, r, Vf, Qv, basis, qv_off, qv_buf);
    team_sync<TEAM>();
  }
  if (valid == 0) return;

  const int64_t code_at = code_off[b] + int64_t(p);

  if (r == 0) {  // raw block: every point is an escape
#pragma unroll
    for (int t = 0; t < WP; ++t) {
      if (t >= W) continue;
      uint32_t ff[PPT];
#pragma unroll
      for (int e = 0; e < PPT; ++e) ff[e] = kEscCode;
      store_bytes<PPT>(codes + code_at + int64_t(t) * M, ff, valid, vec);
#pragma unroll
      for (int e = 0; e < PPT; ++e) {
        if (e >= valid) continue;
        const unsigned long long slot = atomicAdd(esc.count, 1ULL);
        if (slot < esc.cap) {
          esc.key[slot] = key_mark | (uint64_t(b) << 32) | uint64_t(uint32_t(t * M + p + e));
          esc.val[slot] = bits_of<T>(x[t][e]);
        }
      }
    }
    return;
  }

  // projection and coefficient quantization (FP32), row-wise overflow guard
  int32_t qa[RMAX][PPT];
  bool ovf[PPT];
#pragma unroll
  for (int e = 0; e < PPT; ++e) ovf[e] = false;
  const int64_t qa_plane = pad16(int64_t(M) * r);
#pragma unroll
  for (int k = 0; k < RMAX; ++k) {
    if (k >= r) continue;
    float a[PPT];
#pragma unroll
    for (int e = 0; e < PPT; ++e) a[e] = 0.f;
#pragma unroll
    for (int t = 0; t < WP; ++t) {
      if (t < W) {
        const float v = Vf[k][t];
#pragma unroll
        for (int e = 0; e < PPT; ++e) a[e] = fmaf(float(x[t][e]), v, a[e]);
      }
    }
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const float qf = rintf(a[e] * K.inv_eps_f);
      const bool ok = fabsf(qf) < 2147483648.0f;
      ovf[e] = ovf[e] || !ok;
      qa[k][e] = ok ? int32_t(qf) : 0;
    }
    if (coef != nullptr) {
#pragma unroll
      for (int e = 0; e < PPT; ++e)
        if (e < valid) coef[qa_off[b] / 4 + int64_t(k) * M + p + e] = a[e];
    }
  }
#pragma unroll
  for (int k = 0; k < RMAX; ++k) {
    if (k >= r) continue;
    uint32_t z[PPT];
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      if (ovf[e]) qa[k][e] = 0;
      z[e] = zigzag32(qa[k][e]);
    }
    uint8_t* dst = qa_buf + qa_off[b] + int64_t(k) * M + p;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t by[PPT];
#pragma unroll
      for (int e = 0; e < PPT; ++e) by[e] = (z[e] >> (8 * j)) & 0xFF;
      store_bytes<PPT>(dst + j * qa_plane, by, valid, vec);
    }
  }

  // lattice reconstruction (exact in FP64) and residual codes; the per-value
  // work is branch-free (selects), one rarely taken branch per step records
  // that step's escapes
  double qd[RMAX][PPT];
#pragma unroll
  for (int k = 0; k < RMAX; ++k)
#pragma unroll
    for (int e = 0; e < PPT; ++e) qd[k][e] = double(qa[k][e]);
#pragma unroll
  for (int t = 0; t < WP; ++t) {
    if (t >= W) continue;
    uint32_t cd[PPT];
    bool esc_pt[PPT];
    bool any = false;
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      double S = 0.0;
#pragma unroll
      for (int k = 0; k < RMAX; ++k)
        if (k < r) S = fma(Qv[t][k], qd[k][e], S);
      const double xv = double(x[t][e]);
      const double xhat = S * K.c;
      const double dlt = xv - xhat;
      const double q0 = rint(dlt * K.inv2eps);
      const bool big = fabs(q0) > double(kQLimit);
      const double q = big ? 0.0 : q0;
      const double n = fma(q, 131072.0, S);  // q 2^17 is exact: S + q 2^17 rounded once
      const T outv = T(n * K.c);
      esc_pt[e] = big || (fabs(xv - double(outv)) > K.eps);
      const int32_t qi = int32_t(q);
      cd[e] = esc_pt[e] ? uint32_t(kEscCode) : uint32_t((qi << 1) ^ (qi >> 31));  // zigzag, <= 254
      any = any || (esc_pt[e] && e < valid);
    }
    store_bytes<PPT>(codes + code_at + int64_t(t) * M, cd, valid, vec);
    if (any) {
#pragma unroll
      for (int e = 0; e < PPT; ++e) {
        if (!esc_pt[e] || e >= valid) continue;
        const unsigned long long slot = atomicAdd(esc.count, 1ULL);
        if (slot < esc.cap) {
          esc.key[slot] = key_mark | (uint64_t(b) << 32) | uint64_t(uint32_t(t * M + p + e));
          esc.val[slot] = bits_of<T>(x[t][e]);
        }
      }
    }
  }
}


template <int WP, typename T, int PPT, int RMAX, bool DEV, int TEAM>
__device__ __forceinline__ void encode_item(int64_t li, int tid, float (&Vf)[RMAX][WP], double (&Qv)[WP][RMAX],
                                            const T* __restrict__ F, const Dims& dims,
                                            const BlockDesc* __restrict__ desc,
                                            const Item* __restrict__ items,
                                            const int32_t* __restrict__ item_list,
                                            const uint8_t* __restrict__ rank,
                                            const double* __restrict__ basis,
                                            const int64_t* __restrict__ qv_off,
                                            const int64_t* __restrict__ qa_off,
                                            const int64_t* __restrict__ code_off,
                                            const VarConst* __restrict__ vc,
                                            uint8_t* __restrict__ qv_buf,
                                            uint8_t* __restrict__ qa_buf,
                                            uint8_t* __restrict__ codes,
                                            float* __restrict__ coef,
                                            const EscOut& esc, const EncodeWork& work) {
  const Item it = items[item_list[li]];
  const int b = it.block;
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m, r = rank[b];
  const VarConst K = vc[d.var];
  if constexpr (DEV) {  // host-driven launches size the buffers exactly
    if (qv_off[b] + 4 * pad16(int64_t(W) * r) > work.qv_cap || qa_off[b] + 4 * pad16(int64_t(M) * r) > work.qa_cap) {
      if (tid == 0) atomicOr(work.overflow, 1u);
      return;
    }
  }

  const int ps0 = tid * PPT;
  const int valid = ps0 >= it.np ? 0 : ((it.np - ps0) < PPT ? (it.np - ps0) : PPT);
  // the slice's values are loaded first, so that their latency overlaps the
  // basis staging
  T x[WP][PPT];
  load_slice_values<WP, T, PPT>(F, dims, d, it, ps0, valid, x);
  encode_values<WP, T, PPT, RMAX, TEAM>(tid, it, b, d, r, K, ps0, valid, x, Vf, Qv, basis, qv_off, qa_off, code_off,
                                        qv_buf, qa_buf, codes, coef, esc);
}

// DEV = false: host-driven, one item per workgroup; DEV = true:
// device-driven, the grid walks the *work.dcount items of the list
// SMALL: four slices per workgroup, one wavefront each (slices of at most
// 64 * PPT points); otherwise one slice per workgroup.
template <int WP, typename T, int PPT, int RMAX, bool DEV, bool SMALL>
__global__ __launch_bounds__(256) void k_encode(const T* __restrict__ F, Dims dims,
                                                const BlockDesc* __restrict__ desc,
                                                const Item* __restrict__ items,
                                                const int32_t* __restrict__ item_list,
                                                const uint8_t* __restrict__ rank,
                                                const double* __restrict__ basis,
                                                const int64_t* __restrict__ qv_off,
                                                const int64_t* __restrict__ qa_off,
                                                const int64_t* __restrict__ code_off,
                                                const VarConst* __restrict__ vc,
                                                uint8_t* __restrict__ qv_buf,
                                                uint8_t* __restrict__ qa_buf,
                                                uint8_t* __restrict__ codes,
                                                float* __restrict__ coef,
                                                EscOut esc, EncodeWork work) {
  constexpr int TEAM = SMALL ? SmallTeam<WP, T> : 256;
  constexpr int NTEAM = 256 / TEAM;
  __shared__ float Vf[NTEAM][RMAX][WP];    // [k][t]
  __shared__ double Qv[NTEAM][WP][RMAX];   // [t][k], integer valued
  const int team = int(threadIdx.x) / TEAM;
  const int tid = int(threadIdx.x) % TEAM;
  const int64_t first = int64_t(blockIdx.x) * NTEAM + team;
  if constexpr (!DEV) {
    if (SMALL && first >= work.count) return;  // a whole team leaves together
    encode_item<WP, T, PPT, RMAX, false, TEAM>(first, tid, Vf[team], Qv[team], F, dims, desc, items, item_list,
                                               rank, basis, qv_off, qa_off, code_off, vc, qv_buf, qa_buf, codes,
                                               coef, esc, work);
    return;
  }
  const int64_t nwork = int64_t(*work.dcount);
  for (int64_t li = first; li < nwork; li += int64_t(gridDim.x) * NTEAM) {
    if (li != first) team_sync<TEAM>();  // the previous slice's LDS reads are done
    encode_item<WP, T, PPT, RMAX, true, TEAM>(li, tid, Vf[team], Qv[team], F, dims, desc, items, item_list, rank,
                                              basis, qv_off, qa_off, code_off, vc, qv_buf, qa_buf, codes, coef, esc,
                                              work);
  }
}

// ---------------------------------------------------------------------------
// Decode (Alg. 2): lattice values of every point, scattered into the field
// (Eq. (7)); an escaped point gets the value of q = 0 here and is overwritten
// by the escape scatter (k_scatter or k_scatter_keys) that follows.
// ---------------------------------------------------------------------------
// RMAX bounds the rank of every block of the launch (a rank class, or WP).
// TEAM = 0: one workgroup per slice; TEAM = 16: sixteen 16-lane teams per
// 256-thread workgroup, one slice each (slices of at most 16 PPT points),
// entries blockIdx.x * 16 + team of the list, up to count.
template <int WP, typename T, int RMAX, int TEAM>
__global__ __launch_bounds__(256) void k_decode(T* __restrict__ F, Dims dims,
                                                const BlockDesc* __restrict__ desc,
                                                const Item* __restrict__ items,
                                                const int32_t* __restrict__ list,
                                                const uint8_t* __restrict__ rank,
                                                const int64_t* __restrict__ qv_off,
                                                const int64_t* __restrict__ qa_off,
                                                const int64_t* __restrict__ code_off,
                                                const VarConst* __restrict__ vc,
                                                const uint8_t* __restrict__ qv_buf,
                                                const uint8_t* __restrict__ qa_buf,
                                                const uint8_t* __restrict__ codes, int64_t count) {
  // PPT consecutive points per thread: 4-byte code and coefficient-plane
  // loads and 16-byte (FP32) stores for 4-aligned patch rows
  constexpr int PPT = WP == 16 ? 4 : 2;
  constexpr int NT = TEAM ? 256 / TEAM : 1;     // slices per workgroup
  constexpr int LANES = TEAM ? TEAM : 256;     // threads per slice
  __shared__ double Qv_all[NT][WP][RMAX];      // [t][k] per slice
  const int team = TEAM ? int(threadIdx.x) / TEAM : 0;
  const int tl = TEAM ? int(threadIdx.x) % TEAM : int(threadIdx.x);
  const int64_t entry = TEAM ? int64_t(blockIdx.x) * NT + team : int64_t(blockIdx.x);
  const bool live = !TEAM || entry < count;
  const Item it = items[list ? list[live ? entry : 0] : int32_t(live ? entry : 0)];
  const int b = it.block;
  const BlockDesc d = desc[b];
  const int W = d.w(), M = d.m, r = rank[b];
  const VarConst K = vc[d.var];
  const int64_t vplane = pad16(int64_t(W) * r);
  auto& Qv = Qv_all[team];
  for (int idx = tl; idx < WP * RMAX; idx += LANES) {
    const int k = idx / WP, t = idx % WP;
    double v = 0.0;
    if (k < r && t < W) {
      const uint8_t* src = qv_buf + qv_off[b] + k * W + t;
      const uint32_t z = uint32_t(src[0]) | (uint32_t(src[vplane]) << 8) |
                         (uint32_t(src[2 * vplane]) << 16) | (uint32_t(src[3 * vplane]) << 24);
      v = double(unzigzag32(z));
    }
    Qv[t][k] = v;
  }
  __syncthreads();
  if (!live) return;
  const int64_t aplane = pad16(int64_t(M) * r);
  const int64_t nxy = dims.nx * dims.ny;
  T* base = F + fidx(dims, d.var, d.t0, d.z0, d.y0, d.x0);
  const int64_t tstride = dims.nz * nxy;
  const bool vec = d.vec != 0;
  for (int ps0 = tl * PPT; ps0 < it.np; ps0 += LANES * PPT) {
    const int valid = (it.np - ps0) < PPT ? (it.np - ps0) : PPT;
    const bool full = vec && valid == PPT;
    const int p = it.p0 + ps0;
    // coefficients of the PPT points: zigzag codes gathered one byte plane at
    // a time, then decoded in place
    int32_t qa[RMAX][PPT];
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
      uint32_t za[PPT];
#pragma unroll
      for (int e = 0; e < PPT; ++e) za[e] = 0u;
      if (k < r) {
        const uint8_t* src = qa_buf + qa_off[b] + int64_t(k) * M + p;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          uint32_t by[PPT];
          if (full && PPT == 4) {
            const uint32_t w4 = *reinterpret_cast<const uint32_t*>(src + j * aplane);
#pragma unroll
            for (int e = 0; e < PPT; ++e) by[e] = (w4 >> (8 * e)) & 0xFFu;
          } else {
#pragma unroll
            for (int e = 0; e < PPT; ++e) by[e] = e < valid ? uint32_t(src[j * aplane + e]) : 0u;
          }
#pragma unroll
          for (int e = 0; e < PPT; ++e) za[e] |= by[e] << (8 * j);
        }
      }
#pragma unroll
      for (int e = 0; e < PPT; ++e) qa[k][e] = unzigzag32(za[e]);
    }
    int64_t off[PPT];
#pragma unroll
    for (int e = 0; e < PPT; ++e) off[e] = point_off(p + (e < valid ? e : 0), d.px(), d.py(), dims.nx, nxy);
    // the residual codes of every step, all loads issued before any use:
    // byte e of cw[t] is the code of point p + e at step t
    uint32_t cw[WP];
#pragma unroll
    for (int t = 0; t < WP; ++t) {
      cw[t] = 0xFFFFFFFFu;
      if (t < W) {
        const uint8_t* cp = codes + code_off[b] + int64_t(t) * M + p;
        if (full && PPT == 4) {
          cw[t] = *reinterpret_cast<const uint32_t*>(cp);
        } else {
#pragma unroll
          for (int e = 0; e < PPT; ++e)
            if (e < valid) cw[t] = (cw[t] & ~(0xFFu << (8 * e))) | (uint32_t(cp[e]) << (8 * e));
        }
      }
    }
#pragma unroll
    for (int t = 0; t < WP; ++t) {
      if (t >= W) continue;
      uint32_t cd[PPT];
#pragma unroll
      for (int e = 0; e < PPT; ++e) cd[e] = (cw[t] >> (8 * e)) & 0xFFu;
      T outv[PPT];
#pragma unroll
      for (int e = 0; e < PPT; ++e) {
        double S = 0.0;
#pragma unroll
        for (int k = 0; k < RMAX; ++k)
          if (k < r) S = fma(Qv[t][k], double(qa[k][e]), S);
        // escaped points get the lattice value with q = 0 here; the escape
        // scatter that follows overwrites them
        const uint32_t code = cd[e] == kEscCode ? 0u : cd[e];
        const int32_t q = int32_t(code >> 1) ^ -int32_t(code & 1);
        outv[e] = T((S + double(q) * 131072.0) * K.c);
      }
      T* row = base + int64_t(t) * tstride;
      if (full) {
        if constexpr (sizeof(T) == 4 && PPT == 4) {
          *reinterpret_cast<float4*>(row + off[0]) = make_float4(outv[0], outv[1], outv[2], outv[3]);
        } else {
#pragma unroll
          for (int e = 0; e < PPT; ++e) row[off[0] + e] = outv[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < PPT; ++e)
          if (e < valid) row[off[e]] = outv[e];
      }
    }
  }
}

template <int WP, typename T, int PPT, bool SMALL>
void encode_class(int rc, const dim3& g, hipStream_t s, const T* F, const Dims& dims,
                         const BlockDesc* desc, const Item* items, const int32_t* list, const uint8_t* rank,
                         const double* basis, const int64_t* qv_off, const int64_t* qa_off,
                         const int64_t* code_off, const VarConst* vc, uint8_t* qv, uint8_t* qa,
                         uint8_t* codes, float* coef, EscOut esc, const EncodeWork& work) {
  const dim3 bl{256};
#define DLS_ENC(R)                                                                                          \
  do {                                                                                                      \
    if (work.dcount)                                                                                        \
      hipLaunchKernelGGL((k_encode<WP, T, PPT, R, true, SMALL>), g, bl, 0, s, F, dims, desc, items, list,  \
                         rank, basis, qv_off, qa_off, code_off, vc, qv, qa, codes, coef, esc, work);        \
    else                                                                                                    \
      hipLaunchKernelGGL((k_encode<WP, T, PPT, R, false, SMALL>), g, bl, 0, s, F, dims, desc, items, list, \
                         rank, basis, qv_off, qa_off, code_off, vc, qv, qa, codes, coef, esc, work);        \
  } while (0)
  switch (rc) {
    case 0: DLS_ENC(1); break;
    case 1: DLS_ENC(2); break;
    case 2: DLS_ENC(4); break;
    case 3: DLS_ENC(8); break;
    case 4: DLS_ENC(16); break;
    default:
      if constexpr (WP == 32) DLS_ENC(32);
      break;
  }
#undef DLS_ENC
}

// bl: threads per slice (one workgroup each); 64 for the small-slice classes
template <int WP, typename T, int RMAX>
void decode_launch(const dim3& g, const dim3& bl, hipStream_t s, void* F, const Dims& dims,
                          const BlockDesc* desc, const Item* items, const int32_t* list, const uint8_t* rank,
                          const int64_t* qv_off, const int64_t* qa_off, const int64_t* code_off, const VarConst* vc,
                          const uint8_t* qv, const uint8_t* qa, const uint8_t* codes, int64_t count, bool team) {
  if (team) {
    const dim3 gt{unsigned((count + 15) / 16)};
    hipLaunchKernelGGL((k_decode<WP, T, RMAX, 16>), gt, dim3{256}, 0, s, (T*)F, dims, desc, items, list, rank,
                       qv_off, qa_off, code_off, vc, qv, qa, codes, count);
  } else {
    hipLaunchKernelGGL((k_decode<WP, T, RMAX, 0>), g, bl, 0, s, (T*)F, dims, desc, items, list, rank, qv_off,
                       qa_off, code_off, vc, qv, qa, codes, count);
  }
}

#if DLS_CODEC_PART == 3
// ---------------------------------------------------------------------------
// Single-pass encode (reading R28), two kernels:
//
// k_sketch_basis: per block, the rank-1 basis q of its sketch -- the Gram
//   partial of its first slice (the first whole x-rows, at most 1024 points),
//   formed beforehand by k_gram -- by power iteration from the column of the
//   largest diagonal entry; q becomes column 0 of the block's basis, the
//   block's payload regions are the rank-1 ones at their static offsets.
// k_fused: slice i = blockIdx.x (one workgroup per slice: hardware dispatch
//   keeps the slices in flight contiguous, and nothing computed before the
//   slice's work has to stay live across a loop).
//   Every slice is read once into registers, its Gram partial
//   is formed on the matrix cores (FP32 or bf16 operands, FP64 across
//   64-point chunks) and stored, and the slice is encoded at rank 1 with its
//   block's q (the residual codes keep the pointwise bound for any
//   orthonormal basis).  No workgroup waits for another.
// k_verify: per block, the sum of its slices' partials in slice order (as
//   k_eigen forms it) and the test of q on the whole Gram: trace(G) -
//   q^T G q is the exact discarded energy of q, so when it is <= tau the
//   rank rule of Sec. 2.4 Eq. (4) picks rank 1 and the encode stands;
//   otherwise the block is deferred: the two-pass path solves it by Jacobi
//   and encodes it again (its escapes from the single pass carry a mark and
//   are dropped afterwards).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sketch_basis(const double* __restrict__ gpart,
                                                      const int32_t* __restrict__ item_start,
                                                      const Item* __restrict__ items,
                                                      const BlockDesc* __restrict__ desc, int64_t nblocks,
                                                      const double* __restrict__ eps_v,
                                                      const int64_t* __restrict__ r1_off, uint8_t* __restrict__ rank,
                                                      double* __restrict__ lam, double* __restrict__ basis,
                                                      int64_t* __restrict__ qv_size, int64_t* __restrict__ qa_size,
                                                      int64_t* __restrict__ qv_off, int64_t* __restrict__ qa_off,
                                                      unsigned int* __restrict__ state,
                                                      unsigned long long* __restrict__ counters) {
  constexpr int WP = 16;
  __shared__ double sG[16][WP][WP + 1];
  __shared__ double sq[16][WP];
  const int grp = int(threadIdx.x) / WP, row = int(threadIdx.x) % WP;
  const int64_t b = int64_t(blockIdx.x) * 16 + grp;
  if (b >= nblocks) return;  // the whole 16-lane group leaves together
  const BlockDesc d = desc[b];
  const double* gp = gpart + int64_t(item_start[b]) * WP * WP + row * WP;
  double a[WP];
#pragma unroll
  for (int j = 0; j < WP; ++j) {
    a[j] = gp[j];
    sG[grp][row][j] = a[j];
  }
  wave_sync();
  bool fin = true;
#pragma unroll
  for (int j = 0; j < WP; ++j) {
    a[j] = 0.5 * (a[j] + sG[grp][j][row]);
    fin = fin && isfinite(a[j]);
  }
  wave_sync();
#pragma unroll
  for (int j = 0; j < WP; ++j) sG[grp][row][j] = a[j];
  wave_sync();
  fin = row_sum(fin ? 0.0 : 1.0) == 0.0;
  double qi = row == 0 ? 1.0 : 0.0;
  bool pruned = false, likely = true;
  if (fin) {
    int istar = 0;
    double best = sG[grp][0][0];
    for (int j = 1; j < WP; ++j)
      if (sG[grp][j][j] > best) { best = sG[grp][j][j]; istar = j; }
    qi = sG[grp][row][istar];
    double n2 = row_sum(qi * qi);
    if (n2 > 0.0) qi = qi / sqrt(n2);
    else qi = row == istar ? 1.0 : 0.0;
    for (int k = 0; k < kFusedIters; ++k) {
      sq[grp][row] = qi;
      wave_sync();
      double y = 0.0;
#pragma unroll
      for (int j = 0; j < WP; ++j) y = fma(a[j], sq[grp][j], y);
      wave_sync();
      n2 = row_sum(y * y);
      if (n2 > 0.0) qi = y / sqrt(n2);
    }
    // canonical sign: the largest |q_t| positive, the lowest t on a tie
    sq[grp][row] = qi;
    wave_sync();
    double bq = -1.0, sg = 1.0;
    for (int j = 0; j < WP; ++j)
      if (fabs(sq[grp][j]) > bq) { bq = fabs(sq[grp][j]); sg = sq[grp][j] < 0.0 ? -1.0 : 1.0; }
    qi *= sg;
    // the sketch's discarded energy under q, E_s = trace(G_s) - q^T G_s q,
    // is a lower bound of the whole block's (the other points add a PSD
    // Gram), so E_s > tau (by a margin over the FP32 accumulation error of
    // G_s) rules rank 1 out; E_s scaled to the block's points predicts it
    double y = 0.0, di = 0.0;
#pragma unroll
    for (int j = 0; j < WP; ++j) {
      y = fma(a[j], sq[grp][j], y);  // G_s q, q as staged (before the sign)
      di = j == row ? a[j] : di;
    }
    const double tr = row_sum(di);
    const double es = tr - row_sum(sq[grp][row] * y);
    const double eps = eps_v[d.var];
    const double tau = kKappa * eps * eps * double(d.m) * double(d.w());
    const int ms = items[item_start[b]].np;
    pruned = es > 2.0 * tau + 1e-4 * tr;
    likely = es * double(d.m) > tau * double(ms);
  }
  double* bb = basis + b * WP * WP;
  bb[row] = qi;  // column 0 at [0][t]; the other columns are not formed
#pragma unroll
  for (int k = 1; k < WP; ++k) bb[k * WP + row] = 0.0;
  lam[b * WP + row] = 0.0;
  if (row == 0) {
    rank[b] = 1;
    qv_size[b] = 4 * pad16(int64_t(d.w()));
    qa_size[b] = 4 * pad16(int64_t(d.m));
    qv_off[b] = r1_off[b];
    qa_off[b] = r1_off[nblocks + b];
    state[b] = fin && !pruned ? 0u : 3u;  // 3: the block is left to the two-pass path
  }
  // one atomic per wavefront for each count
  const uint64_t lk = __ballot(row == 0 && likely), pr = __ballot(row == 0 && fin && pruned);
  const int lane = int(threadIdx.x & 63);
  if (lane == __ffsll((unsigned long long)__ballot(1)) - 1) {
    if (lk) atomicAdd(counters + kFusedLikely, (unsigned long long)__popcll(lk));
    if (pr) atomicAdd(counters + kFusedPruned, (unsigned long long)__popcll(pr));
  }
}

template <bool BF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_fused(const float* __restrict__ F, Dims dims,
                                               const BlockDesc* __restrict__ desc,
                                               const Item* __restrict__ items, int64_t nitems,
                                               const VarConst* __restrict__ vc, double* __restrict__ gpart,
                                               const unsigned int* __restrict__ state,
                                               const double* __restrict__ basis,
                                               const int64_t* __restrict__ qv_off, const int64_t* __restrict__ qa_off,
                                               const int64_t* __restrict__ code_off, uint8_t* __restrict__ qv_buf,
                                               uint8_t* __restrict__ qa_buf, uint8_t* __restrict__ codes,
                                               float* __restrict__ coef, EscOut esc) {
  constexpr int WP = 16, PPT = 4, LDR = 68;
  __shared__ __align__(16) float stage[4][WP * LDR];
  __shared__ double red[4][4][64];
  __shared__ float Vf[1][WP];
  __shared__ double Qv[WP][1];
  const int tid = int(threadIdx.x), lane = tid & 63, wave = tid >> 6;
  const int tl = lane & 15, q = lane >> 4;
  constexpr uint64_t kSpeculative = uint64_t(1) << 63;
  {
    const int64_t i = blockIdx.x;  // one slice per workgroup (the grid covers every slice)
    if (i >= nitems) return;
    const Item it = items[i];
    const int b = it.block;
    const BlockDesc d = desc[b];
    const unsigned st_b = state[b];  // from k_sketch_basis: 0 usable basis, 3 none
    // thread tid: slice points 4 tid .. 4 tid + 3 (wavefront w: chunks of 64
    // points 4 w .. 4 w + 3), so every step's codes are stored as 256
    // contiguous bytes per wavefront
    const int ps0 = PPT * tid;
    const int valid = ps0 >= it.np ? 0 : ((it.np - ps0) < PPT ? (it.np - ps0) : PPT);
    float x[WP][PPT];
    load_slice_values<WP, float, PPT>(F, dims, d, it, ps0, valid, x);
    // the block's sketch basis, staged while the field loads are in flight
    // (the Gram's barriers below publish it)
    if (st_b == 0u) stage_basis<WP, 1, 256>(tid, it, b, d, 1, Vf, Qv, basis, qv_off, qv_buf);

    // Gram partial of the slice: per 64-point chunk one MFMA accumulation
    // (operands staged through LDS), flushed to FP64 in chunk order
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    float* st = stage[wave];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if ((4 * wave + u) * 64 >= it.np) continue;
      if (q == u) {
#pragma unroll
        for (int t = 0; t < WP; ++t)
          *reinterpret_cast<float4*>(st + t * LDR + 4 * tl) = make_float4(x[t][0], x[t][1], x[t][2], x[t][3]);
      }
      wave_sync();
      float v0[16];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float4 a = *reinterpret_cast<const float4*>(st + tl * LDR + 16 * j + 4 * q);
        v0[4 * j] = a.x; v0[4 * j + 1] = a.y; v0[4 * j + 2] = a.z; v0[4 * j + 3] = a.w;
      }
      wave_sync();
      f32x4 a00 = {0.f, 0.f, 0.f, 0.f};
      if constexpr (BF) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bf16x4 b0 = to_bf16x4(v0 + 4 * j);
          a00 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b0, b0, a00, 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) a00 = __builtin_amdgcn_mfma_f32_16x16x4f32(v0[s2], v0[s2], a00, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] += double(a00[v]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][v][lane] = acc[v];
    __syncthreads();
    if (wave == 0) {
      double* out = gpart + i * WP * WP;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(4 * q + v) * WP + tl] = ((red[0][v][lane] + red[1][v][lane]) + red[2][v][lane]) + red[3][v][lane];
    }
    // the slice encoded at rank 1 with its block's sketch basis (the
    // constants copied to registers: a reference into global memory would be
    // reloaded after every store the encode makes)
    const VarConst K = vc[d.var];
    if (st_b == 0u)
      encode_values<WP, float, PPT, 1, 256, true>(tid, it, b, d, 1, K, ps0, valid, x, Vf, Qv, basis, qv_off,
                                                  qa_off, code_off, qv_buf, qa_buf, codes, coef, esc, kSpeculative);
  }
}

// Verification of the sketch bases: 16 lanes per block (lane = row of the
// Gram), 16 blocks per workgroup.
__global__ __launch_bounds__(256) void k_verify(const double* __restrict__ gpart,
                                                const int32_t* __restrict__ item_start,
                                                const BlockDesc* __restrict__ desc, int64_t nblocks,
                                                const double* __restrict__ eps_v, const double* __restrict__ basis,
                                                double* __restrict__ lam, FusedState fs) {
  constexpr int WP = 16;
  __shared__ double sA[16][WP][WP + 1];
  __shared__ double sq[16][WP];
  const int grp = int(threadIdx.x) / WP, row = int(threadIdx.x) % WP;
  const int64_t b = int64_t(blockIdx.x) * 16 + grp;
  if (b >= nblocks) return;  // the whole 16-lane group leaves together
  const BlockDesc d = desc[b];
  const int i0 = item_start[b], i1 = item_start[b + 1];
  double a[WP];
#pragma unroll
  for (int j = 0; j < WP; ++j) a[j] = 0.0;
  for (int s2 = i0; s2 < i1; ++s2) {  // every entry's loads of a slice issued together
    const double* gp = gpart + int64_t(s2) * WP * WP + row * WP;
#pragma unroll
    for (int j = 0; j < WP; ++j) a[j] += gp[j];
  }
#pragma unroll
  for (int j = 0; j < WP; ++j) sA[grp][row][j] = a[j];
  wave_sync();
  bool fin = true;
#pragma unroll
  for (int j = 0; j < WP; ++j) {
    a[j] = 0.5 * (a[j] + sA[grp][j][row]);
    fin = fin && isfinite(a[j]);
  }
  fin = row_sum(fin ? 0.0 : 1.0) == 0.0;
  const unsigned st_b = fs.state[b];
  bool accept = false;
  double theta = 0.0;
  if (fin && st_b == 0u) {
    const double qi = basis[b * WP * WP + row];
    sq[grp][row] = qi;
    wave_sync();
    double y = 0.0, di = 0.0;
#pragma unroll
    for (int j = 0; j < WP; ++j) {
      y = fma(a[j], sq[grp][j], y);
      di = j == row ? a[j] : di;
    }
    theta = row_sum(qi * y);
    const double tr = row_sum(di);
    const double eps = eps_v[d.var];
    const double tau = kKappa * eps * eps * double(d.m) * double(d.w());
    accept = (tr - theta) <= tau;
  }
  if (row == 0) {
    if (accept) {
      lam[b * WP] = theta;
      fs.state[b] = 1u;
      atomicAdd(fs.counters + kFusedAccepted, 1ULL);
    } else {
      fs.state[b] = 2u;
      const unsigned slot = atomicAdd(fs.ndeferred, 1u);
      fs.deferred[slot] = int32_t(b);
    }
  }
}

// Escapes written by k_fused (marked) for blocks it deferred are dropped:
// their keys become ~0 (sorted last, skipped by the scatter) and are
// counted; the marks of the blocks it kept are cleared.
__global__ __launch_bounds__(256) void k_fix_escapes(uint64_t* __restrict__ key, const unsigned long long* count,
                                                     unsigned long long cap, const unsigned int* __restrict__ state,
                                                     unsigned long long* __restrict__ ndropped) {
  const unsigned long long n = *count < cap ? *count : cap;
  for (unsigned long long i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += uint64_t(gridDim.x) * 256) {
    const uint64_t k = key[i];
    if (!(k >> 63)) continue;
    const uint64_t b = (k >> 32) & 0x7FFFFFFFu;
    if (state[b] == 1u) {
      key[i] = k & ~(uint64_t(1) << 63);
    } else {
      key[i] = ~uint64_t(0);
      atomicAdd(ndropped, 1ULL);
    }
  }
}
#endif

}  // namespace

#if DLS_CODEC_PART == 0
#define DLS_CODEC_SMALL false
#define DLS_CODEC_ENTRY encode_large
#elif DLS_CODEC_PART == 1
#define DLS_CODEC_SMALL true
#define DLS_CODEC_ENTRY encode_small
#endif

#if DLS_CODEC_PART == 3
hipError_t launch_sketch_basis(const double* gpart, const int32_t* item_start, const Item* items,
                               const BlockDesc* desc, int64_t nblocks, const double* eps_v, const int64_t* r1_off,
                               uint8_t* rank, double* lam, double* basis, int64_t* qv_size, int64_t* qa_size,
                               int64_t* qv_off, int64_t* qa_off, unsigned int* state, unsigned long long* counters,
                               hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sketch_basis, dim3{unsigned((nblocks + 15) / 16)}, dim3{256}, 0, s, gpart, item_start, items,
                     desc, nblocks, eps_v, r1_off, rank, lam, basis, qv_size, qa_size, qv_off, qa_off, state,
                     counters);
  return hipGetLastError();
}

hipError_t launch_fused(bool bf16, const float* F, const Dims& dims, const BlockDesc* desc,
                        const Item* items, int64_t nitems, const VarConst* vc, double* gpart,
                        const unsigned int* state, const double* basis, const int64_t* qv_off, const int64_t* qa_off,
                        const int64_t* code_off, uint8_t* qv, uint8_t* qa, uint8_t* codes, float* coef, EscOut esc,
                        hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  if (nitems > int64_t(INT32_MAX)) return hipErrorInvalidValue;  // one workgroup per slice
  const dim3 g{unsigned(nitems)}, bl{256};
  if (bf16)
    hipLaunchKernelGGL(k_fused<true>, g, bl, 0, s, F, dims, desc, items, nitems, vc, gpart, state, basis, qv_off,
                       qa_off, code_off, qv, qa, codes, coef, esc);
  else
    hipLaunchKernelGGL(k_fused<false>, g, bl, 0, s, F, dims, desc, items, nitems, vc, gpart, state, basis, qv_off,
                       qa_off, code_off, qv, qa, codes, coef, esc);
  return hipGetLastError();
}

hipError_t launch_verify(const double* gpart, const int32_t* item_start, const BlockDesc* desc, int64_t nblocks,
                         const double* eps_v, const double* basis, double* lam, const FusedState& fs, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_verify, dim3{unsigned((nblocks + 15) / 16)}, dim3{256}, 0, s, gpart, item_start, desc, nblocks,
                     eps_v, basis, lam, fs);
  return hipGetLastError();
}

hipError_t launch_fix_escapes(uint64_t* key, const unsigned long long* count, unsigned long long cap,
                              const unsigned int* state, unsigned long long* ndropped, hipStream_t s) {
  hipLaunchKernelGGL(k_fix_escapes, dim3{256}, dim3{256}, 0, s, key, count, cap, state, ndropped);
  return hipGetLastError();
}
#endif

#if DLS_CODEC_PART == 0 || DLS_CODEC_PART == 1
hipError_t DLS_CODEC_FN(DLS_CODEC_ENTRY)(int rc, const dim3& g, hipStream_t s, const void* F, const Dims& dims,
                                         const BlockDesc* desc, const Item* items, const int32_t* list,
                                         const uint8_t* rank, const double* basis, const int64_t* qv_off,
                                         const int64_t* qa_off, const int64_t* code_off, const VarConst* vc,
                                         uint8_t* qv, uint8_t* qa, uint8_t* codes, float* coef, EscOut esc,
                                         const EncodeWork& work) {
  using T = DLS_CODEC_T;
  constexpr int WP = DLS_CODEC_WP, PPT = DLS_CODEC_PPT;
  encode_class<WP, T, PPT, DLS_CODEC_SMALL>(rc, g, s, (const T*)F, dims, desc, items, list, rank, basis, qv_off,
                                            qa_off, code_off, vc, qv, qa, codes, coef, esc, work);
  return hipGetLastError();
}
#elif DLS_CODEC_PART == 2
hipError_t DLS_CODEC_FN(decode_part)(int rc, const dim3& g, const dim3& bl, hipStream_t s, void* F,
                                     const Dims& dims, const BlockDesc* desc, const Item* items,
                                     const int32_t* list, const uint8_t* rank, const int64_t* qv_off,
                                     const int64_t* qa_off, const int64_t* code_off, const VarConst* vc,
                                     const uint8_t* qv, const uint8_t* qa, const uint8_t* codes, int64_t count,
                                     bool team) {
  using T = DLS_CODEC_T;
  constexpr int WP = DLS_CODEC_WP;
#define DLS_DEC(R)                                                                                                 \
  decode_launch<WP, T, R>(g, bl, s, F, dims, desc, items, list, rank, qv_off, qa_off, code_off, vc, qv, qa, codes, \
                          count, team)
  switch (rc) {
    case 0: DLS_DEC(1); break;
    case 1: DLS_DEC(2); break;
    case 2: DLS_DEC(4); break;
    case 3: DLS_DEC(8); break;
    case 4: DLS_DEC(16); break;
    default: DLS_DEC(WP); break;  // rc < 0 (every rank) or the r <= 32 class
  }
#undef DLS_DEC
  return hipGetLastError();
}
#endif

}  // namespace dls
