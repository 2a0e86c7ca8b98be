// Device helpers shared by the gfx950 kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dls_internal.h"

namespace dls {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

// four bfloat16 values, each rounded to nearest even (v_cvt_pk_bf16_f32;
// infinity stays infinity, so the eigensolve's finiteness check still sees it)
__device__ __forceinline__ bf16x4 to_bf16x4(const float* v) {
  typedef __bf16 bfv4 __attribute__((ext_vector_type(4)));
  const bfv4 r = {(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
  return __builtin_bit_cast(bf16x4, r);
}

__device__ __forceinline__ int64_t fidx(const Dims& d, int var, int t, int z, int y, int x) {
  return (((int64_t(var) * d.nt + t) * d.nz + z) * d.ny + y) * d.nx + x;
}

// Offset of slice point p (row-major over the patch, x fastest) from the
// patch origin in the field.
__device__ __forceinline__ int64_t point_off(int p, int px, int py, int64_t nx, int64_t nxy) {
  int rho = p / px;
  int i = p - rho * px;
  int k = rho / py;
  int j = rho - k * py;
  return int64_t(k) * nxy + int64_t(j) * nx + i;
}

__device__ __forceinline__ int rr_player(int pos, int step, int n) {
  return pos == 0 ? 0 : ((pos - 1 + step) % (n - 1)) + 1;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Player at position pos of step `step` of the round-robin ordering on n
// players (player 0 fixed, the others rotate), and the inverse map.
__device__ __forceinline__ int rr_slot(int j, int step, int n) {
  return j == 0 ? 0 : ((j - 1 - step) % (n - 1) + (n - 1)) % (n - 1) + 1;
}

// Keeps the compiler from moving LDS accesses across this point.  Lanes of
// one wavefront see each other's earlier LDS writes (a wavefront's LDS
// accesses complete in issue order), so this is all the ordering needed
// between lanes of the same wavefront.
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

// Sum over an aligned group of G lanes (16 or 32), bitwise equal in every
// lane of the group.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  v = row_sum(v);
  if constexpr (G == 32) v += __shfl_xor(v, 16, 64);
  return v;
}

// Parameters of the Jacobi rotation that annihilates apq (Golub & Van Loan,
// symmetric Schur 2x2): t = sign(theta) / (|theta| + sqrt(1 + theta^2)),
// theta = (aqq - app) / (2 apq), c = 1 / sqrt(1 + t^2), s = t c.  Any t
// gives an exactly orthogonal rotation as long as c and s agree, so t comes
// from the hardware reciprocal and square-root estimates; c is then refined
// to full precision by two Newton steps on 1 / sqrt(1 + t^2).
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (!(fabs(apq) > 1e-300)) return;
  const double theta = (aqq - app) * __builtin_amdgcn_rcp(2.0 * apq);
  const double at = fabs(theta);
  double t;
  if (at > 1e150) {
    t = 0.5 * __builtin_amdgcn_rcp(at);
  } else {
    const double u = fma(theta, theta, 1.0);
    t = __builtin_amdgcn_rcp(at + u * __builtin_amdgcn_rsq(u));
  }
  if (theta < 0.0) t = -t;
  const double u = fma(t, t, 1.0);
  double y = __builtin_amdgcn_rsq(u);
  y = y * fma(-0.5 * u * y, y, 1.5);
  y = y * fma(-0.5 * u * y, y, 1.5);
  c = y;
  s = t * y;
}

}  // namespace dls
