// Device helpers shared by the gfx950 kernel files.
#pragma once
#include <hip/hip_runtime.h>

namespace dls {

__device__ __forceinline__ int rr_player(int pos, int step, int n) {
  return pos == 0 ? 0 : ((pos - 1 + step) % (n - 1)) + 1;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Cyclic Jacobi on the symmetric WP x WP matrix A (LDS, leading dimension
// WP + 1), accumulating the rotations into V, with the parallel round-robin
// ordering (WP / 2 disjoint rotations per step, WP - 1 steps per sweep).
// Called by all 64 lanes of a one-wave workgroup.  Stops when the
// off-diagonal norm falls below 1e-13 of the Frobenius norm, or after 12
// sweeps.  Indices whose rows and columns are exactly zero are never
// rotated (their (p, q) entry is 0).
template <int WP>
__device__ inline void jacobi_lds(double* A, double* V, double* alpha, double* beta, int* partner, int tid) {
  constexpr int EPT = WP * WP / 64;
  constexpr int LD = WP + 1;
  for (int sweep = 0; sweep < 12; ++sweep) {
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int idx = tid + 64 * e, i = idx / WP, j = idx % WP;
      const double a = A[i * LD + j];
      tot += a * a;
      if (i != j) off += a * a;
    }
    off = wave_sum(off);
    tot = wave_sum(tot);
    if (!(off > 1e-26 * tot)) break;
    for (int step = 0; step < WP - 1; ++step) {
      if (tid < WP / 2) {
        int p = rr_player(tid, step, WP), q = rr_player(WP - 1 - tid, step, WP);
        if (p > q) { int t = p; p = q; q = t; }
        const double app = A[p * LD + p], aqq = A[q * LD + q], apq = A[p * LD + q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double theta = (aqq - app) / (2.0 * apq);
          double t = 1.0 / (fabs(theta) + sqrt(1.0 + theta * theta));
          if (theta < 0.0) t = -t;
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        partner[p] = q; partner[q] = p;
        alpha[p] = c; beta[p] = -s;
        alpha[q] = c; beta[q] = s;
      }
      __syncthreads();
      double na[EPT], nv[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int idx = tid + 64 * e, i = idx / WP, j = idx % WP;
        const int mi = partner[i], mj = partner[j];
        const double ai = alpha[i], bi = beta[i], aj = alpha[j], bj = beta[j];
        const double ri = fma(aj, A[i * LD + j], bj * A[i * LD + mj]);
        const double rm = fma(aj, A[mi * LD + j], bj * A[mi * LD + mj]);
        na[e] = fma(ai, ri, bi * rm);
        nv[e] = fma(aj, V[i * LD + j], bj * V[i * LD + mj]);
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int idx = tid + 64 * e, i = idx / WP, j = idx % WP;
        A[i * LD + j] = na[e];
        V[i * LD + j] = nv[e];
      }
      __syncthreads();
    }
  }

}

}  // namespace dls
