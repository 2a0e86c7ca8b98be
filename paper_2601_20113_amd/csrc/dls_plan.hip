// Adaptive (quadtree / octree) patch plan, computed from snapshot 0 of each
// variable.  The paper partitions the domain into patches of one size
// (Sec. 2.3, Alg. 1 step 2); the adaptive plan refines a node of edge e > pmin
// into its half-edge children while the mean gradient magnitude over the node
// exceeds the 80th percentile of the snapshot's gradient magnitude.
//
// Device side: gradient magnitude in FP64 (central differences inside,
// one-sided at the ends); the exact order statistic
// sorted(g)[floor(0.8 (n-1))] by radix selection over the FP64 bit patterns;
// per-level node sums and split flags.  FP32 snapshots with rows of a
// multiple of 4 points take the single-read path (the gradient recomputed in
// each of three passes, never stored, the selection finished on the device,
// every variable at once, one host round trip); others store the gradient
// once and select with host-read histograms.  Host side: the depth-first
// walk that emits the split bits and the leaves in (z0, y0, x0) order.
#include <hip/hip_runtime.h>

#include <array>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "dls_internal.h"
#include "dls_kernels.h"

namespace dls {

namespace {

// |grad f| at (x, y, z) of one snapshot, FP64; the same arithmetic everywhere
template <typename T>
__device__ __forceinline__ double grad_mag(const T* __restrict__ f0, int64_t nx, int64_t ny, int64_t nz, int64_t x,
                                           int64_t y, int64_t z) {
  auto at = [&](int64_t zz, int64_t yy, int64_t xx) { return double(f0[(zz * ny + yy) * nx + xx]); };
  double dx = 0.0, dy = 0.0, dz = 0.0;
  if (nx > 1) {
    if (x == 0) dx = at(z, y, 1) - at(z, y, 0);
    else if (x == nx - 1) dx = at(z, y, nx - 1) - at(z, y, nx - 2);
    else dx = (at(z, y, x + 1) - at(z, y, x - 1)) * 0.5;
  }
  if (ny > 1) {
    if (y == 0) dy = at(z, 1, x) - at(z, 0, x);
    else if (y == ny - 1) dy = at(z, ny - 1, x) - at(z, ny - 2, x);
    else dy = (at(z, y + 1, x) - at(z, y - 1, x)) * 0.5;
  }
  if (nz > 1) {
    if (z == 0) dz = at(1, y, x) - at(0, y, x);
    else if (z == nz - 1) dz = at(nz - 1, y, x) - at(nz - 2, y, x);
    else dz = (at(z + 1, y, x) - at(z - 1, y, x)) * 0.5;
  }
  return sqrt(dx * dx + dy * dy + dz * dz);
}

// g = |grad f| of one snapshot, stored once in FP64 (rows over workgroups,
// x over threads: no index divisions).  Workgroups are dealt to the 8 XCDs
// round-robin, so workgroup b runs on XCD b % 8; each XCD is given one
// contiguous eighth of the rows, which its workgroups sweep together, so the
// y and z neighbours of a row are read through the same L2.
template <typename T>
__global__ __launch_bounds__(256) void k_gradient(const T* __restrict__ f0, int64_t nx, int64_t ny, int64_t nz,
                                                  double* __restrict__ g) {
  const int64_t rows = ny * nz;
  const int64_t per_xcd = (rows + 7) / 8;
  const int xcd = int(blockIdx.x % 8);
  const int64_t lo = int64_t(xcd) * per_xcd;
  const int64_t hi = lo + per_xcd < rows ? lo + per_xcd : rows;
  const int64_t step = gridDim.x / 8;
  for (int64_t row = lo + blockIdx.x / 8; row < hi; row += step) {
    const int64_t y = row % ny, z = row / ny;
    for (int64_t x = threadIdx.x; x < nx; x += 256) g[row * nx + x] = grad_mag(f0, nx, ny, nz, x, y, z);
  }
}

// The same gradient for FP32 rows of a multiple of 4 points: each thread
// takes 4 consecutive points (16-byte loads of the row and of its four
// neighbour rows, two scalar loads for the x neighbours), one row per 128
// threads, two rows per workgroup.  Same arithmetic as grad_mag, so the
// values are bitwise equal.
__global__ __launch_bounds__(256) void k_gradient4(const float* __restrict__ f0, int64_t nx, int64_t ny, int64_t nz,
                                                   double* __restrict__ g) {
  const int64_t rows = ny * nz;
  const int64_t nq = nx / 4;  // float4 per row
  const int64_t row = int64_t(blockIdx.x) * 2 + (threadIdx.x >> 7);
  if (row >= rows) return;
  const int64_t y = row % ny, z = row / ny;
  const float* rp = f0 + row * nx;
  for (int64_t qi = threadIdx.x & 127; qi < nq; qi += 128) {
    const int64_t x = 4 * qi;
    const float4 c = *reinterpret_cast<const float4*>(rp + x);
    double v[4] = {c.x, c.y, c.z, c.w};
    double dx[4] = {0.0, 0.0, 0.0, 0.0}, dy[4] = {0.0, 0.0, 0.0, 0.0}, dz[4] = {0.0, 0.0, 0.0, 0.0};
    if (nx > 1) {
      const double l = x > 0 ? double(rp[x - 1]) : 0.0;
      const double r = x + 4 < nx ? double(rp[x + 4]) : 0.0;
      dx[0] = x == 0 ? v[1] - v[0] : (v[1] - l) * 0.5;
      dx[1] = (v[2] - v[0]) * 0.5;
      dx[2] = (v[3] - v[1]) * 0.5;
      dx[3] = x + 4 == nx ? v[3] - v[2] : (r - v[2]) * 0.5;
    }
    auto row4 = [&](int64_t zz, int64_t yy, double* o) {
      const float4 a = *reinterpret_cast<const float4*>(f0 + (zz * ny + yy) * nx + x);
      o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    };
    if (ny > 1) {
      double a[4], b[4];
      if (y == 0) {
        row4(z, 1, a);
        for (int e = 0; e < 4; ++e) dy[e] = a[e] - v[e];
      } else if (y == ny - 1) {
        row4(z, ny - 2, b);
        for (int e = 0; e < 4; ++e) dy[e] = v[e] - b[e];
      } else {
        row4(z, y + 1, a);
        row4(z, y - 1, b);
        for (int e = 0; e < 4; ++e) dy[e] = (a[e] - b[e]) * 0.5;
      }
    }
    if (nz > 1) {
      double a[4], b[4];
      if (z == 0) {
        row4(1, y, a);
        for (int e = 0; e < 4; ++e) dz[e] = a[e] - v[e];
      } else if (z == nz - 1) {
        row4(nz - 2, y, b);
        for (int e = 0; e < 4; ++e) dz[e] = v[e] - b[e];
      } else {
        row4(z + 1, y, a);
        row4(z - 1, y, b);
        for (int e = 0; e < 4; ++e) dz[e] = (a[e] - b[e]) * 0.5;
      }
    }
    double* out = g + row * nx + x;
    for (int e = 0; e < 4; ++e) out[e] = sqrt(dx[e] * dx[e] + dy[e] * dy[e] + dz[e] * dz[e]);
  }
}

// histogram of digit (bits >> shift) & dmask among elements whose bits match
// `prefix` under `pmask`.  With `aggregate`, lanes holding the same digit are
// merged with a ballot first (the exponent pass, where a wave holds few
// distinct digits and LDS atomics on one address would serialise).
__global__ __launch_bounds__(256) void k_radix_hist(const double* __restrict__ g, int64_t n, uint64_t prefix,
                                                    uint64_t pmask, int shift, uint32_t dmask, int aggregate,
                                                    unsigned int* __restrict__ hist) {
  __shared__ unsigned int h[2048];
  for (int j = threadIdx.x; j < 2048; j += 256) h[j] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t stride = int64_t(gridDim.x) * 256;
  const int64_t nround = (n + stride - 1) / stride;
  for (int64_t it = 0; it < nround; ++it) {   // uniform trip count: every lane joins the ballots
    const int64_t i = it * stride + int64_t(blockIdx.x) * 256 + threadIdx.x;
    bool act = false;
    uint32_t d = 0;
    if (i < n) {
      const uint64_t b = uint64_t(__double_as_longlong(g[i]));
      act = (b & pmask) == prefix;
      d = uint32_t(b >> shift) & dmask;
    }
    if (!aggregate) {
      if (act) atomicAdd(&h[d], 1u);
      continue;
    }
    uint64_t pending = __ballot(act);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const uint32_t d0 = __shfl(d, leader, 64);
      const uint64_t same = __ballot(act && d == d0);
      if (lane == leader) atomicAdd(&h[d0], unsigned(__popcll(same)));
      if (d == d0) act = false;
      pending &= ~same;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j <= int(dmask); j += 256)
    if (h[j]) atomicAdd(hist + j, h[j]);
}

// append the bit patterns of g that match `prefix` under `pmask`; one global
// atomic per wavefront (lanes take consecutive slots by their rank in the
// ballot)
__global__ __launch_bounds__(256) void k_radix_compact(const double* __restrict__ g, int64_t n, uint64_t prefix,
                                                       uint64_t pmask, unsigned long long* __restrict__ count,
                                                       uint64_t* __restrict__ out, unsigned long long cap) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = int64_t(gridDim.x) * 256;
  const int64_t nround = (n + stride - 1) / stride;
  for (int64_t it = 0; it < nround; ++it) {
    const int64_t i = it * stride + int64_t(blockIdx.x) * 256 + threadIdx.x;
    uint64_t b = 0;
    bool hit = false;
    if (i < n) {
      b = uint64_t(__double_as_longlong(g[i]));
      hit = (b & pmask) == prefix;
    }
    const uint64_t mask = __ballot(hit);
    if (mask == 0) continue;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (hit) {
      const unsigned long long slot = base + __popcll(mask & ((1ULL << lane) - 1ULL));
      if (slot < cap) out[slot] = b;
    }
  }
}

// finest-level node sums and counts of g.  Nodes of at most 64 points: one
// thread per node; larger nodes: one wavefront per node with a fixed-order
// reduction.  Points are summed in (z, y, x) order within each lane.
__global__ __launch_bounds__(256) void k_node_sums(const double* __restrict__ g, int64_t nx, int64_t ny, int64_t nz,
                                                   int e, int ez, int64_t NX, int64_t NY, int64_t NZ, int per_wave,
                                                   double* __restrict__ sum, int64_t* __restrict__ cnt) {
  const int64_t nn = NX * NY * NZ;
  const int lane = threadIdx.x & 63;
  const int64_t node = per_wave ? int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6) : int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (node >= nn) return;
  const int64_t ix = node % NX, iy = (node / NX) % NY, iz = node / (NX * NY);
  const int64_t x0 = ix * e, y0 = iy * e, z0 = iz * ez;
  const int ex = int((x0 + e < nx ? x0 + e : nx) - x0), ey = int((y0 + e < ny ? y0 + e : ny) - y0),
            ezz = int((z0 + ez < nz ? z0 + ez : nz) - z0);
  double s = 0.0;
  if (!per_wave) {
    for (int zz = 0; zz < ezz; ++zz)
      for (int yy = 0; yy < ey; ++yy) {
        const double* row = g + ((z0 + zz) * ny + y0 + yy) * nx + x0;
        for (int xx = 0; xx < ex; ++xx) s += row[xx];
      }
    sum[node] = s;
    cnt[node] = int64_t(ex) * ey * ezz;
    return;
  }
  const int np = ex * ey * ezz;
  for (int q = lane; q < np; q += 64) {
    const int xx = q % ex, rest = q / ex, yy = rest % ey, zz = rest / ey;
    s += g[((z0 + zz) * ny + y0 + yy) * nx + x0 + xx];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) {
    sum[node] = s;
    cnt[node] = np;
  }
}

// split flag of every node: mean of g over the node > thr
__global__ __launch_bounds__(256) void k_split_flags(const double* __restrict__ sum, const int64_t* __restrict__ cnt,
                                                     int64_t n, double thr, uint8_t* __restrict__ flag) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) flag[i] = (sum[i] / double(cnt[i]) > thr) ? 1 : 0;
}

// parent level from the child level (children in (z, y, x) order)
__global__ __launch_bounds__(256) void k_coarsen(const double* __restrict__ csum, const int64_t* __restrict__ ccnt,
                                                 int64_t CX, int64_t CY, int64_t CZ, int is3d, int64_t NX,
                                                 int64_t NY, int64_t NZ, double* __restrict__ sum,
                                                 int64_t* __restrict__ cnt) {
  const int64_t nn = NX * NY * NZ;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= nn) return;
  const int64_t ix = i % NX, iy = (i / NX) % NY, iz = i / (NX * NY);
  double s = 0.0;
  int64_t c = 0;
  for (int dz = 0; dz < (is3d ? 2 : 1); ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int64_t cx = 2 * ix + dx, cy = 2 * iy + dy, cz = is3d ? 2 * iz + dz : 0;
        if (cx < CX && cy < CY && cz < CZ) {
          const int64_t j = (cz * CY + cy) * CX + cx;
          s += csum[j];
          c += ccnt[j];
        }
      }
  sum[i] = s;
  cnt[i] = c;
}

// ---------------------------------------------------------------------------
// Single-read plan (FP32 snapshots, rows of a multiple of 4 points, finest
// node edge a multiple of 4), every variable at once (grid y = variable):
//   pass 0 reads the snapshot once: finest-level node sums of g, the
//          histogram of bits 52..63 (sign and exponent) of s = g^2 (g is
//          the square root of s, so the order statistic of g is the root of
//          that of s), and the high 32 bits of s stored (4 B per point
//          instead of an 8 B gradient);
//   pass 1 streams the high words: histogram of bits 41..51 of s among the
//          points whose bits 52..63 match;
//   pass 2 streams them again: the points matching bits 41..63 get their
//          exact s recomputed and appended to a candidate list;
// the digit selections and the final selection among the candidates run on
// the device, so the whole plan needs one host round trip (the split flags).
// ---------------------------------------------------------------------------
struct PlanSel {
  uint64_t prefix;        // selected high bits so far
  int64_t k;              // rank sought among the points matching prefix
  unsigned long long ncand;
  uint32_t status;        // 0 ok, 1 rank not found, 2 candidate list full
  uint32_t pad;
  double thr;             // the order statistic
};

// The values one quad of four points x .. x+3 of row (y, z) needs for its
// gradient: the row itself, its y and z neighbour rows and the two x
// neighbours (loaded first, so several quads' loads are in flight together).
struct QuadIn {
  float4 c, ym, yp, zm, zp;
  float l, r;
};

__device__ __forceinline__ void quad_load(const float* __restrict__ f0, int64_t nx, int64_t ny, int64_t nz, int64_t x,
                                          int64_t y, int64_t z, QuadIn& in) {
  // every address clamped into the snapshot and every load unconditional, so
  // the seven loads issue back to back; quad_sq uses only the values the
  // differences need
  const int64_t ym = y > 0 ? y - 1 : y, yp = y + 1 < ny ? y + 1 : y;
  const int64_t zm = z > 0 ? z - 1 : z, zp = z + 1 < nz ? z + 1 : z;
  auto row = [&](int64_t zz, int64_t yy) { return f0 + (zz * ny + yy) * nx; };
  const float* rp = row(z, y);
  in.c = *reinterpret_cast<const float4*>(rp + x);
  in.l = rp[x > 0 ? x - 1 : x];
  in.r = rp[x + 4 < nx ? x + 4 : x + 3];
  in.ym = *reinterpret_cast<const float4*>(row(z, ym) + x);
  in.yp = *reinterpret_cast<const float4*>(row(z, yp) + x);
  in.zm = *reinterpret_cast<const float4*>(row(zm, y) + x);
  in.zp = *reinterpret_cast<const float4*>(row(zp, y) + x);
}

// The same loads for a row interior in y and z (or of a 2D snapshot, sz =
// 0): the neighbour rows at fixed strides from the quad's row rp, so the
// addresses equal the clamped ones of quad_load.
__device__ __forceinline__ void quad_load_in(const float* __restrict__ rp, int64_t nx, int64_t sy, int64_t sz,
                                             int64_t x, QuadIn& in) {
  in.c = *reinterpret_cast<const float4*>(rp + x);
  in.l = rp[x > 0 ? x - 1 : x];
  in.r = rp[x + 4 < nx ? x + 4 : x + 3];
  in.ym = *reinterpret_cast<const float4*>(rp - sy + x);
  in.yp = *reinterpret_cast<const float4*>(rp + sy + x);
  in.zm = *reinterpret_cast<const float4*>(rp - sz + x);
  in.zp = *reinterpret_cast<const float4*>(rp + sz + x);
}

// squared gradient magnitudes s = dx^2 + dy^2 + dz^2 of the quad, with the
// arithmetic of grad_mag / k_gradient4: sqrt(s) is bitwise their g, and the
// order statistics of g are the square roots of those of s (a correctly
// rounded square root is monotone), so the selection never takes a root
template <bool IN = false>
__device__ __forceinline__ void quad_sq(const QuadIn& in, int64_t nx, int64_t ny, int64_t nz, int64_t x, int64_t y,
                                        int64_t z, double (&g)[4]) {
  // each difference as (a - b) * h: the central difference (h = 1/2) inside,
  // the one-sided one (h = 1, exact) at an end, operands selected per lane
  // instead of branched on
  const double v[4] = {in.c.x, in.c.y, in.c.z, in.c.w};
  double dx[4] = {0.0, 0.0, 0.0, 0.0}, dy[4] = {0.0, 0.0, 0.0, 0.0}, dz[4] = {0.0, 0.0, 0.0, 0.0};
  if (nx > 1) {
    const bool lo = x == 0, hi = x + 4 == nx;
    const double l = double(in.l), r = double(in.r);
    dx[0] = ((lo ? v[1] : v[1]) - (lo ? v[0] : l)) * (lo ? 1.0 : 0.5);
    dx[1] = (v[2] - v[0]) * 0.5;
    dx[2] = (v[3] - v[1]) * 0.5;
    dx[3] = ((hi ? v[3] : r) - v[2]) * (hi ? 1.0 : 0.5);
  }
  if (ny > 1) {
    const bool lo = !IN && y == 0, hi = !IN && y == ny - 1;
    const double h = (lo || hi) ? 1.0 : 0.5;
    const double a[4] = {in.yp.x, in.yp.y, in.yp.z, in.yp.w}, b[4] = {in.ym.x, in.ym.y, in.ym.z, in.ym.w};
    for (int e = 0; e < 4; ++e) dy[e] = ((hi ? v[e] : a[e]) - (lo ? v[e] : b[e])) * h;
  }
  if (nz > 1) {
    const bool lo = !IN && z == 0, hi = !IN && z == nz - 1;
    const double h = (lo || hi) ? 1.0 : 0.5;
    const double a[4] = {in.zp.x, in.zp.y, in.zp.z, in.zp.w}, b[4] = {in.zm.x, in.zm.y, in.zm.z, in.zm.w};
    for (int e = 0; e < 4; ++e) dz[e] = ((hi ? v[e] : a[e]) - (lo ? v[e] : b[e])) * h;
  }
  for (int e = 0; e < 4; ++e) g[e] = dx[e] * dx[e] + dy[e] * dy[e] + dz[e] * dz[e];
}

// the squared gradient magnitude of one point, bitwise equal to quad_sq's
// (and to grad_mag before its root)
__device__ __forceinline__ double point_sq(const float* __restrict__ f0, int64_t nx, int64_t ny, int64_t nz, int64_t x,
                                           int64_t y, int64_t z) {
  auto at = [&](int64_t zz, int64_t yy, int64_t xx) { return double(f0[(zz * ny + yy) * nx + xx]); };
  double dx = 0.0, dy = 0.0, dz = 0.0;
  if (nx > 1) {
    if (x == 0) dx = at(z, y, 1) - at(z, y, 0);
    else if (x == nx - 1) dx = at(z, y, nx - 1) - at(z, y, nx - 2);
    else dx = (at(z, y, x + 1) - at(z, y, x - 1)) * 0.5;
  }
  if (ny > 1) {
    if (y == 0) dy = at(z, 1, x) - at(z, 0, x);
    else if (y == ny - 1) dy = at(z, ny - 1, x) - at(z, ny - 2, x);
    else dy = (at(z, y + 1, x) - at(z, y - 1, x)) * 0.5;
  }
  if (nz > 1) {
    if (z == 0) dz = at(1, y, x) - at(0, y, x);
    else if (z == nz - 1) dz = at(nz - 1, y, x) - at(nz - 2, y, x);
    else dz = (at(z + 1, y, x) - at(z - 1, y, x)) * 0.5;
  }
  return dx * dx + dy * dy + dz * dz;
}

struct PassGeom {
  int64_t nx, ny, nz, var_stride;  // snapshot 0 of variable v starts at v * var_stride floats
  int ef, efz, cw;                 // finest node edge (x, y) and (z), x chunk width (multiple of ef)
  int64_t nchunk, NXf, NYf, NZf;   // x chunks; finest node grid
};

// The quads of one pass-0 workgroup: item idx = row * nq + q (row = z * ry
// + y within the chunk), 256 items per step, U steps' loads issued
// together.  A thread's (q, row) and (y, z) advance by fixed increments
// (no division per quad).
template <bool IN>
__device__ __forceinline__ void pass0_quads(const float* __restrict__ f0, const PassGeom& G, int64_t x0, int64_t y0,
                                            int64_t z0, int ry, int nq, int nitem, double* __restrict__ qs,
                                            unsigned int* __restrict__ h, uint32_t* __restrict__ tv) {
  constexpr int U = 2;  // quads per thread whose loads are issued together
  const int dq = 256 % nq, drow = 256 / nq, drm = drow % ry, drz = drow / ry;
  const int64_t sy = G.nx, sz = G.nz > 1 ? G.nx * G.ny : 0;
  int q = int(threadIdx.x) % nq, row = int(threadIdx.x) / nq;
  int ym = row % ry, zq = row / ry;
  for (int base = 0; base < nitem; base += 256 * U) {
    QuadIn in[U];
    int64_t qx[U], qy[U], qz[U], ro[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + 256 * u + int(threadIdx.x);
      qx[u] = x0 + 4 * q;
      qy[u] = y0 + ym;
      qz[u] = z0 + zq;
      ro[u] = (qz[u] * G.ny + qy[u]) * G.nx;  // the quad's row
      if (idx < nitem) {
        if constexpr (IN) quad_load_in(f0 + ro[u], G.nx, sy, sz, qx[u], in[u]);
        else quad_load(f0, G.nx, G.ny, G.nz, qx[u], qy[u], qz[u], in[u]);
      }
      // the next item of this thread: idx + 256
      q += dq;
      const int c = q >= nq ? 1 : 0;
      q -= c ? nq : 0;
      ym += drm + c;
      zq += drz;
      if (ym >= ry) {
        ym -= ry;
        ++zq;
      }
    }
    // exponent digits counted in runs (neighbouring points share them), one
    // LDS atomic per run
    uint32_t run_d = 0xFFFFFFFFu, run_n = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + 256 * u + int(threadIdx.x);
      if (idx >= nitem) continue;
      double sq[4];
      quad_sq<IN>(in[u], G.nx, G.ny, G.nz, qx[u], qy[u], qz[u], sq);
      qs[idx] = ((sqrt(sq[0]) + sqrt(sq[1])) + sqrt(sq[2])) + sqrt(sq[3]);
      uint32_t hi[4];
      for (int e = 0; e < 4; ++e) {
        const uint64_t b = uint64_t(__double_as_longlong(sq[e]));
        hi[e] = uint32_t(b >> 32);
        const uint32_t d = uint32_t(b >> 52);
        if (d != run_d) {
          if (run_n) atomicAdd(&h[run_d], run_n);
          run_d = d;
          run_n = 0;
        }
        ++run_n;
      }
      *reinterpret_cast<uint4*>(tv + ro[u] + qx[u]) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
    }
    if (run_n) atomicAdd(&h[run_d], run_n);
  }
}

// Pass 0, one workgroup per (x chunk, finest node row in y, in z) of one
// variable: the squared gradient s of every point, the finest-level node
// sums of g = sqrt(s), the histogram of bits 52..63 of s, and the high 32
// bits of s stored (4 B per point) for the later passes.
__global__ __launch_bounds__(256) void k_plan_pass0(const float* __restrict__ F, PassGeom G,
                                                    unsigned int* __restrict__ hist, int64_t sum_stride,
                                                    double* __restrict__ sum, int64_t* __restrict__ cnt,
                                                    uint32_t* __restrict__ top) {
  extern __shared__ double qs[];  // quad sums of g, [row][quad]
  __shared__ unsigned int h[4096];
  const int v = blockIdx.y;
  const float* f0 = F + int64_t(v) * G.var_stride;
  uint32_t* tv = top + int64_t(v) * (G.nx * G.ny * G.nz);
  const int64_t wg = blockIdx.x;
  const int64_t chunk = wg % G.nchunk, iy = (wg / G.nchunk) % G.NYf, iz = wg / (G.nchunk * G.NYf);
  const int64_t x0 = chunk * G.cw, y0 = iy * G.ef, z0 = iz * G.efz;
  const int xw = int((x0 + G.cw < G.nx ? x0 + G.cw : G.nx) - x0);
  const int ry = int((y0 + G.ef < G.ny ? y0 + G.ef : G.ny) - y0);
  const int rz = int((z0 + G.efz < G.nz ? z0 + G.efz : G.nz) - z0);
  const int nq = xw / 4, R = ry * rz, nitem = R * nq;
  for (int j = threadIdx.x; j < 4096; j += 256) h[j] = 0;
  __syncthreads();
  // every row of the workgroup interior in y and z (or a 2D snapshot): no
  // boundary differences and no clamped neighbour rows
  const bool interior = G.ny > 2 && y0 > 0 && y0 + ry < G.ny && (G.nz == 1 || (z0 > 0 && z0 + rz < G.nz));
  if (interior) pass0_quads<true>(f0, G, x0, y0, z0, ry, nq, nitem, qs, h, tv);
  else pass0_quads<false>(f0, G, x0, y0, z0, ry, nq, nitem, qs, h, tv);
  __syncthreads();
  unsigned int* gh = hist + int64_t(v) * 4096;
  for (int j = threadIdx.x; j < 4096; j += 256)
    if (h[j]) atomicAdd(gh + j, h[j]);
  // finest-level node sums of the chunk in a fixed order: quads of a node row
  // by row
  const int qpn = G.ef / 4, nnode = (nq + qpn - 1) / qpn;
  for (int j = threadIdx.x; j < nnode; j += 256) {
    const int q0 = j * qpn, q1 = q0 + qpn < nq ? q0 + qpn : nq;
    double acc = 0.0;
    for (int r = 0; r < R; ++r)
      for (int qq = q0; qq < q1; ++qq) acc += qs[r * nq + qq];
    const int64_t ix = x0 / G.ef + j;
    const int64_t node = (iz * G.NYf + iy) * G.NXf + ix;
    sum[int64_t(v) * sum_stride + node] = acc;
    cnt[int64_t(v) * sum_stride + node] = int64_t(R) * (q1 - q0) * 4;
  }
}

// Pass 1 over the stored high words: histogram of bits 41..51 of s among the
// points whose bits 52..63 match the selected digit.
__global__ __launch_bounds__(256) void k_plan_pass1(const uint32_t* __restrict__ top, int64_t n,
                                                    const PlanSel* __restrict__ sel, unsigned int* __restrict__ hist) {
  __shared__ unsigned int h[2048];
  const int v = blockIdx.y;
  const uint32_t* tv = top + int64_t(v) * n;
  for (int j = threadIdx.x; j < 2048; j += 256) h[j] = 0;
  __syncthreads();
  const uint32_t ex = uint32_t(sel[v].prefix >> 52);
  const int64_t n4 = n / 4, stride = int64_t(gridDim.x) * 256;
  constexpr int U = 4;  // loads in flight per thread
  for (int64_t i0 = int64_t(blockIdx.x) * 256 + threadIdx.x; i0 < n4; i0 += U * stride) {
    uint4 t[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      t[u] = i0 + u * stride < n4 ? reinterpret_cast<const uint4*>(tv)[i0 + u * stride] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u * stride >= n4) continue;
      const uint32_t w[4] = {t[u].x, t[u].y, t[u].z, t[u].w};
      // digits of the four consecutive points counted in runs
      uint32_t run_d = 0xFFFFFFFFu, run_n = 0;
      for (int e = 0; e < 4; ++e) {
        if ((w[e] >> 20) != ex) continue;
        const uint32_t d = (w[e] >> 9) & 2047u;
        if (d != run_d) {
          if (run_n) atomicAdd(&h[run_d], run_n);
          run_d = d;
          run_n = 0;
        }
        ++run_n;
      }
      if (run_n) atomicAdd(&h[run_d], run_n);
    }
  }
  __syncthreads();
  unsigned int* gh = hist + int64_t(v) * 4096;
  for (int j = threadIdx.x; j < 2048; j += 256)
    if (h[j]) atomicAdd(gh + j, h[j]);
}

// Pass 2 over the stored high words: the points whose bits 41..63 match the
// selected digits get their exact s recomputed and appended to the
// candidate list (one global atomic per wavefront with hits).
__global__ __launch_bounds__(256) void k_plan_pass2(const uint32_t* __restrict__ top, const float* __restrict__ F,
                                                    PassGeom G, PlanSel* __restrict__ sel,
                                                    uint64_t* __restrict__ cand, unsigned long long cap) {
  const int v = blockIdx.y;
  const int64_t n = G.nx * G.ny * G.nz;
  const uint32_t* tv = top + int64_t(v) * n;
  const float* f0 = F + int64_t(v) * G.var_stride;
  const uint32_t pre = uint32_t(sel[v].prefix >> 41);
  const int lane = threadIdx.x & 63;
  const int64_t n4 = n / 4, stride = int64_t(gridDim.x) * 256;
  constexpr int U = 4;  // loads in flight per thread
  const int64_t nround = (n4 + U * stride - 1) / (U * stride);
  for (int64_t it = 0; it < nround; ++it) {  // uniform trip count: every lane joins the ballots
    uint4 tt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = (it * U + u) * stride + int64_t(blockIdx.x) * 256 + threadIdx.x;
      tt[u] = i < n4 ? reinterpret_cast<const uint4*>(tv)[i]
                     : make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
    const int64_t i = (it * U + u) * stride + int64_t(blockIdx.x) * 256 + threadIdx.x;
    const uint4 t = tt[u];
    const uint32_t w[4] = {t.x, t.y, t.z, t.w};
    const bool any = i < n4 && ((w[0] >> 9) == pre || (w[1] >> 9) == pre || (w[2] >> 9) == pre || (w[3] >> 9) == pre);
    if (__ballot(any) == 0) continue;  // the common case: no hit in the wavefront
    for (int e = 0; e < 4; ++e) {
      const bool hit = i < n4 && (w[e] >> 9) == pre;
      const uint64_t mask = __ballot(hit);
      if (mask == 0) continue;
      const int leader = __ffsll((unsigned long long)mask) - 1;
      unsigned long long slot0 = 0;
      if (lane == leader) slot0 = atomicAdd(&sel[v].ncand, (unsigned long long)__popcll(mask));
      slot0 = __shfl(slot0, leader, 64);
      if (hit) {
        const int64_t pi = 4 * i + e;
        const int64_t x = pi % G.nx, row = pi / G.nx;
        const double sq = point_sq(f0, G.nx, G.ny, G.nz, x, row % G.ny, row / G.ny);
        const unsigned long long slot = slot0 + __popcll(mask & ((1ULL << lane) - 1ULL));
        if (slot < cap) cand[int64_t(v) * int64_t(cap) + int64_t(slot)] = uint64_t(__double_as_longlong(sq));
      }
    }
    }
  }
}

// digit selection: the digit d of the histogram (nbins bins) holding rank k
// (counts of lower digits subtracted); the prefix gains d << shift.  One
// workgroup per variable.
__global__ __launch_bounds__(256) void k_plan_digit(const unsigned int* __restrict__ hist, int nbins, int shift,
                                                    PlanSel* __restrict__ sel) {
  __shared__ unsigned long long part[256];
  const int v = blockIdx.x;
  const unsigned int* hv = hist + int64_t(v) * 4096;
  const int per = (nbins + 255) / 256;
  unsigned long long c = 0;
  for (int j = 0; j < per; ++j) {
    const int b = int(threadIdx.x) * per + j;
    if (b < nbins) c += hv[b];
  }
  part[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    PlanSel S = sel[v];
    if (S.status != 0) return;
    int64_t k = S.k;
    int t = 0;
    for (; t < 256; ++t) {
      if (k < int64_t(part[t])) break;
      k -= int64_t(part[t]);
    }
    int d = -1;
    if (t < 256)
      for (int j = 0; j < per; ++j) {
        const int b = t * per + j;
        if (b >= nbins) break;
        if (k < int64_t(hv[b])) { d = b; break; }
        k -= int64_t(hv[b]);
      }
    if (d < 0) {
      sel[v].status = 1;
      return;
    }
    sel[v].k = k;
    sel[v].prefix = S.prefix | (uint64_t(d) << shift);
  }
}

// the k-th smallest candidate s (all share bits 41..63): radix selection
// over bits 40..0 in digits of 9 and 8 bits, one workgroup of 1024 threads
// per variable, the candidates staged in LDS when they fit (else read with
// four loads in flight per thread); thr = sqrt(s_k)
__global__ __launch_bounds__(1024) void k_plan_cand(const uint64_t* __restrict__ cand, unsigned long long cap,
                                                    PlanSel* __restrict__ sel) {
  constexpr int kStage = 16384, T = 1024;
  __shared__ uint64_t st[kStage];
  __shared__ unsigned int h[512];
  __shared__ int64_t kk;
  __shared__ uint64_t pre;
  __shared__ int dsel;
  const int v = blockIdx.x;
  const PlanSel S = sel[v];
  if (S.status != 0) return;
  if (S.ncand > cap) {
    if (threadIdx.x == 0) sel[v].status = 2;
    return;
  }
  const uint64_t* cv = cand + int64_t(v) * int64_t(cap);
  const int64_t n = int64_t(S.ncand);
  const bool staged = n <= kStage;
  if (staged)
    for (int64_t i = threadIdx.x; i < n; i += T) st[i] = cv[i];
  if (threadIdx.x == 0) { kk = S.k; pre = S.prefix; }
  __syncthreads();
  const int shifts[5] = {32, 24, 16, 8, 0};
  const int widths[5] = {9, 8, 8, 8, 8};
  uint64_t mask = ~((uint64_t(1) << 41) - 1);  // bits already fixed
  for (int pass = 0; pass < 5; ++pass) {
    const int nb = 1 << widths[pass];
    for (int j = threadIdx.x; j < nb; j += T) h[j] = 0;
    __syncthreads();
    const uint64_t pv = pre;
    const uint32_t dm = uint32_t(nb - 1);
    if (staged) {
      for (int64_t i = threadIdx.x; i < n; i += T) {
        const uint64_t b = st[i];
        if ((b & mask) == pv) atomicAdd(&h[uint32_t(b >> shifts[pass]) & dm], 1u);
      }
    } else {
      for (int64_t i0 = threadIdx.x; i0 < n; i0 += 4 * T) {
        uint64_t b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) b[u] = i0 + u * T < n ? cv[i0 + u * T] : ~uint64_t(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u * T < n && (b[u] & mask) == pv) atomicAdd(&h[uint32_t(b[u] >> shifts[pass]) & dm], 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t k = kk;
      int d = -1;
      for (int j = 0; j < nb; ++j) {
        if (k < int64_t(h[j])) { d = j; break; }
        k -= int64_t(h[j]);
      }
      dsel = d;
      if (d >= 0) {
        kk = k;
        pre = pv | (uint64_t(d) << shifts[pass]);
      }
    }
    __syncthreads();
    if (dsel < 0) {
      if (threadIdx.x == 0) sel[v].status = 1;
      return;
    }
    mask |= (uint64_t(nb - 1) << shifts[pass]);
  }
  if (threadIdx.x == 0) {
    sel[v].thr = sqrt(__longlong_as_double((long long)pre));
    sel[v].prefix = pre;
  }
}

// split flags of every node of every variable from the device threshold
__global__ __launch_bounds__(256) void k_plan_flags(const double* __restrict__ sum, const int64_t* __restrict__ cnt,
                                                    int64_t n, const PlanSel* __restrict__ sel,
                                                    uint8_t* __restrict__ flag) {
  const int v = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const double thr = sel[v].thr;
  flag[int64_t(v) * n + i] = (sum[int64_t(v) * n + i] / double(cnt[int64_t(v) * n + i]) > thr) ? 1 : 0;
}

struct DevMem {
  void* p = nullptr;
  size_t n = 0;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
    if (e == hipSuccess) n = bytes;
    return e;
  }
};

}  // namespace

struct PlanScratch {
  DevMem g, cand, hist, sums, cnts, count, flags, sel, top;
  PlanSel* hsel = nullptr;                        // pinned host copy of the selection states
  size_t hsel_n = 0;
  uint8_t* hflags = nullptr;                      // pinned host copy of every variable's split flags
  size_t hflags_n = 0;
  // the split flags of the previous call per variable, with the leaves and
  // bits they produced: equal flags give the same tree, so its walk is skipped
  std::vector<std::vector<uint8_t>> prev_flags, prev_bits;
  std::vector<std::vector<Leaf>> prev_leaves;
  std::vector<std::array<int64_t, 5>> prev_key;  // nx, ny, nz, px, pmin
  unsigned int* hhist = nullptr;                  // pinned host copies of the histogram / count
  unsigned long long* hcount = nullptr;
  ~PlanScratch() {
    if (hhist) (void)hipHostFree(hhist);
    if (hcount) (void)hipHostFree(hcount);
    if (hsel) (void)hipHostFree(hsel);
    if (hflags) (void)hipHostFree(hflags);
  }
};

PlanScratch* plan_scratch_new() { return new PlanScratch(); }
void plan_scratch_delete(PlanScratch* s) { delete s; }

#define PLAN_TRY(expr)                                              \
  do {                                                              \
    hipError_t e_ = (expr);                                         \
    if (e_ != hipSuccess) {                                         \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);      \
      return e_;                                                    \
    }                                                               \
  } while (0)

// Leaves and split bits of every variable of the field, computed from
// snapshot 0.  Returns hipSuccess or the failing HIP error (message in err).
hipError_t adaptive_plan(const Problem& p, const void* F, hipStream_t s, PlanScratch& S, Plan& plan,
                         std::string& err) {
  const int64_t n = p.nx * p.ny * p.nz;
  const bool is3d = p.nz > 1;
  // node grids, coarsest (edge px) to finest (edge pmin)
  std::vector<int> edges;
  for (int e = p.px; e >= p.pmin; e /= 2) edges.push_back(e);
  const int L = int(edges.size());
  std::vector<int64_t> NX(L), NY(L), NZ(L), off(L + 1, 0);
  for (int l = 0; l < L; ++l) {
    NX[l] = (p.nx + edges[l] - 1) / edges[l];
    NY[l] = (p.ny + edges[l] - 1) / edges[l];
    NZ[l] = is3d ? (p.nz + edges[l] - 1) / edges[l] : 1;
    off[l + 1] = off[l] + NX[l] * NY[l] * NZ[l];
  }
  const int64_t nodes = off[L];
  PLAN_TRY(S.sums.ensure(size_t(p.nvars) * size_t(nodes) * sizeof(double)));
  PLAN_TRY(S.cnts.ensure(size_t(p.nvars) * size_t(nodes) * sizeof(int64_t)));
  PLAN_TRY(S.flags.ensure(size_t(p.nvars) * size_t(nodes)));
  PLAN_TRY(S.hist.ensure(2 * size_t(p.nvars) * 4096 * sizeof(unsigned int)));
  double* dsum = static_cast<double*>(S.sums.p);
  int64_t* dcnt = static_cast<int64_t*>(S.cnts.p);
  unsigned int* dhist = static_cast<unsigned int*>(S.hist.p);
  uint8_t* dflag = static_cast<uint8_t*>(S.flags.p);
  const dim3 bl{256};
  plan.leaves.assign(p.nvars, {});
  plan.bits.assign(p.nvars, {});
  const int es = p.esize();
  std::vector<std::vector<uint8_t>> hflag(p.nvars, std::vector<uint8_t>(size_t(nodes)));
  std::vector<char> have(p.nvars, 0);
  const bool timing = std::getenv("DLS_TIMING") != nullptr;
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };

  // the single-read path: every variable at once, one host round trip
  const int ef = edges[L - 1], efz = is3d ? edges[L - 1] : 1;
  int cw = 0;
  {
    const int64_t per_x = 2 * int64_t(ef) * efz;  // LDS bytes of quad sums per point of x
    cw = int(std::min<int64_t>((p.nx + ef - 1) / ef * ef, std::max<int64_t>(ef, 16384 / per_x / ef * ef)));
    cw = (cw + 3) / 4 * 4;
  }
  const int64_t qs_bytes = 2 * int64_t(ef) * efz * cw;
  const bool single_read = p.dtype == 0 && p.nx % 4 == 0 && ef % 4 == 0 && cw % ef == 0 && qs_bytes <= 65536 &&
                           (reinterpret_cast<uintptr_t>(F) & 15) == 0;
  if (single_read) {
    const auto t0 = now();
    const unsigned long long cap = 1ULL << 20;
    PLAN_TRY(S.cand.ensure(size_t(p.nvars) * cap * sizeof(uint64_t)));
    PLAN_TRY(S.sel.ensure(size_t(p.nvars) * sizeof(PlanSel)));
    PLAN_TRY(S.top.ensure(size_t(p.nvars) * size_t(n) * sizeof(uint32_t)));
    uint32_t* dtop = static_cast<uint32_t*>(S.top.p);
    if (S.hsel_n < size_t(p.nvars)) {
      if (S.hsel) (void)hipHostFree(S.hsel);
      S.hsel = nullptr;
      void* q = nullptr;
      PLAN_TRY(hipHostMalloc(&q, size_t(p.nvars) * sizeof(PlanSel), hipHostMallocDefault));
      S.hsel = static_cast<PlanSel*>(q);
      S.hsel_n = size_t(p.nvars);
    }
    if (S.hflags_n < size_t(p.nvars) * size_t(nodes)) {
      if (S.hflags) (void)hipHostFree(S.hflags);
      S.hflags = nullptr;
      void* q = nullptr;
      PLAN_TRY(hipHostMalloc(&q, size_t(p.nvars) * size_t(nodes), hipHostMallocDefault));
      S.hflags = static_cast<uint8_t*>(q);
      S.hflags_n = size_t(p.nvars) * size_t(nodes);
    }
    PlanSel* dsel = static_cast<PlanSel*>(S.sel.p);
    uint64_t* dcand = static_cast<uint64_t*>(S.cand.p);
    const int64_t k0 = int64_t(std::floor(0.8 * double(n - 1)));
    for (int v = 0; v < p.nvars; ++v) S.hsel[v] = PlanSel{0, k0, 0, 0, 0, 0.0};
    PLAN_TRY(hipMemcpyAsync(dsel, S.hsel, size_t(p.nvars) * sizeof(PlanSel), hipMemcpyHostToDevice, s));
    PLAN_TRY(hipMemsetAsync(dhist, 0, 2 * size_t(p.nvars) * 4096 * sizeof(unsigned int), s));
    PassGeom G{p.nx, p.ny, p.nz, p.nt * n, ef, efz, cw, (p.nx + cw - 1) / cw, NX[L - 1], NY[L - 1], NZ[L - 1]};
    const dim3 grid{unsigned(G.nchunk * G.NYf * G.NZf), unsigned(p.nvars)};
    const float* f = static_cast<const float*>(F);
    unsigned int* h0 = dhist;
    unsigned int* h1 = dhist + size_t(p.nvars) * 4096;
    const unsigned sgrid = unsigned(std::min<int64_t>(8192, (n / 4 + 255) / 256));
    const dim3 grid1{sgrid, unsigned(p.nvars)};
    hipLaunchKernelGGL(k_plan_pass0, grid, bl, size_t(qs_bytes), s, f, G, h0, nodes, dsum + off[L - 1],
                       dcnt + off[L - 1], dtop);
    hipLaunchKernelGGL(k_plan_digit, dim3{unsigned(p.nvars)}, bl, 0, s, (const unsigned int*)h0, 4096, 52, dsel);
    hipLaunchKernelGGL(k_plan_pass1, grid1, bl, 0, s, (const uint32_t*)dtop, n, (const PlanSel*)dsel, h1);
    hipLaunchKernelGGL(k_plan_digit, dim3{unsigned(p.nvars)}, bl, 0, s, (const unsigned int*)h1, 2048, 41, dsel);
    hipLaunchKernelGGL(k_plan_pass2, grid1, bl, 0, s, (const uint32_t*)dtop, f, G, dsel, dcand, cap);
    hipLaunchKernelGGL(k_plan_cand, dim3{unsigned(p.nvars)}, dim3{1024}, 0, s, (const uint64_t*)dcand, cap, dsel);
    PLAN_TRY(hipGetLastError());
    for (int v = 0; v < p.nvars; ++v)
      for (int l = L - 2; l >= 0; --l) {
        const int64_t nn = NX[l] * NY[l] * NZ[l];
        double* sv = dsum + int64_t(v) * nodes;
        int64_t* cv = dcnt + int64_t(v) * nodes;
        hipLaunchKernelGGL(k_coarsen, dim3{unsigned((nn + 255) / 256)}, bl, 0, s, (const double*)(sv + off[l + 1]),
                           (const int64_t*)(cv + off[l + 1]), NX[l + 1], NY[l + 1], NZ[l + 1], is3d ? 1 : 0, NX[l],
                           NY[l], NZ[l], sv + off[l], cv + off[l]);
      }
    const dim3 fgrid{unsigned((nodes + 255) / 256), unsigned(p.nvars)};
    hipLaunchKernelGGL(k_plan_flags, fgrid, bl, 0, s, (const double*)dsum, (const int64_t*)dcnt, nodes,
                       (const PlanSel*)dsel, dflag);
    PLAN_TRY(hipGetLastError());
    PLAN_TRY(hipMemcpyAsync(S.hflags, dflag, size_t(p.nvars) * size_t(nodes), hipMemcpyDeviceToHost, s));
    PLAN_TRY(hipMemcpyAsync(S.hsel, dsel, size_t(p.nvars) * sizeof(PlanSel), hipMemcpyDeviceToHost, s));
    PLAN_TRY(hipStreamSynchronize(s));
    for (int v = 0; v < p.nvars; ++v) {
      if (S.hsel[v].status != 0) continue;  // selection not finished on the device: the stored-gradient path below
      std::memcpy(hflag[v].data(), S.hflags + size_t(v) * size_t(nodes), size_t(nodes));
      have[v] = 1;
    }
    if (timing)
      std::fprintf(stderr, "[dls] plan (single read, %d variables): %.3f ms, status %u, %llu candidates\n", p.nvars,
                   ms(t0, now()), S.hsel[0].status, S.hsel[0].ncand);
  }

  // the stored-gradient path, one variable at a time (FP64 snapshots, rows
  // of other widths, or a selection the single-read path did not finish)
  for (int v = 0; v < p.nvars; ++v) {
    if (have[v]) continue;
    const auto t0 = now();
    PLAN_TRY(S.g.ensure(size_t(n) * sizeof(double)));
    PLAN_TRY(S.count.ensure(sizeof(unsigned long long)));
    const unsigned long long cand_cap = 1ULL << 22;
    PLAN_TRY(S.cand.ensure(size_t(cand_cap) * sizeof(uint64_t)));
    unsigned long long* dcount = static_cast<unsigned long long*>(S.count.p);
    uint64_t* dcand = static_cast<uint64_t*>(S.cand.p);
    double* g = static_cast<double*>(S.g.p);
    const uint8_t* f0 = static_cast<const uint8_t*>(F) + size_t(v) * size_t(p.nt) * size_t(n) * es;
    // one row per workgroup up to 2^19 rows (latency-bound rows in flight), a multiple of 8
    const unsigned nrowblk = 8 * unsigned(std::min<int64_t>(65536, (p.ny * p.nz + 7) / 8));
    if (p.dtype == 0 && p.nx % 4 == 0 && (reinterpret_cast<uintptr_t>(f0) & 15) == 0)
      hipLaunchKernelGGL(k_gradient4, dim3{unsigned((p.ny * p.nz + 1) / 2)}, bl, 0, s, (const float*)f0, p.nx, p.ny,
                         p.nz, g);
    else if (p.dtype == 0)
      hipLaunchKernelGGL(k_gradient<float>, dim3{nrowblk}, bl, 0, s, (const float*)f0, p.nx, p.ny, p.nz, g);
    else
      hipLaunchKernelGGL(k_gradient<double>, dim3{nrowblk}, bl, 0, s, (const double*)f0, p.nx, p.ny, p.nz, g);
    PLAN_TRY(hipGetLastError());
    auto hist_pass = [&](uint64_t prefix, uint64_t pmask, int shift, uint32_t dmask, unsigned nblk) {
      hipLaunchKernelGGL(k_radix_hist, dim3{nblk}, bl, 0, s, (const double*)g, n, prefix, pmask, shift, dmask,
                         shift == 53 ? 1 : 0, dhist);
    };
    // exact order statistic k = floor(0.8 (n - 1)): three 11-bit radix passes
    // over g, then the points sharing the 33-bit prefix are gathered and the
    // rest of the selection runs on the host
    int64_t k = int64_t(std::floor(0.8 * double(n - 1)));
    uint64_t prefix = 0, pmask = 0;
    const unsigned nblk = unsigned(std::min<int64_t>(4096, (n + 255) / 256));
    if (S.hhist == nullptr) {
      void* q = nullptr;
      PLAN_TRY(hipHostMalloc(&q, 2048 * sizeof(unsigned int), hipHostMallocDefault));
      S.hhist = static_cast<unsigned int*>(q);
      PLAN_TRY(hipHostMalloc(&q, sizeof(unsigned long long), hipHostMallocDefault));
      S.hcount = static_cast<unsigned long long*>(q);
    }
    unsigned int* h = S.hhist;
    for (int pass = 0; pass < 3; ++pass) {
      const int shift = 53 - 11 * pass;
      const uint32_t dmask = 2047u;
      PLAN_TRY(hipMemsetAsync(dhist, 0, 2048 * sizeof(unsigned int), s));
      hist_pass(prefix, pmask, shift, dmask, nblk);
      PLAN_TRY(hipGetLastError());
      PLAN_TRY(hipMemcpyAsync(h, dhist, 2048 * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
      PLAN_TRY(hipStreamSynchronize(s));
      uint32_t d = 0;
      for (; d <= dmask; ++d) {
        if (k < int64_t(h[d])) break;
        k -= h[d];
      }
      if (d > dmask) {
        err = "radix selection lost its element";
        return hipErrorUnknown;
      }
      prefix |= uint64_t(d) << shift;
      pmask |= uint64_t(dmask) << shift;
    }
    PLAN_TRY(hipMemsetAsync(dcount, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_radix_compact, dim3{nblk}, bl, 0, s, (const double*)g, n, prefix, pmask, dcount, dcand,
                       cand_cap);
    PLAN_TRY(hipGetLastError());
    PLAN_TRY(hipMemcpyAsync(S.hcount, dcount, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    PLAN_TRY(hipStreamSynchronize(s));
    const unsigned long long ncand = *S.hcount;
    uint64_t thr_bits = 0;
    if (ncand <= cand_cap) {
      std::vector<uint64_t> cand(ncand);
      PLAN_TRY(hipMemcpy(cand.data(), dcand, size_t(ncand) * sizeof(uint64_t), hipMemcpyDeviceToHost));
      if (k >= int64_t(ncand)) {
        err = "radix selection lost its element";
        return hipErrorUnknown;
      }
      std::nth_element(cand.begin(), cand.begin() + k, cand.end());
      thr_bits = cand[k];
    } else {
      // too many ties on the prefix: finish with device passes (3 more digits)
      const int shifts[3] = {20, 9, 0};
      const int widths[3] = {11, 11, 9};
      for (int pass = 0; pass < 3; ++pass) {
        const uint32_t dmask = (1u << widths[pass]) - 1u;
        PLAN_TRY(hipMemsetAsync(dhist, 0, 2048 * sizeof(unsigned int), s));
        hist_pass(prefix, pmask, shifts[pass], dmask, nblk);
        PLAN_TRY(hipGetLastError());
        PLAN_TRY(hipMemcpyAsync(h, dhist, 2048 * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
        PLAN_TRY(hipStreamSynchronize(s));
        uint32_t d = 0;
        for (; d <= dmask; ++d) {
          if (k < int64_t(h[d])) break;
          k -= h[d];
        }
        if (d > dmask) {
          err = "radix selection lost its element";
          return hipErrorUnknown;
        }
        prefix |= uint64_t(d) << shifts[pass];
        pmask |= uint64_t(dmask) << shifts[pass];
      }
      thr_bits = prefix;
    }
    double thr;
    std::memcpy(&thr, &thr_bits, 8);
    const auto t1 = now();
    // node sums: finest level directly, coarser levels from their children
    {
      const int l = L - 1;
      const int64_t nn = NX[l] * NY[l] * NZ[l];
      const int64_t node_pts = int64_t(edges[l]) * edges[l] * (is3d ? edges[l] : 1);
      const int per_wave = node_pts > 64 ? 1 : 0;
      const dim3 gs{unsigned(per_wave ? (nn + 3) / 4 : (nn + 255) / 256)};
      hipLaunchKernelGGL(k_node_sums, gs, bl, 0, s, (const double*)g, p.nx, p.ny, p.nz, edges[l], is3d ? edges[l] : 1,
                         NX[l], NY[l], NZ[l], per_wave, dsum + off[l], dcnt + off[l]);
      PLAN_TRY(hipGetLastError());
    }
    for (int l = L - 2; l >= 0; --l) {
      const int64_t nn = NX[l] * NY[l] * NZ[l];
      hipLaunchKernelGGL(k_coarsen, dim3{unsigned((nn + 255) / 256)}, bl, 0, s, (const double*)(dsum + off[l + 1]),
                         (const int64_t*)(dcnt + off[l + 1]), NX[l + 1], NY[l + 1], NZ[l + 1], is3d ? 1 : 0, NX[l],
                         NY[l], NZ[l], dsum + off[l], dcnt + off[l]);
      PLAN_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_split_flags, dim3{unsigned((nodes + 255) / 256)}, bl, 0, s, (const double*)dsum,
                       (const int64_t*)dcnt, nodes, thr, dflag);
    PLAN_TRY(hipGetLastError());
    PLAN_TRY(hipMemcpyAsync(hflag[v].data(), dflag, size_t(nodes), hipMemcpyDeviceToHost, s));
    PLAN_TRY(hipStreamSynchronize(s));
    if (timing)
      std::fprintf(stderr, "[dls] plan var %d (stored gradient): percentile %.3f ms, flags %.3f ms\n", v,
                   ms(t0, t1), ms(t1, now()));
  }

  // the tree walk of every variable from its split flags
  for (int v = 0; v < p.nvars; ++v) {
    // the tree depends only on the flags and the grid: reuse the previous walk
    const std::array<int64_t, 5> key{p.nx, p.ny, p.nz, int64_t(p.px), int64_t(p.pmin)};
    if (S.prev_flags.size() < size_t(p.nvars)) {
      S.prev_flags.resize(p.nvars);
      S.prev_bits.resize(p.nvars);
      S.prev_leaves.resize(p.nvars);
      S.prev_key.resize(p.nvars, std::array<int64_t, 5>{-1, -1, -1, -1, -1});
    }
    if (S.prev_key[v] == key && S.prev_flags[v] == hflag[v]) {
      plan.leaves[v] = S.prev_leaves[v];
      plan.bits[v] = S.prev_bits[v];
      continue;
    }
    // depth-first walk: roots in (z, y, x) order, children in (z, y, x) order
    std::vector<Leaf>& leaves = plan.leaves[v];
    std::vector<uint8_t>& bits = plan.bits[v];
    struct Node { int l; int64_t ix, iy, iz; };
    std::vector<Node> stack;
    for (int64_t iz = 0; iz < NZ[0]; ++iz)
      for (int64_t iy = 0; iy < NY[0]; ++iy)
        for (int64_t ix = 0; ix < NX[0]; ++ix) {
          stack.push_back(Node{0, ix, iy, iz});
          while (!stack.empty()) {
            const Node nd = stack.back();
            stack.pop_back();
            const int e = edges[nd.l];
            const int64_t j = off[nd.l] + (nd.iz * NY[nd.l] + nd.iy) * NX[nd.l] + nd.ix;
            if (e > p.pmin) {
              const bool split = hflag[v][j] != 0;
              bits.push_back(split ? 1 : 0);
              if (split) {
                const int c = nd.l + 1;
                Node kids[8];
                int nk = 0;
                for (int dz = 0; dz < (is3d ? 2 : 1); ++dz)
                  for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                      const int64_t cx = 2 * nd.ix + dx, cy = 2 * nd.iy + dy, cz = is3d ? 2 * nd.iz + dz : 0;
                      if (cx < NX[c] && cy < NY[c] && cz < NZ[c]) kids[nk++] = Node{c, cx, cy, cz};
                    }
                for (int q = nk - 1; q >= 0; --q) stack.push_back(kids[q]);
                continue;
              }
            }
            const int64_t x0 = nd.ix * e, y0 = nd.iy * e, z0 = is3d ? nd.iz * e : 0;
            leaves.push_back(Leaf{int32_t(x0), int32_t(y0), int32_t(z0), int32_t(std::min<int64_t>(e, p.nx - x0)),
                                  int32_t(std::min<int64_t>(e, p.ny - y0)),
                                  int32_t(is3d ? std::min<int64_t>(e, p.nz - z0) : 1)});
          }
        }
    std::stable_sort(leaves.begin(), leaves.end(), [](const Leaf& a, const Leaf& b) {
      if (a.z0 != b.z0) return a.z0 < b.z0;
      if (a.y0 != b.y0) return a.y0 < b.y0;
      return a.x0 < b.x0;
    });
    S.prev_key[v] = key;
    S.prev_flags[v] = hflag[v];
    S.prev_leaves[v] = leaves;
    S.prev_bits[v] = bits;
  }
  return hipSuccess;
}

}  // namespace dls
