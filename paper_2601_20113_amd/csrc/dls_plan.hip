// Adaptive (quadtree / octree) patch plan, computed from snapshot 0 of each
// variable.  The paper partitions the domain into patches of one size
// (Sec. 2.3, Alg. 1 step 2); the adaptive plan refines a node of edge e > pmin
// into its half-edge children while the mean gradient magnitude over the node
// exceeds the 80th percentile of the snapshot's gradient magnitude.
//
// Device side: gradient magnitude in FP64 (central differences inside,
// one-sided at the ends), stored once; the exact order statistic
// sorted(g)[floor(0.8 (n-1))] by radix selection over the FP64 bit patterns
// (three 11-bit digit passes, then the few points sharing the 33-bit prefix
// are gathered and selected on the host); per-level node sums.  Host side: the depth-first walk that emits the split
// bits and the leaves in (z0, y0, x0) order.
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
  DevMem g, cand, hist, sums, cnts, count, flags;
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
  PLAN_TRY(S.g.ensure(size_t(n) * sizeof(double)));
  PLAN_TRY(S.hist.ensure(2048 * sizeof(unsigned int)));
  PLAN_TRY(S.count.ensure(sizeof(unsigned long long)));
  const unsigned long long cand_cap = 1ULL << 22;
  PLAN_TRY(S.cand.ensure(size_t(cand_cap) * sizeof(uint64_t)));
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
  PLAN_TRY(S.sums.ensure(size_t(off[L]) * sizeof(double)));
  PLAN_TRY(S.cnts.ensure(size_t(off[L]) * sizeof(int64_t)));
  PLAN_TRY(S.flags.ensure(size_t(off[L])));
  double* dsum = static_cast<double*>(S.sums.p);
  int64_t* dcnt = static_cast<int64_t*>(S.cnts.p);
  unsigned int* dhist = static_cast<unsigned int*>(S.hist.p);
  unsigned long long* dcount = static_cast<unsigned long long*>(S.count.p);
  uint64_t* dcand = static_cast<uint64_t*>(S.cand.p);
  double* g = static_cast<double*>(S.g.p);
  uint8_t* dflag = static_cast<uint8_t*>(S.flags.p);
  std::vector<uint8_t> hflag(off[L]);
  plan.leaves.assign(p.nvars, {});
  plan.bits.assign(p.nvars, {});
  const int es = p.esize();
  const bool timing = std::getenv("DLS_TIMING") != nullptr;
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  for (int v = 0; v < p.nvars; ++v) {
    const auto t0 = now();
    const uint8_t* f0 = static_cast<const uint8_t*>(F) + size_t(v) * size_t(p.nt) * size_t(n) * es;
    const dim3 bl{256};
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
    hipLaunchKernelGGL(k_split_flags, dim3{unsigned((off[L] + 255) / 256)}, bl, 0, s, (const double*)dsum,
                       (const int64_t*)dcnt, off[L], thr, dflag);
    PLAN_TRY(hipGetLastError());
    PLAN_TRY(hipMemcpyAsync(hflag.data(), dflag, size_t(off[L]), hipMemcpyDeviceToHost, s));
    PLAN_TRY(hipStreamSynchronize(s));
    const auto t2 = now();
    // the tree depends only on the flags and the grid: reuse the previous walk
    const std::array<int64_t, 5> key{p.nx, p.ny, p.nz, int64_t(p.px), int64_t(p.pmin)};
    if (S.prev_flags.size() < size_t(p.nvars)) {
      S.prev_flags.resize(p.nvars);
      S.prev_bits.resize(p.nvars);
      S.prev_leaves.resize(p.nvars);
      S.prev_key.resize(p.nvars, std::array<int64_t, 5>{-1, -1, -1, -1, -1});
    }
    if (S.prev_key[v] == key && S.prev_flags[v] == hflag) {
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
              const bool split = hflag[j] != 0;
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
    S.prev_flags[v] = hflag;
    S.prev_leaves[v] = leaves;
    S.prev_bits[v] = bits;
    if (timing)
      std::fprintf(stderr, "[dls] plan var %d: percentile %.3f ms, node sums %.3f ms, tree %.3f ms, %zu leaves\n", v,
                   ms(t0, t1), ms(t1, t2), ms(t2, now()), leaves.size());
  }
  return hipSuccess;
}

}  // namespace dls
