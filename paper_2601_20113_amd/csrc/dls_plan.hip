// Adaptive (quadtree / octree) patch plan, computed from snapshot 0 of each
// variable.  The paper partitions the domain into patches of one size
// (Sec. 2.3, Alg. 1 step 2); the adaptive plan refines a node of edge e > pmin
// into its half-edge children while the mean gradient magnitude over the node
// exceeds the 80th percentile of the snapshot's gradient magnitude.
//
// Device side: gradient magnitude in FP64 (central differences inside,
// one-sided at the ends), the exact order statistic sorted(g)[floor(0.8 (n-1))]
// by radix selection over the FP64 bit patterns (11-bit digits, 6 passes),
// and per-level node sums.  Host side: the depth-first walk that emits the
// split bits and the leaves in (z0, y0, x0) order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dls_internal.h"
#include "dls_kernels.h"

namespace dls {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_gradient(const T* __restrict__ f0, int64_t nx, int64_t ny, int64_t nz,
                                                  double* __restrict__ g) {
  const int64_t n = nx * ny * nz;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
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
  g[i] = sqrt(dx * dx + dy * dy + dz * dz);
}

// histogram of digit (bits >> shift) & dmask among elements whose bits match
// `prefix` under `pmask`
__global__ __launch_bounds__(256) void k_radix_hist(const double* __restrict__ g, int64_t n, uint64_t prefix,
                                                    uint64_t pmask, int shift, uint32_t dmask,
                                                    unsigned int* __restrict__ hist) {
  __shared__ unsigned int h[2048];
  for (int j = threadIdx.x; j < 2048; j += 256) h[j] = 0;
  __syncthreads();
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const uint64_t b = uint64_t(__double_as_longlong(g[i]));
    if ((b & pmask) == prefix) atomicAdd(&h[(b >> shift) & dmask], 1u);
  }
  __syncthreads();
  for (int j = threadIdx.x; j <= int(dmask); j += 256)
    if (h[j]) atomicAdd(hist + j, h[j]);
}

// finest-level node sums and counts of g (node edge e, node grid NX x NY x NZ)
__global__ __launch_bounds__(256) void k_node_sums(const double* __restrict__ g, int64_t nx, int64_t ny, int64_t nz,
                                                   int e, int ez, int64_t NX, int64_t NY, int64_t NZ,
                                                   double* __restrict__ sum, int64_t* __restrict__ cnt) {
  const int64_t nn = NX * NY * NZ;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= nn) return;
  const int64_t ix = i % NX, iy = (i / NX) % NY, iz = i / (NX * NY);
  const int64_t x0 = ix * e, y0 = iy * e, z0 = iz * ez;
  const int64_t x1 = x0 + e < nx ? x0 + e : nx, y1 = y0 + e < ny ? y0 + e : ny, z1 = z0 + ez < nz ? z0 + ez : nz;
  double s = 0.0;
  for (int64_t z = z0; z < z1; ++z)
    for (int64_t y = y0; y < y1; ++y)
      for (int64_t x = x0; x < x1; ++x) s += g[(z * ny + y) * nx + x];
  sum[i] = s;
  cnt[i] = (x1 - x0) * (y1 - y0) * (z1 - z0);
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
  DevMem g, hist, sums, cnts;
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
  double* dsum = static_cast<double*>(S.sums.p);
  int64_t* dcnt = static_cast<int64_t*>(S.cnts.p);
  unsigned int* dhist = static_cast<unsigned int*>(S.hist.p);
  double* g = static_cast<double*>(S.g.p);
  std::vector<double> hsum(off[L]);
  std::vector<int64_t> hcnt(off[L]);
  plan.leaves.assign(p.nvars, {});
  plan.bits.assign(p.nvars, {});
  const int es = p.esize();
  for (int v = 0; v < p.nvars; ++v) {
    const uint8_t* f0 = static_cast<const uint8_t*>(F) + size_t(v) * size_t(p.nt) * size_t(n) * es;
    const dim3 gn{unsigned((n + 255) / 256)}, bl{256};
    if (p.dtype == 0)
      hipLaunchKernelGGL(k_gradient<float>, gn, bl, 0, s, (const float*)f0, p.nx, p.ny, p.nz, g);
    else
      hipLaunchKernelGGL(k_gradient<double>, gn, bl, 0, s, (const double*)f0, p.nx, p.ny, p.nz, g);
    PLAN_TRY(hipGetLastError());
    // exact order statistic k = floor(0.8 (n - 1)) by radix selection
    int64_t k = int64_t(std::floor(0.8 * double(n - 1)));
    uint64_t prefix = 0, pmask = 0;
    const int shifts[6] = {53, 42, 31, 20, 9, 0};
    const int widths[6] = {11, 11, 11, 11, 11, 9};
    const unsigned nblk = unsigned(std::min<int64_t>(2048, (n + 255) / 256));
    std::vector<unsigned int> h(2048);
    for (int pass = 0; pass < 6; ++pass) {
      const uint32_t dmask = (1u << widths[pass]) - 1u;
      PLAN_TRY(hipMemsetAsync(dhist, 0, 2048 * sizeof(unsigned int), s));
      hipLaunchKernelGGL(k_radix_hist, dim3{nblk}, bl, 0, s, (const double*)g, n, prefix, pmask, shifts[pass],
                         dmask, dhist);
      PLAN_TRY(hipGetLastError());
      PLAN_TRY(hipMemcpyAsync(h.data(), dhist, 2048 * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
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
    double thr;
    std::memcpy(&thr, &prefix, 8);
    // node sums: finest level directly, coarser levels from their children
    {
      const int l = L - 1;
      const int64_t nn = NX[l] * NY[l] * NZ[l];
      hipLaunchKernelGGL(k_node_sums, dim3{unsigned((nn + 255) / 256)}, bl, 0, s, (const double*)g, p.nx, p.ny,
                         p.nz, edges[l], is3d ? edges[l] : 1, NX[l], NY[l], NZ[l], dsum + off[l], dcnt + off[l]);
      PLAN_TRY(hipGetLastError());
    }
    for (int l = L - 2; l >= 0; --l) {
      const int64_t nn = NX[l] * NY[l] * NZ[l];
      hipLaunchKernelGGL(k_coarsen, dim3{unsigned((nn + 255) / 256)}, bl, 0, s, (const double*)(dsum + off[l + 1]),
                         (const int64_t*)(dcnt + off[l + 1]), NX[l + 1], NY[l + 1], NZ[l + 1], is3d ? 1 : 0, NX[l],
                         NY[l], NZ[l], dsum + off[l], dcnt + off[l]);
      PLAN_TRY(hipGetLastError());
    }
    PLAN_TRY(hipMemcpyAsync(hsum.data(), dsum, size_t(off[L]) * sizeof(double), hipMemcpyDeviceToHost, s));
    PLAN_TRY(hipMemcpyAsync(hcnt.data(), dcnt, size_t(off[L]) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PLAN_TRY(hipStreamSynchronize(s));
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
              const bool split = hsum[j] / double(hcnt[j]) > thr;
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
  }
  return hipSuccess;
}

}  // namespace dls
