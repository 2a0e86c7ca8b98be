// Device-side input generators (harness only; no step of the compression
// method lives here).  They evaluate, on the GPU, the same formulas as the
// NumPy generators in synth/__init__.py, with the per-mode constants
// (wave vectors, amplitudes, phases, drifts, decay factors) drawn on the host
// and passed in, so both sides agree up to the last bit of the FP64 cosine.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr double kTwoPi = 6.283185307179586;

// u[t][z][y][x] = T( (sum_j amp_j cos(2 pi ((kz z mod nz)/nz + (ky y mod ny)/ny
//                      + (kx x mod nx)/nx) + phi_j [+ omega_j t])) * dec[t] )
template <typename T>
__global__ __launch_bounds__(256) void k_spectrum(T* __restrict__ out, int64_t nx, int64_t ny, int64_t nz,
                                                  int64_t nt, int nmodes, const int64_t* __restrict__ k,
                                                  const double* __restrict__ amp, const double* __restrict__ phi,
                                                  const double* __restrict__ omega, const double* __restrict__ dec,
                                                  int drift) {
  const int64_t npts = nx * ny * nz;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= npts) return;
  const int64_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
  if (!drift) {
    double base = 0.0;
    for (int j = 0; j < nmodes; ++j) {
      const double pxf = double(((k[3 * j] * x) % nx + nx) % nx) / double(nx);
      const double pyf = double(((k[3 * j + 1] * y) % ny + ny) % ny) / double(ny);
      const double pzf = double(((k[3 * j + 2] * z) % nz + nz) % nz) / double(nz);
      const double ph = kTwoPi * ((pzf + pyf) + pxf);
      base = base + amp[j] * cos(ph + phi[j]);
    }
    for (int64_t t = 0; t < nt; ++t) out[t * npts + i] = T(base * dec[t]);
  } else {
    for (int64_t t = 0; t < nt; ++t) {
      double acc = 0.0;
      for (int j = 0; j < nmodes; ++j) {
        const double pxf = double(((k[3 * j] * x) % nx + nx) % nx) / double(nx);
        const double pyf = double(((k[3 * j + 1] * y) % ny + ny) % ny) / double(ny);
        const double pzf = double(((k[3 * j + 2] * z) % nz + nz) % nz) / double(nz);
        const double ph = kTwoPi * ((pzf + pyf) + pxf) + phi[j];
        acc = acc + amp[j] * cos(ph + omega[j] * double(t));
      }
      out[t * npts + i] = T(acc * dec[t]);
    }
  }
}

// Philox4x32-10 (Salmon et al., SC'11) and one Box-Muller draw per element.
__device__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = uint64_t(0xD2511F53u) * c[0];
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c[2];
    const uint32_t n0 = uint32_t(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = uint32_t(p1);
    const uint32_t n2 = uint32_t(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = uint32_t(p0);
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ inline double philox_normal(uint64_t idx, uint32_t seed, double std) {
  uint32_t c[4] = {uint32_t(idx), uint32_t(idx >> 32), 0u, 0u};
  philox(c, seed, 0x5EEDu);
  const double u1 = (double(c[0]) + 1.0) * 2.3283064365386963e-10;
  const double u2 = double(c[1]) * 2.3283064365386963e-10;
  return std * sqrt(-2.0 * log(u1)) * cos(kTwoPi * u2);
}

// One workgroup per (64 x 64 tile, time step); the tile's blob list holds
// every blob whose truncated box can reach the tile at some time.
template <typename T>
__global__ __launch_bounds__(256) void k_blobs(T* __restrict__ out, int64_t nx, int64_t ny, int tiles_x,
                                               const double* __restrict__ bp, const int32_t* __restrict__ tstart,
                                               const int32_t* __restrict__ tlist, double trunc, uint32_t seed,
                                               double noise_std) {
  const int tile = blockIdx.x, t = blockIdx.y;
  const int64_t tx0 = int64_t(tile % tiles_x) * 64, ty0 = int64_t(tile / tiles_x) * 64;
  const int b0 = tstart[tile], b1 = tstart[tile + 1];
  for (int q = threadIdx.x; q < 64 * 64; q += 256) {
    const int64_t x = tx0 + (q & 63), y = ty0 + (q >> 6);
    if (x >= nx || y >= ny) continue;
    double acc = 0.0;
    for (int j = b0; j < b1; ++j) {
      const int b = tlist[j];
      const double w = bp[5 * b + 2];
      const double cx = bp[5 * b + 0] + bp[5 * b + 3] * double(t);
      const double cy = bp[5 * b + 1] + bp[5 * b + 4] * double(t);
      const double R = trunc * w;
      const double ddx = double(x) - cx, ddy = double(y) - cy;
      if (fabs(ddx) <= R && fabs(ddy) <= R) acc = acc + exp(-(ddx * ddx + ddy * ddy) / (2.0 * w * w));
    }
    const uint64_t idx = uint64_t(t) * uint64_t(ny * nx) + uint64_t(y * nx + x);
    acc = acc + philox_normal(idx, seed, noise_std);
    out[int64_t(t) * nx * ny + y * nx + x] = T(acc);
  }
}

}  // namespace

extern "C" int synth_blobs(void* out, int dtype, int64_t nx, int64_t ny, int64_t nt, const double* d_bp,
                           const int32_t* d_tstart, const int32_t* d_tlist, double trunc, uint32_t seed,
                           double noise_std, void* stream) {
  if (nx <= 0 || ny <= 0 || nt <= 0) return 1;
  const int tiles_x = int((nx + 63) / 64), tiles_y = int((ny + 63) / 64);
  const dim3 g{unsigned(tiles_x * tiles_y), unsigned(nt)}, b{256};
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == 0)
    hipLaunchKernelGGL(k_blobs<float>, g, b, 0, s, (float*)out, nx, ny, tiles_x, d_bp, d_tstart, d_tlist, trunc, seed,
                       noise_std);
  else
    hipLaunchKernelGGL(k_blobs<double>, g, b, 0, s, (double*)out, nx, ny, tiles_x, d_bp, d_tstart, d_tlist, trunc,
                       seed, noise_std);
  return int(hipGetLastError());
}

extern "C" int synth_spectrum(void* out, int dtype, int64_t nx, int64_t ny, int64_t nz, int64_t nt,
                              int nmodes, const int64_t* d_k, const double* d_amp, const double* d_phi,
                              const double* d_omega, const double* d_dec, int drift, void* stream) {
  const int64_t npts = nx * ny * nz;
  if (npts <= 0 || nt <= 0 || nmodes <= 0) return 1;
  const dim3 g{unsigned((npts + 255) / 256)}, b{256};
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == 0)
    hipLaunchKernelGGL(k_spectrum<float>, g, b, 0, s, (float*)out, nx, ny, nz, nt, nmodes, d_k, d_amp, d_phi,
                       d_omega, d_dec, drift);
  else
    hipLaunchKernelGGL(k_spectrum<double>, g, b, 0, s, (double*)out, nx, ny, nz, nt, nmodes, d_k, d_amp, d_phi,
                       d_omega, d_dec, drift);
  return int(hipGetLastError());
}
