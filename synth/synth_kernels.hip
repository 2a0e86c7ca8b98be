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

}  // namespace

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
