// Noise step of the pipeline (arXiv:2412.08265, Sec. 3: the cube gets realistic noise; the paper
// gives no model). Every voxel v of a job's cube gets independent Gaussian noise of variance
// gain * max(C_v, 0) + sigma_floor^2. The standard normal deviate of voxel v is drawn from the
// counter-based Philox-4x32-10 generator (Salmon, Moraes, Dror, Shaw, SC 2011): key = the 64-bit
// seed, counter = (v_lo, v_hi, stream, 0); its first two outputs x0, x1 give u = (x + 1/2) 2^-32
// and eps = sqrt(-2 ln u0) cos(2 pi u1) (Box-Muller, FP64). The result is a pure function of
// (seed, stream, v, C_v): independent of the launch shape and of the other jobs.
//
// An elementwise HBM stream (read and write 4 bytes per voxel) with ~100 integer and FP64 ops per
// voxel; grid-stride blocks of 256 threads, one launch per job.
#include "rubix_internal.h"

namespace rubix {

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ __launch_bounds__(256) void k_noise(float *__restrict__ cube, int64_t n, uint32_t k0,
                                              uint32_t k1, uint32_t stream, double gain,
                                              double floor2) {
  const double two_pi = 6.283185307179586;   // 2 pi rounded to FP64
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
    uint32_t c[4] = {(uint32_t)v, (uint32_t)((uint64_t)v >> 32), stream, 0u};
    philox4x32_10(c, k0, k1);
    const double u0 = ((double)c[0] + 0.5) * 0x1p-32;
    const double u1 = ((double)c[1] + 0.5) * 0x1p-32;
    const double eps = sqrt(-2.0 * log(u0)) * cos(two_pi * u1);
    const double x = (double)cube[v];
    cube[v] = (float)(x + sqrt(gain * fmax(x, 0.0) + floor2) * eps);
  }
}

hipError_t launch_noise(float *cube, int64_t n, uint64_t seed, uint32_t stream, double gain,
                        double sigma_floor, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_noise, dim3((unsigned)blocks), dim3(256), 0, s, cube, n, (uint32_t)seed,
                     (uint32_t)(seed >> 32), stream, gain, sigma_floor * sigma_floor);
  return hipGetLastError();
}

}  // namespace rubix
