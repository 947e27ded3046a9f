// Noise step of the pipeline (arXiv:2412.08265, Sec. 3: the cube gets realistic noise; the paper
// gives no model). Every voxel v of a job's cube gets independent Gaussian noise of variance
// gain * max(C_v, 0) + sigma_floor^2. The standard normal deviates come from the counter-based
// Philox-4x32-10 generator (Salmon, Moraes, Dror, Shaw, SC 2011): key = the 64-bit seed, counter
// = (b_lo, b_hi, stream, 0) for the block b of voxels 4b .. 4b+3. Its outputs x0..x3 give
// u_k = (x_k + 1/2) 2^-32, and the Box-Muller transform turns each pair into two deviates (FP64):
// eps(4b) = r0 cos(2 pi u1), eps(4b+1) = r0 sin(2 pi u1) with r0 = sqrt(-2 ln u0), and likewise
// eps(4b+2), eps(4b+3) from (u2, u3). The result is a pure function of (seed, stream, v, C_v):
// independent of the launch shape and of the other jobs.
//
// An elementwise HBM stream (read and write 4 bytes per voxel). One thread per block of four
// voxels: one Philox block, two logarithms and two sine-cosine pairs (of pi times the argument,
// so no range reduction by 2 pi) per four voxels, and one 16-byte load and store where the cube
// is 16-byte aligned; grid-stride blocks of 256 threads, one launch per job.
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

// Deviates of voxels 4b .. 4b+3.
__device__ __forceinline__ void deviates4(uint64_t b, uint32_t stream, uint32_t k0, uint32_t k1,
                                          double (&e)[4]) {
  uint32_t c[4] = {(uint32_t)b, (uint32_t)(b >> 32), stream, 0u};
  philox4x32_10(c, k0, k1);
  const double u0 = ((double)c[0] + 0.5) * 0x1p-32, u1 = ((double)c[1] + 0.5) * 0x1p-32;
  const double u2 = ((double)c[2] + 0.5) * 0x1p-32, u3 = ((double)c[3] + 0.5) * 0x1p-32;
  const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  double s1, c1, s3, c3;
  sincospi(2.0 * u1, &s1, &c1);
  sincospi(2.0 * u3, &s3, &c3);
  e[0] = r0 * c1;
  e[1] = r0 * s1;
  e[2] = r1 * c3;
  e[3] = r1 * s3;
}

__device__ __forceinline__ float noisy(float x, double eps, double gain, double floor2) {
  const double xd = (double)x;
  return (float)(xd + sqrt(gain * fmax(xd, 0.0) + floor2) * eps);
}

__global__ __launch_bounds__(256) void k_noise(float *__restrict__ cube, int64_t n, uint32_t k0,
                                              uint32_t k1, uint32_t stream, double gain,
                                              double floor2) {
  const int64_t nb = (n + 3) >> 2;
  const bool vec = (reinterpret_cast<uintptr_t>(cube) & 15u) == 0;
  for (int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x; b < nb; b += (int64_t)gridDim.x * 256) {
    double e[4];
    deviates4((uint64_t)b, stream, k0, k1, e);
    const int64_t v = b * 4;
    if (vec && v + 4 <= n) {
      float4 x = *reinterpret_cast<const float4 *>(cube + v);
      x.x = noisy(x.x, e[0], gain, floor2);
      x.y = noisy(x.y, e[1], gain, floor2);
      x.z = noisy(x.z, e[2], gain, floor2);
      x.w = noisy(x.w, e[3], gain, floor2);
      *reinterpret_cast<float4 *>(cube + v) = x;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (v + k < n) cube[v + k] = noisy(cube[v + k], e[k], gain, floor2);
    }
  }
}

hipError_t launch_noise(float *cube, int64_t n, uint64_t seed, uint32_t stream, double gain,
                        double sigma_floor, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(((n + 3) / 4 + 255) / 256, 8192);
  hipLaunchKernelGGL(k_noise, dim3((unsigned)blocks), dim3(256), 0, s, cube, n, (uint32_t)seed,
                     (uint32_t)(seed >> 32), stream, gain, sigma_floor * sigma_floor);
  return hipGetLastError();
}

}  // namespace rubix
