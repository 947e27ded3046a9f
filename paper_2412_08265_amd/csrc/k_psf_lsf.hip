// Step 7 of the pipeline (arXiv:2412.08265, Sec. 3, with the Gaussian PSF/LSF of Sec. 4): a
// separable, zero-padded Gaussian convolution of the cube along lambda (LSF), y and x (PSF).
//
// Each pass is an HBM-bound 1-D stencil. A work item stages its input tile plus a halo of r
// values in LDS with lane-contiguous (coalesced) loads and writes each output once:
//   k_lsf    (spaxel, 256-bin tile): a contiguous run of one spectrum;
//   k_psf<A> (line, 128-spaxel segment, 64-bin tile): 64 lanes span lambda, so every load of a
//            neighbouring spaxel is a contiguous 256-byte row segment.
// The normalised FP32 weights come with the job table (computed on the host in FP64).
#include "rubix_internal.h"

namespace rubix {

__global__ __launch_bounds__(kLsfTL) void k_lsf(const Table *__restrict__ T) {
  __shared__ float buf[kLsfTL + 2 * RUBIX_MAX_RADIUS];
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_LSF]; vb += gridDim.x) {
    const int jj = find_job(T, K_LSF, vb);
    const JobDev &J = jobs[jj];
    const int nt = (J.n_tel + kLsfTL - 1) / kLsfTL;
    const int64_t local = vb - J.vb_start[K_LSF];
    const int64_t s = local / nt;
    const int t = (int)(local - s * nt);
    const int r = J.lsf_r;
    const float *__restrict__ src = J.pl_src[0] + s * J.n_tel;
    float *__restrict__ dst = J.pl_dst[0] + s * J.n_tel;
    const int j0 = t * kLsfTL;
    for (int q = threadIdx.x; q < kLsfTL + 2 * r; q += kLsfTL) {
      const int jj2 = j0 - r + q;
      buf[q] = (jj2 >= 0 && jj2 < J.n_tel) ? src[jj2] : 0.f;
    }
    __syncthreads();
    const int jb = j0 + threadIdx.x;
    if (jb < J.n_tel) {
      float acc = 0.f;
      for (int k = 0; k <= 2 * r; ++k) acc = fmaf(J.lsf_w[k], buf[threadIdx.x + k], acc);
      dst[jb] = acc;
    }
    __syncthreads();
  }
}

// AXIS 0: PSF along y (a line is one x column); AXIS 1: PSF along x (a line is one y row).
template <int AXIS>
__global__ __launch_bounds__(256) void k_psf(const Table *__restrict__ T) {
  __shared__ float buf[(kPsfSeg + 2 * RUBIX_MAX_RADIUS) * kPsfLanes];
  const JobDev *jobs = table_jobs(T);
  const int kind = AXIS == 0 ? K_PSFY : K_PSFX;
  const int lane = threadIdx.x & 63;
  const int grp = threadIdx.x >> 6;
  for (int64_t vb = blockIdx.x; vb < T->h.total[kind]; vb += gridDim.x) {
    const int jj = find_job(T, kind, vb);
    const JobDev &J = jobs[jj];
    const int nseg = AXIS == 0 ? J.n_psf_seg_y : J.n_psf_seg_x;
    const int ntl = J.n_psf_tiles;
    const int64_t local = vb - J.vb_start[kind];
    const int line = (int)(local / ((int64_t)nseg * ntl));
    const int rem = (int)(local - (int64_t)line * nseg * ntl);
    const int seg = rem / ntl;
    const int lt = rem - seg * ntl;
    const int L = AXIS == 0 ? J.ny : J.nx;
    const int q0 = seg * kPsfSeg;
    const int q1 = min(L, q0 + kPsfSeg);
    const int r = J.psf_r;
    const int jb = lt * kPsfLanes + lane;
    const bool act = jb < J.n_tel;
    const float *__restrict__ src = J.pl_src[1 + AXIS];
    float *__restrict__ dst = J.pl_dst[1 + AXIS];
    // spaxel index of position q on this line
    auto spx = [&](int q) -> int64_t {
      return AXIS == 0 ? (int64_t)q * J.nx + line : (int64_t)line * J.nx + q;
    };
    for (int q = q0 - r + grp; q < q1 + r; q += 4) {
      float v = 0.f;
      if (act && q >= 0 && q < L) v = src[spx(q) * J.n_tel + jb];
      buf[(q - (q0 - r)) * kPsfLanes + lane] = v;
    }
    __syncthreads();
    for (int q = q0 + grp; q < q1; q += 4) {
      float acc = 0.f;
      const float *b = buf + (q - q0) * kPsfLanes + lane;
      for (int k = 0; k <= 2 * r; ++k) acc = fmaf(J.psf_w[k], b[k * kPsfLanes], acc);
      if (act) dst[spx(q) * J.n_tel + jb] = acc;
    }
    __syncthreads();
  }
}

// Identity operator (no PSF and no LSF) into a separate output buffer.
__global__ __launch_bounds__(256) void k_copy(const Table *__restrict__ T) {
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_COPY]; vb += gridDim.x) {
    const int jj = find_job(T, K_COPY, vb);
    const JobDev &J = jobs[jj];
    const int64_t base = (vb - J.vb_start[K_COPY]) * 65536;
    for (int q = threadIdx.x; q < 65536; q += 256) {
      const int64_t e = base + q;
      if (e < J.cube_elems) J.copy_dst[e] = J.copy_src[e];
    }
  }
}

static inline int grid_for(int64_t total, int cap) {
  if (total <= 0) return 0;
  int64_t g = total;
  if (cap > 0 && g > cap) g = cap;
  if (g > 0x7fffffff) g = 0x7fffffff;
  return (int)g;
}

hipError_t launch_psf_lsf(const Table *dt, const TableHeader &h, int cap, hipStream_t s) {
  int g;
  if ((g = grid_for(h.total[K_LSF], cap))) hipLaunchKernelGGL(k_lsf, dim3(g), dim3(kLsfTL), 0, s, dt);
  if ((g = grid_for(h.total[K_PSFY], cap))) hipLaunchKernelGGL(k_psf<0>, dim3(g), dim3(256), 0, s, dt);
  if ((g = grid_for(h.total[K_PSFX], cap))) hipLaunchKernelGGL(k_psf<1>, dim3(g), dim3(256), 0, s, dt);
  if ((g = grid_for(h.total[K_COPY], cap))) hipLaunchKernelGGL(k_copy, dim3(g), dim3(256), 0, s, dt);
  return hipGetLastError();
}

}  // namespace rubix
