// Step 7 of the pipeline (arXiv:2412.08265, Sec. 3, with the Gaussian PSF/LSF of Sec. 4): a
// separable, zero-padded Gaussian convolution of the cube along lambda (LSF), y and x (PSF).
//
// Each pass is an HBM-bound 1-D stencil. A work item stages its input tile plus a halo of r values
// in LDS with lane-contiguous (coalesced) loads and writes each output once; every lane computes
// four outputs from one run of LDS values (register blocking), so an LDS value feeds four filter
// taps instead of one:
//   k_lsf    (spaxel, 2048-bin run): thread t owns bins 1024g + 4t .. +3 (g = 0, 1) and reads the
//            staged run with aligned 16-byte LDS loads;
//   k_psf<A> (line, 64-spaxel segment, 64-bin tile): 64 lanes span lambda (every load of a
//            neighbouring spaxel is a contiguous 256-byte row segment); wave w owns 16 output
//            positions of the segment, four at a time.
// The normalised FP32 weights come with the job table (computed on the host in FP64), padded with
// kWPad zeros on both sides so a blocked filter needs no branch at the ends of its window.
#include "rubix_internal.h"

namespace rubix {

// staging loads per thread in flight together: the LSF's whole run with any radius in one
// batch; the PSF's 64 + 2r + 4 rows in one batch for r <= 14
constexpr int kLsfBatch = (kLsfOut + 2 * RUBIX_MAX_RADIUS + 4 + 255) / 256;
constexpr int kPsfBatch = 24;

__global__ __launch_bounds__(256) void k_lsf(const Table *__restrict__ T) {
  __shared__ __attribute__((aligned(16))) float buf[kLsfOut + 2 * RUBIX_MAX_RADIUS + 8];
  const JobDev *jobs = table_jobs(T);
  const int tid = threadIdx.x;
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_LSF]; vb += gridDim.x) {
    const int jj = find_job(T, K_LSF, vb);
    const JobDev &J = jobs[jj];
    const int nt = (J.n_tel + kLsfOut - 1) / kLsfOut;
    const int64_t local = vb - J.vb_start[K_LSF];
    const int64_t s = local / nt;
    const int t = (int)(local - s * nt);
    const int r = J.lsf_r;
    const float *__restrict__ src = J.pl_src[0] + s * J.n_tel;
    float *__restrict__ dst = J.pl_dst[0] + s * J.n_tel;
    const int j0 = t * kLsfOut;
    const int nload = kLsfOut + 2 * r + 4;       // + 4: the last float4 of a lane's window
    // staging in batches of kLsfBatch loads per thread, all in flight before the LDS writes:
    // each load reads a clamped, always valid index and a bit mask zeroes what lies outside the
    // row (no load sits behind a branch)
    for (int q0 = tid; q0 < nload; q0 += 256 * kLsfBatch) {
      uint32_t v[kLsfBatch];
#pragma unroll
      for (int b = 0; b < kLsfBatch; ++b) {
        const int jj2 = j0 - r + q0 + 256 * b;
        const uint32_t x = __float_as_uint(src[min(max(jj2, 0), J.n_tel - 1)]);
        v[b] = x & ((jj2 >= 0 && jj2 < J.n_tel) ? 0xffffffffu : 0u);
      }
#pragma unroll
      for (int b = 0; b < kLsfBatch; ++b)
        if (q0 + 256 * b < nload) buf[q0 + 256 * b] = __uint_as_float(v[b]);
    }
    __syncthreads();
    // thread t owns the runs of 4 bins at 1024 g + 4t, g = 0 .. kLsfOut/1024 - 1:
    // out[4t + i] = sum_{k=0..2r} w_k buf[4t + i + k] = sum_o wp[o - i] buf[4t + o], o = 0..2r+3,
    // wp[m] = weight of offset m (zero outside 0..2r)
    for (int g = 0; g < kLsfOut / 1024; ++g) {
    const int t4 = 1024 * g + 4 * tid;
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
    const float *wp = J.lsf_w + kWPad;            // wp[m], m in [-kWPad, 2r + kWPad]
    const int nq = (2 * r + 4 + 3) / 4;
    for (int m = 0; m < nq; ++m) {
      const float4 x = *reinterpret_cast<const float4 *>(&buf[t4 + 4 * m]);
      const int o = 4 * m;
      acc0 = fmaf(wp[o], x.x, acc0);
      acc1 = fmaf(wp[o - 1], x.x, acc1);
      acc2 = fmaf(wp[o - 2], x.x, acc2);
      acc3 = fmaf(wp[o - 3], x.x, acc3);
      acc0 = fmaf(wp[o + 1], x.y, acc0);
      acc1 = fmaf(wp[o], x.y, acc1);
      acc2 = fmaf(wp[o - 1], x.y, acc2);
      acc3 = fmaf(wp[o - 2], x.y, acc3);
      acc0 = fmaf(wp[o + 2], x.z, acc0);
      acc1 = fmaf(wp[o + 1], x.z, acc1);
      acc2 = fmaf(wp[o], x.z, acc2);
      acc3 = fmaf(wp[o - 1], x.z, acc3);
      acc0 = fmaf(wp[o + 3], x.w, acc0);
      acc1 = fmaf(wp[o + 2], x.w, acc1);
      acc2 = fmaf(wp[o + 1], x.w, acc2);
      acc3 = fmaf(wp[o], x.w, acc3);
    }
    const int jb = j0 + t4;
    if (jb + 3 < J.n_tel && (((uintptr_t)(dst + jb)) & 15) == 0) {
      *reinterpret_cast<float4 *>(dst + jb) = make_float4(acc0, acc1, acc2, acc3);
    } else {
      if (jb < J.n_tel) dst[jb] = acc0;
      if (jb + 1 < J.n_tel) dst[jb + 1] = acc1;
      if (jb + 2 < J.n_tel) dst[jb + 2] = acc2;
      if (jb + 3 < J.n_tel) dst[jb + 3] = acc3;
    }
    }
    __syncthreads();
  }
}

// AXIS 0: PSF along y (a line is one x column); AXIS 1: PSF along x (a line is one y row).
// Dynamic LDS: (kPsfSeg + 2 * max_psf_r) rows of kPsfLanes floats.
template <int AXIS>
__global__ __launch_bounds__(256) void k_psf(const Table *__restrict__ T) {
  extern __shared__ float buf[];
  const JobDev *jobs = table_jobs(T);
  const int kind = AXIS == 0 ? K_PSFY : K_PSFX;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
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
    auto spx = [&](int q) -> int64_t {
      return AXIS == 0 ? (int64_t)q * J.nx + line : (int64_t)line * J.nx + q;
    };
    // rows q0 - r .. q0 + kPsfSeg + r + 3 (the last rows only feed masked blocked outputs)
    const int nrow = kPsfSeg + 2 * r + 4;
    // staging in batches of kPsfBatch rows per wave with every load in flight before the LDS
    // writes: each load reads a clamped, always valid element of the line, and the zero padding
    // is a bit mask on the loaded value (no load sits behind a branch)
    // (the row of each load is wave-uniform: its base is scalar, the lane offset is shared)
    const int jc = min(jb, J.n_tel - 1);
    for (int t0 = __builtin_amdgcn_readfirstlane(w); t0 < nrow; t0 += 4 * kPsfBatch) {
      uint32_t v[kPsfBatch];
#pragma unroll
      for (int b = 0; b < kPsfBatch; ++b) {
        const int q = q0 - r + t0 + 4 * b;
        const float *row = src + spx(min(max(q, 0), L - 1)) * J.n_tel;
        const uint32_t x = __float_as_uint(row[jc]);
        v[b] = x & ((act && q >= 0 && q < L) ? 0xffffffffu : 0u);
      }
#pragma unroll
      for (int b = 0; b < kPsfBatch; ++b)
        if (t0 + 4 * b < nrow) buf[(t0 + 4 * b) * kPsfLanes + lane] = __uint_as_float(v[b]);
    }
    __syncthreads();
    const float *wp = J.psf_w + kWPad;
    for (int b = 0; b < 4; ++b) {
      const int qr = 16 * w + 4 * b;                  // first of 4 output rows (segment-relative)
      if (q0 + qr >= q1) break;                       // wave-uniform
      float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
      const float *col = buf + qr * kPsfLanes + lane;
      for (int o = 0; o < 2 * r + 4; ++o) {
        const float v = col[o * kPsfLanes];
        acc0 = fmaf(wp[o], v, acc0);
        acc1 = fmaf(wp[o - 1], v, acc1);
        acc2 = fmaf(wp[o - 2], v, acc2);
        acc3 = fmaf(wp[o - 3], v, acc3);
      }
      if (act) {
        const int q = q0 + qr;
        dst[spx(q) * J.n_tel + jb] = acc0;
        if (q + 1 < q1) dst[spx(q + 1) * J.n_tel + jb] = acc1;
        if (q + 2 < q1) dst[spx(q + 2) * J.n_tel + jb] = acc2;
        if (q + 3 < q1) dst[spx(q + 3) * J.n_tel + jb] = acc3;
      }
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
  const size_t psf_lds = sizeof(float) * kPsfLanes * (kPsfSeg + 2 * h.max_psf_r + 4);
  if ((g = grid_for(h.total[K_LSF], cap))) hipLaunchKernelGGL(k_lsf, dim3(g), dim3(256), 0, s, dt);
  if ((g = grid_for(h.total[K_PSFY], cap)))
    hipLaunchKernelGGL(k_psf<0>, dim3(g), dim3(256), psf_lds, s, dt);
  if ((g = grid_for(h.total[K_PSFX], cap)))
    hipLaunchKernelGGL(k_psf<1>, dim3(g), dim3(256), psf_lds, s, dt);
  if ((g = grid_for(h.total[K_COPY], cap))) hipLaunchKernelGGL(k_copy, dim3(g), dim3(256), 0, s, dt);
  return hipGetLastError();
}

int psf_lsf_kernel_kind(const void *f) {
  if (f == (const void *)k_lsf) return K_LSF;
  if (f == (const void *)k_psf<0>) return K_PSFY;
  if (f == (const void *)k_psf<1>) return K_PSFX;
  if (f == (const void *)k_copy) return K_COPY;
  return -1;
}

}  // namespace rubix
