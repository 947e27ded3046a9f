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
//   k_psf_lsf_fused (lambda tile of kFuseL bins, x segment of kFuseX spaxels): all three filters
//            in one pass that reads the cube once and writes it once. The work item walks the y
//            rows in order; per row it stages kFuseX + 2 kFuseR x positions by kFuseL + 2 r_lsf
//            bins in LDS, filters them along lambda and then along x, and adds the row into
//            2 kFuseR partial output rows per lane held in registers (the y filter, updated in
//            place: rows run in unrolled blocks of kFuseU, each compiled for its phase), storing
//            the output row that the new row completes. The next row's loads are in flight
//            while the current row is filtered. Jobs whose radii exceed the fused bounds, and
//            jobs with an LSF only, run the 1-D passes.
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

// Bijection on [0, total) that hands each XCD a contiguous run of work items: blocks are dispatched
// to the XCDs round robin by index, so block b runs on XCD b mod 8, and neighbouring tiles (which
// share halo rows) then meet in that XCD's L2.
__device__ __forceinline__ int64_t xcd_run(int64_t vb, int64_t total) {
  const int64_t full = total & ~int64_t(7);
  if (vb >= full) return vb;
  return (vb & 7) * (full >> 3) + (vb >> 3);
}

// Weight of offset m - kFuseR (m = 0 .. 2 kFuseR) of a filter of radius r <= kFuseR; zero beyond r.
__device__ __forceinline__ float fuse_weight(const float *w, int r, int m) {
  const int o = m - kFuseR;
  return (o >= -r && o <= r) ? w[kWPad + o + r] : 0.f;
}

// LDS copy of the LSF weights: WL[4 + m] = weight of offset m - r (m = 0 .. 2r), zero for the
// other m in -4 .. 2 kFuseLsfR + 7, so a block of four outputs reads them as aligned float4s
constexpr int kFuseWL = 2 * kFuseLsfR + 16;

// One row of the y filter at phase ph (a compile-time constant after unrolling): partial k of
// output row y - R + k lives in P[i][(k + ph) % 2R]. The complete partial (k = 0) takes
// wpx[2R] t and leaves; each other partial k + 1 takes wpx[2R - 1 - k] t in place and becomes
// partial k of the next row; the freed slot starts the new last partial with wpx[0] t. These
// are the FMAs of a shift register, with the registers renamed instead of moved.
__device__ __forceinline__ void fuse_y_step(int ph, float (&P)[4][2 * kFuseR], const float (&t)[4],
                                            const float (&wpx)[2 * kFuseR + 1], float (&done)[4]) {
  constexpr int L = 2 * kFuseR;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    done[i] = fmaf(wpx[L], t[i], P[i][ph]);
    P[i][ph] = wpx[0] * t[i];
#pragma unroll
    for (int k = 0; k < L - 1; ++k)
      P[i][(k + 1 + ph) % L] = fmaf(wpx[L - 1 - k], t[i], P[i][(k + 1 + ph) % L]);
  }
}

__global__ __launch_bounds__(256) void k_psf_lsf_fused(const Table *__restrict__ T) {
  __shared__ __attribute__((aligned(16))) float S[kFuseRows * kFuseW];   // staged input row
  __shared__ __attribute__((aligned(16))) float M[kFuseRows * kFuseL];   // after the LSF
  __shared__ __attribute__((aligned(16))) float WL[kFuseWL];
  const JobDev *jobs = table_jobs(T);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar x offsets
  typedef __attribute__((address_space(1))) float GOut;     // global stores, scalar row base
  const int64_t total = T->h.total[K_FUSE];
  for (int64_t vb0 = blockIdx.x; vb0 < total; vb0 += gridDim.x) {
    const int64_t vb = xcd_run(vb0, total);
    const int jj = find_job(T, K_FUSE, vb);
    const JobDev &J = jobs[jj];
    const int nt = J.n_tel, nx = J.nx, ny = J.ny;
    const int nxs = (nx + kFuseX - 1) / kFuseX;
    const int64_t local = vb - J.vb_start[K_FUSE];
    const int lt = (int)(local / nxs);
    const int x0 = (int)(local - (int64_t)lt * nxs) * kFuseX;
    const int l0 = lt * kFuseL;
    const int rl = J.lsf_r;
    const int wc = kFuseL + 2 * rl + 4;          // staged bins per x position (+ 4: see k_lsf)
    const int64_t plane = (int64_t)nx * nt;      // floats per y row of the cube
    for (int i = tid; i < kFuseWL; i += 256) {
      const int m = i - 4;
      WL[i] = (m >= 0 && m <= 2 * rl) ? J.lsf_w[kWPad + m] : 0.f;
    }
    // staging: wave w stages x positions x0 - kFuseR + w + 4 i (i = 0..7), lane l the bins
    // l0 - rl + l and, for l + 64 < wc, l0 - rl + l + 64. A row is read through a buffer
    // resource over its y plane (one with no bytes for x positions outside the cube), the x
    // position's offset in the scalar offset and the bin's in the lane offset; lanes whose bin
    // lies outside the spectrum or past the staged width take an offset past the plane (the
    // router keeps planes below 2^31 bytes, so the sum cannot wrap), and all of these read 0
    uint32_t loff[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = lane + 64 * h;
      const int g = l0 - rl + c;
      loff[h] = (c < wc && g >= 0 && g < nt) ? 4u * (uint32_t)g : 0x80000000u;
    }
    // the x and y filters padded to radius kFuseR
    float wpx[2 * kFuseR + 1];
#pragma unroll
    for (int m = 0; m <= 2 * kFuseR; ++m) wpx[m] = fuse_weight(J.psf_w, J.psf_r, m);
    const int nq = (2 * rl + 4 + 3) / 4;
    const float *__restrict__ src = J.fuse_src;
    float *__restrict__ dst = J.fuse_dst;
    // outputs of this thread: x = x0 + 4 w + i (i = 0..3), bin l0 + lane
    const int lb = l0 + lane;
    const bool lok = lb < nt;
    // P[i][.]: partial sums of output rows y - kFuseR .. y + kFuseR - 1 before row y is added.
    // At the start of each block of kFuseU rows partial k (of output row y - kFuseR + k) sits in
    // P[i][k], before the block's u-th row in P[i][(k + u) % 2 kFuseR]: each row updates every
    // partial in place and only its phase u decides which one is complete
    float P[4][2 * kFuseR];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int k = 0; k < 2 * kFuseR; ++k) P[i][k] = 0.f;
    float pf[kFuseRows / 4][2];
    auto load_row = [&](int y) {
      const float *rowp = src + (int64_t)y * plane;
      const __amdgpu_buffer_rsrc_t rin =
          __builtin_amdgcn_make_buffer_rsrc((void *)rowp, (short)0, (int)(plane * 4), 0x00020000);
      const __amdgpu_buffer_rsrc_t rout =
          __builtin_amdgcn_make_buffer_rsrc((void *)rowp, (short)0, 0, 0x00020000);
#pragma unroll
      for (int i = 0; i < kFuseRows / 4; ++i) {
        const int gx = x0 - kFuseR + w + 4 * i;
        const bool xin = gx >= 0 && gx < nx;
        const __amdgpu_buffer_rsrc_t rx = xin ? rin : rout;
        const int so = xin ? gx * nt * 4 : 0;
        pf[i][0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, loff[0], so, 0));
        pf[i][1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, loff[1], so, 0));
      }
    };
    // one input row: stage it (its loads were issued one row earlier), issue the next row's
    // loads, filter along lambda and then along x: t[i] = sum_m wpx[m] M[4w + i + m][lane]
    auto filter_row = [&](int y, float (&t)[4]) {
#pragma unroll
      for (int i = 0; i < kFuseRows / 4; ++i) {
        float *srow = S + (w + 4 * i) * kFuseW + lane;
        srow[0] = pf[i][0];
        if (lane < kFuseW - 64) srow[64] = pf[i][1];
      }
      if (y + 1 < ny) load_row(y + 1);
      __syncthreads();
      // LSF along lambda for staged x positions xx = tid/16 and tid/16 + 16, bins 4 (tid % 16)
      // + 0..3: out_i = sum_o wl[o - i] S[xx][b4 + o], the weights read from LDS as float4s
      {
        const int b4 = 4 * (tid & 15);
        const float *r0 = S + (tid >> 4) * kFuseW + b4;
        const float *r1 = r0 + 16 * kFuseW;
        float a[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        float4 wa = *reinterpret_cast<const float4 *>(WL);
        for (int m = 0; m < nq; ++m) {
          const float4 wb = *reinterpret_cast<const float4 *>(WL + 4 * m + 4);
          const float4 xs[2] = {*reinterpret_cast<const float4 *>(r0 + 4 * m),
                                *reinterpret_cast<const float4 *>(r1 + 4 * m)};
#pragma unroll
          for (int g = 0; g < 2; ++g) {
            const float4 x = xs[g];
            // wa = wl[o-4 .. o-1], wb = wl[o .. o+3] with o = 4m
            a[g][0] = fmaf(wb.x, x.x, a[g][0]);
            a[g][0] = fmaf(wb.y, x.y, a[g][0]);
            a[g][0] = fmaf(wb.z, x.z, a[g][0]);
            a[g][0] = fmaf(wb.w, x.w, a[g][0]);
            a[g][1] = fmaf(wa.w, x.x, a[g][1]);
            a[g][1] = fmaf(wb.x, x.y, a[g][1]);
            a[g][1] = fmaf(wb.y, x.z, a[g][1]);
            a[g][1] = fmaf(wb.z, x.w, a[g][1]);
            a[g][2] = fmaf(wa.z, x.x, a[g][2]);
            a[g][2] = fmaf(wa.w, x.y, a[g][2]);
            a[g][2] = fmaf(wb.x, x.z, a[g][2]);
            a[g][2] = fmaf(wb.y, x.w, a[g][2]);
            a[g][3] = fmaf(wa.y, x.x, a[g][3]);
            a[g][3] = fmaf(wa.z, x.y, a[g][3]);
            a[g][3] = fmaf(wa.w, x.z, a[g][3]);
            a[g][3] = fmaf(wb.x, x.w, a[g][3]);
          }
          wa = wb;
        }
#pragma unroll
        for (int g = 0; g < 2; ++g)
          *reinterpret_cast<float4 *>(M + ((tid >> 4) + 16 * g) * kFuseL + b4) =
              make_float4(a[g][0], a[g][1], a[g][2], a[g][3]);
      }
      __syncthreads();
      // PSF along x: t[i] = sum_m wpx[m] M[4w + i + m][lane]
#pragma unroll
      for (int o = 0; o < 2 * kFuseR + 4; ++o) {
        const float v = M[(4 * w + o) * kFuseL + lane];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (o - i >= 0 && o - i <= 2 * kFuseR) t[i] = fmaf(wpx[o - i], v, t[i]);
      }
    };
    if (ny > 0) load_row(0);
    // rows in blocks of kFuseU: within a block the y update of its u-th row is compiled for
    // phase u, so partials stay in place; one rotation per block restores the order
    const int ysteps = ny + kFuseR;
    for (int yb = 0; yb < ysteps; yb += kFuseU) {
#pragma unroll
      for (int u = 0; u < kFuseU; ++u) {
        const int y = yb + u;
        if (y >= ysteps) break;                                      // block-uniform
        float t[4] = {0.f, 0.f, 0.f, 0.f};
        if (y < ny) filter_row(y, t);                               // block-uniform
        // PSF along y: row y adds wpx[2R - k] t to output row y - R + k; row y - R is then
        // complete
        float done[4];
        fuse_y_step(u, P, t, wpx, done);
        const int yo = y - kFuseR;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int x = x0 + 4 * w + i;
          // the row base is wave-uniform (scalar registers), the lane's bin its offset
          GOut *orow = (GOut *)(dst + (int64_t)yo * plane + (int64_t)x * nt + l0);
          if (yo >= 0 && x < nx && lok) orow[lane] = done[i];
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float r[2 * kFuseR];
#pragma unroll
        for (int k = 0; k < 2 * kFuseR; ++k) r[k] = P[i][(k + kFuseU) % (2 * kFuseR)];
#pragma unroll
        for (int k = 0; k < 2 * kFuseR; ++k) P[i][k] = r[k];
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
  if ((g = grid_for(h.total[K_FUSE], cap)))
    hipLaunchKernelGGL(k_psf_lsf_fused, dim3(g), dim3(256), 0, s, dt);
  return hipGetLastError();
}

int psf_lsf_kernel_kind(const void *f) {
  if (f == (const void *)k_lsf) return K_LSF;
  if (f == (const void *)k_psf<0>) return K_PSFY;
  if (f == (const void *)k_psf<1>) return K_PSFX;
  if (f == (const void *)k_copy) return K_COPY;
  if (f == (const void *)k_psf_lsf_fused) return K_FUSE;
  return -1;
}

}  // namespace rubix
