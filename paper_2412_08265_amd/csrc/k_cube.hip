// Steps 3-6 of the pipeline (arXiv:2412.08265, Sec. 3): SSP lookup, Doppler shift, resampling to
// the telescope grid and the per-spaxel sum.
//
// Data flow (all on the caller's stream, in this order):
//   k_chunks  one block per job: splits every spaxel's particle range into chunks of at most
//             kCubeChunk particles (load balance for dense central spaxels); chunks of a spaxel
//             with several chunks get partial-sum slots.
//   k_vbound  streams the particles in input order: the job's largest Doppler slope and window
//             flag for the cube kernel, and a packed 16-byte (mass, age, [M/H], v_los) record each.
//   k_prep_sorted  one block per kPrepBlock sorted in-field particles: gathers each one's packed
//             record through perm once (into LDS), takes each position's spaxel from the segment
//             offsets (no gather of keys), orders the block by (spaxel, SSP cell) in LDS,
//             and writes in that order a 32-byte record {flux row, Doppler slope g, 4 corner
//             weights, window flag}; consecutive particles of a spaxel then share template rows
//             (L1 hits in the cube kernel and the adjoint).
//   k_cube    one block per (lambda tile of kCubeTL bins, chunk); each wave owns 62 consecutive
//             telescope bins and walks the chunk's particles, kCubeGroup at a time:
//               stage    lane l computes the particle's bilinear spectrum at SSP node n0 + l,
//                        S = sum_c a_c T_c[n0 + l] (four coalesced row loads from the template
//                        slice in L1/L2; in the interior path global loads whose row base sits
//                        in scalar registers, so no VALU work forms their addresses), into the
//                        wave's own 64-float LDS slot; n0 is lane 0's shifted node index, so the
//                        slot covers both taps of all 62 bins;
//               resample each lane reads (S[k - n0], S[k - n0 + 1]) with one ds_read2 and
//                        accumulates the linear interpolant in registers (no atomics).
//             Slots are private to a wave, so no block barrier is needed; particle records
//             come through the scalar cache and a group's 16 row loads are in flight together.
//             A wave whose windows stay inside the SSP grid for every slope of the job (most of
//             them) runs without range checks; the others range-check each tap; a particle
//             whose span does not fit a window gathers its taps directly.
//             Blocks are ordered lambda-tile major, so the blocks resident on one XCD at a time
//             share one tile's slice of the template grid in that XCD's L2.
//   k_cube_bin  bin-mean jobs in place of k_cube: the same work items on tiles of kBinTL bins,
//             each bin's value the integral of the shifted spectrum over the bin.
//   k_combine sums a multi-chunk spaxel's partial spectra in chunk order (deterministic).
// The adjoint's records come from k_pack (the packing half of k_vbound) and k_prep_sorted in
// mode 1 (plain bilinear weights, the particle's spaxel and input index).
//
// Resampling index: for bin centre lam_j the node index of the rest-frame wavelength is
//   q = (lam_j/((1+z)(1+beta)) - lam0)/dlam = Q_j - lam_j * g,
//   Q_j = (lam_j/(1+z) - lam0)/dlam,  g = beta/(1+beta) / ((1+z) dlam).
// Q_j is formed in FP64 per lane (split_index, with the job's reciprocals of 1+z and dlam) and
// split into an integer and an FP32 fraction; only the small Doppler term lam_j*g is FP32, so q
// carries an absolute error of ~1e-6 nodes instead of the ~1e-3 that an FP32 lam/(1+beta) would
// give at 9000 A. The integer part k = floor(q) is taken in FP32 from this form; the adjoint
// carries the same rest index in 40-bit fixed point instead (another rounding of the same q). A q
// within the index error of a node may land on either side of it, and both are correct results.
#include "rubix_internal.h"

namespace rubix {

constexpr double kCkms = 299792.458;

// Largest k in [0, n-2] with thr[k] <= x, clamped; returns the fraction computed by `frac`.
__device__ __forceinline__ int cell_of(const double *thr, int n, double x) {
  if (!(x > thr[0])) return 0;
  if (x >= thr[n - 1]) return n - 2;
  int lo = 0, hi = n - 1;             // thr[lo] <= x < thr[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (thr[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ double clamp01(double t) { return fmin(1.0, fmax(0.0, t)); }

// Doppler slope g of the node index (FP32, from FP64) and whether the node span of one wave's
// kCubeWaveBins bins fits its 64-node window: q advances by bin_slope/(1+beta) nodes per bin, so
// when 61 steps stay below 61.9 nodes the node indices of 62 consecutive bins span at most 63
// nodes (0.1 node of margin is far above the FP32 error of q). k_prep_sorted and k_vbound both use it.
// On log grids the Doppler term is the constant index shift ln(1+beta)/dln and the node step per
// bin does not depend on beta.
__device__ __forceinline__ void doppler_slope(const JobDev &J, const SspDev &S, double v, float &g,
                                              bool &fits) {
  const double beta = v / kCkms;
  double beff;
  if (J.log_lambda) {
    g = (float)(log1p(beta) / S.lam_step);
    beff = (beta > -1.0) ? J.bin_slope : -1.0;
  } else {
    const double opz = 1.0 + J.z_sys;
    g = (float)(beta / (1.0 + beta) / (opz * S.lam_step));
    beff = J.bin_slope / (1.0 + beta);
  }
  fits = isfinite((double)g) && beff > 0.0 && 61.0 * beff <= 61.9;
}

// mode 0: forward weights flux_scale*m*J*w_c; mode 1: plain bilinear weights w_c.
// The record of sorted particle i (mode 0: forward weights flux_scale*m*J*w_c, or
// flux_scale*m*dlam_ssp/dlam_tel*w_c for the bin mean; mode 1: plain bilinear weights w_c).
// Record of the particle with input index j, packed properties pr (mass, age, [M/H], vlos; packed
// in input order by k_vbound in the forward and k_pack in the backward) and spaxel key.
// The SSP cell (ja, jz) is cell_of's for the age and metallicity thresholds; the node arrays
// (age thresholds, log10 age nodes, metallicity nodes) are the grid's, here copies in LDS.
__device__ __forceinline__ PrepRec make_record(const JobDev &J, const SspDev &S, int j, float4 pr,
                                               int key, int mode, int ja, int jz,
                                               const double *age_thr, const double *log_age,
                                               const double *met_nodes) {
  const double m = pr.x, age = pr.y, met = pr.z, v = pr.w;
  double ta;
  if (!(age > age_thr[0])) ta = 0.0;
  else if (age >= age_thr[S.n_age - 1]) ta = 1.0;
  else ta = clamp01((log10(age) - log_age[ja]) / (log_age[ja + 1] - log_age[ja]));
  double tz;
  if (!(met > met_nodes[0])) tz = 0.0;
  else if (met >= met_nodes[S.n_met - 1]) tz = 1.0;
  else tz = clamp01((met - met_nodes[jz]) / (met_nodes[jz + 1] - met_nodes[jz]));
  const double beta = v / kCkms;
  const double opz = 1.0 + J.z_sys;
  const double jac = 1.0 / (opz * (1.0 + beta));
  // a line-of-sight velocity that is not finite: the particle adds nothing (zero weights; the
  // Jacobian would be NaN) and its Doppler slope is set to 0 below, so every kernel that reads
  // the record sees finite indices and no NaN reaches a bin
  const bool moving = isfinite(v);
  const double scale = !moving ? 0.0
                       : mode != 0 ? 1.0
                       : J.resample ? J.flux_scale * m * J.bin_scale : J.flux_scale * m * jac;
  PrepRec r;
  r.row = (ja * S.n_met + jz) * S.n_lam;
  bool fits;
  doppler_slope(J, S, v, r.g, fits);
  if (!moving) r.g = 0.f;
  r.a[0] = (float)(scale * (1.0 - ta) * (1.0 - tz));
  r.a[1] = (float)(scale * (1.0 - ta) * tz);
  r.a[2] = (float)(scale * ta * (1.0 - tz));
  r.a[3] = (float)(scale * ta * tz);
  r.spaxel = mode == 0 ? -1 : key;
  if (!fits) r.row = ~r.row;
  r.pad = mode == 0 ? 0 : j;     // backward: the particle's input index (where its dots go)
  return r;
}


// Per job, over all its particles in input order: the largest |g| of a particle whose span fits,
// and whether any particle's span does not fit (doppler_slope, exactly as k_prep_sorted
// decides). The cube kernel uses them to find lambda tiles where every particle's window lies
// inside the SSP grid. One atomic per work item; k_chunks zeroes counts[2..3] before this kernel
// runs. The same pass packs each particle's (mass, age, [M/H], vlos) into one 16-byte record, so
// that k_prep_sorted gathers one record per sorted particle instead of four scattered floats.
__global__ __launch_bounds__(256) void k_vbound(const Table *__restrict__ T) {
  __shared__ int s_g[4], s_f[4];
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_VB]; vb += gridDim.x) {
    const int jj = find_job(T, K_VB, vb);
    const JobDev &J = jobs[jj];
    const int64_t base = (vb - J.vb_start[K_VB]) * kVbParticles;
    int gmax = 0, nofit = 0;
    for (int q = threadIdx.x; q < kVbParticles; q += 256) {
      const int64_t i = base + q;
      if (i < J.n) {
        const float vl = J.vlos[i];
        J.pay[i] = make_float4(J.mass[i], J.age[i], J.met[i], vl);
        float g;
        bool fits;
        doppler_slope(J, S, (double)vl, g, fits);
        if (fits) gmax = max(gmax, __float_as_int(fabsf(g)));   // non-negative: int order
        else nofit = 1;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      gmax = max(gmax, __shfl_xor(gmax, off));
      nofit |= __shfl_xor(nofit, off);
    }
    if ((threadIdx.x & 63) == 0) { s_g[threadIdx.x >> 6] = gmax; s_f[threadIdx.x >> 6] = nofit; }
    __syncthreads();
    if (threadIdx.x == 0) {
      atomicMax(&J.counts[2], max(max(s_g[0], s_g[1]), max(s_g[2], s_g[3])));
      if (s_f[0] | s_f[1] | s_f[2] | s_f[3]) atomicOr(&J.counts[3], 1);
    }
    __syncthreads();
  }
}

// The backward pass's packing of (mass, age, [M/H], vlos) in input order (k_vbound's packing
// without its Doppler bounds, which only the forward sum uses).
__global__ __launch_bounds__(256) void k_pack(const Table *__restrict__ T) {
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_VB]; vb += gridDim.x) {
    const int jj = find_job(T, K_VB, vb);
    const JobDev &J = jobs[jj];
    const int64_t base = (vb - J.vb_start[K_VB]) * kVbParticles;
    for (int q = threadIdx.x; q < kVbParticles; q += 256) {
      const int64_t i = base + q;
      if (i < J.n) J.pay[i] = make_float4(J.mass[i], J.age[i], J.met[i], J.vlos[i]);
    }
  }
}

// One block of 1024 threads per job: chunk list, partial slots, combine list.
__global__ __launch_bounds__(1024) void k_chunks(const Table *__restrict__ T) {
  __shared__ uint32_t sc[1024], ss[1024], sb[1024];
  const JobDev *jobs = table_jobs(T);
  const int t = threadIdx.x;
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_CHUNK]; vb += gridDim.x) {
    const int jj = find_job(T, K_CHUNK, vb);
    const JobDev &J = jobs[jj];
    const int n_s = J.n_s;
    const int per = (n_s + 1023) / 1024;
    const int s0 = min(n_s, t * per), s1 = min(n_s, s0 + per);
    uint32_t nc = 0, nslot = 0, ncomb = 0;
    for (int s = s0; s < s1; ++s) {
      const int cnt = J.seg_off[s + 1] - J.seg_off[s];
      const int nch = cnt <= kCubeChunk ? 1 : (cnt + kCubeChunk - 1) / kCubeChunk;
      nc += nch;
      if (nch > 1) { nslot += nch; ncomb += 1; }
    }
    sc[t] = nc; ss[t] = nslot; sb[t] = ncomb;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      uint32_t a = 0, b = 0, c = 0;
      if (t >= off) { a = sc[t - off]; b = ss[t - off]; c = sb[t - off]; }
      __syncthreads();
      sc[t] += a; ss[t] += b; sb[t] += c;
      __syncthreads();
    }
    uint32_t co = sc[t] - nc, so = ss[t] - nslot, bo = sb[t] - ncomb;
    if (t == 1023) { J.counts[0] = (int32_t)sc[t]; J.counts[1] = (int32_t)sb[t]; }
    if (t == 0) { J.counts[2] = 0; J.counts[3] = 0; }          // k_vbound's reductions
    __syncthreads();
    for (int s = s0; s < s1; ++s) {
      const int p0 = J.seg_off[s], p1 = J.seg_off[s + 1];
      const int cnt = p1 - p0;
      const int nch = cnt <= kCubeChunk ? 1 : (cnt + kCubeChunk - 1) / kCubeChunk;
      if (nch == 1) {
        J.chunks[co++] = ChunkRec{s, p0, p1, -1};
      } else {
        J.combs[bo++] = CombRec{s, (int32_t)so, nch, 0};
        for (int c = 0; c < nch; ++c) {
          const int a = p0 + c * kCubeChunk;
          J.chunks[co++] = ChunkRec{s, a, min(p1, a + kCubeChunk), (int32_t)so++};
        }
      }
    }
  }
}


// The template grid is read through a buffer resource: one uniform descriptor and a 32-bit byte
// offset per lane; offsets past the end of the grid read 0 instead of faulting. The per-particle
// part of the offset is added to the lane part in a VGPR rather than passed as the scalar
// offset: a window that starts before node 0 of the first row has a negative per-particle part,
// which must wrap modulo 2^32 together with the lane part (only the lane offset does). Even where
// the offset is known to be non-negative the scalar-offset form is slower on gfx950: on the
// 1e7-particle workload 39.5 ms against 29.0 ms for the interior path below.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t flux_rsrc(const SspDev &S) {
  const uint32_t bytes = (uint32_t)S.n_age * (uint32_t)S.n_met * (uint32_t)S.n_lam * 4u;
  return __builtin_amdgcn_make_buffer_rsrc((void *)S.flux, (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float ldf(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff + off, 0, 0));
}
typedef __attribute__((address_space(4))) const int CInt;         // read-only: scalar loads

// The next lane's value (lane l receives lane l+1's; lane 63 keeps its own), by a wave-wide DPP
// shift: a VALU move instead of a cross-lane permute through the LDS unit.
__device__ __forceinline__ int next_lane_i(int x) {
  return __builtin_amdgcn_update_dpp(x, x, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ float next_lane_f(float x) {
  return __builtin_bit_cast(float, next_lane_i(__builtin_bit_cast(int, x)));
}

// Particle records in blocks of kPrepBlock sorted in-field particles, each block ordered by
// (spaxel, SSP cell) (stable), so that the particles a wave walks in turn mostly share their four
// template rows: consecutive row loads then hit in the vector L1. Sorting inside a block keeps
// every spaxel's particles at the positions its segment held, so every chunk of the cube kernel
// still sums particles of one spaxel and every spaxel keeps its particles; only the order of the
// FP32 sums changes. Keys (spaxel rank in the block, cell, position) are bitonic-sorted in LDS;
// each record is then built for its sorted position and written once.
__global__ __launch_bounds__(256) void k_prep_sorted(const Table *__restrict__ T, int mode) {
  __shared__ uint64_t key[kPrepBlock];
  __shared__ float4 spay[kPrepBlock];    // the block's packed properties, gathered once
  __shared__ int sidx[kPrepBlock];       // and input indices, by position in sorted order
  __shared__ uint32_t srank[kPrepBlock]; // spaxel of each position, relative to the first one
  __shared__ uint32_t scan_lds[256];
  // the grid's node arrays, so the cell searches and weights read LDS instead of global memory
  __shared__ double l_age_thr[RUBIX_MAX_AGE_NODES], l_log_age[RUBIX_MAX_AGE_NODES];
  __shared__ double l_met[RUBIX_MAX_MET_NODES];
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  const int t = threadIdx.x;
  static_assert(kPrepBlock == 4 * 256, "four positions per thread in the spaxel scan");
  for (int i = t; i < S.n_age; i += 256) {
    l_age_thr[i] = S.age_thr[i];
    l_log_age[i] = S.log_age[i];
  }
  for (int i = t; i < S.n_met; i += 256) l_met[i] = S.met[i];
  __syncthreads();
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_PREP]; vb += gridDim.x) {
    const int jj = find_job(T, K_PREP, vb);
    const JobDev &J = jobs[jj];
    const int n_in = J.seg_off[J.n_s];
    const int64_t p0 = (vb - J.vb_start[K_PREP]) * kPrepBlock;
    if (p0 >= n_in) continue;
    const int n = (int)min((int64_t)kPrepBlock, (int64_t)n_in - p0);
    const int s0 = J.key[J.perm[p0]];
    // The spaxel of every position from the segment offsets rather than a gather of keys
    // through perm: mark where each later spaxel's segment starts inside the block (an empty
    // spaxel starts where the next one does), then a prefix sum gives the spaxel's offset from
    // s0. Segments after s0 start past p0; seg_off[n_s] = n_in ends every thread's walk.
    for (int i = t; i < kPrepBlock; i += 256) srank[i] = 0;
    __syncthreads();
    for (int s = s0 + 1 + t; s <= J.n_s; s += 256) {
      const int b = J.seg_off[s];
      if (b >= p0 + n) break;
      atomicAdd(&srank[b - p0], 1u);
    }
    __syncthreads();
    {
      uint32_t c[4], run = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        run += srank[4 * t + q];
        c[q] = run;
      }
      uint32_t excl;
      block_exclusive_scan_256(run, scan_lds, excl);
#pragma unroll
      for (int q = 0; q < 4; ++q) srank[4 * t + q] = excl + c[q];
    }
    __syncthreads();
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = t; i < np; i += 256) {
      uint64_t k = ~0ull;
      if (i < n) {
        const int j = J.perm[p0 + i];
        const float4 pr = J.pay[j];
        const int ja = cell_of(l_age_thr, S.n_age, (double)pr.y);
        const int jz = cell_of(l_met, S.n_met, (double)pr.z);
        k = ((uint64_t)srank[i] << 32) | ((uint64_t)(ja * S.n_met + jz) << 12) | (uint64_t)i;
        spay[i] = pr;
        sidx[i] = j;
      }
      key[i] = k;
    }
    __syncthreads();
    for (int size = 2; size <= np; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int q = t; q < (np >> 1); q += 256) {
          const int lo = 2 * q - (q & (stride - 1));
          const int hi = lo + stride;
          const uint64_t a = key[lo], b = key[hi];
          if ((a > b) == ((lo & size) == 0)) { key[lo] = b; key[hi] = a; }
        }
        __syncthreads();
      }
    }
    // the records from the LDS copies: no second gather through the permutation
    for (int i = t; i < n; i += 256) {
      const uint64_t k = key[i];
      const int src = (int)(k & 4095u);
      const int cell = (int)((k >> 12) & 0xfffffu);
      const int ja = cell / S.n_met, jz = cell - ja * S.n_met;
      J.prep[p0 + i] = make_record(J, S, sidx[src], spay[src], s0 + (int)(k >> 32), mode, ja, jz,
                                   l_age_thr, l_log_age, l_met);
    }
    __syncthreads();   // the LDS arrays are reused by the block's next item
  }
}


// A particle record through the scalar cache (the records are read-only in this kernel).
__device__ __forceinline__ PrepRec load_rec(const PrepRec *p) {
  CInt *q = (CInt *)p;
  PrepRec r;
  r.row = q[0];
  r.g = __int_as_float(q[1]);
  r.a[0] = __int_as_float(q[2]);
  r.a[1] = __int_as_float(q[3]);
  r.a[2] = __int_as_float(q[4]);
  r.a[3] = __int_as_float(q[5]);
  r.spaxel = q[6];
  r.pad = 0;
  return r;
}

// One particle's resampled contribution to the lane's bin with both taps gathered from the
// template grid (particles whose node span does not fit a wave window, coarse telescope grids).
__device__ __forceinline__ float direct_contrib(const PrepRec &r, __amdgpu_buffer_rsrc_t rs,
                                               int nl, int o1, int o2, int o3, int qi, float qf,
                                               float lamf, bool act) {
  const float tq = fmaf(-lamf, r.g, qf);
  const float fl = floorf(tq);
  const float tau = tq - fl;
  const int k = qi + (int)fminf(fmaxf(fl, -1.0e8f), 1.0e8f);
  const bool ok = act && (k >= 0) && ((k < nl - 1) || (k == nl - 1 && tau == 0.f));
  if (!ok) return 0.f;
  const int kk = min(k, nl - 2);
  const float tt = (k > kk) ? 1.f : tau;
  const uint32_t e = (uint32_t)(prep_row(r.row) + kk) * 4u;
  const uint32_t b1 = (uint32_t)o1 * 4u, b2 = (uint32_t)o2 * 4u, b3 = (uint32_t)o3 * 4u;
  const float p0 = ldf(rs, e, 0), q0 = ldf(rs, e + 4u, 0);
  const float p1 = ldf(rs, e + b1, 0), q1 = ldf(rs, e + b1 + 4u, 0);
  const float p2 = ldf(rs, e + b2, 0), q2 = ldf(rs, e + b2 + 4u, 0);
  const float p3 = ldf(rs, e + b3, 0), q3 = ldf(rs, e + b3 + 4u, 0);
  float v = r.a[0] * fmaf(tt, q0 - p0, p0);
  v = fmaf(r.a[1], fmaf(tt, q1 - p1, p1), v);
  v = fmaf(r.a[2], fmaf(tt, q2 - p2, p2), v);
  v = fmaf(r.a[3], fmaf(tt, q3 - p3, p3), v);
  return v;
}

// One particle through the wave's LDS slot, with range checks for windows that reach past the
// SSP wavelength grid. All 64 lanes must be active (n0 is lane 0's node index).
__device__ __forceinline__ float slot_contrib(const PrepRec &r, __amdgpu_buffer_rsrc_t rs,
                                             int nl, const uint32_t lb[4], int qi, float qf,
                                             float lamf, bool act, float *slot, int lane) {
  const float t = fmaf(-lamf, r.g, qf);
  const float fl = floorf(t);
  const float tau = t - fl;
  const int k = qi + (int)fl;
  const int n0 = __builtin_amdgcn_readfirstlane(k);
  const bool inside = (n0 >= 0) && (n0 + 63 <= nl - 1);
  // nodes outside the grid stage values that only out-of-range lanes read (masked below)
  const uint32_t so = (uint32_t)(r.row + n0) * 4u;
  float S = r.a[0] * ldf(rs, lb[0], so);
  S = fmaf(r.a[1], ldf(rs, lb[1], so), S);
  S = fmaf(r.a[2], ldf(rs, lb[2], so), S);
  S = fmaf(r.a[3], ldf(rs, lb[3], so), S);
  slot[lane] = S;
  __builtin_amdgcn_wave_barrier();
  const int idx = min(max(k - n0, 0), 62);
  const float s0 = slot[idx], s1 = slot[idx + 1];
  __builtin_amdgcn_wave_barrier();
  if (inside) return fmaf(tau, s1 - s0, s0);
  const bool ok = act && (k >= 0) && ((k < nl - 1) || (k == nl - 1 && tau == 0.f));
  if (!ok) return 0.f;
  return (k == nl - 1) ? s0 : fmaf(tau, s1 - s0, s0);
}

__global__ __launch_bounds__(kCubeThreads) void k_cube(const Table *__restrict__ T) {
  __shared__ float slots[kCubeThreads / 64][kCubeGroup][64];
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  const __amdgpu_buffer_rsrc_t rs = flux_rsrc(S);
  const float *__restrict__ flux = S.flux;
  const int nl = S.n_lam;
  const int o1 = nl, o2 = S.n_met * nl, o3 = o2 + nl;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float *wslot = &slots[w][0][0];
  // byte offsets of this lane's node in the four corner rows relative to corner (ja, jz)
  const uint32_t lb[4] = {(uint32_t)lane * 4u, (uint32_t)(lane + o1) * 4u,
                          (uint32_t)(lane + o2) * 4u, (uint32_t)(lane + o3) * 4u};
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_CUBE]; vb += gridDim.x) {
    const int jj = find_job(T, K_CUBE, vb);
    const JobDev &J = jobs[jj];
    const int64_t local = vb - J.vb_start[K_CUBE];
    const int tile = (int)(local / J.n_chunk_ub);
    const int c = (int)(local - (int64_t)tile * J.n_chunk_ub);
    if (c >= ((CInt *)J.counts)[0]) continue;
    const int jw = tile * kCubeTL + w * kCubeWaveBins;     // first bin of this wave
    if (jw >= J.n_tel) continue;                           // wave-uniform: nothing to do
    CInt *chp = (CInt *)(J.chunks + c);
    const ChunkRec ch{chp[0], chp[1], chp[2], chp[3]};
    const int jb = jw + lane;
    const bool act = (lane < kCubeWaveBins) && (jb < J.n_tel);
    // lanes 62, 63 only stage nodes; they and lanes past the band take the constants of the
    // wave's last bin, so every lane's node index stays within the 64-node window
    int qi;
    float qf, lamf;
    split_index(J, S, min(jw + min(lane, kCubeWaveBins - 1), J.n_tel - 1), qi, qf, lamf);
    const int qi0 = __builtin_amdgcn_readfirstlane(qi);
    const uint32_t abase = (uint32_t)(qi - qi0) * 4u;   // + LDS byte address of the slots
    const bool direct_job = J.cube_direct != 0;
    const PrepRec *prep = J.prep;
    float acc = 0.f, tot = 0.f;
    int since = 0;
    int p = ch.p0;
    // Interior wave: every particle of the job fits a window and, with |g| at most the job's
    // largest, lane 0's window [n0, n0 + 63] lies inside the SSP grid for any g in [-gmax, gmax]
    // (n0 is monotone in g), so the groups below need no per-particle checks.
    bool interior = false;
    if (!direct_job && ((CInt *)J.counts)[3] == 0) {
      const float gm = __int_as_float(((CInt *)J.counts)[2]);
      const float lam0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(lamf)));
      const float qf0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(qf)));
      const int lo = __builtin_amdgcn_readfirstlane(qi0 + floor_i32(fmaf(-lam0, gm, qf0)));
      const int hi = __builtin_amdgcn_readfirstlane(qi0 + floor_i32(fmaf(lam0, gm, qf0)));
      interior = lo >= 0 && hi + 63 <= nl - 1;
    }
    uint32_t lo[4] = {lb[0], lb[1], lb[2], lb[3]};
    if (interior) {
      // blocks of groups that end on the partial-sum boundaries (every kCubeSubsum particles of
      // the chunk the partial sum moves into the total)
      while (p + kCubeGroup <= ch.p1) {
        const int pe = p + min(kCubeSubsum - since, (ch.p1 - p) / kCubeGroup * kCubeGroup);
        since += pe - p;
        for (; p < pe; p += kCubeGroup) {
          // the lane offsets pass through an empty asm each iteration, so their widening to
          // 64 bits stays next to the loads and the loads take the scalar-base form
          asm volatile("" : "+v"(lo[0]), "+v"(lo[1]), "+v"(lo[2]), "+v"(lo[3]));
          PrepRec r[kCubeGroup];
#pragma unroll
          for (int u = 0; u < kCubeGroup; ++u) r[u] = load_rec(prep + p + u);
          float tau[kCubeGroup];
          uint32_t dl[kCubeGroup], so[kCubeGroup];
#pragma unroll
          for (int u = 0; u < kCubeGroup; ++u) {
            const float t = fmaf(-lamf, r[u].g, qf);
            tau[u] = __builtin_amdgcn_fractf(t);
            const int fi = floor_i32(t);
            const int fi0 = __builtin_amdgcn_readfirstlane(fi);
            dl[u] = (uint32_t)(fi - fi0) * 4u;
            so[u] = (uint32_t)(r[u].row + qi0 + fi0) * 4u;      // window base, >= 0 here
          }
          float v[kCubeGroup][4];
#pragma unroll
          for (int u = 0; u < kCubeGroup; ++u) {
            // in range here: global loads with the window's row base in scalar registers and the
            // lane's 32-bit offset in a VGPR (no per-particle VALU add)
            const GChar *wb = (const GChar *)flux + so[u];
#pragma unroll
            for (int c = 0; c < 4; ++c) v[u][c] = *(const GFloat *)(wb + lo[c]);
          }
#pragma unroll
          for (int u = 0; u < kCubeGroup; ++u) {
            float Sv = r[u].a[0] * v[u][0];
            Sv = fmaf(r[u].a[1], v[u][1], Sv);
            Sv = fmaf(r[u].a[2], v[u][2], Sv);
            Sv = fmaf(r[u].a[3], v[u][3], Sv);
            wslot[u * 64 + lane] = Sv;
          }
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int u = 0; u < kCubeGroup; ++u) {
            const float *sp = (const float *)((const char *)wslot + abase + dl[u]) + u * 64;
            const float s0 = sp[0], s1 = sp[1];
            acc += fmaf(tau[u], s1 - s0, s0);
          }
          __builtin_amdgcn_wave_barrier();
        }
        if (since >= kCubeSubsum) { tot += acc; acc = 0.f; since = 0; }
      }
    }
    // full groups: straight-line code, all row loads of the group in flight together
    for (; p + kCubeGroup <= ch.p1; p += kCubeGroup) {
      PrepRec r[kCubeGroup];
#pragma unroll
      for (int u = 0; u < kCubeGroup; ++u) r[u] = load_rec(prep + p + u);
      // every window fits <=> no row offset carries the "does not fit" sign
      int32_t orow = 0;
#pragma unroll
      for (int u = 0; u < kCubeGroup; ++u) orow |= r[u].row;
      if (!direct_job && orow >= 0) {
        // every span fits a window: the group's 16 row loads in flight together, as in the
        // interior, with each tap range-checked (a window may start before node 0 or reach past
        // the last node; its out-of-grid nodes are only read by bins that the check zeroes)
        float tau[kCubeGroup];
        int fi[kCubeGroup], fi0[kCubeGroup];
        float v[kCubeGroup][4];
#pragma unroll
        for (int u = 0; u < kCubeGroup; ++u) {
          const float t = fmaf(-lamf, r[u].g, qf);
          tau[u] = __builtin_amdgcn_fractf(t);
          fi[u] = floor_i32(t);
          fi0[u] = __builtin_amdgcn_readfirstlane(fi[u]);
          // window base: lane 0's node; the offset wraps modulo 2^32 with the lane part when the
          // window starts before node 0 of the first row (past the grid's bytes: reads 0)
          const uint32_t so = (uint32_t)(r[u].row + qi0 + fi0[u]) * 4u;
#pragma unroll
          for (int c = 0; c < 4; ++c) v[u][c] = ldf(rs, lb[c], so);
        }
#pragma unroll
        for (int u = 0; u < kCubeGroup; ++u) {
          float Sv = r[u].a[0] * v[u][0];
          Sv = fmaf(r[u].a[1], v[u][1], Sv);
          Sv = fmaf(r[u].a[2], v[u][2], Sv);
          Sv = fmaf(r[u].a[3], v[u][3], Sv);
          wslot[u * 64 + lane] = Sv;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int u = 0; u < kCubeGroup; ++u) {
          // k - n0 = (qi - qi0) + (fi - fi0), in [0, 62] for every lane (the clamp guards LDS)
          const int idx = min(max((qi - qi0) + (fi[u] - fi0[u]), 0), 62);
          const float s0 = wslot[u * 64 + idx], s1 = wslot[u * 64 + idx + 1];
          const int k = qi + fi[u];
          const bool ok = act && (k >= 0) && ((k < nl - 1) || (k == nl - 1 && tau[u] == 0.f));
          const float val = (k == nl - 1) ? s0 : fmaf(tau[u], s1 - s0, s0);
          acc += ok ? val : 0.f;
        }
        __builtin_amdgcn_wave_barrier();
      } else {
#pragma unroll
        for (int u = 0; u < kCubeGroup; ++u) {
          if (!direct_job && r[u].row >= 0)
            acc += slot_contrib(r[u], rs, nl, lb, qi, qf, lamf, act, wslot, lane);
          else
            acc += direct_contrib(r[u], rs, nl, o1, o2, o3, qi, qf, lamf, act);
        }
      }
      since += kCubeGroup;
      if (since >= kCubeSubsum) { tot += acc; acc = 0.f; since = 0; }
    }
    // the last < kCubeGroup particles one at a time
    for (; p < ch.p1; ++p) {
      const PrepRec r = load_rec(prep + p);
      if (!direct_job && r.row >= 0)
        acc += slot_contrib(r, rs, nl, lb, qi, qf, lamf, act, wslot, lane);
      else
        acc += direct_contrib(r, rs, nl, o1, o2, o3, qi, qf, lamf, act);
    }
    tot += acc;
    if (act) {
      if (ch.slot < 0) J.cube_raw[(int64_t)ch.s * J.n_tel + jb] = tot;
      else J.partial[(int64_t)ch.slot * J.n_tel + jb] = tot;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Bin-mean resampling (flux conserving): cube_raw[s][j] = sum over the spaxel's particles of
//   a_i . integral of the particle's piecewise-linear spectrum over the rest-frame node interval
//   [q_lo, q_hi] of bin j (a_i = corner weights x flux_scale m dlam_ssp/dlam_tel),
// with the interval clipped to [0, n-1] (the spectrum is zero outside the grid). On a node
// segment k the integral from fraction x to y is S_k (y - x) + (S_{k+1} - S_k)(y^2 - x^2)/2.
// Work items as k_cube's, on tiles of kBinTL bins: each wave owns kBinWaveBins bins and stages
// the particle's spectrum at 64 consecutive nodes n0 .. n0+63 in its LDS slot (n0 = lane 0's
// clipped lower node), which covers every lane's interval when the bins span at most 63 nodes
// and no bin spans more than two segments; otherwise the particle's segments are gathered from
// the template grid directly (both cases give the same sum of the same terms). Per particle a lane
// splits one bin edge (its own, edge jw + l) and takes its bin's upper edge from the next lane,
// so neighbouring bins see the same edge.
// Log grids: the spectrum is linear in the log-grid index and the bin's integral runs over rest
// wavelength, lambda(q) = lambda_0 e^{q dln}, so a segment's integral from its node k to fraction
// a carries the weight e^{t dln} dln: lambda_k (S_k E1(a dln) + (S_{k+1} - S_k) a Phi(a dln)) with
// E1(h) = e^h - 1 and Phi(h) = e^h - (e^h - 1)/h, both by their Taylor series (four terms; the
// ABI admits steps up to 0.05, where the next terms are below 1e-7), and each bin's sum is divided
// by its width in wavelength.
// ---------------------------------------------------------------------------------------------
// One instance per grid kind (every job of a call shares the SSP grid's kind), so the linear
// kernel carries none of the log path's registers.
template <bool kLog>
__global__ __launch_bounds__(kCubeThreads) void k_cube_bin(const Table *__restrict__ T) {
  __shared__ float slots[kCubeThreads / 64][kCubeGroup][64];
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  const __amdgpu_buffer_rsrc_t rs = flux_rsrc(S);
  const int nl = S.n_lam;
  const int o1 = nl, o2 = S.n_met * nl, o3 = o2 + nl;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float *wslot = &slots[w][0][0];     // one particle at a time
  float *gslot = &slots[w][0][0];     // a group: kCubeGroup rows of 64
  const uint32_t lb[4] = {(uint32_t)lane * 4u, (uint32_t)(lane + o1) * 4u,
                          (uint32_t)(lane + o2) * 4u, (uint32_t)(lane + o3) * 4u};
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_CUBEB]; vb += gridDim.x) {
    const int jj = find_job(T, K_CUBEB, vb);
    const JobDev &J = jobs[jj];
    const int64_t local = vb - J.vb_start[K_CUBEB];
    const int tile = (int)(local / J.n_chunk_ub);
    const int c = (int)(local - (int64_t)tile * J.n_chunk_ub);
    if (c >= ((CInt *)J.counts)[0]) continue;
    if ((J.log_lambda != 0) != kLog) continue;             // the other instance's job
    const int jw = tile * kBinTL + w * kBinWaveBins;
    if (jw >= J.n_tel) continue;                           // wave-uniform
    CInt *chp = (CInt *)(J.chunks + c);
    const ChunkRec ch{chp[0], chp[1], chp[2], chp[3]};
    const int jb = jw + lane;
    const bool act = (lane < kBinWaveBins) && (jb < J.n_tel);
    // lane l holds edge jw + l (the lower edge of bin jw + l, the upper edge of bin jw + l - 1);
    // lanes past the wave's last edge take it, so the node span stays that of the bins
    int qe;
    float fe, le;
    bin_edge(J, S, min(jw + min(lane, kBinWaveBins), J.n_tel), qe, fe, le);
    // log grids: the node wavelengths' base and step, the wavelength of the lane's edge node at
    // rest (a node k's is lam_e e^{(k - qe) dln}, the exponent small), the whole-segment series,
    // and 1 / the bin's width in wavelength
    constexpr bool lg = kLog;
    const float lam0 = (float)S.lam_start, dln = (float)S.lam_step;
    const float lam_e = lg ? (float)(S.lam_start * exp((double)qe * S.lam_step)) : 0.f;
    const float e1h = expm1_small(dln), phh = phi_small(dln);
    const float inv_w = lg ? (float)(1.0 / (J.tel_start * exp((double)min(jb, J.n_tel - 1) * J.tel_step) *
                                            2.0 * sinh(0.5 * J.tel_step)))
                           : 1.f;
    const PrepRec *prep = J.prep;
    float acc = 0.f, tot = 0.f;
    int since = 0;
    // one particle's edge geometry: the node interval and fraction of the lane's edge (clipped to
    // the grid), the bin's upper edge from the next lane, the wave's lowest node n0, and whether
    // the wave's bins fit one 64-node window with at most two segments per bin
    struct Edge {
      int klo, khi, n0;
      float a, b;
      bool empty, window;
    };
    auto edge_of = [&](const PrepRec &r) {
      Edge e;
      const float tl = fmaf(-le, r.g, fe);
      e.klo = qe + floor_i32(tl);
      e.a = __builtin_amdgcn_fractf(tl);
      clip_node(e.klo, e.a, nl);
      e.khi = next_lane_i(e.klo);
      e.b = next_lane_f(e.a);
      e.empty = (e.klo > e.khi) || (e.klo == e.khi && !(e.a < e.b));
      e.n0 = __builtin_amdgcn_readfirstlane(e.klo);
      const int nmax = __builtin_amdgcn_readlane(e.khi, 63) + 1;    // last bin's upper node
      const bool two = !e.empty && (e.khi - e.klo > 1);
      e.window = (nmax - e.n0 <= 63) && !__builtin_amdgcn_ballot_w64(two);
      return e;
    };
    // a bin's value from the staged values s0, s1 of its lower edge's segment: the integral over
    // the lane's edge segment from its node to the edge (P) and over the whole segment (Tn); the
    // bin's value is P(upper edge) - P(lower edge), plus the lower segment's Tn when the upper
    // edge lies in the next segment
    auto window_bin = [&](const Edge &e, float s0, float s1) {
      float P, Tn;
      if (lg) {
        const float lamk = node_lambda(e.klo, qe, lam_e, lam0, dln);
        P = log_partial(lamk, s0, s1 - s0, e.a, dln);
        Tn = lamk * fmaf(s0, e1h, (s1 - s0) * phh);
      } else {
        P = e.a * fmaf(0.5f * e.a, s1 - s0, s0);
        Tn = 0.5f * (s0 + s1);
      }
      const float Ph = next_lane_f(P);
      const float vv = (Ph - P) + (e.khi > e.klo ? Tn : 0.f);
      return e.empty ? 0.f : vv;
    };
    // one particle: its window staged through the wave's first slot row, or (spans that do not
    // fit a window) its segments gathered from the template grid
    auto one = [&](const PrepRec &r, const Edge &e) {
      const int row = prep_row(r.row);
      float v = 0.f;
      if (e.window) {
        const uint32_t so = (uint32_t)(row + e.n0) * 4u;
        float Sv = r.a[0] * ldf(rs, lb[0], so);
        Sv = fmaf(r.a[1], ldf(rs, lb[1], so), Sv);
        Sv = fmaf(r.a[2], ldf(rs, lb[2], so), Sv);
        Sv = fmaf(r.a[3], ldf(rs, lb[3], so), Sv);
        wslot[lane] = Sv;
        __builtin_amdgcn_wave_barrier();
        const int i0 = min(max(e.klo - e.n0, 0), 62);
        const float s0 = wslot[i0], s1 = wslot[i0 + 1];
        __builtin_amdgcn_wave_barrier();
        v = window_bin(e, s0, s1);
      } else if (!e.empty) {
        // any number of segments, gathered from the template grid
        for (int k = e.klo; k <= e.khi; ++k) {
          const uint32_t ek = (uint32_t)(row + k) * 4u;
          const uint32_t b1 = (uint32_t)o1 * 4u, b2 = (uint32_t)o2 * 4u, b3 = (uint32_t)o3 * 4u;
          float s0 = r.a[0] * ldf(rs, ek, 0);
          s0 = fmaf(r.a[1], ldf(rs, ek + b1, 0), s0);
          s0 = fmaf(r.a[2], ldf(rs, ek + b2, 0), s0);
          s0 = fmaf(r.a[3], ldf(rs, ek + b3, 0), s0);
          float s1 = r.a[0] * ldf(rs, ek + 4u, 0);
          s1 = fmaf(r.a[1], ldf(rs, ek + b1 + 4u, 0), s1);
          s1 = fmaf(r.a[2], ldf(rs, ek + b2 + 4u, 0), s1);
          s1 = fmaf(r.a[3], ldf(rs, ek + b3 + 4u, 0), s1);
          const float x = k == e.klo ? e.a : 0.f, y = k == e.khi ? e.b : 1.f;
          if (lg) {
            const float lamk = node_lambda(k, qe, lam_e, lam0, dln);
            v += log_partial(lamk, s0, s1 - s0, y, dln) - log_partial(lamk, s0, s1 - s0, x, dln);
          } else {
            v += seg_integral(s0, s1, x, y);
          }
        }
      }
      return v;
    };
    int p = ch.p0;
    // log grids: groups of kCubeGroup particles whose windows all lie inside the rows, the
    // group's 16 row loads in flight together from scalar row bases (as in k_cube's interior
    // path); the values, their order of summation and so the result are those of the
    // one-particle path. (On linear grids, with fewer instructions per particle, the groups
    // measured slower than one particle at a time: 59.0 against 54.9 ms on the large galaxy.)
    uint32_t lo[4] = {lb[0], lb[1], lb[2], lb[3]};
    for (; kLog && p + kCubeGroup <= ch.p1; p += kCubeGroup) {
      asm volatile("" : "+v"(lo[0]), "+v"(lo[1]), "+v"(lo[2]), "+v"(lo[3]));
      PrepRec r[kCubeGroup];
      Edge e[kCubeGroup];
      bool all = true;
#pragma unroll
      for (int u = 0; u < kCubeGroup; ++u) {
        r[u] = load_rec(prep + p + u);
        e[u] = edge_of(r[u]);
        all = all && e[u].window && e[u].n0 + 63 <= nl - 1;      // wave-uniform
      }
      if (all) {
        float v[kCubeGroup][4];
#pragma unroll
        for (int u = 0; u < kCubeGroup; ++u) {
          // n0 >= 0 (clipped) and n0 + 63 <= n - 1: every lane's load lies in its row
          const GChar *wb = (const GChar *)S.flux + (uint32_t)(prep_row(r[u].row) + e[u].n0) * 4u;
#pragma unroll
          for (int c = 0; c < 4; ++c) v[u][c] = *(const GFloat *)(wb + lo[c]);
        }
#pragma unroll
        for (int u = 0; u < kCubeGroup; ++u) {
          float Sv = r[u].a[0] * v[u][0];
          Sv = fmaf(r[u].a[1], v[u][1], Sv);
          Sv = fmaf(r[u].a[2], v[u][2], Sv);
          Sv = fmaf(r[u].a[3], v[u][3], Sv);
          gslot[u * 64 + lane] = Sv;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int u = 0; u < kCubeGroup; ++u) {
          const int i0 = min(max(e[u].klo - e[u].n0, 0), 62);
          const float s0 = gslot[u * 64 + i0], s1 = gslot[u * 64 + i0 + 1];
          acc += window_bin(e[u], s0, s1);
        }
        __builtin_amdgcn_wave_barrier();
      } else {
#pragma unroll
        for (int u = 0; u < kCubeGroup; ++u) acc += one(r[u], e[u]);
      }
      since += kCubeGroup;
      if (since >= kCubeSubsum) { tot += acc; acc = 0.f; since = 0; }
    }
    // one particle at a time (the rest of a log-grid chunk, a whole linear-grid chunk); on linear
    // grids the next particle's record is loaded while this one is summed (on log grids that
    // measured slower: 81.5 against 70.9 ms)
    if constexpr (kLog) {
      for (; p < ch.p1; ++p) {
        const PrepRec r = load_rec(prep + p);
        acc += one(r, edge_of(r));
        if (++since == kCubeSubsum) { tot += acc; acc = 0.f; since = 0; }
      }
    } else {
      PrepRec rn;
      if (p < ch.p1) rn = load_rec(prep + p);
      for (; p < ch.p1; ++p) {
        const PrepRec r = rn;
        rn = load_rec(prep + min(p + 1, ch.p1 - 1));
        acc += one(r, edge_of(r));
        if (++since == kCubeSubsum) { tot += acc; acc = 0.f; since = 0; }
      }
    }
    tot = (tot + acc) * inv_w;
    if (act) {
      if (ch.slot < 0) J.cube_raw[(int64_t)ch.s * J.n_tel + jb] = tot;
      else J.partial[(int64_t)ch.slot * J.n_tel + jb] = tot;
    }
  }
}

__global__ __launch_bounds__(kCubeThreads) void k_combine(const Table *__restrict__ T) {
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_COMB]; vb += gridDim.x) {
    const int jj = find_job(T, K_COMB, vb);
    const JobDev &J = jobs[jj];
    const int64_t local = vb - J.vb_start[K_COMB];
    const int tile = (int)(local / J.n_comb_ub);
    const int e = (int)(local - (int64_t)tile * J.n_comb_ub);
    if (e >= J.counts[1]) continue;
    const CombRec cr = J.combs[e];
    if ((int)threadIdx.x >= kCubeTL) continue;
    const int jb = tile * kCubeTL + threadIdx.x;
    if (jb >= J.n_tel) continue;
    float sum = 0.f;
    for (int q = 0; q < cr.n_slots; ++q) sum += J.partial[(int64_t)(cr.first_slot + q) * J.n_tel + jb];
    J.cube_raw[(int64_t)cr.s * J.n_tel + jb] = sum;
  }
}

thread_local hipEvent_t t_cube_events[2] = {nullptr, nullptr};

static inline int grid_for(int64_t total, int cap) {
  if (total <= 0) return 0;
  int64_t g = total;
  if (cap > 0 && g > cap) g = cap;
  if (g > 0x7fffffff) g = 0x7fffffff;
  return (int)g;
}

hipError_t launch_cube(const Table *dt, const TableHeader &h, int cap, hipStream_t s) {
  int g;
  if ((g = grid_for(h.total[K_CHUNK], cap)))
    hipLaunchKernelGGL(k_chunks, dim3(g), dim3(1024), 0, s, dt);
  if ((g = grid_for(h.total[K_VB], cap)))
    hipLaunchKernelGGL(k_vbound, dim3(g), dim3(256), 0, s, dt);
  if ((g = grid_for(h.total[K_PREP], cap)))
    hipLaunchKernelGGL(k_prep_sorted, dim3(g), dim3(256), 0, s, dt, 0);
  // the summation kernels (bin-centre and bin-mean jobs), timed together when requested
  const bool timed = t_cube_events[0] && t_cube_events[1];
  if (timed) (void)hipEventRecord(t_cube_events[0], s);
  if ((g = grid_for(h.total[K_CUBE], cap)))
    hipLaunchKernelGGL(k_cube, dim3(g), dim3(kCubeThreads), 0, s, dt);
  if ((g = grid_for(h.total[K_CUBEB], cap)))
  {
    // the instance of the SSP grid's kind; both (each skipping the other kind's jobs) when the
    // table lives only on the device and its kind is not known here (log_lambda = -1)
    if (h.ssp.log_lambda != 1)
      hipLaunchKernelGGL(k_cube_bin<false>, dim3(g), dim3(kCubeThreads), 0, s, dt);
    if (h.ssp.log_lambda != 0)
      hipLaunchKernelGGL(k_cube_bin<true>, dim3(g), dim3(kCubeThreads), 0, s, dt);
  }
  if (timed) (void)hipEventRecord(t_cube_events[1], s);
  if ((g = grid_for(h.total[K_COMB], cap)))
    hipLaunchKernelGGL(k_combine, dim3(g), dim3(kCubeThreads), 0, s, dt);
  return hipGetLastError();
}

// Backward needs the same per-particle records with plain bilinear weights.
hipError_t launch_prep_backward(const Table *dt, const TableHeader &h, int cap, hipStream_t s) {
  int g;
  if ((g = grid_for(h.total[K_VB], cap)))
    hipLaunchKernelGGL(k_pack, dim3(g), dim3(256), 0, s, dt);
  if ((g = grid_for(h.total[K_PREP], cap)))
    hipLaunchKernelGGL(k_prep_sorted, dim3(g), dim3(256), 0, s, dt, 1);
  return hipGetLastError();
}

int cube_kernel_kind(const void *f) {
  if (f == (const void *)k_prep_sorted) return K_PREP;
  if (f == (const void *)k_chunks) return K_CHUNK;
  if (f == (const void *)k_vbound) return K_VB;
  if (f == (const void *)k_cube_bin<false> || f == (const void *)k_cube_bin<true>) return K_CUBEB;
  if (f == (const void *)k_cube) return K_CUBE;
  if (f == (const void *)k_combine) return K_COMB;
  return -1;
}

}  // namespace rubix
