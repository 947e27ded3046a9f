// Steps 1-2 of the pipeline (arXiv:2412.08265, Sec. 3): orient the galaxy and assign particles to
// spaxels, then a stable LSD radix sort of the particle indices by spaxel key.
//
// Design for gfx950: the work is HBM streaming (24 B in, 8 B out per particle for the rotation,
// ~20 B per particle per 8-bit sort pass), so every kernel reads and writes with unit-stride,
// lane-contiguous accesses and keeps the per-tile histograms in LDS. Ranks inside a tile are found
// with wave64 ballots (one ballot per digit bit), which is stable by construction: a wave handles
// 64 consecutive keys per round and rounds in order, waves hold consecutive 1024-key ranges.
#include "rubix_internal.h"

namespace rubix {

// ---------------------------------------------------------------------------------------------
// rotation, spaxel key, line-of-sight velocity
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int32_t rotate_one(const JobDev &J, int i) {
  double x = J.x[i], y = J.y[i], z = J.z[i];
  double vx = J.vx[i], vy = J.vy[i], vz = J.vz[i];
  int32_t key;
  double vl;
  {
#pragma clang fp contract(off)
    // fixed grouping, no fused multiply-add: the key is an exact function of the inputs
    double xp = (J.R[0] * x + J.R[1] * y) + J.R[2] * z;
    double yp = (J.R[3] * x + J.R[4] * y) + J.R[5] * z;
    double tx = xp / J.spaxel + J.half_nx;
    double ty = yp / J.spaxel + J.half_ny;
    double fx = floor(tx), fy = floor(ty);
    bool in = (fx >= 0.0) && (fx < (double)J.nx) && (fy >= 0.0) && (fy < (double)J.ny);
    key = in ? (int32_t)fy * J.nx + (int32_t)fx : J.n_s;
    vl = (J.R[6] * vx + J.R[7] * vy) + J.R[8] * vz;
  }
  J.key[i] = key;
  J.vlos[i] = (float)vl;
  return key;
}

// One sort tile per work item; the tile's digit histogram of the first sort pass is counted in
// LDS on the way (the first pass needs no separate histogram kernel).
__global__ __launch_bounds__(kSortThreads) void k_rotate(const Table *__restrict__ T) {
  __shared__ uint32_t h[256];
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_ROT]; vb += gridDim.x) {
    const int j = find_job(T, K_ROT, vb);
    const JobDev &J = jobs[j];
    const int tile = (int)(vb - J.vb_start[K_ROT]);
    const int64_t base = (int64_t)tile * kSortTile;
    h[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll 4
    for (int it = 0; it < kSortItems; ++it) {
      int64_t i = base + it * kSortThreads + threadIdx.x;
      if (i < J.n) atomicAdd(&h[(uint32_t)rotate_one(J, (int)i) & 255u], 1u);
    }
    __syncthreads();
    J.hist[(int64_t)threadIdx.x * J.n_sort_tiles + tile] = h[threadIdx.x];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// radix sort: per-tile digit histograms
// ---------------------------------------------------------------------------------------------
// A buffer resource over the part of a 32-bit array that one sort tile covers: elements
// [base, min(base + kSortTile, n)). Loads past its end return 0 instead of reading memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const uint32_t *p, int64_t base,
                                                           int64_t n) {
  const int64_t cnt = n - base < (int64_t)kSortTile ? n - base : (int64_t)kSortTile;
  return __builtin_amdgcn_make_buffer_rsrc((void *)(p + base), (short)0, (int)(cnt * 4), 0x00020000);
}

__device__ __forceinline__ uint32_t ld_u32(__amdgpu_buffer_rsrc_t rs, int idx) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (uint32_t)idx * 4u, 0, 0);
}

__device__ __forceinline__ const uint32_t *sort_src_keys(const JobDev &J, int pass) {
  return pass == 0 ? reinterpret_cast<const uint32_t *>(J.key) : J.kbuf[(pass - 1) & 1];
}

__global__ __launch_bounds__(kSortThreads) void k_hist(const Table *__restrict__ T, int pass) {
  __shared__ uint32_t h[256];
  const JobDev *jobs = table_jobs(T);
  const int shift = 8 * pass;
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_ROT]; vb += gridDim.x) {
    const int j = find_job(T, K_ROT, vb);
    const JobDev &J = jobs[j];
    if (pass >= J.passes) continue;          // uniform: this job needs fewer passes
    const int tile = (int)(vb - J.vb_start[K_ROT]);
    const uint32_t *src = sort_src_keys(J, pass);
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)tile * kSortTile;
    // every key of the tile loaded first through the tile's buffer resource (no load behind a
    // branch; entries past the end read 0 and are not counted), then counted
    const __amdgpu_buffer_rsrc_t rk = tile_rsrc(src, base, J.n);
    uint32_t dg[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it)
      dg[it] = (ld_u32(rk, it * kSortThreads + threadIdx.x) >> shift) & 255u;
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const int64_t i = base + it * kSortThreads + threadIdx.x;
      if (i < J.n) atomicAdd(&h[dg[it]], 1u);
    }
    __syncthreads();
    J.hist[(int64_t)threadIdx.x * J.n_sort_tiles + tile] = h[threadIdx.x];
    __syncthreads();
  }
}

// Exclusive scan of hist[d][0..n_sort_tiles) in place, one work item per (job, digit d).
__global__ __launch_bounds__(256) void k_scan(const Table *__restrict__ T, int pass) {
  __shared__ uint32_t lds[256];
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_SCAN]; vb += gridDim.x) {
    const int j = find_job(T, K_SCAN, vb);
    const JobDev &J = jobs[j];
    if (pass >= J.passes) continue;
    const int d = (int)(vb - J.vb_start[K_SCAN]);
    uint32_t *row = J.hist + (int64_t)d * J.n_sort_tiles;
    const int nb = J.n_sort_tiles;
    const int per = (nb + 255) / 256;
    const int b0 = threadIdx.x * per;
    const int b1 = min(nb, b0 + per);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += row[b];
    uint32_t excl;
    uint32_t total = block_exclusive_scan_256(sum, lds, excl);
    uint32_t run = excl;
    for (int b = b0; b < b1; ++b) {
      uint32_t c = row[b];
      row[b] = run;
      run += c;
    }
    if (threadIdx.x == 0) J.dtot[d] = total;
    __syncthreads();
  }
}

// Stable scatter of one tile: 4 waves x 16 rounds x 64 lanes. The ranks put the tile in digit
// order in LDS first; the tile is then written out in that order, so the lanes of a store write
// consecutive positions of a few digit runs instead of 64 scattered ones.
__global__ __launch_bounds__(kSortThreads) void k_scatter(const Table *__restrict__ T,
                                                          int pass) {
  __shared__ uint32_t wcnt[4][256];
  __shared__ uint32_t gdelta[256];
  __shared__ uint32_t scan_lds[256];
  __shared__ uint32_t sk[kSortTile];
  __shared__ uint32_t sv[kSortTile];
  const JobDev *jobs = table_jobs(T);
  const int shift = 8 * pass;
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int lane = t & 63;
  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_ROT]; vb += gridDim.x) {
    const int j = find_job(T, K_ROT, vb);
    const JobDev &J = jobs[j];
    if (pass >= J.passes) continue;
    const int tile = (int)(vb - J.vb_start[K_ROT]);
    const bool last = (pass == J.passes - 1);
    const uint32_t *src_k = sort_src_keys(J, pass);
    const uint32_t *src_v = pass == 0 ? nullptr : J.vbuf[(pass - 1) & 1];
    uint32_t *dst_k = J.kbuf[pass & 1];
    uint32_t *dst_v = last ? reinterpret_cast<uint32_t *>(J.perm) : J.vbuf[pass & 1];

    // global position of this tile's first key of digit t: digit offset + the tile's prefix in
    // the digit (thread t owns digit t)
    uint32_t excl;
    block_exclusive_scan_256(J.dtot[t], scan_lds, excl);
    const uint32_t gbase = excl + J.hist[(int64_t)t * J.n_sort_tiles + tile];
    wcnt[0][t] = 0; wcnt[1][t] = 0; wcnt[2][t] = 0; wcnt[3][t] = 0;
    __syncthreads();

    uint32_t keys[kSortItems], vals[kSortItems], rank[kSortItems];
    const int64_t base = (int64_t)tile * kSortTile + w * (64 * kSortItems);
    // the wave's keys loaded first through the tile's buffer resource, so all of them are in
    // flight together (entries past the end read 0 and are masked below); the values follow in
    // one batch once the ranks are known
    const int64_t tbase = (int64_t)tile * kSortTile;
    const int woff = w * (64 * kSortItems);
    {
      const __amdgpu_buffer_rsrc_t rk = tile_rsrc(src_k, tbase, J.n);
#pragma unroll
      for (int r = 0; r < kSortItems; ++r) keys[r] = ld_u32(rk, woff + r * 64 + lane);
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const int64_t e = base + r * 64 + lane;
      const bool valid = e < J.n;
      const uint32_t k = keys[r];
      uint32_t d = (k >> shift) & 255u;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        peers &= bit ? bb : ~bb;
      }
      const uint32_t below = __popcll(peers & lt_mask);
      const uint32_t cnt = __popcll(peers);
      uint32_t c0 = 0;
      if (valid) c0 = wcnt[w][d];
      __builtin_amdgcn_wave_barrier();
      if (valid && below == 0) wcnt[w][d] = c0 + cnt;   // lowest lane of each digit group
      __builtin_amdgcn_wave_barrier();
      rank[r] = valid ? (c0 + below) : 0xffffffffu;
    }
    __syncthreads();
    // digit t: exclusive prefix over the 4 waves, then over the digits of the tile (the tile's
    // digit-ordered position of each wave's first key of digit t)
    uint32_t run = 0;
    uint32_t wpre[4];
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) {
      wpre[ww] = run;
      run += wcnt[ww][t];
    }
    uint32_t toff;
    block_exclusive_scan_256(run, scan_lds, toff);
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) wcnt[ww][t] = toff + wpre[ww];
    gdelta[t] = gbase - toff;
    __syncthreads();
    if (pass == 0) {
#pragma unroll
      for (int r = 0; r < kSortItems; ++r) vals[r] = (uint32_t)(base + r * 64 + lane);
    } else {
      const __amdgpu_buffer_rsrc_t rv = tile_rsrc(src_v, tbase, J.n);
#pragma unroll
      for (int r = 0; r < kSortItems; ++r) vals[r] = ld_u32(rv, woff + r * 64 + lane);
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      if (rank[r] != 0xffffffffu) {
        const uint32_t d = (keys[r] >> shift) & 255u;
        const uint32_t lpos = wcnt[w][d] + rank[r];
        sk[lpos] = keys[r];
        sv[lpos] = vals[r];
      }
    }
    __syncthreads();
    // the tile in digit order: position q goes to gdelta[digit] + q
    const int nv = (int)min((int64_t)kSortTile, J.n - tbase);
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const int q = r * kSortThreads + t;
      if (q < nv) {
        const uint32_t k = sk[q];
        const uint32_t pos = gdelta[(k >> shift) & 255u] + (uint32_t)q;
        dst_k[pos] = k;
        dst_v[pos] = sv[q];
      }
    }
    __syncthreads();
  }
}

// seg_off[s] = number of sorted keys < s (lower bound), s = 0..n_s.
__global__ __launch_bounds__(256) void k_segoff(const Table *__restrict__ T) {
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_SEG]; vb += gridDim.x) {
    const int j = find_job(T, K_SEG, vb);
    const JobDev &J = jobs[j];
    const int64_t s = (vb - J.vb_start[K_SEG]) * 256 + threadIdx.x;
    if (s > J.n_s) continue;
    int lo = 0, hi = J.n;
    if (J.n > 0) {
      const uint32_t *sk = J.kbuf[(J.passes - 1) & 1];
      while (lo < hi) {
        int mid = (int)(((int64_t)lo + hi) >> 1);
        if ((int64_t)sk[mid] < s) lo = mid + 1; else hi = mid;
      }
    }
    J.seg_off[s] = lo;
  }
}

static inline int grid_for(int64_t total, int cap) {
  if (total <= 0) return 0;
  int64_t g = total;
  if (cap > 0 && g > cap) g = cap;
  if (g > 0x7fffffff) g = 0x7fffffff;
  return (int)g;
}

hipError_t launch_rotate_bin(const Table *dt, const TableHeader &h, int cap, hipStream_t s) {
  const int max_passes = h.max_passes;
  int g = grid_for(h.total[K_ROT], cap);
  if (g) hipLaunchKernelGGL(k_rotate, dim3(g), dim3(kSortThreads), 0, s, dt);
  for (int p = 0; p < max_passes; ++p) {
    // the first pass's histograms come from k_rotate
    if (g && p > 0) hipLaunchKernelGGL(k_hist, dim3(g), dim3(kSortThreads), 0, s, dt, p);
    int gs = grid_for(h.total[K_SCAN], cap);
    if (gs) hipLaunchKernelGGL(k_scan, dim3(gs), dim3(256), 0, s, dt, p);
    if (g) hipLaunchKernelGGL(k_scatter, dim3(g), dim3(kSortThreads), 0, s, dt, p);
  }
  int gseg = grid_for(h.total[K_SEG], cap);
  if (gseg) hipLaunchKernelGGL(k_segoff, dim3(gseg), dim3(256), 0, s, dt);
  return hipGetLastError();
}

int rotate_bin_kernel_kind(const void *f) {
  if (f == (const void *)k_rotate || f == (const void *)k_hist || f == (const void *)k_scatter)
    return K_ROT;
  if (f == (const void *)k_scan) return K_SCAN;
  if (f == (const void *)k_segoff) return K_SEG;
  return -1;
}

}  // namespace rubix
