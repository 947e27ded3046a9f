// Steps 3-6 of the pipeline (arXiv:2412.08265, Sec. 3): SSP lookup, Doppler shift, resampling to
// the telescope grid and the per-spaxel sum.
//
// Data flow (all on the caller's stream):
//   k_prep    one thread per sorted in-field particle: gathers (mass, age, [M/H], v_los) through
//             perm, finds the SSP cell, and writes a 32-byte record {flux row, Doppler slope g,
//             4 corner weights, spaxel, node-offset bounds} in spaxel order.
//   k_chunks  one block per job: splits every spaxel's particle range into chunks of at most
//             kCubeChunk particles (load balance for dense central spaxels); chunks of a spaxel
//             with several chunks get partial-sum slots.
//   k_cube    one block per (lambda tile of at most kCubeMaxTL bins, chunk), particles taken in
//             batches of kCubeBatch:
//               phase 1  lanes span SSP nodes: each staged particle's bilinear spectrum
//                        S_i[n] = sum_c a_ic T_c[n] over the tile's node window goes to LDS
//                        (four coalesced row loads per node, the template slice sits in L2);
//               phase 2  lanes span telescope bins: the Doppler-shifted node index and one
//                        ds_read2 of (S_i[k], S_i[k+1]) give the resampled value, accumulated in
//                        registers (no atomics).
//             Blocks are ordered lambda-tile major, so the blocks resident on one XCD at a time
//             share one tile's slice of the template grid in that XCD's L2.
//   k_combine sums a multi-chunk spaxel's partial spectra in chunk order (deterministic).
//
// Resampling index: for bin centre lam_j the node index of the rest-frame wavelength is
//   q = (lam_j/((1+z)(1+beta)) - lam0)/dlam = Q_j - lam_j * g,
//   Q_j = (lam_j/(1+z) - lam0)/dlam,  g = beta/(1+beta) / ((1+z) dlam).
// Q_j is formed in FP64 per lane and split into an integer and an FP32 fraction; only the small
// Doppler term lam_j*g is FP32, so q carries an absolute error of ~1e-6 nodes instead of the
// ~1e-3 that an FP32 lam/(1+beta) would give at 9000 A. The integer part k = floor(q) is the
// same FP32 decision in every kernel (forward and adjoint).
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

// mode 0: forward weights flux_scale*m*J*w_c; mode 1: plain bilinear weights w_c.
__global__ __launch_bounds__(kPrepThreads) void k_prep(const Table *__restrict__ T, int mode) {
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_PREP]; vb += gridDim.x) {
    const int jj = find_job(T, K_PREP, vb);
    const JobDev &J = jobs[jj];
    const int64_t i = (vb - J.vb_start[K_PREP]) * kPrepThreads + threadIdx.x;
    const int n_in = J.seg_off[J.n_s];
    if (i >= n_in) continue;
    const int j = J.perm[i];
    const double age = J.age[j], m = J.mass[j], met = J.met[j], v = J.vlos[j];
    const int ja = cell_of(S.age_thr, S.n_age, age);
    double ta;
    if (!(age > S.age_thr[0])) ta = 0.0;
    else if (age >= S.age_thr[S.n_age - 1]) ta = 1.0;
    else ta = clamp01((log10(age) - S.log_age[ja]) / (S.log_age[ja + 1] - S.log_age[ja]));
    const int jz = cell_of(S.met, S.n_met, met);
    double tz;
    if (!(met > S.met[0])) tz = 0.0;
    else if (met >= S.met[S.n_met - 1]) tz = 1.0;
    else tz = clamp01((met - S.met[jz]) / (S.met[jz + 1] - S.met[jz]));
    const double beta = v / kCkms;
    const double opz = 1.0 + J.z_sys;
    const double jac = 1.0 / (opz * (1.0 + beta));
    const double scale = mode == 0 ? J.flux_scale * m * jac : 1.0;
    PrepRec r;
    r.row = (ja * S.n_met + jz) * S.n_lam;
    r.g = (float)(beta / (1.0 + beta) / (opz * S.lam_step));
    r.a[0] = (float)(scale * (1.0 - ta) * (1.0 - tz));
    r.a[1] = (float)(scale * (1.0 - ta) * tz);
    r.a[2] = (float)(scale * ta * (1.0 - tz));
    r.a[3] = (float)(scale * ta * tz);
    r.spaxel = J.key[j];
    // floor(q) - floor(Q_j) = floor(fl32(Qf_j - lam_j g)) with Qf_j in [0, 1] and lam_j over the
    // band: bounded by the band ends, with one node of margin each side for FP32 rounding and one
    // more below, so that the interval (k-1, k) used at the last SSP node is inside the window
    const double glo = (double)r.g;
    const double l0 = (double)(float)J.tel_start;
    const double l1 = (double)(float)(J.tel_start + (J.n_tel - 1) * J.tel_step);
    const double e0 = -l0 * glo, e1 = -l1 * glo;
    const double mn = fmin(e0, e1), mx = fmax(e0, e1);
    if (isfinite(mn) && isfinite(mx) && mn > -30000.0 && mx < 30000.0) {
      const int dlo = (int)floor(mn) - 2;
      const int dhi = (int)floor(mx) + 2;
      r.lohi = (int32_t)((uint32_t)(dlo & 0xffff) | ((uint32_t)dhi << 16));
    } else {
      r.lohi = kLohiBad;
    }
    J.prep[i] = r;
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

// One particle's resampled contribution to bin jb with both taps gathered from the template grid
// (particles without a bounded node window, and jobs whose telescope grid is much coarser than
// the SSP grid).
__device__ __forceinline__ float direct_contrib(const PrepRec &r, const float *__restrict__ flux,
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
  const float *b = flux + r.row + kk;
  float v = r.a[0] * fmaf(tt, b[1] - b[0], b[0]);
  v = fmaf(r.a[1], fmaf(tt, b[o1 + 1] - b[o1], b[o1]), v);
  v = fmaf(r.a[2], fmaf(tt, b[o2 + 1] - b[o2], b[o2]), v);
  v = fmaf(r.a[3], fmaf(tt, b[o3 + 1] - b[o3], b[o3]), v);
  return v;
}

__device__ __forceinline__ void split_index(const JobDev &J, const SspDev &S, int jb, int &qi,
                                            float &qf, float &lamf) {
  const double lam = J.tel_start + (double)jb * J.tel_step;
  const double Q = (lam / (1.0 + J.z_sys) - S.lam_start) / S.lam_step;
  const double Qfl = floor(Q);
  qi = (int)fmin(fmax(Qfl, -1.0e9), 1.0e9);
  qf = (float)(Q - Qfl);
  lamf = (float)lam;
}

__global__ __launch_bounds__(kCubeThreads) void k_cube(const Table *__restrict__ T) {
  __shared__ float sbuf[kCubeBatch * kCubeSlot];
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  const float *__restrict__ flux = S.flux;
  const int nl = S.n_lam;
  const int o1 = nl, o2 = S.n_met * nl, o3 = o2 + nl;
  const int tid = threadIdx.x;
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_CUBE]; vb += gridDim.x) {
    const int jj = find_job(T, K_CUBE, vb);
    const JobDev &J = jobs[jj];
    const int64_t local = vb - J.vb_start[K_CUBE];
    const int tile = (int)(local / J.n_chunk_ub);
    const int c = (int)(local - (int64_t)tile * J.n_chunk_ub);
    if (c >= J.counts[0]) continue;
    const ChunkRec ch = J.chunks[c];
    const int TL = J.cube_tl;
    const int j0 = tile * TL;
    const int jl = min(j0 + TL, J.n_tel) - 1;
    const int jb = j0 + tid;
    const bool act = (tid < TL) && (jb < J.n_tel);
    const bool direct_job = J.cube_direct != 0;
    int qi, qi0, qil;
    float qf, lamf, qf_u, lam_u;
    split_index(J, S, jb, qi, qf, lamf);
    split_index(J, S, j0, qi0, qf_u, lam_u);     // tile-uniform node index range
    split_index(J, S, jl, qil, qf_u, lam_u);
    const int span = qil - qi0;
    const int lrel = qi - qi0;
    float acc = 0.f, tot = 0.f;
    int since = 0;
    const PrepRec *__restrict__ prep = J.prep;
    for (int pb = ch.p0; pb < ch.p1; pb += kCubeBatch) {
      const int nb = min(kCubeBatch, ch.p1 - pb);
      // phase 1: node windows of the batch's spectra into LDS
#pragma unroll
      for (int b = 0; b < kCubeBatch; ++b) {
        if (b < nb) {
          const PrepRec r = prep[pb + b];
          const int dlo = (int)(int16_t)(r.lohi & 0xffff), dhi = r.lohi >> 16;
          const int W = span + dhi - dlo + 2;
          if (!direct_job && r.lohi != kLohiBad && W <= kCubeSlot) {
            const int n0 = qi0 + dlo;
            const bool inside = (n0 >= 0) && (n0 + W <= nl);
            const float *__restrict__ rp = flux + r.row;
            for (int m = tid; m < W; m += kCubeThreads) {
              int node = n0 + m;
              if (!inside) node = min(max(node, 0), nl - 1);
              float v = r.a[0] * rp[node];
              v = fmaf(r.a[1], rp[o1 + node], v);
              v = fmaf(r.a[2], rp[o2 + node], v);
              v = fmaf(r.a[3], rp[o3 + node], v);
              sbuf[b * kCubeSlot + m] = v;
            }
          }
        }
      }
      __syncthreads();
      // phase 2: Doppler-shifted linear resampling from the staged spectra
#pragma unroll
      for (int b = 0; b < kCubeBatch; ++b) {
        if (b < nb) {
          const PrepRec r = prep[pb + b];
          const int dlo = (int)(int16_t)(r.lohi & 0xffff), dhi = r.lohi >> 16;
          const int W = span + dhi - dlo + 2;
          if (!direct_job && r.lohi != kLohiBad && W <= kCubeSlot) {
            const int n0 = qi0 + dlo;
            const bool inside = (n0 >= 0) && (n0 + W <= nl);
            const float tq = fmaf(-lamf, r.g, qf);
            const float fl = floorf(tq);
            const float tau = tq - fl;
            const int fi = (int)fminf(fmaxf(fl, -30000.f), 30000.f);
            if (inside) {
              // every node of the window exists: no range test; the clamp only guards lanes
              // past the end of the band, whose results are discarded
              const int idx = min(max(lrel + fi - dlo, 0), kCubeSlot - 2);
              const float s0 = sbuf[b * kCubeSlot + idx];
              const float s1 = sbuf[b * kCubeSlot + idx + 1];
              acc += fmaf(tau, s1 - s0, s0);
            } else {
              const int k = qi + fi;
              const bool ok = act && (k >= 0) && ((k < nl - 1) || (k == nl - 1 && tau == 0.f));
              if (ok) {
                const int kk = min(k, nl - 2);
                const float tt = (k > kk) ? 1.f : tau;
                const int idx = min(max(kk - n0, 0), kCubeSlot - 2);
                const float s0 = sbuf[b * kCubeSlot + idx];
                const float s1 = sbuf[b * kCubeSlot + idx + 1];
                acc += fmaf(tt, s1 - s0, s0);
              }
            }
          } else {
            acc += direct_contrib(r, flux, nl, o1, o2, o3, qi, qf, lamf, act);
          }
        }
      }
      since += nb;
      if (since >= kCubeSubsum) { tot += acc; acc = 0.f; since = 0; }
      __syncthreads();
    }
    tot += acc;
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
    if ((int)threadIdx.x >= J.cube_tl) continue;
    const int jb = tile * J.cube_tl + threadIdx.x;
    if (jb >= J.n_tel) continue;
    float sum = 0.f;
    for (int q = 0; q < cr.n_slots; ++q) sum += J.partial[(int64_t)(cr.first_slot + q) * J.n_tel + jb];
    J.cube_raw[(int64_t)cr.s * J.n_tel + jb] = sum;
  }
}

static inline int grid_for(int64_t total, int cap) {
  if (total <= 0) return 0;
  int64_t g = total;
  if (cap > 0 && g > cap) g = cap;
  if (g > 0x7fffffff) g = 0x7fffffff;
  return (int)g;
}

hipError_t launch_cube(const Table *dt, const TableHeader &h, int cap, hipStream_t s) {
  int g;
  if ((g = grid_for(h.total[K_PREP], cap)))
    hipLaunchKernelGGL(k_prep, dim3(g), dim3(kPrepThreads), 0, s, dt, 0);
  if ((g = grid_for(h.total[K_CHUNK], cap)))
    hipLaunchKernelGGL(k_chunks, dim3(g), dim3(1024), 0, s, dt);
  if ((g = grid_for(h.total[K_CUBE], cap)))
    hipLaunchKernelGGL(k_cube, dim3(g), dim3(kCubeThreads), 0, s, dt);
  if ((g = grid_for(h.total[K_COMB], cap)))
    hipLaunchKernelGGL(k_combine, dim3(g), dim3(kCubeThreads), 0, s, dt);
  return hipGetLastError();
}

// Backward needs the same per-particle records with plain bilinear weights.
hipError_t launch_prep_backward(const Table *dt, const TableHeader &h, int cap, hipStream_t s) {
  int g;
  if ((g = grid_for(h.total[K_PREP], cap)))
    hipLaunchKernelGGL(k_prep, dim3(g), dim3(kPrepThreads), 0, s, dt, 1);
  return hipGetLastError();
}

}  // namespace rubix
