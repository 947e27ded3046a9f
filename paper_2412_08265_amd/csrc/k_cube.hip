// Steps 3-6 of the pipeline (arXiv:2412.08265, Sec. 3): SSP lookup, Doppler shift, resampling to
// the telescope grid and the per-spaxel sum.
//
// Data flow (all on the caller's stream):
//   k_prep    one thread per sorted in-field particle: gathers (mass, age, [M/H], v_los) through
//             perm, finds the SSP cell, and writes a 32-byte record {flux row, Doppler slope g,
//             4 corner weights} in spaxel order.
//   k_chunks  one block per job: splits every spaxel's particle range into chunks of at most
//             kCubeChunk particles (load balance for dense central spaxels); chunks of a spaxel
//             with several chunks get partial-sum slots.
//   k_cube    one block per (lambda tile of kCubeTL bins, chunk): lanes own telescope bins and
//             loop over the chunk's particles, accumulating in registers (no atomics). Blocks are
//             ordered lambda-tile major, so the blocks resident on one XCD at a time share one
//             tile's slice of the template grid in that XCD's L2.
//   k_combine sums a multi-chunk spaxel's partial spectra in chunk order (deterministic).
//
// Resampling index: for bin centre lam_j the node index of the rest-frame wavelength is
//   q = (lam_j/((1+z)(1+beta)) - lam0)/dlam = Q_j - lam_j * g,
//   Q_j = (lam_j/(1+z) - lam0)/dlam,  g = beta/(1+beta) / ((1+z) dlam).
// Q_j is formed in FP64 per lane and split into an integer and an FP32 fraction; only the small
// Doppler term lam_j*g is FP32, so q carries an absolute error of ~1e-6 nodes instead of the
// ~1e-3 that an FP32 lam/(1+beta) would give at 9000 A.
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
    r.pad = 0;
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

__global__ __launch_bounds__(kCubeTL) void k_cube(const Table *__restrict__ T) {
  const SspDev &S = T->h.ssp;
  const JobDev *jobs = table_jobs(T);
  const float *__restrict__ flux = S.flux;
  const int nl = S.n_lam;
  const int o1 = nl, o2 = S.n_met * nl, o3 = o2 + nl;
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_CUBE]; vb += gridDim.x) {
    const int jj = find_job(T, K_CUBE, vb);
    const JobDev &J = jobs[jj];
    const int64_t local = vb - J.vb_start[K_CUBE];
    const int tile = (int)(local / J.n_chunk_ub);
    const int c = (int)(local - (int64_t)tile * J.n_chunk_ub);
    if (c >= J.counts[0]) continue;
    const ChunkRec ch = J.chunks[c];
    const int jb = tile * kCubeTL + threadIdx.x;
    const bool act = jb < J.n_tel;
    const double lam = J.tel_start + (double)jb * J.tel_step;
    const double Q = (lam / (1.0 + J.z_sys) - S.lam_start) / S.lam_step;
    const double Qfl = floor(Q);
    const int qi = (int)fmin(fmax(Qfl, -1.0e9), 1.0e9);
    const float qf = (float)(Q - Qfl);
    const float lamf = (float)lam;
    float acc = 0.f, tot = 0.f;
    const PrepRec *__restrict__ prep = J.prep;
    for (int p = ch.p0; p < ch.p1; ++p) {
      const PrepRec r = prep[p];
      const float tq = fmaf(-lamf, r.g, qf);
      const float fl = floorf(tq);
      const float tau = tq - fl;
      const int k = qi + (int)fminf(fmaxf(fl, -1.0e8f), 1.0e8f);
      const bool ok = act && (k >= 0) && ((k < nl - 1) || (k == nl - 1 && tau == 0.f));
      if (ok) {
        const int kk = min(k, nl - 2);
        const float tt = (k > kk) ? 1.f : tau;
        const float *b = flux + r.row + kk;
        const float v0 = fmaf(tt, b[1] - b[0], b[0]);
        const float v1 = fmaf(tt, b[o1 + 1] - b[o1], b[o1]);
        const float v2 = fmaf(tt, b[o2 + 1] - b[o2], b[o2]);
        const float v3 = fmaf(tt, b[o3 + 1] - b[o3], b[o3]);
        acc = fmaf(r.a[0], v0, acc);
        acc = fmaf(r.a[1], v1, acc);
        acc = fmaf(r.a[2], v2, acc);
        acc = fmaf(r.a[3], v3, acc);
      }
      if (((p - ch.p0) & (kCubeSubsum - 1)) == kCubeSubsum - 1) { tot += acc; acc = 0.f; }
    }
    tot += acc;
    if (act) {
      if (ch.slot < 0) J.cube_raw[(int64_t)ch.s * J.n_tel + jb] = tot;
      else J.partial[(int64_t)ch.slot * J.n_tel + jb] = tot;
    }
  }
}

__global__ __launch_bounds__(kCubeTL) void k_combine(const Table *__restrict__ T) {
  const JobDev *jobs = table_jobs(T);
  for (int64_t vb = blockIdx.x; vb < T->h.total[K_COMB]; vb += gridDim.x) {
    const int jj = find_job(T, K_COMB, vb);
    const JobDev &J = jobs[jj];
    const int64_t local = vb - J.vb_start[K_COMB];
    const int tile = (int)(local / J.n_comb_ub);
    const int e = (int)(local - (int64_t)tile * J.n_comb_ub);
    if (e >= J.counts[1]) continue;
    const CombRec cr = J.combs[e];
    const int jb = tile * kCubeTL + threadIdx.x;
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
    hipLaunchKernelGGL(k_cube, dim3(g), dim3(kCubeTL), 0, s, dt);
  if ((g = grid_for(h.total[K_COMB], cap)))
    hipLaunchKernelGGL(k_combine, dim3(g), dim3(kCubeTL), 0, s, dt);
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
