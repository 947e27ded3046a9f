// Internal layout shared by the HIP translation units of librubix: the device job table that every
// kernel reads, work-item ("virtual block") bookkeeping and launch helpers.
//
// Every kernel walks virtual blocks vb = blockIdx.x, blockIdx.x + gridDim.x, ... < table->total[K]
// and maps vb to (job, local block) with the per-job prefix jobs[j].vb_start[K]. A launch whose grid
// equals the total is an ordinary one-pass launch; a smaller grid makes the same kernel persistent.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rubix.h"

namespace rubix {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per sort work item
constexpr int kPrepThreads = 256;
constexpr int kPrepBlock = 1024;    // sorted particles per record block (ordered by spaxel, SSP cell)
constexpr int kCubeThreads = 256;   // threads per cube work item (4 waves)
constexpr int kCubeWaveBins = 62;   // telescope bins per wave; its 64 lanes stage a 64-node window
constexpr int kCubeTL = 4 * kCubeWaveBins;  // telescope bins per cube tile
constexpr int kCubeGroup = 4;       // particles staged per wave at once (their loads overlap)
constexpr int kCubeChunk = 2048;    // max particles per cube work item
constexpr int kBinWaveBins = 60;    // bin-mean kernel: telescope bins per wave
constexpr int kBinTL = 4 * kBinWaveBins;
constexpr int kCubeSubsum = 256;    // particles per inner FP32 partial sum
constexpr int kWPad = 4;            // zero weights before a padded filter
constexpr int kWArray = 2 * RUBIX_MAX_RADIUS + 1 + 16;   // padded filter array (zeros after)
constexpr int kLsfOut = 2048;       // bins per LSF work item (two runs of 4 per thread)
constexpr int kPsfLanes = 64;       // bins per PSF work item
constexpr int kPsfSeg = 64;         // spaxels of a line per PSF work item (16 per wave)
// fused PSF+LSF pass: a work item owns kFuseX x positions by kFuseL bins and walks every y row;
// it takes jobs whose PSF radius is 1..kFuseR and whose LSF radius is at most kFuseLsfR
constexpr int kFuseX = 16;
constexpr int kFuseL = 64;
constexpr int kFuseR = 8;
constexpr int kFuseU = 4;          // fused pass: rows per unrolled block of the y update
constexpr int kFuseLsfR = 22;
constexpr int kFuseRows = kFuseX + 2 * kFuseR;          // staged x positions per row
constexpr int kFuseW = kFuseL + 2 * kFuseLsfR + 4;      // LDS floats per staged x position
constexpr int kBwdParticles = 16;   // particles per backward work item (4 per wave)
constexpr int kFinThreads = 256;
constexpr int kVbParticles = 16384; // particles per Doppler-bound work item

enum Kind : int {
  K_ROT = 0,   // rotate/key and radix-sort tiles (per kSortTile particles)
  K_SCAN,      // per (job, digit)
  K_SEG,       // seg_off, per 256 spaxels
  K_PREP,      // per kPrepBlock sorted particles
  K_CHUNK,     // one per job
  K_CUBE,      // per (lambda tile, chunk slot)
  K_COMB,      // per (lambda tile, combine slot)
  K_LSF,       // per (spaxel, lambda tile)
  K_PSFY,      // per (x column, y segment, lambda tile)
  K_PSFX,      // per (y row, x segment, lambda tile)
  K_COPY,      // per 64k floats of a cube (identity PSF/LSF)
  K_FUSE,      // fused PSF+LSF, per (lambda tile of kFuseL bins, x segment of kFuseX)
  K_BINTAB,    // per 256 bin edges of a bin-mean job
  K_BWD,       // per kBwdParticles sorted particles
  K_FIN,       // per kFinThreads sorted particles
  K_ANG,       // one per job
  K_VB,        // per kVbParticles particles (Doppler bounds for the cube kernel)
  K_CUBEB,     // per (lambda tile of kBinTL bins, chunk slot): bin-mean resampling jobs
  K_BWDB,      // per kBwdParticles sorted particles of a bin-mean job (K_BWD covers the others)
  NK
};

// Per-particle record written by the prep kernel, in sorted order (32 bytes).
struct PrepRec {
  int32_t row;      // flux offset of corner (ja, jz): (ja*n_met + jz)*n_lam, stored as ~offset
                    // (negative) when the particle's node span does not fit a wave window (see
                    // prep_row): the 62 node indices of a wave's bins then span more than 63 nodes
  float g;          // Doppler term of the node index: beta/(1+beta) / ((1+z_sys) dlam_ssp)
                    // per Angstrom of bin wavelength, or ln(1+beta)/dln_ssp on log grids
  float a[4];       // corner weights (forward: flux_scale m J w_c; backward: w_c)
  int32_t spaxel;   // key of the particle (backward records; -1 in forward records)
  int32_t pad;      // backward records: the particle's input index; 0 in forward records
};

// Flux offset of a record's corner (ja, jz) whatever its window flag.
__host__ __device__ inline int32_t prep_row(int32_t row) { return row < 0 ? ~row : row; }

struct ChunkRec {
  int32_t s, p0, p1, slot;   // spaxel, sorted particle range [p0, p1), partial slot or -1
};

struct CombRec {
  int32_t s, first_slot, n_slots, pad;
};

typedef __attribute__((address_space(1))) const float GFloat;     // global memory
typedef __attribute__((address_space(1))) const char GChar;

struct SspDev {
  const float *flux;
  int32_t n_age, n_met, n_lam, log_lambda;   // log_lambda: nodes lam_start * exp(k lam_step)
  double lam_start, lam_step;
  double age_thr[RUBIX_MAX_AGE_NODES];   // 10^(log age node), FP64 cell thresholds in Gyr
  double log_age[RUBIX_MAX_AGE_NODES];   // log10 age nodes (FP64 copies of the FP32 inputs)
  double met[RUBIX_MAX_MET_NODES];
};

struct JobDev {
  // inputs
  const float *x, *y, *z, *vx, *vy, *vz, *mass, *age, *met;
  int32_t n, nx, ny, n_s;
  double R[9];        // rotation matrix, row major
  double dR2[9];      // dR[2][:]/dphi_k for k = 0, 1, 2 (row k)
  double spaxel, half_nx, half_ny;
  double tel_start, tel_step, z_sys, flux_scale;
  double lsf_sigma_bins, psf_sigma;
  // normalised weights of offsets -r..r at [kWPad + k + r], zero-padded by kWPad on both sides
  // so register-blocked filters can read weights of out-of-range offsets without a branch
  float lsf_w[kWArray];
  float psf_w[kWArray];
  int32_t n_tel, passes, n_sort_tiles, n_tiles;     // n_tiles: cube lambda tiles of kCubeTL bins
  int32_t cube_direct, log_lambda;                   // 1 = gather taps from global (coarse grids);
                                                     // 1 = both grids uniform in ln(lambda)
  double q_off, q_ratio;  // log grids: rest-frame node index of bin j is q_off + j * q_ratio
  int32_t resample, n_tiles_b;  // 1 = bin-mean resampling; its tiles of kBinTL bins
  double bin_scale;             // bin mean: dlam_ssp / dlam_tel (linear grids), 1 (log grids)
  double bin_slope;                                  // d(node index)/d(bin) at rest
  double inv_opz, inv_ds;  // 1/(1+z_sys) and 1/dlam_ssp (linear grids: the rest-frame index)
  // rest-frame node index at zero velocity of bin centre j in 40-bit fixed point:
  // Q_j * 2^40 = q0x + j * qrx (linear and log grids), for the adjoint's per-window split
  int64_t q0x, qrx;
  int32_t n_chunk_ub, n_comb_ub, lsf_r, psf_r;
  int32_t n_psf_tiles, n_psf_seg_y, n_psf_seg_x, n_fin_blocks;
  // outputs
  int32_t *key, *perm, *seg_off;
  float *vlos, *cube_raw;
  // PSF/LSF passes: source and destination of the lambda, y and x passes (null = skipped);
  // copy_src/copy_dst for a job with no pass at all
  const float *pl_src[3];
  float *pl_dst[3];
  const float *copy_src;
  float *copy_dst;
  // fused PSF+LSF pass (replaces the three passes where the radii allow it)
  const float *fuse_src;
  float *fuse_dst;
  int64_t cube_elems;
  // backward I/O
  const float *grad_raw;
  float *d_mass, *d_age, *d_met, *d_vlos, *d_vel;
  double *d_angles;     // 3 doubles for this job
  // workspace (per job)
  uint32_t *kbuf[2], *vbuf[2];
  uint32_t *hist;       // [256][n_sort_tiles], digit major
  uint32_t *dtot;       // [256]
  PrepRec *prep;        // [n]
  float4 *pay;          // [n]: (mass, age, [M/H], vlos) in input order
  ChunkRec *chunks;     // [n_chunk_ub]
  CombRec *combs;       // [n_comb_ub]
  int32_t *counts;      // [0] chunks, [1] combine entries, [2] bits of the largest |Doppler
                        // slope| of the job, [3] nonzero if some particle's span does not fit
  float *partial;       // [n_comb_slots_ub][n_tel]
  float *tmp_cube;      // [cube_elems]
  float4 *bintab;       // [n_tel + 1] bin edges of a bin-mean job: (node index integer part
                        // as int bits, frac, lambda, 0)
  double *dots;         // [n][4]: s_m, s_a, s_z, Y per in-field particle, in input order
  double *ang_part;     // [n_fin_blocks][3]
  int64_t vb_start[NK];
};

struct TableHeader {
  int32_t n_jobs, max_passes;   // max_passes: most radix-sort passes any job of the table needs
  int32_t max_psf_r, max_lsf_r; // largest PSF / LSF radius of the table (sizes LDS)
  int64_t total[NK];
  SspDev ssp;
};

struct Table {
  TableHeader h;
  // JobDev jobs[n_jobs] follows, 16-byte aligned
};

__host__ __device__ inline const JobDev *table_jobs(const Table *t) {
  return reinterpret_cast<const JobDev *>(reinterpret_cast<const char *>(t) +
                                          ((sizeof(Table) + 255) & ~size_t(255)));
}

__host__ __device__ inline size_t table_bytes(int n_jobs) {
  return ((sizeof(Table) + 255) & ~size_t(255)) + size_t(n_jobs) * sizeof(JobDev);
}

// Largest job index j with jobs[j].vb_start[kind] <= vb (vb is wave-uniform).
__device__ inline int find_job(const Table *t, int kind, int64_t vb) {
  const JobDev *jobs = table_jobs(t);
  int lo = 0, hi = t->h.n_jobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].vb_start[kind] <= vb) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// floor(t) as an integer in one instruction (floor-and-convert); t is finite and far inside the
// int range here.
__device__ __forceinline__ int floor_i32(float t) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(t));
  return r;
}

// Bin-mean resampling helpers, shared by the forward sum and its adjoint so both see the same
// bin edges. Integral over a node segment of the linear interpolant between s0 and s1, from
// fraction x to fraction y.
__device__ __forceinline__ float seg_integral(float s0, float s1, float x, float y) {
  return fmaf(s0, y - x, 0.5f * (s1 - s0) * (y * y - x * x));
}

// Node interval and fraction of an edge, clipped to [0, n-1] as (k, t) with k in [0, n-2].
__device__ __forceinline__ void clip_node(int &k, float &t, int nl) {
  if (k < 0) { k = 0; t = 0.f; }
  else if (k > nl - 2) { k = nl - 2; t = 1.f; }
}

// Rest-frame node index at zero velocity of wavelength lam on a linear grid,
// Q = (lam/(1+z) - lam0_ssp)/dlam_ssp with the two divisions taken as multiplications by the
// job's reciprocals, split into its integer part qi and FP32 fraction qf.
__device__ __forceinline__ void split_q(double Q, int &qi, float &qf) {
  const double Qfl = floor(Q);
  qi = (int)fmin(fmax(Qfl, -1.0e9), 1.0e9);
  qf = (float)(Q - Qfl);
}
__device__ __forceinline__ double rest_q(const JobDev &J, const SspDev &S, double lam) {
  return (lam * J.inv_opz - S.lam_start) * J.inv_ds;
}

// Rest-frame node index of telescope bin jb's centre, split into an integer and an FP32
// fraction, and the factor lamf that multiplies the particle's Doppler term g (the particle's
// index is qi + qf - lamf g): the bin wavelength on linear grids; 1 on log grids, where
// Q = q_off + jb q_ratio. The forward sums and the bin-mean edges take it from here; the adjoint
// walks the bins with the fixed-point form of the same rest index (q0x, qrx in JobDev).
__device__ __forceinline__ void split_index(const JobDev &J, const SspDev &S, int jb, int &qi,
                                            float &qf, float &lamf) {
  if (J.log_lambda) {
    split_q(J.q_off + (double)jb * J.q_ratio, qi, qf);
    lamf = 1.0f;
  } else {
    const double lam = J.tel_start + (double)jb * J.tel_step;
    split_q(rest_q(J, S, lam), qi, qf);
    lamf = (float)lam;
  }
}

// The same for telescope bin edge e (the lower edge of bin e, the upper edge of bin e - 1): at
// wavelength start + (e - 1/2) step on linear grids; on log grids at ln lambda = ln start +
// (e - 1/2) step, where Q = q_off + (e - 1/2) q_ratio and the Doppler factor is 1.
__device__ __forceinline__ void bin_edge(const JobDev &J, const SspDev &S, int e, int &qi,
                                         float &qf, float &lamf) {
  if (J.log_lambda) {
    split_q(J.q_off + ((double)e - 0.5) * J.q_ratio, qi, qf);
    lamf = 1.0f;
    return;
  }
  const double lam = J.tel_start + ((double)e - 0.5) * J.tel_step;
  split_q(rest_q(J, S, lam), qi, qf);
  lamf = (float)lam;
}

// Log grids (bin mean): the weight of rest wavelength over a segment, by Taylor series in
// h = (fraction) * dln: E1(h) = e^h - 1 and Phi(h) = e^h - (e^h - 1)/h, four terms each (the ABI
// admits SSP steps up to 0.05, where the next terms are below 1e-7).
__device__ __forceinline__ float expm1_small(float h) {
  return h * fmaf(h, fmaf(h, fmaf(h, 1.f / 24.f, 1.f / 6.f), 0.5f), 1.f);
}
__device__ __forceinline__ float phi_small(float h) {
  return h * fmaf(h, fmaf(h, fmaf(h, 1.f / 30.f, 0.125f), 1.f / 3.f), 0.5f);
}
// wavelength of node k from the lane's reference node qe (wavelength lam_e): a short series in
// the small exponent (k - qe) dln, or the exponential itself where the exponent is not small
__device__ __forceinline__ float node_lambda(int k, int qe, float lam_e, float lam0, float dln) {
  const float x = (float)(k - qe) * dln;
  if (fabsf(x) <= 0.05f) return fmaf(lam_e, expm1_small(x), lam_e);
  return lam0 * expf((float)k * dln);
}
// integral over rest wavelength of the segment from node k (value s0, slope d) to fraction a
__device__ __forceinline__ float log_partial(float lamk, float s0, float d, float a, float dln) {
  const float h = a * dln;
  return lamk * fmaf(s0, expm1_small(h), d * a * phi_small(h));
}

// Launchers (one per translation unit); grid = number of blocks (persistent if < total).
hipError_t launch_upload(const void *host_table, size_t bytes, void *dev_table, hipStream_t s);
hipError_t launch_rotate_bin(const Table *dt, const TableHeader &h, int grid_cap, hipStream_t s);
hipError_t launch_cube(const Table *dt, const TableHeader &h, int grid_cap, hipStream_t s);
// When both are non-null, launch_cube records them on its stream right before and right after
// the cube-summation kernel (a measurement aid; set per call by the ABI, null otherwise).
extern thread_local hipEvent_t t_cube_events[2];
hipError_t launch_psf_lsf(const Table *dt, const TableHeader &h, int grid_cap, hipStream_t s);
hipError_t launch_backward(const Table *dt, const TableHeader &h, int grid_cap, hipStream_t s);

hipError_t launch_noise(float *cube, int64_t n, uint64_t seed, uint32_t stream, double gain,
                        double sigma_floor, hipStream_t s);

// Work-item kind (Kind) whose total sets the grid of a forward kernel, or -1 if `func` is not one
// of that file's forward kernels (identifies the kernel nodes of a captured forward sequence).
int rotate_bin_kernel_kind(const void *func);
int cube_kernel_kind(const void *func);
int psf_lsf_kernel_kind(const void *func);

// Block-wide exclusive scan of one value per thread (256 threads); returns the block total.
__device__ __forceinline__ uint32_t block_exclusive_scan_256(uint32_t v, uint32_t *lds,
                                                             uint32_t &excl) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    uint32_t add = (t >= off) ? lds[t - off] : 0u;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  uint32_t incl = lds[t];
  uint32_t total = lds[255];
  __syncthreads();
  excl = incl - v;
  return total;
}

}  // namespace rubix
