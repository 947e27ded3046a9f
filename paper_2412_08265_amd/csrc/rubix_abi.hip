// Host side of the C ABI declared in include/rubix.h: argument validation, workspace layout, the
// device job table and the launch sequences. No allocation, no host<->device copies of data; the
// job table reaches the device through kernel arguments (k_upload), so a call can be captured in
// a HIP graph as is.
#include <math.h>
#include <stdarg.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <cstdio>
#include <string>
#include <vector>

#include "rubix_internal.h"

namespace rubix {

hipError_t launch_prep_backward(const Table *dt, const TableHeader &h, int cap, hipStream_t s);

// ---------------------------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------------------------
static thread_local std::string g_err;
// cube-kernel timer (measurement aid): on/off and the event pairs recorded since the last read
static thread_local bool g_timer_on = false;
static thread_local std::vector<std::pair<hipEvent_t, hipEvent_t>> g_timer_ev;

static int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// ---------------------------------------------------------------------------------------------
// upload of the job table through kernel arguments
// ---------------------------------------------------------------------------------------------
struct UploadChunk {
  uint32_t offset_words, n_words;
  uint32_t w[880];
};

__global__ void k_upload(UploadChunk c, uint32_t *dst) {
  for (uint32_t i = threadIdx.x; i < c.n_words; i += blockDim.x) dst[c.offset_words + i] = c.w[i];
}

hipError_t launch_upload(const void *host_table, size_t bytes, void *dev_table, hipStream_t s) {
  const uint32_t *src = static_cast<const uint32_t *>(host_table);
  const size_t words = (bytes + 3) / 4;
  UploadChunk c;
  for (size_t off = 0; off < words; off += 880) {
    c.offset_words = (uint32_t)off;
    c.n_words = (uint32_t)std::min<size_t>(880, words - off);
    memcpy(c.w, src + off, c.n_words * 4);
    hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, c, static_cast<uint32_t *>(dev_table));
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// sizes and layout
// ---------------------------------------------------------------------------------------------
static inline size_t al(size_t b) { return (b + 255) & ~size_t(255); }
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

enum Call { CALL_ROTATE, CALL_CUBE, CALL_PSF, CALL_BWD, CALL_SIZE, CALL_PACK };

struct JobSizes {
  int64_t n, n_s, n_tel, cube_elems;
  int passes, n_sort_tiles, n_tiles, n_tiles_b, n_chunk_ub, n_comb_ub, n_slot_ub;
  int lsf_r, psf_r, n_psf_tiles, n_psf_seg_y, n_psf_seg_x, n_fin_blocks;
  double lsf_sigma_bins;
  // byte offsets inside the job's workspace region
  size_t o_k0, o_k1, o_v0, o_v1, o_hist, o_dtot;                       // sort
  size_t o_prep, o_chunks, o_combs, o_counts, o_partial, o_pay;       // cube
  size_t o_tmp;                                                       // psf/lsf
  size_t o_bintab, o_dots, o_ang;                                     // backward (+ o_prep)
  size_t region;
  size_t psf_region;                                                  // psf/lsf alone
};

static int radius_of(double sigma) { return sigma > 0.0 ? (int)(4.0 * sigma + 0.5) : 0; }

// LSF width in telescope bins; on a log grid taken at the central wavelength (constant in bins).
static double lsf_bins(const rubix_job &j) {
  if (j.tel.log_spaced) {
    const double lam_c = j.tel.start * exp(j.tel.step * (j.tel.n - 1) / 2.0);
    return j.lsf_sigma_A / (lam_c * j.tel.step);
  }
  return j.lsf_sigma_A / j.tel.step;
}

static JobSizes sizes_of(const rubix_job &j) {
  JobSizes z{};
  z.n = j.p.n;
  z.n_s = (int64_t)j.grid.nx * j.grid.ny;
  z.n_tel = j.tel.n;
  z.cube_elems = z.n_s * z.n_tel;
  int bits = 0;
  while ((int64_t(1) << bits) <= z.n_s) ++bits;      // keys are 0..n_s
  z.passes = std::max(1, (bits + 7) / 8);
  z.n_sort_tiles = (int)cdiv(z.n, kSortTile);
  z.n_tiles = (int)cdiv(z.n_tel, kCubeTL);
  z.n_tiles_b = (int)cdiv(z.n_tel, kBinTL);
  z.n_chunk_ub = (int)(z.n_s + cdiv(z.n, kCubeChunk));
  z.n_comb_ub = z.n > kCubeChunk ? (int)(z.n / (kCubeChunk + 1) + 1) : 0;
  z.n_slot_ub = (int)(2 * cdiv(z.n, kCubeChunk) + 2);
  z.lsf_sigma_bins = lsf_bins(j);
  z.lsf_r = radius_of(z.lsf_sigma_bins);
  z.psf_r = radius_of(j.psf_sigma_spx);
  z.n_psf_tiles = (int)cdiv(z.n_tel, kPsfLanes);
  z.n_psf_seg_y = (int)cdiv(j.grid.ny, kPsfSeg);
  z.n_psf_seg_x = (int)cdiv(j.grid.nx, kPsfSeg);
  z.n_fin_blocks = (int)cdiv(z.n, kFinThreads);
  const size_t n4 = al(4 * (size_t)z.n);
  // sort region
  size_t o = 0;
  z.o_k0 = o; o += n4;
  z.o_k1 = o; o += n4;
  z.o_v0 = o; o += n4;
  z.o_v1 = o; o += n4;
  z.o_hist = o; o += al(4ull * 256 * z.n_sort_tiles);
  z.o_dtot = o; o += al(4 * 256);
  size_t sort_end = o;
  // cube region
  o = 0;
  z.o_prep = o; o += al(sizeof(PrepRec) * (size_t)z.n);
  z.o_chunks = o; o += al(sizeof(ChunkRec) * (size_t)z.n_chunk_ub);
  z.o_combs = o; o += al(sizeof(CombRec) * (size_t)std::max(1, z.n_comb_ub));
  z.o_counts = o; o += al(16);
  z.o_partial = o; o += z.n_comb_ub > 0 ? al(4ull * z.n_slot_ub * z.n_tel) : 0;
  z.o_pay = o; o += al(16ull * z.n);
  size_t cube_end = o;
  // psf/lsf region
  z.o_tmp = 0;
  size_t psf_end = al(4ull * z.cube_elems);
  z.psf_region = psf_end;
  // backward region (prep at the same offset as in the cube region)
  o = al(sizeof(PrepRec) * (size_t)z.n);
  z.o_bintab = o; o += al(16ull * (z.n_tel + 1));  // n_tel + 1 bin edges for bin-mean jobs
  z.o_dots = o; o += al(32ull * z.n);
  z.o_ang = o; o += al(24ull * std::max(1, z.n_fin_blocks));
  size_t bwd_end = o;
  z.region = std::max(std::max(sort_end, cube_end), std::max(psf_end, bwd_end));
  return z;
}

// The fused PSF+LSF pass takes PSF radii 1..kFuseR, LSF radii up to kFuseLsfR and y rows
// (nx * n_tel floats) addressed with 32-bit byte offsets.
static bool fused_psf_lsf(const rubix_job &j, const JobSizes &z) {
  return z.psf_r >= 1 && z.psf_r <= kFuseR && z.lsf_r <= kFuseLsfR &&
         (int64_t)j.grid.nx * z.n_tel * 4 < (int64_t(1) << 31);
}

static bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

static int validate_ssp(const rubix_ssp *ssp) {
  if (!ssp) return fail(RUBIX_EINVAL, "ssp is NULL");
  if (ssp->n_age < 2 || ssp->n_age > RUBIX_MAX_AGE_NODES)
    return fail(RUBIX_EINVAL, "ssp.n_age=%d outside [2, %d]", ssp->n_age, RUBIX_MAX_AGE_NODES);
  if (ssp->n_met < 2 || ssp->n_met > RUBIX_MAX_MET_NODES)
    return fail(RUBIX_EINVAL, "ssp.n_met=%d outside [2, %d]", ssp->n_met, RUBIX_MAX_MET_NODES);
  if (!ssp->log_age_nodes || !ssp->met_nodes || !ssp->flux)
    return fail(RUBIX_EINVAL, "ssp node or flux pointer is NULL");
  for (int i = 0; i < ssp->n_age; ++i) {
    if (!isfinite(ssp->log_age_nodes[i]) || (i && !(ssp->log_age_nodes[i] > ssp->log_age_nodes[i - 1])))
      return fail(RUBIX_EINVAL, "ssp.log_age_nodes must be finite and strictly increasing (index %d)", i);
  }
  for (int i = 0; i < ssp->n_met; ++i) {
    if (!isfinite(ssp->met_nodes[i]) || (i && !(ssp->met_nodes[i] > ssp->met_nodes[i - 1])))
      return fail(RUBIX_EINVAL, "ssp.met_nodes must be finite and strictly increasing (index %d)", i);
  }
  if (ssp->lam.n < 2) return fail(RUBIX_EINVAL, "ssp.lam.n=%d < 2", ssp->lam.n);
  if (!finite_pos(ssp->lam.step) || !isfinite(ssp->lam.start))
    return fail(RUBIX_EINVAL, "ssp.lam start/step invalid");
  if (ssp->lam.log_spaced != 0 && ssp->lam.log_spaced != 1)
    return fail(RUBIX_EINVAL, "ssp.lam.log_spaced must be 0 or 1");
  if (ssp->lam.log_spaced && !finite_pos(ssp->lam.start))
    return fail(RUBIX_EINVAL, "a log-spaced SSP grid needs start > 0");
  // the kernels address the template grid through 32-bit byte offsets
  if ((int64_t)ssp->n_age * ssp->n_met * ssp->lam.n >= ((int64_t)1 << 30))
    return fail(RUBIX_ERANGE, "ssp grid has 2^30 or more values (32-bit byte offsets)");
  return RUBIX_OK;
}

static int validate_jobs(const rubix_job *jobs, int n_jobs, Call call) {
  if (!jobs) return fail(RUBIX_EINVAL, "jobs is NULL");
  if (n_jobs < 1 || n_jobs > RUBIX_MAX_JOBS)
    return fail(RUBIX_EINVAL, "n_jobs=%d outside [1, %d]", n_jobs, RUBIX_MAX_JOBS);
  for (int k = 0; k < n_jobs; ++k) {
    const rubix_job &j = jobs[k];
    if (j.p.n < 0) return fail(RUBIX_EINVAL, "job %d: n=%lld < 0", k, (long long)j.p.n);
    if (j.p.n > INT32_MAX) return fail(RUBIX_ERANGE, "job %d: more than 2^31-1 particles", k);
    if (j.grid.nx < 1 || j.grid.ny < 1)
      return fail(RUBIX_EINVAL, "job %d: grid %dx%d is empty", k, j.grid.nx, j.grid.ny);
    if ((int64_t)j.grid.nx * j.grid.ny >= INT32_MAX)
      return fail(RUBIX_ERANGE, "job %d: too many spaxels", k);
    if (!finite_pos(j.grid.spaxel_kpc)) return fail(RUBIX_EINVAL, "job %d: spaxel_kpc must be > 0", k);
    if (j.tel.n < 1) return fail(RUBIX_EINVAL, "job %d: tel.n=%d < 1", k, j.tel.n);
    if (!finite_pos(j.tel.step) || !isfinite(j.tel.start))
      return fail(RUBIX_EINVAL, "job %d: telescope grid start/step invalid", k);
    if (j.tel.log_spaced != 0 && j.tel.log_spaced != 1)
      return fail(RUBIX_EINVAL, "job %d: tel.log_spaced must be 0 or 1", k);
    if (j.tel.log_spaced && !finite_pos(j.tel.start))
      return fail(RUBIX_EINVAL, "job %d: a log-spaced telescope grid needs start > 0", k);
    if (j.resample != 0 && j.resample != 1)
      return fail(RUBIX_EINVAL, "job %d: resample must be 0 or 1", k);
    if (!(j.z_sys > -1.0) || !isfinite(j.z_sys)) return fail(RUBIX_EINVAL, "job %d: z_sys must be > -1", k);
    if (!isfinite(j.flux_scale)) return fail(RUBIX_EINVAL, "job %d: flux_scale not finite", k);
    for (int a = 0; a < 3; ++a)
      if (!isfinite(j.angles_rad[a])) return fail(RUBIX_EINVAL, "job %d: angle %d not finite", k, a);
    if (!(j.psf_sigma_spx >= 0.0) || !(j.lsf_sigma_A >= 0.0) || !isfinite(j.psf_sigma_spx) ||
        !isfinite(j.lsf_sigma_A))
      return fail(RUBIX_EINVAL, "job %d: PSF/LSF sigma must be finite and >= 0", k);
    if (radius_of(j.psf_sigma_spx) > RUBIX_MAX_RADIUS ||
        radius_of(lsf_bins(j)) > RUBIX_MAX_RADIUS)
      return fail(RUBIX_ERANGE, "job %d: PSF/LSF radius exceeds %d", k, RUBIX_MAX_RADIUS);
    if (call == CALL_SIZE) continue;
    const bool need_pos = call == CALL_ROTATE || call == CALL_PACK;
    const bool need_props = call == CALL_CUBE || call == CALL_BWD || call == CALL_PACK;
    const bool need_vel = need_pos || call == CALL_BWD;
    if (j.p.n > 0) {
      if (need_pos && (!j.p.x || !j.p.y || !j.p.z))
        return fail(RUBIX_EINVAL, "job %d: position pointer is NULL", k);
      if (need_vel && (!j.p.vx || !j.p.vy || !j.p.vz))
        return fail(RUBIX_EINVAL, "job %d: velocity pointer is NULL", k);
      if (need_props && (!j.p.mass || !j.p.age || !j.p.met))
        return fail(RUBIX_EINVAL, "job %d: mass/age/met pointer is NULL", k);
    }
    if (call == CALL_ROTATE || call == CALL_CUBE || call == CALL_BWD || call == CALL_PACK) {
      if ((!j.key || !j.perm || !j.vlos) && j.p.n > 0)
        return fail(RUBIX_EINVAL, "job %d: key/perm/vlos pointer is NULL", k);
      if (!j.seg_off) return fail(RUBIX_EINVAL, "job %d: seg_off is NULL", k);
    }
    if ((call == CALL_CUBE || call == CALL_PACK) && !j.cube_raw)
      return fail(RUBIX_EINVAL, "job %d: cube_raw is NULL", k);
    if (call == CALL_PACK && !j.cube) return fail(RUBIX_EINVAL, "job %d: cube is NULL", k);
  }
  return RUBIX_OK;
}

// Every telescope grid must be of the SSP grid's kind (both uniform in lambda or in ln lambda).
static int check_grid_kinds(const rubix_job *jobs, int n_jobs, const rubix_ssp *ssp) {
  for (int k = 0; k < n_jobs; ++k) {
    if (jobs[k].tel.log_spaced != ssp->lam.log_spaced)
      return fail(RUBIX_EINVAL, "job %d: telescope grid %s but SSP grid %s", k,
                  jobs[k].tel.log_spaced ? "log-spaced" : "linear",
                  ssp->lam.log_spaced ? "log-spaced" : "linear");
    // the bin-mean kernel's segment weights on log grids are series in the SSP step
    if (jobs[k].resample == 1 && ssp->lam.log_spaced && !(ssp->lam.step <= 0.05))
      return fail(RUBIX_EINVAL, "job %d: bin-mean resampling on log grids needs an SSP step "
                  "of at most 0.05 in ln(lambda)", k);
  }
  return RUBIX_OK;
}

static size_t workspace_bytes(const rubix_job *jobs, int n_jobs) {
  size_t b = al(table_bytes(n_jobs));
  for (int k = 0; k < n_jobs; ++k) b += al(sizes_of(jobs[k]).region);
  return b;
}

// Table plus the PSF/LSF intermediate cube of every job: all that rubix_psf_lsf's kernels use.
static size_t psf_scratch_bytes(const rubix_job *jobs, int n_jobs) {
  size_t b = al(table_bytes(n_jobs));
  for (int k = 0; k < n_jobs; ++k) b += al(sizes_of(jobs[k]).psf_region);
  return b;
}

static int check_ws(const rubix_job *jobs, int n_jobs, void *ws, size_t ws_bytes) {
  const size_t need = workspace_bytes(jobs, n_jobs);
  if (!ws) return fail(RUBIX_EWORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(RUBIX_EWORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < need) return fail(RUBIX_EWORKSPACE, "workspace of %zu bytes < %zu needed", ws_bytes, need);
  return RUBIX_OK;
}

static int check_ws_regions(const rubix_job *jobs, int n_jobs, void *ws, size_t ws_bytes) {
  const size_t need = workspace_bytes(jobs, n_jobs) - al(table_bytes(n_jobs));
  if (!ws) return fail(RUBIX_EWORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(RUBIX_EWORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < need) return fail(RUBIX_EWORKSPACE, "workspace of %zu bytes < %zu needed", ws_bytes, need);
  return RUBIX_OK;
}

// ---------------------------------------------------------------------------------------------
// table construction
// ---------------------------------------------------------------------------------------------
static void rotation(const double ang[3], double R[9], double dR2[9]) {
#pragma clang fp contract(off)
  const double c1 = cos(ang[0]), s1 = sin(ang[0]);
  const double c2 = cos(ang[1]), s2 = sin(ang[1]);
  const double c3 = cos(ang[2]), s3 = sin(ang[2]);
  // R = Rz(phi3) Ry(phi2) Rx(phi1), each entry written as the closed-form product
  R[0] = c3 * c2;  R[1] = (c3 * s2) * s1 - s3 * c1;  R[2] = (c3 * s2) * c1 + s3 * s1;
  R[3] = s3 * c2;  R[4] = (s3 * s2) * s1 + c3 * c1;  R[5] = (s3 * s2) * c1 - c3 * s1;
  R[6] = -s2;      R[7] = c2 * s1;                   R[8] = c2 * c1;
  // d(row 2)/dphi_k
  dR2[0] = 0.0;  dR2[1] = c2 * c1;  dR2[2] = -c2 * s1;
  dR2[3] = -c2;  dR2[4] = -s2 * s1; dR2[5] = -s2 * c1;
  dR2[6] = 0.0;  dR2[7] = 0.0;      dR2[8] = 0.0;
}

// Normalised sampled Gaussian of radius r at w[kWPad + k + r], k = -r..r; zeros elsewhere.
static void gauss_weights(double sigma, int r, float *w) {
  for (int i = 0; i < kWArray; ++i) w[i] = 0.f;
  if (r == 0) { w[kWPad] = 1.f; return; }
  double tmp[2 * RUBIX_MAX_RADIUS + 1], sum = 0.0;
  for (int k = -r; k <= r; ++k) { tmp[k + r] = exp(-0.5 * (k / sigma) * (k / sigma)); sum += tmp[k + r]; }
  for (int k = 0; k <= 2 * r; ++k) w[kWPad + k] = (float)(tmp[k] / sum);
}

static void fill_ssp(SspDev &S, const rubix_ssp *ssp) {
  memset(&S, 0, sizeof S);
  if (!ssp) return;
  S.flux = ssp->flux;
  S.n_age = ssp->n_age; S.n_met = ssp->n_met; S.n_lam = ssp->lam.n;
  S.lam_start = ssp->lam.start; S.lam_step = ssp->lam.step;
  S.log_lambda = ssp->lam.log_spaced;
  for (int i = 0; i < ssp->n_age; ++i) {
    S.log_age[i] = (double)ssp->log_age_nodes[i];
    S.age_thr[i] = pow(10.0, S.log_age[i]);
  }
  for (int i = 0; i < ssp->n_met; ++i) S.met[i] = (double)ssp->met_nodes[i];
}

struct PslfIO { const float *const *in; float *const *out; };
struct BwdIO {
  const float *const *grad_raw;
  float *const *d_mass, *const *d_age, *const *d_met, *const *d_vlos, *const *d_vel;
  double *d_angles;
};

// Builds the table (host bytes) for `jobs` with per-job workspace regions placed after the table
// region of `ws`. Per-call I/O (PSF/LSF in/out, backward buffers) is optional.
static std::vector<uint8_t> build_table(const rubix_job *jobs, int n_jobs, const rubix_ssp *ssp,
                                        void *ws, const PslfIO *pl, const BwdIO *bw,
                                        bool table_in_ws = true, bool psf_only = false) {
  std::vector<uint8_t> buf(table_bytes(n_jobs), 0);
  Table *t = reinterpret_cast<Table *>(buf.data());
  JobDev *J = reinterpret_cast<JobDev *>(buf.data() + ((sizeof(Table) + 255) & ~size_t(255)));
  t->h.n_jobs = n_jobs;
  fill_ssp(t->h.ssp, ssp);
  // per-job regions follow the table when the table is uploaded to the workspace head
  uint8_t *region = static_cast<uint8_t *>(ws) + (table_in_ws ? al(table_bytes(n_jobs)) : 0);
  int64_t start[NK] = {0};
  int max_passes = 1;
  for (int k = 0; k < n_jobs; ++k) {
    const rubix_job &j = jobs[k];
    const JobSizes z = sizes_of(j);
    JobDev &d = J[k];
    d.x = j.p.x; d.y = j.p.y; d.z = j.p.z; d.vx = j.p.vx; d.vy = j.p.vy; d.vz = j.p.vz;
    d.mass = j.p.mass; d.age = j.p.age; d.met = j.p.met;
    d.n = (int32_t)z.n; d.nx = j.grid.nx; d.ny = j.grid.ny; d.n_s = (int32_t)z.n_s;
    rotation(j.angles_rad, d.R, d.dR2);
    d.spaxel = j.grid.spaxel_kpc;
    d.half_nx = j.grid.nx / 2.0; d.half_ny = j.grid.ny / 2.0;
    d.tel_start = j.tel.start; d.tel_step = j.tel.step; d.z_sys = j.z_sys; d.flux_scale = j.flux_scale;
    d.lsf_sigma_bins = z.lsf_sigma_bins; d.psf_sigma = j.psf_sigma_spx;
    d.lsf_r = z.lsf_r; d.psf_r = z.psf_r;
    gauss_weights(z.lsf_sigma_bins, z.lsf_r, d.lsf_w);
    gauss_weights(j.psf_sigma_spx, z.psf_r, d.psf_w);
    d.n_tel = (int32_t)z.n_tel; d.passes = z.passes; d.n_sort_tiles = z.n_sort_tiles; d.n_tiles = z.n_tiles;
    d.log_lambda = j.tel.log_spaced;
    d.resample = j.resample;
    d.n_tiles_b = z.n_tiles_b;
    d.bin_scale = (ssp && !j.tel.log_spaced) ? ssp->lam.step / j.tel.step : 1.0;
    if (ssp && j.tel.log_spaced) {
      // node index of bin j at rest: q_off + j q_ratio (exact when the two grids coincide)
      d.q_off = ((log(j.tel.start) - log(ssp->lam.start)) - log1p(j.z_sys)) / ssp->lam.step;
      d.q_ratio = j.tel.step / ssp->lam.step;
      d.bin_slope = d.q_ratio;
    } else {
      d.bin_slope = ssp ? j.tel.step / ((1.0 + j.z_sys) * ssp->lam.step) : 1.0;
    }
    d.inv_opz = 1.0 / (1.0 + j.z_sys);
    d.inv_ds = ssp ? 1.0 / ssp->lam.step : 1.0;
    {
      // fixed-point rest index: Q_j = Q_0 + j r exactly as the FP64 form groups it for bin 0,
      // the slope r per bin; 40 fraction bits keep j r within 2e-9 node over 2^22 bins
      double q0, r;
      if (ssp && j.tel.log_spaced) { q0 = d.q_off; r = d.q_ratio; }
      else if (ssp) { q0 = (j.tel.start * d.inv_opz - ssp->lam.start) * d.inv_ds;
                      r = j.tel.step * d.inv_opz * d.inv_ds; }
      else { q0 = 0.0; r = 0.0; }
      d.q0x = (int64_t)llround(q0 * 1099511627776.0);
      d.qrx = (int64_t)llround(r * 1099511627776.0);
    }
    // a telescope grid coarser than the SSP grid needs node windows wider than a wave; such jobs
    // gather their two taps per corner directly from the template grid
    d.cube_direct = d.bin_slope > 1.0 ? 1 : 0;
    d.n_chunk_ub = z.n_chunk_ub; d.n_comb_ub = z.n_comb_ub;
    d.n_psf_tiles = z.n_psf_tiles; d.n_psf_seg_y = z.n_psf_seg_y; d.n_psf_seg_x = z.n_psf_seg_x;
    d.n_fin_blocks = z.n_fin_blocks;
    d.key = j.key; d.perm = j.perm; d.seg_off = j.seg_off; d.vlos = j.vlos; d.cube_raw = j.cube_raw;
    d.cube_elems = z.cube_elems;
    max_passes = std::max(max_passes, z.passes);
    // workspace
    d.kbuf[0] = reinterpret_cast<uint32_t *>(region + z.o_k0);
    d.kbuf[1] = reinterpret_cast<uint32_t *>(region + z.o_k1);
    d.vbuf[0] = reinterpret_cast<uint32_t *>(region + z.o_v0);
    d.vbuf[1] = reinterpret_cast<uint32_t *>(region + z.o_v1);
    d.hist = reinterpret_cast<uint32_t *>(region + z.o_hist);
    d.dtot = reinterpret_cast<uint32_t *>(region + z.o_dtot);
    d.prep = reinterpret_cast<PrepRec *>(region + z.o_prep);
    d.chunks = reinterpret_cast<ChunkRec *>(region + z.o_chunks);
    d.combs = reinterpret_cast<CombRec *>(region + z.o_combs);
    d.counts = reinterpret_cast<int32_t *>(region + z.o_counts);
    d.partial = reinterpret_cast<float *>(region + z.o_partial);
    d.pay = reinterpret_cast<float4 *>(region + z.o_pay);
    d.tmp_cube = reinterpret_cast<float *>(region + z.o_tmp);
    d.bintab = reinterpret_cast<float4 *>(region + z.o_bintab);
    d.dots = reinterpret_cast<double *>(region + z.o_dots);
    d.ang_part = reinterpret_cast<double *>(region + z.o_ang);
    region += al(psf_only ? z.psf_region : z.region);
    // PSF/LSF routing: one fused pass where the radii and the row size allow it, else a lambda
    // pass, a y pass and an x pass, the last active one writing `out`
    int64_t n_lsf = 0, n_psfy = 0, n_psfx = 0, n_copy = 0, n_fuse = 0;
    if (pl && fused_psf_lsf(j, z)) {
      d.fuse_src = pl->in[k];
      d.fuse_dst = pl->out[k];
      n_fuse = cdiv(z.n_tel, kFuseL) * cdiv(j.grid.nx, kFuseX);
    } else if (pl) {
      const float *in = pl->in[k];
      float *out = pl->out[k];
      const bool L = z.lsf_r > 0, P = z.psf_r > 0;
      const int n_pass = (L ? 1 : 0) + (P ? 2 : 0);
      // destinations alternate between out and tmp so that the final pass lands in out
      float *bufs[2] = {out, d.tmp_cube};
      int which = (n_pass % 2 == 1) ? 0 : 1;   // first destination
      const float *cur = in;
      const bool act[3] = {L, P, P};
      for (int q = 0; q < 3; ++q) {
        if (!act[q]) continue;
        d.pl_src[q] = cur;
        d.pl_dst[q] = bufs[which];
        cur = bufs[which];
        which ^= 1;
      }
      if (L) n_lsf = z.n_s * cdiv(z.n_tel, kLsfOut);
      if (P) {
        n_psfy = (int64_t)j.grid.nx * z.n_psf_seg_y * z.n_psf_tiles;
        n_psfx = (int64_t)j.grid.ny * z.n_psf_seg_x * z.n_psf_tiles;
      }
      if (n_pass == 0 && in != out) {
        d.copy_src = in; d.copy_dst = out;
        n_copy = cdiv(z.cube_elems, 65536);
      }
    }
    if (bw) {
      d.grad_raw = bw->grad_raw[k];
      d.d_mass = bw->d_mass[k]; d.d_age = bw->d_age[k]; d.d_met = bw->d_met[k];
      d.d_vlos = bw->d_vlos[k]; d.d_vel = bw->d_vel ? bw->d_vel[k] : nullptr;
      d.d_angles = bw->d_angles + 3 * k;
    }
    const int64_t cnt[NK] = {
        /*K_ROT*/ z.n_sort_tiles,
        /*K_SCAN*/ z.n > 0 ? 256 : 0,
        /*K_SEG*/ cdiv(z.n_s + 1, 256),
        /*K_PREP*/ cdiv(z.n, kPrepBlock),
        /*K_CHUNK*/ 1,
        /*K_CUBE*/ j.resample ? 0 : (int64_t)z.n_tiles * z.n_chunk_ub,
        /*K_COMB*/ (int64_t)z.n_tiles * z.n_comb_ub,
        /*K_LSF*/ n_lsf,
        /*K_PSFY*/ n_psfy,
        /*K_PSFX*/ n_psfx,
        /*K_COPY*/ n_copy,
        /*K_FUSE*/ n_fuse,
        /*K_BINTAB*/ j.resample ? cdiv(z.n_tel + 1, 256) : 0,
        /*K_BWD*/ j.resample ? 0 : cdiv(z.n, kBwdParticles),
        /*K_FIN*/ z.n_fin_blocks,
        /*K_ANG*/ 1,
        /*K_VB*/ cdiv(z.n, kVbParticles),
        /*K_CUBEB*/ j.resample ? (int64_t)z.n_tiles_b * z.n_chunk_ub : 0,
        /*K_BWDB*/ j.resample ? cdiv(z.n, kBwdParticles) : 0,
    };
    for (int q = 0; q < NK; ++q) {
      d.vb_start[q] = start[q];
      start[q] += cnt[q];
    }
  }
  for (int q = 0; q < NK; ++q) t->h.total[q] = start[q];
  t->h.max_passes = max_passes;
  for (int k = 0; k < n_jobs; ++k) {
    t->h.max_psf_r = std::max(t->h.max_psf_r, J[k].psf_r);
    t->h.max_lsf_r = std::max(t->h.max_lsf_r, J[k].lsf_r);
  }
  return buf;
}

static int device_status(hipError_t e, const char *what) {
  if (e == hipSuccess) return RUBIX_OK;
  return fail(RUBIX_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

using Launcher = hipError_t (*)(const Table *, const TableHeader &, int, hipStream_t);

static int run(const std::vector<uint8_t> &tab, void *ws, hipStream_t s, Launcher fn,
               const char *what) {
  hipError_t e = launch_upload(tab.data(), tab.size(), ws, s);
  if (e != hipSuccess) return device_status(e, "job table upload");
  const Table *host = reinterpret_cast<const Table *>(tab.data());
  e = fn(static_cast<const Table *>(ws), host->h, 0, s);
  return device_status(e, what);
}

static int validate_psf_io(const rubix_job *jobs, int n_jobs, const float *const *in,
                           float *const *out) {
  int rc;
  if ((rc = validate_jobs(jobs, n_jobs, CALL_PSF))) return rc;
  if (!in || !out) return fail(RUBIX_EINVAL, "in/out arrays are NULL");
  for (int k = 0; k < n_jobs; ++k) {
    if (!in[k] || !out[k]) return fail(RUBIX_EINVAL, "job %d: in/out cube is NULL", k);
    const int64_t bytes = (int64_t)jobs[k].grid.nx * jobs[k].grid.ny * jobs[k].tel.n * 4;
    const char *a = reinterpret_cast<const char *>(in[k]);
    const char *b = reinterpret_cast<const char *>(out[k]);
    if (a < b + bytes && b < a + bytes) return fail(RUBIX_EINVAL, "job %d: in and out overlap", k);
  }
  return RUBIX_OK;
}

// Scratch of the allocation-free entry point: the job table and the PSF/LSF intermediate cubes,
// in a file-scope device array that every GPU the library runs on holds until the process ends.
// In host code `scratch` names a host-side stand-in, never the device memory: the device address
// comes from hipGetSymbolAddress, taken once per device with that device current, and only that
// address is handed to kernels. Calls that overlap on one GPU share the array and race.
static __device__ __align__(256) uint8_t scratch[RUBIX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices];

static int scratch_on_current_device(void **ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_status(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(RUBIX_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return device_status(e, "hipGetSymbolAddress(scratch)");
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255))
      return fail(RUBIX_EDEVICE, "scratch symbol address unusable");
    g_scratch_dev[dev] = p;
  }
  *ptr = g_scratch_dev[dev];
  return RUBIX_OK;
}

}  // namespace rubix

using namespace rubix;

extern "C" {

const char *rubix_last_error(void) { return g_err.c_str(); }

const char *rubix_version(void) { return "rubix-mi355x 0.1.0 (gfx950)"; }

int rubix_workspace_size(const rubix_job *jobs, int n_jobs, const rubix_ssp *ssp, size_t *bytes) {
  g_err.clear();
  if (!bytes) return fail(RUBIX_EINVAL, "bytes is NULL");
  int rc = validate_jobs(jobs, n_jobs, CALL_SIZE);
  if (rc) return rc;
  if (ssp && (rc = validate_ssp(ssp))) return rc;
  if (ssp && (rc = check_grid_kinds(jobs, n_jobs, ssp))) return rc;
  *bytes = workspace_bytes(jobs, n_jobs);
  return RUBIX_OK;
}

int rubix_rotate_bin(const rubix_job *jobs, int n_jobs, void *ws, size_t ws_bytes, void *stream) {
  g_err.clear();
  int rc;
  if ((rc = validate_jobs(jobs, n_jobs, CALL_ROTATE))) return rc;
  if ((rc = check_ws(jobs, n_jobs, ws, ws_bytes))) return rc;
  auto tab = build_table(jobs, n_jobs, nullptr, ws, nullptr, nullptr);
  return run(tab, ws, static_cast<hipStream_t>(stream), launch_rotate_bin, "rubix_rotate_bin");
}

int rubix_cube(const rubix_job *jobs, int n_jobs, const rubix_ssp *ssp, void *ws, size_t ws_bytes,
               void *stream) {
  g_err.clear();
  int rc;
  if ((rc = validate_jobs(jobs, n_jobs, CALL_CUBE))) return rc;
  if ((rc = validate_ssp(ssp))) return rc;
  if ((rc = check_grid_kinds(jobs, n_jobs, ssp))) return rc;
  if ((rc = check_ws(jobs, n_jobs, ws, ws_bytes))) return rc;
  auto tab = build_table(jobs, n_jobs, ssp, ws, nullptr, nullptr);
  if (!g_timer_on) return run(tab, ws, static_cast<hipStream_t>(stream), launch_cube, "rubix_cube");
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e != hipSuccess) {
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    return device_status(e, "cube timer events");
  }
  t_cube_events[0] = ev[0];
  t_cube_events[1] = ev[1];
  rc = run(tab, ws, static_cast<hipStream_t>(stream), launch_cube, "rubix_cube");
  t_cube_events[0] = t_cube_events[1] = nullptr;
  g_timer_ev.push_back({ev[0], ev[1]});
  return rc;
}

int rubix_cube_timer(int enable) {
  g_err.clear();
  g_timer_on = enable != 0;
  return RUBIX_OK;
}

int rubix_cube_timer_read(double *total_ms, int *count) {
  g_err.clear();
  if (!total_ms || !count) return fail(RUBIX_EINVAL, "total_ms/count is NULL");
  double sum = 0.0;
  hipError_t e = hipSuccess;
  for (auto &p : g_timer_ev) {
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventSynchronize(p.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
    sum += ms;
  }
  *count = (int)g_timer_ev.size();
  *total_ms = sum;
  for (auto &p : g_timer_ev) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  g_timer_ev.clear();
  return device_status(e, "cube timer read");
}

int rubix_psf_lsf(const rubix_job *jobs, int n_jobs, const float *const *in, float *const *out,
                  void *ws, size_t ws_bytes, void *stream) {
  g_err.clear();
  int rc;
  if ((rc = validate_psf_io(jobs, n_jobs, in, out))) return rc;
  if ((rc = check_ws(jobs, n_jobs, ws, ws_bytes))) return rc;
  PslfIO io{in, out};
  auto tab = build_table(jobs, n_jobs, nullptr, ws, &io, nullptr);
  return run(tab, ws, static_cast<hipStream_t>(stream), launch_psf_lsf, "rubix_psf_lsf");
}

int rubix_psf_lsf_noalloc(const rubix_job *jobs, int n_jobs, const float *const *in,
                          float *const *out, void *stream) {
  g_err.clear();
  int rc;
  if ((rc = validate_psf_io(jobs, n_jobs, in, out))) return rc;
  const size_t need = psf_scratch_bytes(jobs, n_jobs);
  if (need > (size_t)RUBIX_NOALLOC_SCRATCH_BYTES)
    return fail(RUBIX_ERANGE, "rubix_psf_lsf_noalloc: the batch needs %zu bytes of scratch "
                "(job table and intermediate cubes) > the static %d", need,
                RUBIX_NOALLOC_SCRATCH_BYTES);
  void *ws = nullptr;
  if ((rc = scratch_on_current_device(&ws))) return rc;
  PslfIO io{in, out};
  auto tab = build_table(jobs, n_jobs, nullptr, ws, &io, nullptr, true, /*psf_only=*/true);
  return run(tab, ws, static_cast<hipStream_t>(stream), launch_psf_lsf, "rubix_psf_lsf_noalloc");
}

int rubix_cube_backward(const rubix_job *jobs, int n_jobs, const rubix_ssp *ssp,
                        const float *const *grad_raw, float *const *d_mass, float *const *d_age,
                        float *const *d_met, float *const *d_vlos, float *const *d_vel,
                        double *d_angles, void *ws, size_t ws_bytes, void *stream) {
  g_err.clear();
  int rc;
  if ((rc = validate_jobs(jobs, n_jobs, CALL_BWD))) return rc;
  if ((rc = validate_ssp(ssp))) return rc;
  if ((rc = check_grid_kinds(jobs, n_jobs, ssp))) return rc;
  if (!grad_raw || !d_mass || !d_age || !d_met || !d_vlos || !d_angles)
    return fail(RUBIX_EINVAL, "gradient array argument is NULL");
  for (int k = 0; k < n_jobs; ++k) {
    if (!grad_raw[k]) return fail(RUBIX_EINVAL, "job %d: grad_raw is NULL", k);
    if (jobs[k].p.n > 0 && (!d_mass[k] || !d_age[k] || !d_met[k] || !d_vlos[k]))
      return fail(RUBIX_EINVAL, "job %d: a gradient output is NULL", k);
  }
  if ((rc = check_ws(jobs, n_jobs, ws, ws_bytes))) return rc;
  BwdIO io{grad_raw, d_mass, d_age, d_met, d_vlos, d_vel, d_angles};
  auto tab = build_table(jobs, n_jobs, ssp, ws, nullptr, &io);
  return run(tab, ws, static_cast<hipStream_t>(stream), launch_backward, "rubix_cube_backward");
}

int rubix_add_noise(const rubix_job *jobs, int n_jobs, const rubix_noise *noise,
                    float *const *cubes, void *stream) {
  g_err.clear();
  if (!jobs || !noise || !cubes) return fail(RUBIX_EINVAL, "jobs/noise/cubes is NULL");
  if (n_jobs < 1 || n_jobs > RUBIX_MAX_JOBS)
    return fail(RUBIX_EINVAL, "n_jobs=%d outside [1, %d]", n_jobs, RUBIX_MAX_JOBS);
  for (int k = 0; k < n_jobs; ++k) {
    const rubix_noise &p = noise[k];
    if (!cubes[k]) return fail(RUBIX_EINVAL, "job %d: cube is NULL", k);
    if (jobs[k].grid.nx < 1 || jobs[k].grid.ny < 1 || jobs[k].tel.n < 1)
      return fail(RUBIX_EINVAL, "job %d: empty cube shape", k);
    if (!(p.gain >= 0.0) || !isfinite(p.gain) || !(p.sigma_floor >= 0.0) || !isfinite(p.sigma_floor))
      return fail(RUBIX_EINVAL, "job %d: gain and sigma_floor must be finite and >= 0", k);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int k = 0; k < n_jobs; ++k) {
    const int64_t n = (int64_t)jobs[k].grid.nx * jobs[k].grid.ny * jobs[k].tel.n;
    hipError_t e = launch_noise(cubes[k], n, noise[k].seed, noise[k].stream, noise[k].gain,
                                noise[k].sigma_floor, s);
    if (e != hipSuccess) return device_status(e, "rubix_add_noise");
  }
  return RUBIX_OK;
}

size_t rubix_table_bytes(int n_jobs) {
  if (n_jobs < 1 || n_jobs > RUBIX_MAX_JOBS) return 0;
  return al(table_bytes(n_jobs));
}

int rubix_forward_pack(const rubix_job *jobs, int n_jobs, const rubix_ssp *ssp, void *ws,
                       size_t ws_bytes, void *host_table, size_t host_table_bytes,
                       int max_psf_radius, int max_sort_passes) {
  g_err.clear();
  int rc;
  if ((rc = validate_jobs(jobs, n_jobs, CALL_PACK))) return rc;
  if ((rc = validate_ssp(ssp))) return rc;
  if ((rc = check_grid_kinds(jobs, n_jobs, ssp))) return rc;
  if ((rc = check_ws_regions(jobs, n_jobs, ws, ws_bytes))) return rc;
  if (!host_table) return fail(RUBIX_EINVAL, "host_table is NULL");
  if (host_table_bytes < al(table_bytes(n_jobs)))
    return fail(RUBIX_EINVAL, "host_table of %zu bytes < %zu needed", host_table_bytes,
                al(table_bytes(n_jobs)));
  std::vector<const float *> in(n_jobs);
  std::vector<float *> out(n_jobs);
  for (int k = 0; k < n_jobs; ++k) { in[k] = jobs[k].cube_raw; out[k] = jobs[k].cube; }
  PslfIO io{in.data(), out.data()};
  auto tab = build_table(jobs, n_jobs, ssp, ws, &io, nullptr, /*table_in_ws=*/false);
  const Table *t = reinterpret_cast<const Table *>(tab.data());
  if (t->h.max_psf_r > max_psf_radius || t->h.max_lsf_r > RUBIX_MAX_RADIUS)
    return fail(RUBIX_ERANGE, "a job's PSF radius %d exceeds the packed launch's %d",
                t->h.max_psf_r, max_psf_radius);
  if (t->h.max_passes > max_sort_passes)
    return fail(RUBIX_ERANGE, "a job needs %d sort passes, the packed launch runs %d",
                t->h.max_passes, max_sort_passes);
  memcpy(host_table, tab.data(), tab.size());
  return RUBIX_OK;
}

int rubix_forward_packed(const void *dev_table, int grid_blocks, int max_psf_radius,
                         int max_sort_passes, void *stream) {
  g_err.clear();
  if (!dev_table) return fail(RUBIX_EINVAL, "dev_table is NULL");
  if (grid_blocks < 1) return fail(RUBIX_EINVAL, "grid_blocks=%d < 1", grid_blocks);
  if (max_psf_radius < 0 || max_psf_radius > RUBIX_MAX_RADIUS)
    return fail(RUBIX_EINVAL, "max_psf_radius=%d outside [0, %d]", max_psf_radius, RUBIX_MAX_RADIUS);
  if (max_sort_passes < 1 || max_sort_passes > 4)
    return fail(RUBIX_EINVAL, "max_sort_passes=%d outside [1, 4]", max_sort_passes);
  // launch shapes that do not depend on the table: every kind gets grid_blocks blocks and walks
  // the totals it reads from the device table
  TableHeader h;
  memset(&h, 0, sizeof h);
  for (int q = 0; q < NK; ++q) h.total[q] = grid_blocks;
  h.ssp.log_lambda = -1;       // grid kind known only to the device table
  h.max_passes = max_sort_passes;
  h.max_psf_r = max_psf_radius;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Table *dt = static_cast<const Table *>(dev_table);
  hipError_t e = launch_rotate_bin(dt, h, grid_blocks, s);
  if (e == hipSuccess) e = launch_cube(dt, h, grid_blocks, s);
  if (e == hipSuccess) e = launch_psf_lsf(dt, h, grid_blocks, s);
  return device_status(e, "rubix_forward_packed");
}

struct rubix_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipGraphNode_t> nodes;      // kernel nodes, in no particular order
  std::vector<hipKernelNodeParams> params;
  std::vector<int> kinds;                 // work-item kind that sets each node's grid
  const void *dev_table = nullptr;
  int max_jobs = 0, max_psf_r = 0, max_passes = 0;
};

static void graph_free(rubix_graph g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

int rubix_graph_create(const void *dev_table, int max_jobs, int max_psf_radius,
                       int max_sort_passes, rubix_graph *out) {
  g_err.clear();
  if (!out) return fail(RUBIX_EINVAL, "out is NULL");
  *out = nullptr;
  if (!dev_table) return fail(RUBIX_EINVAL, "dev_table is NULL");
  if (reinterpret_cast<uintptr_t>(dev_table) & 255)
    return fail(RUBIX_EINVAL, "dev_table not 256-byte aligned");
  if (max_jobs < 1 || max_jobs > RUBIX_MAX_JOBS)
    return fail(RUBIX_EINVAL, "max_jobs=%d outside [1, %d]", max_jobs, RUBIX_MAX_JOBS);
  if (max_psf_radius < 0 || max_psf_radius > RUBIX_MAX_RADIUS)
    return fail(RUBIX_EINVAL, "max_psf_radius=%d outside [0, %d]", max_psf_radius, RUBIX_MAX_RADIUS);
  if (max_sort_passes < 1 || max_sort_passes > 4)
    return fail(RUBIX_EINVAL, "max_sort_passes=%d outside [1, 4]", max_sort_passes);
  rubix_graph g = new rubix_graph_s;
  g->dev_table = dev_table;
  g->max_jobs = max_jobs;
  g->max_psf_r = max_psf_radius;
  g->max_passes = max_sort_passes;
  // capture every forward kernel once with a one-block grid on a private stream
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) { graph_free(g); return device_status(e, "capture stream"); }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    TableHeader h;
    memset(&h, 0, sizeof h);
    for (int q = 0; q < NK; ++q) h.total[q] = 1;
    h.ssp.log_lambda = -1;     // grid kind known only to the device table
    h.max_passes = max_sort_passes;
    h.max_psf_r = max_psf_radius;
    const Table *dt = static_cast<const Table *>(dev_table);
    hipError_t el = launch_rotate_bin(dt, h, 0, cs);
    if (el == hipSuccess) el = launch_cube(dt, h, 0, cs);
    if (el == hipSuccess) el = launch_psf_lsf(dt, h, 0, cs);
    e = hipStreamEndCapture(cs, &g->graph);
    if (el != hipSuccess) e = el;
  }
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) { graph_free(g); return device_status(e, "forward graph capture"); }
  size_t n = 0;
  e = hipGraphGetNodes(g->graph, nullptr, &n);
  std::vector<hipGraphNode_t> all(n);
  if (e == hipSuccess && n) e = hipGraphGetNodes(g->graph, all.data(), &n);
  if (e != hipSuccess) { graph_free(g); return device_status(e, "graph nodes"); }
  for (hipGraphNode_t nd : all) {
    hipGraphNodeType ty;
    if ((e = hipGraphNodeGetType(nd, &ty)) != hipSuccess) break;
    if (ty != hipGraphNodeTypeKernel) {
      graph_free(g);
      return fail(RUBIX_EDEVICE, "forward graph holds a node of type %d (kernels only)", (int)ty);
    }
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof kp);
    if ((e = hipGraphKernelNodeGetParams(nd, &kp)) != hipSuccess) break;
    int kind = rotate_bin_kernel_kind(kp.func);
    if (kind < 0) kind = cube_kernel_kind(kp.func);
    if (kind < 0) kind = psf_lsf_kernel_kind(kp.func);
    if (kind < 0) {
      graph_free(g);
      return fail(RUBIX_EDEVICE, "forward graph holds an unknown kernel");
    }
    g->nodes.push_back(nd);
    g->params.push_back(kp);
    g->kinds.push_back(kind);
  }
  if (e != hipSuccess) { graph_free(g); return device_status(e, "graph kernel nodes"); }
  // rotate/bin: rotate (with the first pass's histograms), a histogram for every later pass,
  // scan and scatter per pass, segment offsets; cube: chunks, bounds, cell-ordered
  // prep, the bin-centre sum, the bin-mean sum's two instances (linear and log grids), combine;
  // PSF/LSF: the three 1-D passes, the copy and the fused pass
  const size_t expect = 3u * max_sort_passes + 1 + 7 + 5;
  if (g->nodes.size() != expect) {
    const size_t got = g->nodes.size();
    graph_free(g);
    return fail(RUBIX_EDEVICE, "forward graph holds %zu kernels, expected %zu", got, expect);
  }
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) { graph_free(g); return device_status(e, "graph instantiation"); }
  *out = g;
  return RUBIX_OK;
}

int rubix_graph_launch(rubix_graph g, const void *host_table, size_t host_table_bytes,
                       void *stream) {
  g_err.clear();
  if (!g || !g->exec) return fail(RUBIX_EINVAL, "graph is NULL");
  if (!host_table) return fail(RUBIX_EINVAL, "host_table is NULL");
  if (host_table_bytes < sizeof(Table)) return fail(RUBIX_EINVAL, "host_table too small");
  const Table *t = static_cast<const Table *>(host_table);
  const int nj = t->h.n_jobs;
  if (nj < 1 || nj > g->max_jobs)
    return fail(RUBIX_EINVAL, "table holds %d jobs; the graph takes 1..%d", nj, g->max_jobs);
  const size_t tb = table_bytes(nj);
  if (host_table_bytes < tb)
    return fail(RUBIX_EINVAL, "host_table of %zu bytes < %zu", host_table_bytes, tb);
  if (t->h.max_passes > g->max_passes || t->h.max_psf_r > g->max_psf_r)
    return fail(RUBIX_ERANGE, "table needs %d sort passes and PSF radius %d; the graph has %d, %d",
                t->h.max_passes, t->h.max_psf_r, g->max_passes, g->max_psf_r);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(const_cast<void *>(g->dev_table), host_table, tb,
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return device_status(e, "table copy");
  for (size_t i = 0; i < g->nodes.size(); ++i) {
    hipKernelNodeParams kp = g->params[i];
    const int64_t tot = t->h.total[g->kinds[i]];
    kp.gridDim = dim3((unsigned)std::min<int64_t>(std::max<int64_t>(tot, 1), 0x7fffffff));
    e = hipGraphExecKernelNodeSetParams(g->exec, g->nodes[i], &kp);
    if (e != hipSuccess) return device_status(e, "graph grid update");
  }
  return device_status(hipGraphLaunch(g->exec, s), "graph launch");
}

int rubix_graph_destroy(rubix_graph g) {
  g_err.clear();
  graph_free(g);
  return RUBIX_OK;
}

}  // extern "C"
