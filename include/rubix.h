/*
 * rubix.h -- C ABI of the MI355X (gfx950) IFU datacube forward model.
 *
 * The operations follow the pipeline of arXiv:2412.08265, Sec. 3 ("RUBIX Codebase"): orient the
 * galaxy, assign particles to spaxels, look up SSP spectra, Doppler-shift them by the line-of-sight
 * velocity, resample to the telescope wavelength grid, sum per spaxel, convolve with a PSF and an
 * LSF (Gaussian, Sec. 4 "Qualitative Analysis"); plus the gradient of a cube loss with respect to
 * the particle properties and viewing angles (Abstract and Sec. 1: gradients through the whole
 * pipeline). The paper fixes no formula; the conventions taken are stated per entry point.
 *
 * Conventions shared by every entry point
 *  - Pointers marked DEVICE are HIP device pointers owned by the caller; HOST pointers are read
 *    during the call only. The library allocates nothing and keeps no state between calls.
 *  - Every call runs asynchronously on `stream` (a hipStream_t; NULL = the null stream) and returns
 *    once its kernels are enqueued. Device faults surface at the caller's next synchronisation.
 *  - Every call takes an array of `n_jobs` job descriptors (1 <= n_jobs <= RUBIX_MAX_JOBS) and
 *    processes all of them in the same launches; a single galaxy is a batch of one. Each job's
 *    results depend only on that job's inputs (bitwise identical alone or in a batch).
 *  - `ws` is a caller-owned DEVICE workspace of at least rubix_workspace_size() bytes, 256-byte
 *    aligned. Its contents need not survive between calls. Concurrent calls need distinct
 *    workspaces.
 *  - Return value: RUBIX_OK (0) or a negative status; rubix_last_error() then returns a message
 *    (thread-local, valid until the next call on the same thread). Host-visible arguments are
 *    validated before any launch. Device data is not inspected, and no value of it makes a
 *    kernel access memory out of range: a particle whose rotated position is not finite falls
 *    outside the field (key nx*ny); one whose line-of-sight velocity is not finite contributes
 *    nothing to the cube; a NaN age or [M/H] takes the first node of its axis (infinities clamp
 *    to the matching end); a non-finite mass makes the voxels its spectrum reaches non-finite.
 *  - Sizes: particle counts up to 2^31-1 per job; int32 spaxel keys and offsets; SSP grids of
 *    fewer than 2^30 values (their byte offsets are 32-bit), larger ones fail with RUBIX_ERANGE.
 *  - Line-of-sight velocities: a particle whose v_los is not finite adds nothing to the cube in
 *    either resampling mode, and rubix_cube_backward gives it zero gradients and no share of the
 *    angle gradients.
 */
#ifndef RUBIX_H
#define RUBIX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RUBIX_OK          0
#define RUBIX_EINVAL     -1   /* bad argument (null pointer, bad size, non-increasing nodes ...) */
#define RUBIX_EWORKSPACE -2   /* workspace missing, misaligned or too small                      */
#define RUBIX_EDEVICE    -3   /* a HIP call failed; the message carries hipGetErrorString        */
#define RUBIX_ERANGE     -4   /* a size exceeds what the library supports                        */

#define RUBIX_MAX_JOBS       64
#define RUBIX_MAX_AGE_NODES  256
#define RUBIX_MAX_MET_NODES  64
#define RUBIX_MAX_RADIUS     64   /* PSF/LSF kernel radius int(4 sigma + 0.5) must not exceed it */

/* Square spaxels of side `spaxel_kpc` on an nx x ny grid centred on the origin of the rotated
 * frame; spaxel (ix, iy) has key iy*nx + ix; particles outside the grid get key nx*ny. */
typedef struct {
  int32_t nx, ny;
  double  spaxel_kpc;
} rubix_grid;

/* Wavelength grid, k = 0..n-1, step > 0:
 *   log_spaced = 0: value k is start + k*step [Angstrom] (uniform in lambda);
 *   log_spaced = 1: value k is start * exp(k*step), start > 0 [Angstrom], step in ln(lambda)
 *                   (uniform in ln lambda: a Doppler shift is then a constant index shift).
 * The SSP grid and every telescope grid used with it must be of the same kind. */
typedef struct {
  double  start;
  double  step;
  int32_t n;
  int32_t log_spaced;
} rubix_lgrid;

/* SSP template library (the paper's "simple stellar population (SSP) library", Sec. 3).
 * flux[ia][iz][k]: template of age node ia and metallicity node iz at wavelength node k, FP32,
 * wavelength contiguous. Age nodes are log10(age / Gyr); metallicity nodes are [M/H] in dex; both
 * strictly increasing, n_age, n_met >= 2. lam.n >= 2. */
typedef struct {
  int32_t      n_age, n_met;
  const float *log_age_nodes;   /* HOST  [n_age] */
  const float *met_nodes;       /* HOST  [n_met] */
  rubix_lgrid  lam;
  const float *flux;            /* DEVICE [n_age][n_met][lam.n] */
} rubix_ssp;

/* Star particles, structure of arrays, FP32, all DEVICE [n]. */
typedef struct {
  int64_t      n;
  const float *x, *y, *z;       /* kpc */
  const float *vx, *vy, *vz;    /* km/s */
  const float *mass;            /* Msun */
  const float *age;             /* Gyr, > 0 */
  const float *met;             /* [M/H] = log10(Z/Zsun), dex */
} rubix_particles;

/* One galaxy observation. Outputs are DEVICE buffers owned by the caller; a call writes only the
 * outputs it documents and reads the ones an earlier call produced. */
typedef struct {
  rubix_particles p;
  double      angles_rad[3];    /* phi1 about x (inclination), phi2 about y, phi3 about z      */
  rubix_grid  grid;
  rubix_lgrid tel;              /* telescope bin centres, tel.n >= 1                            */
  double      z_sys;            /* systemic redshift (> -1); 0 for a galaxy at rest            */
  double      flux_scale;       /* overall flux factor (e.g. distance dimming); 1 by default   */
  double      psf_sigma_spx;    /* Gaussian PSF sigma in spaxels; 0 = none                     */
  double      lsf_sigma_A;      /* Gaussian LSF sigma in Angstrom; 0 = none. On a log-spaced
                                   telescope grid it is converted to bins at the grid's central
                                   wavelength start*exp(step*(n-1)/2) and held constant in bins
                                   (a constant velocity width)                                   */
  int32_t    *key;              /* [n]           written by rubix_rotate_bin                   */
  int32_t    *perm;             /* [n]           written by rubix_rotate_bin                   */
  int32_t    *seg_off;          /* [nx*ny + 1]   written by rubix_rotate_bin                   */
  float      *vlos;             /* [n]           written by rubix_rotate_bin                   */
  float      *cube_raw;         /* [ny][nx][tel.n] written by rubix_cube                       */
  float      *cube;             /* [ny][nx][tel.n] optional; rubix_psf_lsf may write it        */
  int32_t     resample;         /* 0: bin-centre sampling (below); 1: bin mean (flux conserving;
                                   on log grids the SSP step must be <= 0.05)                   */
  int32_t     reserved;         /* 0                                                            */
} rubix_job;

/* Bytes of workspace that every entry point below needs for these jobs (the maximum over all
 * entry points, so one workspace serves a whole forward + backward sequence).
 * Returns RUBIX_OK and sets *bytes, or an error for invalid jobs / SSP. */
int rubix_workspace_size(const rubix_job *jobs, int n_jobs, const rubix_ssp *ssp,
                         size_t *bytes);

/* Steps 1-2 of Sec. 3: orientation and spaxel assignment.
 *  - R = Rz(phi3) Ry(phi2) Rx(phi1) (column vectors), entries from the C library's cos/sin;
 *    x' = ((R00 x + R01 y) + R02 z), y' likewise, in FP64 without fused multiply-add.
 *  - key[i] = iy*nx + ix with ix = floor(x'/s + nx/2), iy = floor(y'/s + ny/2) when
 *    0 <= ix < nx and 0 <= iy < ny (half-open cells), else nx*ny.
 *  - vlos[i] = ((R20 vx + R21 vy) + R22 vz) in FP64, rounded to FP32; positive = receding.
 *  - perm = stable ascending sort of the indices by key (equal keys keep input order; the
 *    out-of-field sentinel sorts last); seg_off[s] = number of particles with key < s,
 *    s = 0..nx*ny, so spaxel s owns sorted positions [seg_off[s], seg_off[s+1]).
 * key, perm, seg_off are exact integers (bit-reproducible). */
int rubix_rotate_bin(const rubix_job *jobs, int n_jobs, void *ws, size_t ws_bytes,
                     void *stream);

/* Steps 3-6 of Sec. 3: SSP lookup, Doppler shift, resampling, spaxel sum. Reads perm, seg_off
 * and vlos from rubix_rotate_bin and writes cube_raw (every voxel; empty spaxels get 0).
 *  - SSP lookup: bilinear in (u_a = log10(age/Gyr), u_z = [M/H]), clamped to the node range.
 *    The age cell is chosen by comparing age with the node ages 10^node (FP64); the fraction in
 *    the cell is linear in u_a. The metallicity cell compares [M/H] with the nodes directly.
 *  - Doppler + resampling: f_i(lam_j) = flux_scale m_i J_i Slin_i(q_ij) with
 *    q_ij = (lam_j / ((1+z_sys)(1+beta_i)) - lam0_ssp) / dlam_ssp, beta_i = vlos_i / c,
 *    J_i = 1/((1+z_sys)(1+beta_i)) (flux-density Jacobian), Slin the linear interpolant of the
 *    bilinear SSP spectrum between wavelength nodes, 0 for q < 0 or q > n-1 (resample = 0; on
 *    log-spaced grids q_ij = Q_j - ln(1+beta_i)/dln_ssp).
 *    resample = 1 (linear grids): the mean of the observed flux density over bin j,
 *    f_i(j) = flux_scale m_i (dlam_ssp / tel.step) * integral of Slin_i over the rest-frame node
 *    interval [q_ij(lam_j - step/2), q_ij(lam_j + step/2)] (exact for the piecewise-linear
 *    spectrum; the sum over bins conserves the flux of any shift inside the band).
 *    resample = 1 (log grids): the same mean over bin j = [ln lam_j - step/2, ln lam_j + step/2],
 *    f_i(j) = flux_scale m_i / dlam_j * integral of Slin_i over rest wavelength between the bin's
 *    rest-frame edges, Slin linear in the log-grid index, dlam_j = 2 lam_j sinh(step/2) (each
 *    segment's exponential weight evaluated by a four-term series, so the SSP step must be at
 *    most 0.05).
 *  - cube_raw[s][j] = sum of f_i(lam_j) over the particles of spaxel s, FP32, accumulated per
 *    work item in a fixed order (deterministic; independent of the other jobs in the batch). */
int rubix_cube(const rubix_job *jobs, int n_jobs, const rubix_ssp *ssp, void *ws,
               size_t ws_bytes, void *stream);

/* Step 7 of Sec. 3: LSF then PSF, out[j] = A in[j] for each job j (in[j], out[j] DEVICE cubes of
 * that job's shape, not overlapping). Separable sampled Gaussians exp(-k^2/(2 sigma^2)),
 * |k| <= int(4 sigma + 0.5), normalised to unit sum, zero padding outside the cube: along lambda
 * with sigma = lsf_sigma_A / tel.step bins (log grids: see rubix_job.lsf_sigma_A), then along y
 * and along x with sigma = psf_sigma_spx.
 * sigma = 0 skips that axis. The operator is symmetric, so the same call applies its adjoint. */
int rubix_psf_lsf(const rubix_job *jobs, int n_jobs, const float *const *in, float *const *out,
                  void *ws, size_t ws_bytes, void *stream);

/* Adjoint of rubix_cube (gradients through the pipeline, Abstract / Sec. 1). Given
 * grad_raw[j] = dL/dcube_raw (DEVICE, cube shape), writes per particle, in input order:
 *   d_mass, d_age (per Gyr), d_met (per dex), d_vlos (per km/s)   DEVICE [n] each;
 *   d_vel  (optional, may be NULL)  DEVICE [3][n], dL/dv = d_vlos * R[2][:] (SoA x, y, z);
 *   d_angles DEVICE double [3 * n_jobs], dL/dphi_k = sum_i d_vlos_i (dR/dphi_k v_i)_z with the
 *   spaxel assignment held fixed (binning is piecewise constant).
 * Particles outside the field get 0. Derivatives at SSP nodes / wavelength nodes take the
 * right-hand cell; clamped age or metallicity gives 0 along that axis. Positions get no gradient.
 * Bin-mean jobs (resample = 1): the integrand does not depend on beta, the bin's limits do, so
 * d_vlos is the Leibniz sum over the bin edges of the integrand at the edge times its dq/dbeta
 * (on log grids the integrand is Slin lam dln and dq/dbeta = -1/((1+beta) dln)); an edge
 * clipped to the SSP grid's end (q <= 0 or q >= n-1) contributes nothing.
 * Reads key, perm, seg_off, vlos from rubix_rotate_bin. Per-particle dot products are reduced in
 * FP64 in a fixed order (deterministic). */
int rubix_cube_backward(const rubix_job *jobs, int n_jobs, const rubix_ssp *ssp,
                        const float *const *grad_raw, float *const *d_mass,
                        float *const *d_age, float *const *d_met, float *const *d_vlos,
                        float *const *d_vel, double *d_angles, void *ws, size_t ws_bytes,
                        void *stream);

/* Noise (Sec. 3 ends with realistic noise; the paper gives no model). Reading taken: every voxel
 * v of the cube gets independent Gaussian noise of variance gain * max(C_v, 0) + sigma_floor^2.
 * Voxels v = 4b .. 4b+3 (C order in [ny][nx][tel.n]) take their deviates from one block of
 * Philox-4x32-10 (Salmon et al., SC 2011) keyed by `seed` (low word first) with counter
 * (b_lo, b_hi, stream, 0): its outputs x0..x3 give u = (x + 1/2) 2^-32 and, by Box-Muller in
 * FP64, eps(4b) = r0 cos(2 pi u1), eps(4b+1) = r0 sin(2 pi u1), eps(4b+2) = r1 cos(2 pi u3),
 * eps(4b+3) = r1 sin(2 pi u3), r0 = sqrt(-2 ln u0), r1 = sqrt(-2 ln u2); the noisy value is
 * rounded to FP32 once. It depends only on (seed, stream, v, C_v). */
typedef struct {
  uint64_t seed;
  uint32_t stream;        /* independent sequences for one seed (e.g. one per observation)     */
  uint32_t reserved;      /* 0                                                                  */
  double   gain;          /* noise variance per unit of cube value, >= 0                       */
  double   sigma_floor;   /* standard deviation of the floor, >= 0                             */
} rubix_noise;

/* Adds noise in place to cubes[k] (DEVICE, the shape of jobs[k]) with noise[k] (HOST array of
 * n_jobs). Only the jobs' grid and tel.n are read. No workspace. */
int rubix_add_noise(const rubix_job *jobs, int n_jobs, const rubix_noise *noise,
                    float *const *cubes, void *stream);

/* ---- Allocation-free PSF/LSF ------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, hosts that forbid hipMalloc): rubix_psf_lsf without a workspace argument. The job table
 * and the intermediate cubes live in a static device array of RUBIX_NOALLOC_SCRATCH_BYTES that
 * each GPU the library runs on holds until the process ends; the call allocates nothing and
 * clears nothing (every byte it reads there it has written first). The caller still owns in[k]
 * and out[k]. Fails with RUBIX_ERANGE, before any device work, if the batch needs more scratch
 * than that: the aligned job table plus 4 * nx * ny * tel.n bytes (rounded up to 256) per job.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU (other
 * threads, or other streams not ordered with this one) race; calls ordered on one stream do not.
 * Results equal rubix_psf_lsf's bit for bit. */
#define RUBIX_NOALLOC_SCRATCH_BYTES (64 << 20)
int rubix_psf_lsf_noalloc(const rubix_job *jobs, int n_jobs, const float *const *in,
                          float *const *out, void *stream);

/* ---- Batched forward pass for replayed launches (serving) -----------------------------------
 * The calls above upload their job table through kernel arguments. For a serving loop that
 * replays one captured launch sequence (a HIP graph) for every batch, the table instead lives in
 * a caller-owned device buffer that the caller refreshes before each replay:
 *   1. rubix_forward_pack writes the table for a batch into a host buffer (ideally pinned);
 *   2. the caller copies it to its device table buffer (e.g. hipMemcpyAsync on the stream);
 *   3. rubix_forward_packed launches rotate/bin -> cube -> PSF/LSF (cube_raw -> cube) for every
 *      job of that table. Its launch arguments depend only on (dev_table, grid_blocks,
 *      max_psf_radius, max_sort_passes), never on the table's contents, so the launches can be
 *      captured once and replayed: each kernel runs grid_blocks blocks that stride over the work
 *      items the table describes (block b takes items b, b + grid_blocks, ...; persistent
 *      blocks). The table holds no state the launches consume: copy it before a replay only when
 *      the batch changes.
 * The jobs' workspace regions are laid out inside `ws` (size: rubix_workspace_size minus
 * rubix_table_bytes), which must stay valid until the launches complete. */

/* Bytes of a packed table for n_jobs jobs (0 if n_jobs is out of range). */
size_t rubix_table_bytes(int n_jobs);

/* Validates the jobs (they need positions, velocities, properties and every output, including
 * cube) and writes their table into host_table (>= rubix_table_bytes(n_jobs) bytes). Fails with
 * RUBIX_ERANGE if a job needs a larger PSF radius or more sort passes than the replayed launch
 * will provide. */
int rubix_forward_pack(const rubix_job *jobs, int n_jobs, const rubix_ssp *ssp, void *ws,
                       size_t ws_bytes, void *host_table, size_t host_table_bytes,
                       int max_psf_radius, int max_sort_passes);

/* Enqueues the forward pass of the packed table at dev_table (DEVICE, 256-byte aligned) on
 * `stream`: grid_blocks blocks per kernel (>= 1), LDS sized for max_psf_radius (0..64),
 * max_sort_passes (1..4) radix passes (jobs needing fewer skip the rest). Results are those of
 * rubix_rotate_bin + rubix_cube + rubix_psf_lsf(cube_raw -> cube), bit for bit. */
int rubix_forward_packed(const void *dev_table, int grid_blocks, int max_psf_radius,
                         int max_sort_passes, void *stream);

/* ---- Forward graph (serving) ------------------------------------------------------------------
 * A forward graph holds the whole forward launch sequence (rotate/bin, cube, PSF/LSF with
 * cube_raw -> cube) of packed tables at one device address, captured once as a HIP graph and
 * instantiated. Each launch copies a packed table (rubix_forward_pack) to that address, sets
 * every kernel's grid to the table's work-item count, and launches the graph: the kernels run
 * exactly as in the plain entry points (one block per work item), so results are bitwise those of
 * rubix_rotate_bin + rubix_cube + rubix_psf_lsf, at the host cost of one graph launch.
 * Unlike the rest of this library a graph is state: it owns a HIP graph and its instantiation
 * (host and driver resources; no device memory is allocated) until rubix_graph_destroy. */
typedef struct rubix_graph_s *rubix_graph;

/* Captures and instantiates the forward sequence for tables of up to max_jobs jobs at dev_table
 * (DEVICE, >= rubix_table_bytes(max_jobs) bytes, 256-byte aligned, valid for the graph's life),
 * with LDS for PSF radii up to max_psf_radius (0..64) and max_sort_passes (1..4) radix passes.
 * Capture runs on a private stream and launches nothing. *out = NULL on failure. */
int rubix_graph_create(const void *dev_table, int max_jobs, int max_psf_radius,
                       int max_sort_passes, rubix_graph *out);

/* Enqueues on `stream`: the copy of host_table (written by rubix_forward_pack with the same radius
 * and pass limits; pinned host memory makes the copy asynchronous; it must stay unchanged until
 * the copy has run) to the graph's dev_table, then the graph with grids from that table. The
 * jobs' buffers and the workspace named in the table must stay valid until the graph completes.
 * The graph's previous launch must have completed before the next call (its grids are updated
 * in place). */
int rubix_graph_launch(rubix_graph g, const void *host_table, size_t host_table_bytes,
                       void *stream);

/* Releases the graph (NULL is ignored). Its launches must have completed. */
int rubix_graph_destroy(rubix_graph g);

/* ---- Measurement aid -------------------------------------------------------------------------
 * rubix_cube_timer(1) makes the following rubix_cube calls on this thread record a HIP event pair
 * on their stream right before and right after the cube-summation kernels (the step that sums
 * the resampled spectra, bin-centre and bin-mean jobs; rubix_cube also runs short preparation
 * and combine kernels around it).
 * rubix_cube_timer(0) stops recording. rubix_cube_timer_read waits for every pair recorded since
 * the last read, returns their summed elapsed time in ms and their count, and releases them.
 * The pairs are library state (HIP events), held until read. Graph launches are never timed. */
int rubix_cube_timer(int enable);
int rubix_cube_timer_read(double *total_ms, int *count);

/* Message for the last non-zero status returned on this thread ("" if none). */
const char *rubix_last_error(void);

/* Version string of the library build. */
const char *rubix_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RUBIX_H */
