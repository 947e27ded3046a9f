"""Plain, slow, FP64 CPU oracle of the IFU datacube forward model (arXiv:2412.08265).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's CPU-baseline
leg, never by the product path. It shares no code with the HIP library (no kernels, headers,
helpers, tables or constants); it reads the same FP32 input arrays (promoted to FP64).

The paper describes the method in one paragraph of Sec. 3 ("RUBIX Codebase"): orient the galaxy in
the field of view, assign particles to IFU spaxels, look each star's spectrum up in an SSP library,
Doppler-shift it by the line-of-sight velocity (and galaxy distance), resample it to the telescope
wavelength grid, sum the spectra per spaxel, then convolve with a PSF and an LSF (Gaussian, Sec. 4
"Qualitative Analysis"). Gradients through the whole pipeline are the paper's second claim
(Abstract, Sec. 1). The paper gives no formula for any step; the readings this oracle takes where
it is silent are stated at each function and collected in the design notes of the repository.

Conventions (all readings):
  * rotation R = Rz(phi3) Ry(phi2) Rx(phi1), column vectors; phi1 is the inclination;
  * line of sight = rotated +z, v_los = (R v)_z, positive = receding = redshift;
  * spaxel index ix = floor(x'/s + nx/2) (grid centred on the origin, half-open cells);
  * SSP lookup = bilinear interpolation in (log10 age/Gyr, [M/H]), clamped to the node range;
  * Doppler: a rest-frame wavelength lam_r is observed at lam_r (1+z_sys)(1+v_los/c); the observed
    flux density is f_obs(lam) = J f_rest(lam / ((1+z_sys)(1+beta))), J = 1/((1+z_sys)(1+beta));
  * resampling = linear interpolation of the shifted spectrum at telescope bin centres, zero outside
    the SSP wavelength range;
  * PSF / LSF = sampled, normalised Gaussians truncated at radius int(4 sigma + 0.5), zero padding;
  * loss (differentiation workload) = 0.5 || A C_raw - T* ||^2 with A = PSF o LSF.
"""
from __future__ import annotations

import math
import os
from typing import Dict, Optional, Sequence

import numpy as np

C_KMS = 299792.458  # km/s

__all__ = [
    "C_KMS", "rotation_matrix", "rotation_matrix_derivs", "rotate_positions", "los_velocity",
    "spaxel_keys", "sort_by_key", "ssp_cell", "ssp_weights", "interp_templates",
    "rest_index", "doppler_index", "doppler_index_dbeta", "node_cell", "node_ties",
    "one_sided_cells", "cell_linear", "resample_linear", "particle_spectra_bounds",
    "integral_linear", "linear_at", "bin_edge_indices", "bin_edge_indices_log",
    "integral_log_weighted", "particle_spectra", "cube_raw", "gaussian_weights",
    "convolve_axis", "psf_lsf", "forward", "loss", "loss_grad_cube", "adjoint",
    "OracleConfig", "config_from_workload", "ForkedPool",
]


# --------------------------------------------------------------------------------------------------
# configuration
# --------------------------------------------------------------------------------------------------
class OracleConfig:
    """Plain container of the run's hyper-parameters (the paper's JSON configuration, Sec. 3)."""

    def __init__(self, angles_rad, nx, ny, spaxel_kpc, tel_start, tel_step, n_tel,
                 log_age_nodes, met_nodes, ssp_lam_start, ssp_lam_step, ssp_flux,
                 psf_sigma_spx=0.0, lsf_sigma_A=0.0, z_sys=0.0, flux_scale=1.0,
                 log_lambda=False, resample=0):
        self.angles_rad = tuple(float(a) for a in angles_rad)
        self.nx, self.ny = int(nx), int(ny)
        self.spaxel_kpc = float(spaxel_kpc)
        self.tel_start, self.tel_step, self.n_tel = float(tel_start), float(tel_step), int(n_tel)
        self.log_age_nodes = np.asarray(log_age_nodes, dtype=np.float64)
        self.met_nodes = np.asarray(met_nodes, dtype=np.float64)
        self.ssp_lam_start, self.ssp_lam_step = float(ssp_lam_start), float(ssp_lam_step)
        self.ssp_flux = np.asarray(ssp_flux, dtype=np.float64)
        self.psf_sigma_spx = float(psf_sigma_spx)
        self.lsf_sigma_A = float(lsf_sigma_A)
        self.z_sys = float(z_sys)
        self.flux_scale = float(flux_scale)
        # both wavelength grids uniform in ln(lambda): value k is start * exp(k * step)
        self.log_lambda = bool(log_lambda)
        # resampling reading: 0 = the shifted spectrum sampled at bin centres (linear
        # interpolation); 1 = its average over each telescope bin (flux conserving)
        self.resample = int(resample)
        if self.resample not in (0, 1):
            raise ValueError("resample must be 0 or 1")

    @property
    def n_spaxels(self):
        return self.nx * self.ny

    def tel_lambda(self):
        k = np.arange(self.n_tel, dtype=np.float64)
        if self.log_lambda:
            return self.tel_start * np.exp(self.tel_step * k)
        return self.tel_start + self.tel_step * k

    def ssp_lambda(self):
        k = np.arange(self.ssp_flux.shape[2], dtype=np.float64)
        if self.log_lambda:
            return self.ssp_lam_start * np.exp(self.ssp_lam_step * k)
        return self.ssp_lam_start + self.ssp_lam_step * k

    def lsf_sigma_bins(self):
        """LSF width in telescope bins. On a log grid a bin is lambda * step wide; the width is
        taken at the grid's central wavelength and held constant in bins (a constant velocity
        width), so the LSF stays one fixed kernel."""
        if self.log_lambda:
            lam_c = self.tel_start * math.exp(self.tel_step * (self.n_tel - 1) / 2.0)
            return self.lsf_sigma_A / (lam_c * self.tel_step)
        return self.lsf_sigma_A / self.tel_step


def config_from_workload(w) -> OracleConfig:
    """Adapter from a synthetic workload description (plain attribute access only)."""
    s = w.ssp
    return OracleConfig(w.angles_rad, w.nx, w.ny, w.spaxel_kpc, w.tel_start, w.tel_step, w.n_tel,
                        s.log_age_nodes, s.met_nodes, s.lam_start, s.lam_step, s.flux,
                        w.psf_sigma_spx, w.lsf_sigma_A, w.z_sys, w.flux_scale,
                        getattr(w, "log_lambda", False), getattr(w, "resample", 0))


def _p64(p, name):
    return np.asarray(getattr(p, name), dtype=np.float64)


# --------------------------------------------------------------------------------------------------
# step 1: orientation (Sec. 3, "orientate the galaxy in the field of view")
# --------------------------------------------------------------------------------------------------
def rotation_matrix(phi1: float, phi2: float, phi3: float) -> np.ndarray:
    """R = Rz(phi3) @ Ry(phi2) @ Rx(phi1), entries written out as the closed-form product.

    cos/sin come from the C math library through Python's `math` module. The closed form fixes
    the floating-point grouping of each entry, so any other implementation that writes the same
    products reaches the same doubles.
    """
    c1, s1 = math.cos(phi1), math.sin(phi1)
    c2, s2 = math.cos(phi2), math.sin(phi2)
    c3, s3 = math.cos(phi3), math.sin(phi3)
    return np.array([
        [c3 * c2, (c3 * s2) * s1 - s3 * c1, (c3 * s2) * c1 + s3 * s1],
        [s3 * c2, (s3 * s2) * s1 + c3 * c1, (s3 * s2) * c1 - c3 * s1],
        [-s2, c2 * s1, c2 * c1],
    ], dtype=np.float64)


def rotation_matrix_derivs(phi1: float, phi2: float, phi3: float) -> np.ndarray:
    """dR/dphi_k for k = 0, 1, 2 (array [3, 3, 3]), from the same closed form."""
    c1, s1 = math.cos(phi1), math.sin(phi1)
    c2, s2 = math.cos(phi2), math.sin(phi2)
    c3, s3 = math.cos(phi3), math.sin(phi3)
    d1 = np.array([
        [0.0, c3 * s2 * c1 + s3 * s1, -c3 * s2 * s1 + s3 * c1],
        [0.0, s3 * s2 * c1 - c3 * s1, -s3 * s2 * s1 - c3 * c1],
        [0.0, c2 * c1, -c2 * s1],
    ])
    d2 = np.array([
        [-c3 * s2, c3 * c2 * s1, c3 * c2 * c1],
        [-s3 * s2, s3 * c2 * s1, s3 * c2 * c1],
        [-c2, -s2 * s1, -s2 * c1],
    ])
    d3 = np.array([
        [-s3 * c2, -s3 * s2 * s1 - c3 * c1, -s3 * s2 * c1 + c3 * s1],
        [c3 * c2, c3 * s2 * s1 - s3 * c1, c3 * s2 * c1 + s3 * s1],
        [0.0, 0.0, 0.0],
    ])
    return np.stack([d1, d2, d3])


def rotate_positions(p, R: np.ndarray):
    """x' = R x in FP64, each component summed left to right without fused multiply-add:
    x'_a = ((R[a,0] x + R[a,1] y) + R[a,2] z)."""
    x, y, z = _p64(p, "x"), _p64(p, "y"), _p64(p, "z")
    xp = R[0, 0] * x + R[0, 1] * y + R[0, 2] * z
    yp = R[1, 0] * x + R[1, 1] * y + R[1, 2] * z
    zp = R[2, 0] * x + R[2, 1] * y + R[2, 2] * z
    return xp, yp, zp


def los_velocity(p, R: np.ndarray) -> np.ndarray:
    """v_los = (R v)_z in km/s (positive = receding)."""
    vx, vy, vz = _p64(p, "vx"), _p64(p, "vy"), _p64(p, "vz")
    return R[2, 0] * vx + R[2, 1] * vy + R[2, 2] * vz


# --------------------------------------------------------------------------------------------------
# step 2: spaxel assignment (Sec. 3, "particles are assigned to the IFU spaxels")
# --------------------------------------------------------------------------------------------------
def spaxel_keys(xp: np.ndarray, yp: np.ndarray, nx: int, ny: int, spaxel: float) -> np.ndarray:
    """Nearest-grid-point binning on an nx x ny grid of square spaxels of side `spaxel` centred on
    the origin. ix = floor(x'/s + nx/2), iy likewise; in the field iff 0 <= ix < nx and
    0 <= iy < ny (half-open: a particle exactly on the upper border is outside).
    key = iy*nx + ix for particles in the field, nx*ny (the sentinel) otherwise."""
    tx = xp / spaxel + nx / 2.0
    ty = yp / spaxel + ny / 2.0
    ix = np.floor(tx)
    iy = np.floor(ty)
    inside = (ix >= 0) & (ix < nx) & (iy >= 0) & (iy < ny)
    key = np.full(xp.shape, nx * ny, dtype=np.int64)
    key[inside] = iy[inside].astype(np.int64) * nx + ix[inside].astype(np.int64)
    return key


def sort_by_key(key: np.ndarray, n_spaxels: int):
    """perm = stable argsort of the keys (equal keys keep input order, the sentinel sorts last);
    seg_off[s] = number of particles with key < s, for s = 0..n_spaxels."""
    perm = np.argsort(key, kind="stable")
    seg_off = np.searchsorted(key[perm], np.arange(n_spaxels + 1), side="left")
    return perm.astype(np.int64), seg_off.astype(np.int64)


# --------------------------------------------------------------------------------------------------
# step 3: SSP lookup (Sec. 3, "lookup from a simple stellar population library")
# --------------------------------------------------------------------------------------------------
def ssp_cell(u: np.ndarray, nodes: np.ndarray, x: Optional[np.ndarray] = None,
             thr: Optional[np.ndarray] = None):
    """Cell index j and fraction t of u on strictly increasing nodes, clamped to the node range.

    The cell is decided by comparing x with thresholds thr (by default x = u, thr = nodes):
    j = largest k in [0, n-2] with thr[k] <= x; x <= thr[0] gives (j=0, t=0) and x >= thr[-1]
    gives (j=n-2, t=1). Inside the range t = (u - nodes[j]) / (nodes[j+1] - nodes[j]), clipped to
    [0, 1]. Also returns the mask of values inside [thr[0], thr[-1]] (not clamped)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = u if x is None else x
    thr = nodes if thr is None else np.asarray(thr, dtype=np.float64)
    n = nodes.shape[0]
    j = np.clip(np.searchsorted(thr, x, side="right") - 1, 0, n - 2)
    t = np.clip((u - nodes[j]) / (nodes[j + 1] - nodes[j]), 0.0, 1.0)
    t = np.where(x <= thr[0], 0.0, np.where(x >= thr[-1], 1.0, t))
    inside = (x >= thr[0]) & (x <= thr[-1])
    return j, t, inside


def ssp_weights(age: np.ndarray, met: np.ndarray, log_age_nodes, met_nodes):
    """Bilinear weights on the (log10 age/Gyr, [M/H]) grid. Corner order:
    (ja, jz), (ja, jz+1), (ja+1, jz), (ja+1, jz+1). Returns ja, jz, ta, tz, w[n, 4] and masks.

    The age cell is found by comparing the age with the node ages 10^node (FP64), the fraction
    is linear in log10(age); the [M/H] cell compares [M/H] with its nodes directly."""
    age = np.asarray(age, dtype=np.float64)
    la = np.asarray(log_age_nodes, dtype=np.float64)
    ua = np.log10(age)
    uz = np.asarray(met, dtype=np.float64)
    ja, ta, ina = ssp_cell(ua, la, x=age, thr=10.0 ** la)
    jz, tz, inz = ssp_cell(uz, np.asarray(met_nodes, dtype=np.float64))
    w = np.stack([(1 - ta) * (1 - tz), (1 - ta) * tz, ta * (1 - tz), ta * tz], axis=-1)
    return ja, jz, ta, tz, w, ina, inz


def interp_templates(flux: np.ndarray, ja, jz, w) -> np.ndarray:
    """S_i = sum over the 4 corners of w_ic * T[corner_c], shape [n, n_lam_ssp]."""
    return (w[:, 0:1] * flux[ja, jz] + w[:, 1:2] * flux[ja, jz + 1]
            + w[:, 2:3] * flux[ja + 1, jz] + w[:, 3:4] * flux[ja + 1, jz + 1])


# --------------------------------------------------------------------------------------------------
# steps 4-5: Doppler shift and resampling (Sec. 3)
# --------------------------------------------------------------------------------------------------
def rest_index(cfg: OracleConfig) -> np.ndarray:
    """SSP node index of each telescope bin centre for a source at rest in the galaxy frame (beta
    = 0), FP64: Q_j = (lam_j/(1+z_sys) - lam0_ssp)/dlam_ssp on linear grids; on log grids
    Q_j = off + j * ratio with off = (ln lam0_tel - ln lam0_ssp - ln(1+z_sys))/dln_ssp and
    ratio = dln_tel/dln_ssp (this grouping is exact when the two grids coincide)."""
    j = np.arange(cfg.n_tel, dtype=np.float64)
    if cfg.log_lambda:
        off = ((math.log(cfg.tel_start) - math.log(cfg.ssp_lam_start)) - math.log1p(cfg.z_sys)) \
            / cfg.ssp_lam_step
        return off + j * (cfg.tel_step / cfg.ssp_lam_step)
    return (cfg.tel_lambda() / (1.0 + cfg.z_sys) - cfg.ssp_lam_start) / cfg.ssp_lam_step


def doppler_index(cfg: OracleConfig, vlos: np.ndarray) -> np.ndarray:
    """Fractional SSP node index of the rest-frame wavelength seen at each telescope bin centre,
    shape [n, n_tel]: the rest wavelength is lam_j / ((1+z_sys)(1+beta_i)), so
    q_ij = (lam_j / ((1+z_sys)(1+beta_i)) - lam0_ssp) / dlam_ssp on linear grids and
    q_ij = Q_j - ln(1+beta_i) / dln_ssp on log grids (a Doppler shift is a constant shift of the
    log-grid index)."""
    beta = np.asarray(vlos, dtype=np.float64) / C_KMS
    if cfg.log_lambda:
        return rest_index(cfg)[None, :] - np.log1p(beta)[:, None] / cfg.ssp_lam_step
    lam_rest = cfg.tel_lambda()[None, :] / ((1.0 + cfg.z_sys) * (1.0 + beta[:, None]))
    return (lam_rest - cfg.ssp_lam_start) / cfg.ssp_lam_step


def doppler_index_dbeta(cfg: OracleConfig, vlos: np.ndarray) -> np.ndarray:
    """dq_ij/dbeta_i: -lam_j/((1+z)(1+beta)^2 dlam) on linear grids, -1/((1+beta) dln) on log
    grids; shape [n, n_tel] (broadcast)."""
    beta = np.asarray(vlos, dtype=np.float64) / C_KMS
    if cfg.log_lambda:
        return np.broadcast_to(-1.0 / ((1.0 + beta[:, None]) * cfg.ssp_lam_step),
                               (beta.shape[0], cfg.n_tel))
    return -cfg.tel_lambda()[None, :] / ((1.0 + cfg.z_sys) * (1.0 + beta[:, None]) ** 2
                                         * cfg.ssp_lam_step)


def node_cell(q: np.ndarray, n_nodes: int):
    """The node interval [k, k+1] holding q and whether q lies on the SSP grid, in FP64:
    valid iff 0 <= q <= n-1, k = floor(q) with the last node mapped to (k = n-2, tau = 1)."""
    valid = (q >= 0.0) & (q <= n_nodes - 1)
    k = np.minimum(np.floor(np.where(valid, q, 0.0)), n_nodes - 2).astype(np.int64)
    return k, valid


def node_ties(q: np.ndarray, d: np.ndarray, n_nodes: int, ties):
    """Pairs whose node interval is decided by rounding, for a method that computes q with an
    absolute error of at most eps = eps_abs + eps_rel |d| (`ties` = (eps_abs, eps_rel); d is the
    Doppler part of q, its change from the particle at rest). Such a method may put a q within eps
    of a node r in [0, n-1] on either side of r: in the interval left of r (r-1, which is off the
    grid for r = 0) or right of it (r, off the grid for r = n-1). Returns the mask and r.

    At an interior node the interpolated value is continuous, so only its slope (the adjoint)
    depends on the side; at the two ends of the SSP range the value itself does (in the band or
    zero). Every one-sided result is a correct result there (several correct results)."""
    eps_abs, eps_rel = ties
    r = np.rint(np.where(np.isfinite(q), q, -2.0))
    eps = eps_abs + eps_rel * np.abs(np.where(np.isfinite(d), d, 0.0))
    tie = (np.abs(q - r) <= eps) & (r >= 0) & (r <= n_nodes - 1)
    return tie, r.astype(np.int64)


def one_sided_cells(q: np.ndarray, d: np.ndarray, n_nodes: int, ties):
    """The FP64 cell (node_cell) and, for the pairs tied at a node r (node_ties), the cell left of
    r (r-1) and the cell right of r (r), each on the grid iff it lies in [0, n-2]; untied pairs
    keep the FP64 cell on both sides. Returns (k, valid), (k_left, valid_left),
    (k_right, valid_right) and the tie mask. The FP64 cell of a tied pair is one of the two."""
    k, valid = node_cell(q, n_nodes)
    tie, r = node_ties(q, d, n_nodes, ties)
    left = (np.where(tie, r - 1, k), np.where(tie, r >= 1, valid))
    right = (np.where(tie, r, k), np.where(tie, r <= n_nodes - 2, valid))
    return (k, valid), left, right, tie


def cell_linear(S: np.ndarray, q: np.ndarray, k: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """The linear function of node interval [k, k+1] of row i of S evaluated at q (tau = q - k),
    zero where the interval is off the grid (valid false)."""
    kk = np.where(valid, k, 0)
    tau = np.where(valid, q - kk, 0.0)
    s0 = np.take_along_axis(S, kk, axis=1)
    s1 = np.take_along_axis(S, kk + 1, axis=1)
    return np.where(valid, (1.0 - tau) * s0 + tau * s1, 0.0)


def resample_linear(S: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Piecewise-linear interpolation of row i of S at fractional node positions q[i, :];
    zero where q < 0 or q > n-1. The last node maps to (k = n-2, tau = 1)."""
    return cell_linear(S, q, *node_cell(q, S.shape[1]))


def integral_linear(S: np.ndarray, q_lo: np.ndarray, q_hi: np.ndarray) -> np.ndarray:
    """Integral of the piecewise-linear interpolant of row i of S (in node-index units) over
    [q_lo[i, j], q_hi[i, j]], with the interpolant zero outside [0, n-1]; FP64. Uses the exact
    antiderivative: F(q) = C_k + S_k t + (S_{k+1} - S_k) t^2 / 2 on segment k (t = q - k), C_k
    the trapezoid sum of segments 0..k-1, q clipped to [0, n-1]."""
    n = S.shape[1]
    C = np.zeros_like(S)
    C[:, 1:] = np.cumsum(0.5 * (S[:, :-1] + S[:, 1:]), axis=1)

    def F(q):
        q = np.clip(q, 0.0, n - 1.0)
        k = np.minimum(np.floor(q), n - 2).astype(np.int64)
        t = q - k
        s0 = np.take_along_axis(S, k, axis=1)
        s1 = np.take_along_axis(S, k + 1, axis=1)
        return np.take_along_axis(C, k, axis=1) + s0 * t + (s1 - s0) * t * t / 2.0

    return F(q_hi) - F(q_lo)


def bin_edge_indices(cfg: OracleConfig, vlos: np.ndarray):
    """Rest-frame SSP node index of the lower and upper edge of every telescope bin (centre
    lam_j, width dlam), shape [n, n_tel] each; linear grids."""
    beta = np.asarray(vlos, dtype=np.float64) / C_KMS
    f = (1.0 + cfg.z_sys) * (1.0 + beta[:, None])
    lam = cfg.tel_lambda()[None, :]
    lo = ((lam - 0.5 * cfg.tel_step) / f - cfg.ssp_lam_start) / cfg.ssp_lam_step
    hi = ((lam + 0.5 * cfg.tel_step) / f - cfg.ssp_lam_start) / cfg.ssp_lam_step
    return lo, hi


def bin_edge_indices_log(cfg: OracleConfig, vlos: np.ndarray):
    """Log grids: rest-frame SSP node index of the lower and upper edge of every telescope bin,
    shape [n, n_tel] each. Bin j spans ln lam in [ln lam_j - dln/2, ln lam_j + dln/2] (uniform in
    ln lam, centred on lam_j); an edge's rest index is
    (ln lam_edge - ln(1+z) - ln(1+beta) - ln lam0_ssp) / dln_ssp."""
    beta = np.asarray(vlos, dtype=np.float64) / C_KMS
    j = np.arange(cfg.n_tel, dtype=np.float64)[None, :]
    base = (math.log(cfg.tel_start) - math.log1p(cfg.z_sys) - math.log(cfg.ssp_lam_start))
    shift = np.log1p(beta)[:, None]
    lo = (base + (j - 0.5) * cfg.tel_step - shift) / cfg.ssp_lam_step
    hi = (base + (j + 0.5) * cfg.tel_step - shift) / cfg.ssp_lam_step
    return lo, hi


def integral_log_weighted(S: np.ndarray, q_lo: np.ndarray, q_hi: np.ndarray, lam0: float,
                          dln: float) -> np.ndarray:
    """Log grids: integral over rest wavelength of the spectrum whose value is linear in the node
    index between nodes (row i of S), over the rest-frame index interval [q_lo, q_hi] clipped to
    [0, n-1] (zero outside), FP64. With lam(q) = lam0 exp(q dln), dlam = lam dln dq, and on segment
    k (t = q - k) the integrand (S_k + t d_k) lam0 e^{k dln} e^{t dln} dln, whose antiderivative in
    t is lam0 e^{k dln} (S_k + t d_k - d_k/dln) e^{t dln}."""
    n = S.shape[1]
    k_all = np.arange(n - 1, dtype=np.float64)
    d = S[:, 1:] - S[:, :-1]
    lamk = lam0 * np.exp(k_all * dln)                     # rest wavelength of node k

    def G(k, t):
        # antiderivative on segment k at fraction t, per row (k, t arrays of the row's shape)
        sk = np.take_along_axis(S, k, axis=1)
        dk = np.take_along_axis(d, k, axis=1)
        return lamk[k] * (sk + t * dk - dk / dln) * np.exp(t * dln)

    # whole segments: G_k(1) - G_k(0), summed from node 0
    full = lamk[None, :] * ((S[:, :-1] + d - d / dln) * math.exp(dln) - (S[:, :-1] - d / dln))
    C = np.zeros((S.shape[0], n))
    C[:, 1:] = np.cumsum(full, axis=1)

    def F(q):
        q = np.clip(q, 0.0, n - 1.0)
        k = np.minimum(np.floor(q), n - 2).astype(np.int64)
        t = q - k
        zero = np.zeros_like(t)
        return np.take_along_axis(C, k, axis=1) + G(k, t) - G(k, zero)

    return F(q_hi) - F(q_lo)


def particle_spectra(p, idx: np.ndarray, vlos: np.ndarray, cfg: OracleConfig) -> np.ndarray:
    """Observed spectrum of each particle in `idx` on the telescope grid, shape [len(idx), n_tel].

    resample 0: f_i(lam_j) = flux_scale m_i J_i Slin_i(q_ij), J_i = 1/((1+z_sys)(1+beta_i)).
    resample 1: the mean of the observed flux density over bin j,
      f_i(j) = (1/dlam) int_{bin j} flux_scale m_i J_i Slin_i(q(lam)) dlam
             = flux_scale m_i (dlam_ssp / dlam) int_{q_lo}^{q_hi} Slin_i(q) dq
    (the substitution lam -> q cancels J); summed over bins this conserves the flux exactly.
    On log grids the same mean, with the spectrum linear in the log-grid index: f_i(j) =
    (flux_scale m_i / dlam_j) x the integral of Slin_i over the rest wavelength between the bin's
    edges (integral_log_weighted), dlam_j the bin's width in wavelength."""
    age = _p64(p, "age")[idx]
    met = _p64(p, "met")[idx]
    mass = _p64(p, "mass")[idx]
    v = vlos[idx]
    ja, jz, ta, tz, w, _, _ = ssp_weights(age, met, cfg.log_age_nodes, cfg.met_nodes)
    S = interp_templates(cfg.ssp_flux, ja, jz, w)
    if cfg.resample == 1 and cfg.log_lambda:
        # the mean of the observed flux density over bin j, of width
        # dlam_j = lam_j (e^{dln/2} - e^{-dln/2}): the substitution of the rest wavelength cancels
        # J, leaving (flux_scale m / dlam_j) x the integral of Slin over the rest wavelength
        q_lo, q_hi = bin_edge_indices_log(cfg, v)
        width = cfg.tel_lambda() * (2.0 * math.sinh(0.5 * cfg.tel_step))
        return ((cfg.flux_scale * mass)[:, None] / width[None, :]) * integral_log_weighted(
            S, q_lo, q_hi, cfg.ssp_lam_start, cfg.ssp_lam_step)
    if cfg.resample == 1:
        q_lo, q_hi = bin_edge_indices(cfg, v)
        scale = cfg.flux_scale * mass * (cfg.ssp_lam_step / cfg.tel_step)
        return scale[:, None] * integral_linear(S, q_lo, q_hi)
    q = doppler_index(cfg, v)
    J = 1.0 / ((1.0 + cfg.z_sys) * (1.0 + v / C_KMS))
    return (cfg.flux_scale * mass * J)[:, None] * resample_linear(S, q)


def particle_spectra_bounds(p, idx: np.ndarray, vlos: np.ndarray, cfg: OracleConfig, ties):
    """particle_spectra together with the range of its correct results where the node interval
    is decided by rounding (node_ties with `ties` = (eps_abs, eps_rel)): returns f, lo, hi and the
    number of tied (particle, bin) pairs, lo/hi the smaller/larger of the two one-sided values
    (equal to f elsewhere). Only bin-centre sampling has such pairs that matter: the bin mean is an
    integral, continuous in its edges' positions, so there lo = hi = f."""
    f = particle_spectra(p, idx, vlos, cfg)
    if cfg.resample == 1:
        return f, f, f, 0
    v = vlos[idx]
    q = doppler_index(cfg, v)
    n = cfg.ssp_flux.shape[2]
    tie, r = node_ties(q, q - rest_index(cfg)[None, :], n, ties)
    ti, tj = np.nonzero(tie)
    if ti.size == 0:
        return f, f, f, 0
    # the one-sided values at the tied pairs only (the cells left and right of node r)
    sub = np.asarray(idx)[ti]
    age, met = _p64(p, "age")[sub], _p64(p, "met")[sub]
    ja, jz, _, _, w, _, _ = ssp_weights(age, met, cfg.log_age_nodes, cfg.met_nodes)
    S = interp_templates(cfg.ssp_flux, ja, jz, w)          # one row per tied pair
    qt, rt = q[ti, tj][:, None], r[ti, tj][:, None]
    J = 1.0 / ((1.0 + cfg.z_sys) * (1.0 + v[ti] / C_KMS))
    scale = cfg.flux_scale * _p64(p, "mass")[sub] * J
    fl = scale * cell_linear(S, qt, rt - 1, rt >= 1)[:, 0]
    fr = scale * cell_linear(S, qt, rt, rt <= n - 2)[:, 0]
    lo, hi = f.copy(), f.copy()
    lo[ti, tj] = np.minimum(fl, fr)
    hi[ti, tj] = np.maximum(fl, fr)
    return f, lo, hi, int(ti.size)


# --------------------------------------------------------------------------------------------------
# step 6: spaxel sum (Sec. 3, "the stellar spectra in each spaxel are summed up")
# --------------------------------------------------------------------------------------------------
def _cube_rows(args):
    s_lo, s_hi, chunk, ties = args
    st = _POOL_STATE
    p, key, perm, seg_off, vlos, cfg = (st["p"], st["key"], st["perm"], st["seg_off"],
                                        st["vlos"], st["cfg"])
    out = np.zeros((s_hi - s_lo, cfg.n_tel))
    lo_out = np.zeros_like(out) if ties is not None else None
    hi_out = np.zeros_like(out) if ties is not None else None
    n_tied = 0
    i0, i1 = int(seg_off[s_lo]), int(seg_off[s_hi])
    for c0 in range(i0, i1, chunk):
        idx = perm[c0:min(i1, c0 + chunk)]
        k = key[idx] - s_lo
        starts = np.flatnonzero(np.r_[True, k[1:] != k[:-1]])
        if ties is None:
            f = particle_spectra(p, idx, vlos, cfg)
        else:
            f, lo, hi, nt = particle_spectra_bounds(p, idx, vlos, cfg, ties)
            n_tied += nt
            lo_out[k[starts]] += np.add.reduceat(lo, starts, axis=0)
            hi_out[k[starts]] += np.add.reduceat(hi, starts, axis=0)
        out[k[starts]] += np.add.reduceat(f, starts, axis=0)
    return s_lo, out, lo_out, hi_out, n_tied


_POOL_STATE: Dict = {}


class ForkedPool:
    """A fork-context process pool whose children run no garbage collection of the parent's
    objects: the parent collects its garbage first and freezes the rest (a caller that holds
    device resources, e.g. a GPU test, would otherwise see a child finalise them)."""

    def __init__(self, ctx, workers):
        import gc
        gc.collect()
        gc.freeze()
        try:
            self.pool = ctx.Pool(workers)
        except BaseException:
            gc.unfreeze()
            raise

    def __enter__(self):
        return self.pool.__enter__()

    def __exit__(self, *exc):
        import gc
        try:
            return self.pool.__exit__(*exc)
        finally:
            gc.unfreeze()


def cube_raw(p, key, perm, seg_off, vlos, cfg: OracleConfig, workers: Optional[int] = None,
             chunk: int = 1024, ties=None):
    """C_raw[s, j] = sum over particles with key s of f_i(lam_j), FP64, shape [ny*nx, n_tel].

    Works over spaxel ranges; with workers > 1 the ranges run in forked processes.
    With `ties` = (eps_abs, eps_rel) it returns (C_raw, C_lo, C_hi, n_tied) instead: C_lo / C_hi
    sum every particle's smaller / larger one-sided value at the pairs whose node interval is
    decided by rounding (particle_spectra_bounds), so any choice of sides per pair lies between
    them."""
    n_s = cfg.n_spaxels
    n_in = int(seg_off[n_s])
    workers = workers if workers is not None else int(os.environ.get("ORACLE_WORKERS", "1"))
    _POOL_STATE.update(p=p, key=key, perm=perm, seg_off=seg_off, vlos=vlos, cfg=cfg)
    # split spaxels into ranges holding roughly equal particle counts
    n_ranges = max(1, workers * 8) if workers > 1 else 1
    bounds = np.searchsorted(seg_off, np.linspace(0, n_in, n_ranges + 1), side="left")
    bounds[0], bounds[-1] = 0, n_s
    bounds = np.unique(np.clip(bounds, 0, n_s))
    tasks = [(int(a), int(b), chunk, ties) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    out = np.zeros((n_s, cfg.n_tel))
    lo = np.zeros_like(out) if ties is not None else None
    hi = np.zeros_like(out) if ties is not None else None
    n_tied = 0

    def put(res):
        nonlocal n_tied
        s_lo, rows, rlo, rhi, nt = res
        out[s_lo:s_lo + rows.shape[0]] = rows
        if ties is not None:
            lo[s_lo:s_lo + rows.shape[0]] = rlo
            hi[s_lo:s_lo + rows.shape[0]] = rhi
            n_tied += nt

    if workers > 1 and len(tasks) > 1:
        import multiprocessing as mp
        with ForkedPool(mp.get_context("fork"), workers) as pool:
            for res in pool.imap_unordered(_cube_rows, tasks):
                put(res)
    else:
        for t in tasks:
            put(_cube_rows(t))
    _POOL_STATE.clear()
    if ties is None:
        return out
    return out, lo, hi, n_tied


# --------------------------------------------------------------------------------------------------
# step 7: PSF and LSF (Sec. 3 "point-spread function (PSF) and line-spread function (LSF)
# convolution"; Gaussian per Sec. 4 "Qualitative Analysis")
# --------------------------------------------------------------------------------------------------
def gaussian_weights(sigma: float) -> np.ndarray:
    """Sampled Gaussian exp(-k^2 / (2 sigma^2)) for |k| <= r, r = int(4 sigma + 0.5), normalised
    to unit sum. sigma = 0 gives the identity kernel [1]."""
    if sigma <= 0.0:
        return np.ones(1)
    r = int(4.0 * sigma + 0.5)
    k = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * (k / sigma) ** 2)
    return w / w.sum()


def convolve_axis(a: np.ndarray, w: np.ndarray, axis: int) -> np.ndarray:
    """out[..., i, ...] = sum_k w[k + r] a[..., i + k, ...], zero outside the array."""
    r = (w.shape[0] - 1) // 2
    a = np.moveaxis(np.asarray(a, dtype=np.float64), axis, 0)
    n = a.shape[0]
    out = np.zeros_like(a)
    for k in range(-r, r + 1):
        lo, hi = max(0, -k), min(n, n - k)
        if hi > lo:
            out[lo:hi] += w[k + r] * a[lo + k:hi + k]
    return np.moveaxis(out, 0, axis)


def psf_lsf(c_raw: np.ndarray, cfg: OracleConfig) -> np.ndarray:
    """A C_raw: LSF along lambda (sigma in bins = sigma_A / dlam_tel), then the PSF along y and
    along x (sigma in spaxels). Input/output shape [ny*nx, n_tel]."""
    c = c_raw.reshape(cfg.ny, cfg.nx, cfg.n_tel)
    c = convolve_axis(c, gaussian_weights(cfg.lsf_sigma_bins()), 2)
    wp = gaussian_weights(cfg.psf_sigma_spx)
    c = convolve_axis(c, wp, 0)
    c = convolve_axis(c, wp, 1)
    return c.reshape(cfg.ny * cfg.nx, cfg.n_tel)


# --------------------------------------------------------------------------------------------------
# whole forward pass
# --------------------------------------------------------------------------------------------------
def forward(p, cfg: OracleConfig, workers: Optional[int] = None, frozen_key=None,
            with_cube=True, ties=None) -> Dict[str, np.ndarray]:
    """Run steps 1-7. Returns key, perm, seg_off, vlos (FP64), cube_raw and cube (FP64).

    `frozen_key` replaces the binning result (used when differentiating w.r.t. angles).
    With `ties` = (eps_abs, eps_rel) (node_ties) it also returns the range of correct cubes:
    cube_raw_lo / cube_raw_hi (cube_raw's bounds) and cube_lo / cube_hi (their PSF/LSF images,
    which bound the cube since the Gaussian weights are positive), and n_ties."""
    R = rotation_matrix(*cfg.angles_rad)
    xp, yp, _ = rotate_positions(p, R)
    vlos = los_velocity(p, R)
    key = spaxel_keys(xp, yp, cfg.nx, cfg.ny, cfg.spaxel_kpc) if frozen_key is None \
        else np.asarray(frozen_key, dtype=np.int64)
    perm, seg_off = sort_by_key(key, cfg.n_spaxels)
    out = dict(R=R, key=key, perm=perm, seg_off=seg_off, vlos=vlos)
    if with_cube:
        if ties is None:
            c = cube_raw(p, key, perm, seg_off, vlos, cfg, workers=workers)
        else:
            c, lo, hi, nt = cube_raw(p, key, perm, seg_off, vlos, cfg, workers=workers, ties=ties)
            out.update(cube_raw_lo=lo, cube_raw_hi=hi, cube_lo=psf_lsf(lo, cfg),
                       cube_hi=psf_lsf(hi, cfg), n_ties=nt)
        out["cube_raw"] = c
        out["cube"] = psf_lsf(c, cfg)
    return out


# --------------------------------------------------------------------------------------------------
# loss and adjoint (gradients through the pipeline: Abstract, Sec. 1)
# --------------------------------------------------------------------------------------------------
def loss(cube: np.ndarray, target: np.ndarray) -> float:
    """L = 0.5 * || A C_raw - T* ||^2 (cube = A C_raw)."""
    r = np.asarray(cube, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return 0.5 * float(np.sum(r * r))


def loss_grad_cube(cube: np.ndarray, target: np.ndarray, cfg: OracleConfig) -> np.ndarray:
    """G = dL/dC_raw = A^T (A C_raw - T*) = A (A C_raw - T*), since A is a symmetric operator."""
    return psf_lsf(np.asarray(cube, dtype=np.float64) - np.asarray(target, dtype=np.float64), cfg)


def adjoint(p, cfg: OracleConfig, G: np.ndarray, fw: Optional[Dict] = None,
            idx: Optional[np.ndarray] = None, chunk: int = 512,
            workers: int = 1, ties=None) -> Dict[str, np.ndarray]:
    """Analytic gradients of L given G = dL/dC_raw, for particles `idx` (default: all). For the
    bin-mean resampling see _adjoint_bin_mean; the bin-centre form is below.

    Per particle i in the field (spaxel s), as sums over the telescope bins j of per-bin terms,
    with the bilinear spectrum Slin_i = sum_c w_ic Tlin_c and its cell-direction derivatives
    Sa_i = sum_c (dw_c/dt_a) Tlin_c, Sz_i = sum_c (dw_c/dt_z) Tlin_c (all at q_ij):
      dL/dm_i      = flux_scale J_i sum_j G[s,j] Slin_i
      dL/dage_i    = flux_scale m_i J_i sum_j G[s,j] Sa_i / (du_a) / (age_i ln 10)
      dL/dmet_i    = flux_scale m_i J_i sum_j G[s,j] Sz_i / (du_z)
      dL/dvlos_i   = (1/c) sum_j G[s,j] flux_scale m_i [dJ/dbeta Slin_i(q_ij)
                                          + J_i Slin_i'(q_ij) dq_ij/dbeta]
    with Slin' the slope of the linear interpolant on the node interval holding q (node_cell: the
    right-hand one at a node), zero outside the SSP range, and clamped axes giving zero. Angles use
    frozen keys:
      dL/dphi_k = sum_i dL/dvlos_i (dR/dphi_k v_i)_z,   dL/dv_i = dL/dvlos_i R[2, :].
    Particles outside the field get zero. Positions get no gradient (binning is piecewise
    constant).

    With `ties` = (eps_abs, eps_rel) (node_ties) the result also holds, per quantity, `<name>_lo`
    and `<name>_hi`: the range of correct gradients when each (particle, bin) pair whose node
    interval is decided by rounding may take either side (a bin's terms from the left or the right
    interval; for the bin mean, an edge at either end of the SSP range inside or outside it), and
    n_ties, the number of such pairs (edges)."""
    if fw is None:
        fw = forward(p, cfg, with_cube=False)
    R, key, vlos = fw["R"], fw["key"], fw["vlos"]
    n = key.shape[0]
    if idx is None:
        idx = np.arange(n)
    idx = np.asarray(idx, dtype=np.int64)
    names = ("mass", "age", "met", "vlos")
    if workers > 1 and idx.shape[0] > 4 * chunk:
        # the per-particle gradients are independent: evaluate index ranges in forked processes
        import multiprocessing as mp
        parts = np.array_split(idx, workers * 4)
        _POOL_STATE.update(adj=(p, cfg, G, fw, chunk, ties))
        with ForkedPool(mp.get_context("fork"), workers) as pool:
            res = pool.map(_adjoint_part, parts)
        _POOL_STATE.clear()
        keys = names if ties is None else names + tuple(f"{k}_{e}" for k in names
                                                         for e in ("lo", "hi"))
        out = {k: np.concatenate([r[k] for r in res]) for k in keys}
        if ties is not None:
            out["n_ties"] = sum(r["n_ties"] for r in res)
        return _adjoint_angles(p, cfg, R, idx, out)
    n_s = cfg.n_spaxels
    out = {k: np.zeros(idx.shape[0]) for k in names}
    if ties is not None:
        out.update({f"{k}_{e}": np.zeros(idx.shape[0]) for k in names for e in ("lo", "hi")})
        out["n_ties"] = 0
    nl = cfg.ssp_flux.shape[2]
    T = cfg.ssp_flux
    la_nodes, mz_nodes = cfg.log_age_nodes, cfg.met_nodes
    inf = key[idx] < n_s
    Q = rest_index(cfg)[None, :]
    for c0 in range(0, idx.shape[0], chunk):
        sel = np.arange(c0, min(idx.shape[0], c0 + chunk))
        sel = sel[inf[sel]]
        if sel.size == 0:
            continue
        ii = idx[sel]
        age, met, mass = _p64(p, "age")[ii], _p64(p, "met")[ii], _p64(p, "mass")[ii]
        v = vlos[ii]
        beta = v / C_KMS
        ja, jz, ta, tz, w, ina, inz = ssp_weights(age, met, la_nodes, mz_nodes)
        if cfg.resample == 1:
            fn = _adjoint_bin_mean_log if cfg.log_lambda else _adjoint_bin_mean
            fn(cfg, G, key[ii], age, mass, v, ja, jz, ta, tz, w, ina, inz, out, sel, ties)
            continue
        q = doppler_index(cfg, v)
        g = G[key[ii]]                                   # [m, n_tel]
        corners = [(ja, jz), (ja, jz + 1), (ja + 1, jz), (ja + 1, jz + 1)]
        fs = cfg.flux_scale
        J = 1.0 / ((1.0 + cfg.z_sys) * (1.0 + beta))
        dJ = -J / (1.0 + beta)
        dq = doppler_index_dbeta(cfg, v)
        dwa = np.stack([-(1 - tz), -tz, (1 - tz), tz], axis=-1)
        dwz = np.stack([-(1 - ta), (1 - ta), -ta, ta], axis=-1)
        du_a = la_nodes[ja + 1] - la_nodes[ja]
        du_z = mz_nodes[jz + 1] - mz_nodes[jz]
        c_age = np.where(ina, fs * mass * J / du_a / (age * math.log(10.0)), 0.0)[:, None]
        c_met = np.where(inz, fs * mass * J / du_z, 0.0)[:, None]

        def terms(k, valid):
            # per-bin terms of the four gradients with node interval k (valid: on the grid)
            Sl = np.zeros_like(q)
            Sa = np.zeros_like(q)
            Sz = np.zeros_like(q)
            dS = np.zeros_like(q)                        # slope of Slin per node index
            kk = np.where(valid, k, 0)
            for c, (a_, z_) in enumerate(corners):
                row = T[a_, z_]                           # [m, nl]
                tl = cell_linear(row, q, k, valid)
                Sl += w[:, c:c + 1] * tl
                Sa += dwa[:, c:c + 1] * tl
                Sz += dwz[:, c:c + 1] * tl
                t0 = np.take_along_axis(row, kk, axis=1)
                t1 = np.take_along_axis(row, kk + 1, axis=1)
                dS += w[:, c:c + 1] * np.where(valid, t1 - t0, 0.0)
            return (fs * J[:, None] * g * Sl, c_age * g * Sa, c_met * g * Sz,
                    fs * mass[:, None] * g * (dJ[:, None] * Sl + J[:, None] * dS * dq) / C_KMS)

        if ties is None:
            base = terms(*node_cell(q, nl))
            for name, t in zip(names, base):
                out[name][sel] = np.sum(t, axis=1)
            continue
        cell, left, right, tie = one_sided_cells(q, q - Q, nl, ties)
        base, tl_, tr_ = terms(*cell), terms(*left), terms(*right)
        out["n_ties"] += int(tie.sum())
        for name, t, a_, b_ in zip(names, base, tl_, tr_):
            out[name][sel] = np.sum(t, axis=1)
            out[f"{name}_lo"][sel] = np.sum(np.where(tie, np.minimum(a_, b_), t), axis=1)
            out[f"{name}_hi"][sel] = np.sum(np.where(tie, np.maximum(a_, b_), t), axis=1)
    return _adjoint_angles(p, cfg, R, idx, out)


def linear_at(S: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Value of the piecewise-linear interpolant of row i of S at q[i, j], for q in [0, n-1]
    (clipped there; callers mask what lies outside)."""
    n = S.shape[1]
    q = np.clip(q, 0.0, n - 1.0)
    k = np.minimum(np.floor(q), n - 2).astype(np.int64)
    t = q - k
    s0 = np.take_along_axis(S, k, axis=1)
    s1 = np.take_along_axis(S, k + 1, axis=1)
    return s0 + t * (s1 - s0)


def _adjoint_bin_mean(cfg, G, keys, age, mass, v, ja, jz, ta, tz, w, ina, inz, out, sel,
                      ties=None):
    """Gradients for the bin-mean resampling (reading 1), particles `sel` of the chunk.

    f_i(j) = B m_i sum_c w_ic I_c(j), B = flux_scale dlam_ssp/dlam, I_c(j) the integral of the
    linear interpolant of corner c over [q_lo,ij, q_hi,ij] clipped to [0, n-1]. With
    X_ic = sum_j G[s, j] I_c(j):
      dL/dm_i    = B sum_c w_ic X_ic,
      dL/dage_i  = B m_i sum_c (dw_c/dt_a) X_ic / du_a / (age_i ln 10), dL/dmet_i likewise;
    the integrand does not depend on beta, the limits do (Leibniz rule): with Slin_i the
    bilinear spectrum's interpolant,
      dL/dbeta_i = B m_i sum_j G[s, j] (Slin_i(q_hi) dq_hi/dbeta - Slin_i(q_lo) dq_lo/dbeta),
    an edge outside (0, n-1) being clipped and contributing nothing, and
    dq/dbeta = -lam_edge / ((1+z)(1+beta)^2 dlam_ssp) at the bin edge lam_edge = lam_j -/+ dlam/2.
    The integrals are continuous in the edges' positions, so only the Leibniz term of an edge at
    either end of the SSP range depends on rounding (edge_terms)."""
    T = cfg.ssp_flux
    nl = T.shape[2]
    la_nodes, mz_nodes = cfg.log_age_nodes, cfg.met_nodes
    g = G[keys]                                            # [m, n_tel]
    q_lo, q_hi = bin_edge_indices(cfg, v)
    corners = [(ja, jz), (ja, jz + 1), (ja + 1, jz), (ja + 1, jz + 1)]
    X = np.zeros((keys.shape[0], 4))
    for c, (a_, z_) in enumerate(corners):
        X[:, c] = np.sum(g * integral_linear(T[a_, z_], q_lo, q_hi), axis=1)
    B = cfg.flux_scale * cfg.ssp_lam_step / cfg.tel_step
    out["mass"][sel] = B * np.sum(w * X, axis=1)
    dwa = np.stack([-(1 - tz), -tz, (1 - tz), tz], axis=-1)
    dwz = np.stack([-(1 - ta), (1 - ta), -ta, ta], axis=-1)
    du_a = la_nodes[ja + 1] - la_nodes[ja]
    du_z = mz_nodes[jz + 1] - mz_nodes[jz]
    out["age"][sel] = np.where(ina, B * mass * np.sum(dwa * X, axis=1) / du_a
                               / (age * math.log(10.0)), 0.0)
    out["met"][sel] = np.where(inz, B * mass * np.sum(dwz * X, axis=1) / du_z, 0.0)
    S = interp_templates(T, ja, jz, w)
    beta = np.asarray(v, dtype=np.float64) / C_KMS
    lam = cfg.tel_lambda()[None, :]
    f2 = (1.0 + cfg.z_sys) * (1.0 + beta[:, None]) ** 2 * cfg.ssp_lam_step
    rest_lo, rest_hi = bin_edge_indices(cfg, np.zeros(1))
    scale = (B * mass / C_KMS)[:, None] * g
    edges = [(q_hi, q_hi - rest_hi, scale * linear_at(S, q_hi) * (-(lam + 0.5 * cfg.tel_step) / f2)),
             (q_lo, q_lo - rest_lo, -scale * linear_at(S, q_lo) * (-(lam - 0.5 * cfg.tel_step) / f2))]
    edge_terms(edges, nl, ties, out, sel)


def edge_terms(edges, nl, ties, out, sel):
    """The Leibniz terms of the bin-mean velocity gradient: per edge (q, d, y), y the edge's term
    in every bin if the edge lies strictly inside (0, n-1) and 0 otherwise (a clipped edge does
    not move the integral). With `ties` an edge within eps of either end of the range (node_ties'
    eps, d the Doppler part of q) may count as inside or outside, and the bounds take both."""
    total = 0.0
    lo = hi = 0.0
    n_tied = 0
    for q, d, y in edges:
        inside = (q > 0.0) & (q < nl - 1.0)
        t = np.where(inside, y, 0.0)
        total = total + t
        if ties is not None:
            eps = ties[0] + ties[1] * np.abs(np.where(np.isfinite(d), d, 0.0))
            tie = (np.abs(q) <= eps) | (np.abs(q - (nl - 1.0)) <= eps)
            n_tied += int(tie.sum())
            lo = lo + np.where(tie, np.minimum(y, 0.0), t)
            hi = hi + np.where(tie, np.maximum(y, 0.0), t)
    out["vlos"][sel] = np.sum(total, axis=1)
    if ties is not None:
        out["vlos_lo"][sel] = np.sum(lo, axis=1)
        out["vlos_hi"][sel] = np.sum(hi, axis=1)
        out["n_ties"] += n_tied
        for k in ("mass", "age", "met"):
            out[f"{k}_lo"][sel] = out[k][sel]
            out[f"{k}_hi"][sel] = out[k][sel]


def _adjoint_bin_mean_log(cfg, G, keys, age, mass, v, ja, jz, ta, tz, w, ina, inz, out, sel,
                          ties=None):
    """Gradients for the bin-mean resampling on log grids, particles `sel` of the chunk.

    f_i(j) = fs m_i / dlam_j sum_c w_ic I_c(j), I_c(j) the integral over rest wavelength of
    corner c's interpolant (linear in the log-grid index) between the bin's rest-frame edges,
    clipped to the grid. With X_ic = sum_j G[s, j] I_c(j) / dlam_j the mass, age and [M/H]
    gradients take the form of the linear-grid bin mean with B = fs. The integrand
    Slin(q) lam(q) dln_ssp does not depend on beta; the limits move with
    dq/dbeta = -1/((1+beta) dln_ssp) at both edges (Leibniz rule), so
      dL/dbeta_i = -fs m_i / (1+beta_i) sum_j G[s, j] / dlam_j
                   (Slin_i(q_hi) lam(q_hi) [q_hi inside] - Slin_i(q_lo) lam(q_lo) [q_lo inside]),
    an edge outside (0, n-1) being clipped and contributing nothing (edge_terms)."""
    T = cfg.ssp_flux
    nl = T.shape[2]
    la_nodes, mz_nodes = cfg.log_age_nodes, cfg.met_nodes
    width = cfg.tel_lambda() * (2.0 * math.sinh(0.5 * cfg.tel_step))
    g = G[keys] / width[None, :]                           # [m, n_tel]
    q_lo, q_hi = bin_edge_indices_log(cfg, v)
    corners = [(ja, jz), (ja, jz + 1), (ja + 1, jz), (ja + 1, jz + 1)]
    X = np.zeros((keys.shape[0], 4))
    for c, (a_, z_) in enumerate(corners):
        X[:, c] = np.sum(g * integral_log_weighted(T[a_, z_], q_lo, q_hi, cfg.ssp_lam_start,
                                                   cfg.ssp_lam_step), axis=1)
    B = cfg.flux_scale
    out["mass"][sel] = B * np.sum(w * X, axis=1)
    dwa = np.stack([-(1 - tz), -tz, (1 - tz), tz], axis=-1)
    dwz = np.stack([-(1 - ta), (1 - ta), -ta, ta], axis=-1)
    du_a = la_nodes[ja + 1] - la_nodes[ja]
    du_z = mz_nodes[jz + 1] - mz_nodes[jz]
    out["age"][sel] = np.where(ina, B * mass * np.sum(dwa * X, axis=1) / du_a
                               / (age * math.log(10.0)), 0.0)
    out["met"][sel] = np.where(inz, B * mass * np.sum(dwz * X, axis=1) / du_z, 0.0)
    S = interp_templates(T, ja, jz, w)
    beta = np.asarray(v, dtype=np.float64) / C_KMS
    rest_lo, rest_hi = bin_edge_indices_log(cfg, np.zeros(1))
    scale = (-B * mass / (1.0 + beta) / C_KMS)[:, None] * g
    edges = []
    for q, rest, sgn in ((q_hi, rest_hi, 1.0), (q_lo, rest_lo, -1.0)):
        lam_r = cfg.ssp_lam_start * np.exp(np.clip(q, 0.0, nl - 1.0) * cfg.ssp_lam_step)
        edges.append((q, q - rest, sgn * scale * linear_at(S, q) * lam_r))
    edge_terms(edges, nl, ties, out, sel)


def _adjoint_part(part):
    p, cfg, G, fw, chunk, ties = _POOL_STATE["adj"]
    return adjoint(p, cfg, G, fw, idx=part, chunk=chunk, workers=1, ties=ties)


def _adjoint_angles(p, cfg, R, idx, out):
    """dL/dphi_k = sum_i dL/dvlos_i (dR/dphi_k v_i)_z and dL/dv_i = dL/dvlos_i R[2, :]; with
    bounds on dL/dvlos_i (vlos_lo / vlos_hi) also the bounds of both that follow from them."""
    dR = rotation_matrix_derivs(*cfg.angles_rad)
    vx, vy, vz = _p64(p, "vx")[idx], _p64(p, "vy")[idx], _p64(p, "vz")[idx]
    coef = [dR[k, 2, 0] * vx + dR[k, 2, 1] * vy + dR[k, 2, 2] * vz for k in range(3)]
    dv = out["vlos"]
    out["angles"] = np.array([np.sum(dv * coef[k]) for k in range(3)])
    out["vel"] = dv[None, :] * R[2, :, None]
    if "vlos_lo" in out:
        lo, hi = out["vlos_lo"], out["vlos_hi"]
        out["angles_lo"] = np.array([np.sum(np.minimum(lo * c, hi * c)) for c in coef])
        out["angles_hi"] = np.array([np.sum(np.maximum(lo * c, hi * c)) for c in coef])
        a, b = lo[None, :] * R[2, :, None], hi[None, :] * R[2, :, None]
        out["vel_lo"], out["vel_hi"] = np.minimum(a, b), np.maximum(a, b)
    return out
