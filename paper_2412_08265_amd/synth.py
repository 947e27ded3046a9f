"""Seeded synthetic inputs: star-particle galaxies, SSP template grids and workload configs.

This module only *draws* inputs. It holds none of the forward model's arithmetic (no rotation,
binning, interpolation, Doppler shift, resampling or convolution), so that both the HIP path and the
FP64 CPU oracle can consume the very same arrays without sharing any method code.

Every array that leaves this module is FP32 (rounded to nearest even from an FP64 draw); both sides
read the same FP32 values, so input rounding is not part of any parity comparison.

Stand-ins: the paper's inputs are TNG50-1 star particles (Sec. 4, "Qualitative Analysis") and the
MaStar SSP library; neither is available, so these generators produce galaxies and templates with
the shapes, ranges and structure those inputs have (disk + bulge particle sets, log-spaced SSP ages,
metallicity axis, uniform wavelength grids).
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Dict, Optional

import numpy as np

C_KMS = 299792.458  # speed of light [km/s]


# --------------------------------------------------------------------------------------------------
# particles
# --------------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Particles:
    """Structure-of-arrays star particles, FP32. Units: kpc, km/s, Msun, Gyr, dex ([M/H])."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    mass: np.ndarray
    age: np.ndarray
    met: np.ndarray

    FIELDS = ("x", "y", "z", "vx", "vy", "vz", "mass", "age", "met")

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return [getattr(self, f) for f in self.FIELDS]

    def as_dict(self) -> Dict[str, np.ndarray]:
        return {f: getattr(self, f) for f in self.FIELDS}

    def subset(self, idx) -> "Particles":
        return Particles(*[np.ascontiguousarray(a[idx]) for a in self.arrays()])

    def replace(self, **kw) -> "Particles":
        d = self.as_dict()
        d.update({k: np.ascontiguousarray(v, dtype=np.float32) for k, v in kw.items()})
        return Particles(**d)

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in self.arrays():
            h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
        return h.hexdigest()

    @staticmethod
    def concat(parts) -> "Particles":
        return Particles(*[np.concatenate([getattr(p, f) for p in parts]) for f in Particles.FIELDS])


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _stellar_props(rng: np.random.Generator, n: int):
    logm = rng.uniform(4.0, 6.0, n)          # log10 mass [Msun], log-uniform 1e4..1e6
    age = rng.uniform(0.1, 13.0, n)          # Gyr
    met = rng.uniform(-2.0, 0.3, n)          # [M/H] = log10(Z/Zsun)
    return 10.0 ** logm, age, met


def make_disk(rng: np.random.Generator, n: int, scale_kpc=3.0, height_kpc=0.3,
              vcirc=200.0, sigma_v=30.0):
    """Exponential disk with surface density ~ exp(-R/h): R ~ Gamma(2, h), z ~ Laplace(0, h_z).

    Velocity: circular `vcirc` counter-clockwise about +z plus an isotropic Gaussian dispersion.
    Draw order is frozen: R, phi, z, 3 dispersion components, mass, age, met.
    """
    R = rng.gamma(2.0, scale_kpc, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    z = rng.laplace(0.0, height_kpc, n)
    disp = rng.normal(0.0, sigma_v, (3, n))
    mass, age, met = _stellar_props(rng, n)
    x = R * np.cos(phi)
    y = R * np.sin(phi)
    vx = -vcirc * np.sin(phi) + disp[0]
    vy = vcirc * np.cos(phi) + disp[1]
    vz = disp[2]
    return Particles(*[_f32(a) for a in (x, y, z, vx, vy, vz, mass, age, met)])


def make_bulge(rng: np.random.Generator, n: int, a_kpc=1.0, sigma_v=150.0):
    """Hernquist sphere (untruncated), isotropic Gaussian velocities.

    r = a*sqrt(u)/(1-sqrt(u)) inverts M(<r) ~ r^2/(r+a)^2. Draw order: u, cos(theta), phi,
    3 velocity components, mass, age, met.
    """
    u = rng.uniform(0.0, 1.0, n)
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    vel = rng.normal(0.0, sigma_v, (3, n))
    mass, age, met = _stellar_props(rng, n)
    su = np.sqrt(u)
    r = a_kpc * su / (1.0 - su)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    x = r * sth * np.cos(phi)
    y = r * sth * np.sin(phi)
    z = r * cth
    return Particles(*[_f32(a) for a in (x, y, z, vel[0], vel[1], vel[2], mass, age, met)])


def make_galaxy(n: int, seed: int, bulge_frac: float = 0.2) -> Particles:
    """Disk + bulge galaxy of `n` particles in total; the bulge holds round(bulge_frac*n)."""
    rng = np.random.default_rng(seed)
    nb = int(round(bulge_frac * n))
    nd = n - nb
    disk = make_disk(rng, nd)
    if nb == 0:
        return disk
    bulge = make_bulge(rng, nb)
    return Particles.concat([disk, bulge])


# --------------------------------------------------------------------------------------------------
# SSP template grids
# --------------------------------------------------------------------------------------------------
@dataclasses.dataclass
class SSPGrid:
    """SSP template grid. flux[n_age][n_met][n_lam] FP32, lambda contiguous.

    Nodes: log10(age/Gyr) (strictly increasing), [M/H] (strictly increasing); lambda nodes
    lam_start + k*lam_step [Angstrom], or lam_start * exp(k*lam_step) when log_lambda.
    """
    log_age_nodes: np.ndarray
    met_nodes: np.ndarray
    lam_start: float
    lam_step: float
    flux: np.ndarray
    log_lambda: bool = False

    @property
    def n_age(self):
        return int(self.log_age_nodes.shape[0])

    @property
    def n_met(self):
        return int(self.met_nodes.shape[0])

    @property
    def n_lam(self):
        return int(self.flux.shape[2])

    def lam(self) -> np.ndarray:
        k = np.arange(self.n_lam, dtype=np.float64)
        if self.log_lambda:
            return self.lam_start * np.exp(self.lam_step * k)
        return self.lam_start + self.lam_step * k


def _planck_lambda(lam_A, T):
    # B_lambda up to a constant: lam^-5 / (exp(hc/(lam k T)) - 1), hc/k = 1.4387769e8 A K
    x = 1.4387769e8 / (lam_A * T)
    return lam_A ** -5 / np.expm1(x)


def make_ssp(n_age: int, n_met: int, lam_start: float, lam_step: float, n_lam: int,
             n_lines: int = 20, line_seed: int = 12345, age_range=(0.1, 13.0),
             met_range=(-2.0, 0.3), log_lambda: bool = False) -> SSPGrid:
    """Synthetic SSP grid: blackbody-like continuum whose temperature falls with age and rises
    with decreasing metallicity, times 20 Gaussian absorption lines whose depths grow with age and
    metallicity. The lines are shared by all templates (seeded once)."""
    ages = np.geomspace(age_range[0], age_range[1], n_age)
    mets = np.linspace(met_range[0], met_range[1], n_met)
    k = np.arange(n_lam, dtype=np.float64)
    lam = lam_start * np.exp(lam_step * k) if log_lambda else lam_start + lam_step * k
    lam_lo, lam_hi = lam[0], lam[-1]
    lrng = np.random.default_rng(line_seed)
    margin = min(50.0, 0.25 * (lam_hi - lam_lo))
    mu = lrng.uniform(lam_lo + margin, lam_hi - margin, n_lines)
    sig = lrng.uniform(2.0, 6.0, n_lines)
    dep = lrng.uniform(0.1, 0.5, n_lines)
    prof = np.exp(-0.5 * ((lam[None, :] - mu[:, None]) / sig[:, None]) ** 2)  # [lines, lam]
    flux = np.empty((n_age, n_met, n_lam), dtype=np.float64)
    for ia, a in enumerate(ages):
        xa = math.log10(a / 0.1) / math.log10(130.0)
        for iz, m in enumerate(mets):
            teff = 4000.0 + 16000.0 * (a / 0.1) ** -0.45 - 500.0 * m
            cont = _planck_lambda(lam, teff) / _planck_lambda(5500.0, teff) * (a / 1.0) ** -0.7
            xz = (m + 2.0) / 2.3
            depth = np.minimum(0.9, dep * (0.6 + 0.4 * xa) * (0.6 + 0.4 * xz))
            absorb = np.prod(1.0 - depth[:, None] * prof, axis=0)
            flux[ia, iz] = cont * absorb
    return SSPGrid(_f32(np.log10(ages)), _f32(mets), float(lam_start), float(lam_step),
                   _f32(flux), bool(log_lambda))


def make_line_ssp(lam_start: float, lam_step: float, n_lam: int, line_center: float,
                  line_sigma: float, n_age=2, n_met=2, amplitude=1.0,
                  log_lambda: bool = False) -> SSPGrid:
    """Emission-line-only templates (compact support, zero continuum): every template is the same
    Gaussian line. Used by the line-position and flux-conservation invariants."""
    k = np.arange(n_lam, dtype=np.float64)
    lam = lam_start * np.exp(lam_step * k) if log_lambda else lam_start + lam_step * k
    prof = amplitude * np.exp(-0.5 * ((lam - line_center) / line_sigma) ** 2)
    prof[prof < 1e-30] = 0.0
    flux = np.broadcast_to(prof, (n_age, n_met, n_lam)).copy()
    ages = np.geomspace(0.1, 13.0, n_age)
    mets = np.linspace(-2.0, 0.3, n_met)
    return SSPGrid(_f32(np.log10(ages)), _f32(mets), float(lam_start), float(lam_step),
                   _f32(flux), bool(log_lambda))


# --------------------------------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    """One forward-model run: particles + viewing angles + spaxel grid + telescope grid + SSP."""
    name: str
    particles: Particles
    angles_deg: tuple            # (phi1 about x = inclination, phi2 about y, phi3 about z)
    nx: int
    ny: int
    spaxel_kpc: float
    tel_start: float             # telescope bin centre of bin 0 [A]
    tel_step: float              # [A], or the ln(lambda) step when log_lambda
    n_tel: int
    ssp: SSPGrid
    psf_sigma_spx: float = 0.0
    lsf_sigma_A: float = 0.0
    z_sys: float = 0.0
    flux_scale: float = 1.0
    log_lambda: bool = False     # telescope bins tel_start * exp(k * tel_step) (as the SSP grid)
    resample: int = 0            # 0 bin-centre sampling, 1 bin mean (flux conserving)

    @property
    def angles_rad(self):
        return tuple(math.radians(a) for a in self.angles_deg)

    @property
    def n_spaxels(self):
        return self.nx * self.ny


_SSP_CACHE: Dict[tuple, SSPGrid] = {}


def cached_ssp(*args, **kw) -> SSPGrid:
    key = (args, tuple(sorted(kw.items())))
    if key not in _SSP_CACHE:
        _SSP_CACHE[key] = make_ssp(*args, **kw)
    return _SSP_CACHE[key]


def tiny_workload(seed=1, n=1000) -> Workload:
    """1000-particle exponential disk (no bulge), 16x16 spaxels of 1 kpc, SSP 10x5x500 on
    3600..7400 A, telescope grid = SSP nodes, no PSF/LSF, inclination 60 deg."""
    rng = np.random.default_rng(seed)
    p = make_disk(rng, n)
    lam = np.linspace(3600.0, 7400.0, 500)
    ssp = cached_ssp(10, 5, 3600.0, float(lam[1] - lam[0]), 500)
    return Workload("tiny-1e3", p, (60.0, 0.0, 0.0), 16, 16, 1.0,
                    3600.0, float(lam[1] - lam[0]), 500, ssp)


def medium_workload(seed=2, n=1_000_000) -> Workload:
    """1e6 particles (80 % disk, 20 % Hernquist bulge), 50x50 spaxels of 0.6 kpc (30 kpc FoV),
    SSP 100x12x3000 on 3600..7400 A, telescope grid = SSP nodes, PSF 1.5 spx, LSF 2.5 A."""
    p = make_galaxy(n, seed)
    step = (7400.0 - 3600.0) / 2999.0
    ssp = cached_ssp(100, 12, 3600.0, step, 3000)
    return Workload("disk+bulge-1e6", p, (60.0, 0.0, 0.0), 50, 50, 0.6,
                    3600.0, step, 3000, ssp, psf_sigma_spx=1.5, lsf_sigma_A=2.5)


def log_workload(seed=5, n=200_000) -> Workload:
    """Wavelength grids uniform in ln(lambda): 2e5 particles (disk + bulge), 30x30 spaxels of
    1 kpc, SSP 40x8x3000 from 3600 A with dln = 1.2e-4 (36 km/s per node), telescope 3300 bins of
    dln = 1e-4 starting 0.37 node above the SSP start, systemic z 0.002, PSF 1 spx, LSF 1.2 A."""
    p = make_galaxy(n, seed)
    ssp = cached_ssp(40, 8, 3600.0, 1.2e-4, 3000, log_lambda=True)
    return Workload("loglam-2e5", p, (60.0, 0.0, 0.0), 30, 30, 1.0,
                    3600.0 * math.exp(0.37 * 1.2e-4), 1.0e-4, 3300, ssp, psf_sigma_spx=1.0,
                    lsf_sigma_A=1.2, z_sys=0.002, log_lambda=True)


def large_log_workload(seed=3, n=10_000_000, spaxel_kpc=0.2) -> Workload:
    """The 1e7-particle galaxy on grids uniform in ln(lambda): 4563 SSP nodes and telescope bins
    from 4700 A with dln = 1.6e-4 (48 km/s per bin; 4700-9763 A), SSP 106x12, PSF 2 spx,
    LSF 2.7 A at the central wavelength."""
    p = make_galaxy(n, seed)
    ssp = cached_ssp(106, 12, 4700.0, 1.6e-4, 4563, log_lambda=True)
    return Workload("disk+bulge-1e7-loglam", p, (60.0, 0.0, 0.0), 150, 150, spaxel_kpc,
                    4700.0, 1.6e-4, 4563, ssp, psf_sigma_spx=2.0, lsf_sigma_A=2.7,
                    log_lambda=True)


def large_workload(seed=3, n=10_000_000, spaxel_kpc=0.2) -> Workload:
    """1e7 particles (80 % disk, 20 % bulge), 150x150 spaxels of 0.2 kpc (30 kpc FoV), telescope
    4563 bins at 1.25 A from 4700 A, SSP 106x12x4563 on the same centres, PSF 2 spx, LSF 2.7 A."""
    p = make_galaxy(n, seed)
    ssp = cached_ssp(106, 12, 4700.0, 1.25, 4563)
    return Workload("disk+bulge-1e7", p, (60.0, 0.0, 0.0), 150, 150, spaxel_kpc,
                    4700.0, 1.25, 4563, ssp, psf_sigma_spx=2.0, lsf_sigma_A=2.7)


def differentiation_target_params(p: Particles):
    """Perturbed parameters of the differentiation workload's target cube: masses +10 %,
    ages +0.5 Gyr (capped at 13 Gyr), [M/H] +0.1 dex, inclination +5 deg."""
    return p.replace(mass=p.mass.astype(np.float64) * 1.1,
                     age=np.minimum(p.age.astype(np.float64) + 0.5, 13.0),
                     met=p.met.astype(np.float64) + 0.1), (65.0, 0.0, 0.0)


# --------------------------------------------------------------------------------------------------
# serving trace
# --------------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    workload: Workload


def serving_ssp() -> SSPGrid:
    """Resident grid shared by all serving requests: 100 ages x 12 [M/H] x 4563 lambda
    (4700 + 1.25 k A)."""
    return cached_ssp(100, 12, 4700.0, 1.25, 4563)


def serving_request(i: int, ssp: Optional[SSPGrid] = None, n_max: float = 5e6,
                    n_min: float = 1e4) -> Workload:
    """Request i (seed 4000+i): N log-uniform in [n_min, n_max], square grid side uniform in
    {20..100} over a 30 kpc FoV, a telescope window of 1500..4563 contiguous resident nodes at a
    random start, inclination uniform in [0, 90) deg, PSF 2 spx, LSF 2.7 A."""
    ssp = ssp or serving_ssp()
    rng = np.random.default_rng(4000 + i)
    n = int(round(10.0 ** rng.uniform(math.log10(n_min), math.log10(n_max))))
    side = int(rng.integers(20, 101))
    n_lam = int(rng.integers(1500, ssp.n_lam + 1))
    start = int(rng.integers(0, ssp.n_lam - n_lam + 1))
    incl = float(rng.uniform(0.0, 90.0))
    gal_seed = int(rng.integers(0, 2 ** 31 - 1))
    p = make_galaxy(n, gal_seed)
    return Workload(f"req{i}", p, (incl, 0.0, 0.0), side, side, 30.0 / side,
                    ssp.lam_start + ssp.lam_step * start, ssp.lam_step, n_lam, ssp,
                    psf_sigma_spx=2.0, lsf_sigma_A=2.7)


def poisson_arrivals(n: int, rate_hz: float, seed: int = 4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))
