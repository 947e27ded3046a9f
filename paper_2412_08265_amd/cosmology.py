"""Placing a galaxy at a distance: the observation scalars that depend on it.

The forward model takes a galaxy distance among its configuration (arXiv:2412.08265, Sec. 3:
the Doppler shift depends on the galaxy distance and the line-of-sight velocity; the
configuration names the galaxy distance). Here the distance enters as a cosmological redshift z
in a flat Lambda-CDM universe:
  - systemic redshift z_sys = z (every wavelength stretched by 1+z; the kernels also apply the
    flux-density factor 1/(1+z) through the Jacobian J);
  - spaxel size in kpc from an angular size: s = theta * D_A, D_A = D_C / (1+z);
  - flux dimming: flux_scale = 1 / (4 pi D_L^2) with D_L = (1+z) D_C in Mpc, so the cube holds
    template luminosity density x Msun / (4 pi Mpc^2);
  - D_C = (c/H0) * integral_0^z dz' / E(z'), E(z) = sqrt(Om (1+z)^3 + 1 - Om), by 64-point
    Gauss-Legendre quadrature (the integrand is smooth and positive).
These are host-side scalars computed once per observation; no part of the per-particle path runs
here.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_KMS = 299792.458
ARCSEC_RAD = math.pi / 648000.0

_GL_X, _GL_W = np.polynomial.legendre.leggauss(64)


@dataclasses.dataclass(frozen=True)
class FlatLCDM:
    H0: float = 70.0        # km/s/Mpc
    Om: float = 0.3

    def E(self, z):
        z = np.asarray(z, dtype=np.float64)
        return np.sqrt(self.Om * (1.0 + z) ** 3 + (1.0 - self.Om))

    def comoving_distance_mpc(self, z: float) -> float:
        if z < 0:
            raise ValueError("z must be >= 0")
        if z == 0:
            return 0.0
        zz = 0.5 * z * (_GL_X + 1.0)
        return float(C_KMS / self.H0 * 0.5 * z * np.sum(_GL_W / self.E(zz)))

    def luminosity_distance_mpc(self, z: float) -> float:
        return (1.0 + z) * self.comoving_distance_mpc(z)

    def angular_diameter_distance_mpc(self, z: float) -> float:
        return self.comoving_distance_mpc(z) / (1.0 + z)


def place_at_redshift(obs, z: float, spaxel_arcsec: float, cosmo: FlatLCDM = FlatLCDM()):
    """A copy of `obs` (an Observation) for the galaxy at redshift z observed with square
    spaxels of `spaxel_arcsec`: z_sys = z, spaxel_kpc = theta D_A, flux_scale multiplied by
    1/(4 pi D_L^2) [Mpc^-2]."""
    if not (z > 0):
        raise ValueError("z must be > 0 (a galaxy at z = 0 has no finite flux dimming)")
    d_a_kpc = cosmo.angular_diameter_distance_mpc(z) * 1.0e3
    d_l = cosmo.luminosity_distance_mpc(z)
    return dataclasses.replace(obs, z_sys=float(z),
                               spaxel_kpc=float(spaxel_arcsec * ARCSEC_RAD * d_a_kpc),
                               flux_scale=float(obs.flux_scale / (4.0 * math.pi * d_l * d_l)))
