"""Oracle of the distance scalars (test infrastructure; not imported by the product path).

The galaxy distance of the forward model's configuration (arXiv:2412.08265, Sec. 3) as a redshift
in a flat Lambda-CDM universe, computed plainly and independently of the library's helper:
  D_C(z) = (c/H0) integral_0^z dz'/sqrt(Om (1+z')^3 + 1 - Om)   (adaptive quadrature, scipy),
  D_L = (1+z) D_C,  D_A = D_C/(1+z),
  spaxel_kpc = theta[rad] * D_A[kpc],  flux_scale = 1/(4 pi D_L[Mpc]^2),  z_sys = z.
"""
from __future__ import annotations

import math

import scipy.integrate

C_KMS = 299792.458


def comoving_distance_mpc(z: float, H0: float = 70.0, Om: float = 0.3) -> float:
    f = lambda x: 1.0 / math.sqrt(Om * (1.0 + x) ** 3 + (1.0 - Om))
    val, _ = scipy.integrate.quad(f, 0.0, z, epsabs=0.0, epsrel=1e-13, limit=200)
    return C_KMS / H0 * val


def luminosity_distance_mpc(z: float, H0: float = 70.0, Om: float = 0.3) -> float:
    return (1.0 + z) * comoving_distance_mpc(z, H0, Om)


def angular_diameter_distance_mpc(z: float, H0: float = 70.0, Om: float = 0.3) -> float:
    return comoving_distance_mpc(z, H0, Om) / (1.0 + z)


def observation_scalars(z: float, spaxel_arcsec: float, H0: float = 70.0, Om: float = 0.3):
    """(z_sys, spaxel_kpc, flux_scale) of a galaxy at redshift z seen with spaxels of the given
    angular size."""
    theta = spaxel_arcsec * math.pi / (180.0 * 3600.0)
    d_a_kpc = angular_diameter_distance_mpc(z, H0, Om) * 1000.0
    d_l = luminosity_distance_mpc(z, H0, Om)
    return z, theta * d_a_kpc, 1.0 / (4.0 * math.pi * d_l ** 2)
