"""Distance scalars: the oracle's flat Lambda-CDM distances against closed forms and a series,
and the library's host-side helper against the oracle."""
import math

import numpy as np
import pytest

from oracle import cosmology as OC
from paper_2412_08265_amd import ops
from paper_2412_08265_amd.cosmology import FlatLCDM, place_at_redshift

C = OC.C_KMS


@pytest.mark.parametrize("z", [0.01, 0.3, 1.0, 4.0])
def test_oracle_einstein_de_sitter_and_empty_closed_forms(z):
    # Om = 1: D_C = 2 (c/H0) (1 - 1/sqrt(1+z));  Om = 0 (E = 1): D_C = c z / H0
    assert abs(OC.comoving_distance_mpc(z, 70.0, 1.0)
               - 2 * C / 70.0 * (1 - 1 / math.sqrt(1 + z))) <= 1e-12 * C / 70.0
    assert abs(OC.comoving_distance_mpc(z, 67.0, 0.0) - C * z / 67.0) <= 1e-12 * C / 67.0 * z


def test_oracle_low_redshift_series():
    """D_L = (c/H0) (z + (1 - q0) z^2 / 2 + O(z^3)), q0 = Om/2 - (1 - Om) for flat LCDM."""
    Om = 0.3
    q0 = Om / 2 - (1 - Om)
    for z in (1e-3, 3e-3, 1e-2):
        series = C / 70.0 * (z + (1 - q0) * z * z / 2)
        assert abs(OC.luminosity_distance_mpc(z, 70.0, Om) - series) <= 2 * C / 70.0 * z ** 3


@pytest.mark.parametrize("Om", [0.3, 1.0, 0.05])
def test_library_distances_match_oracle(Om):
    cosmo = FlatLCDM(68.0, Om)
    for z in (1e-3, 0.02, 0.1, 1.0, 3.0):
        ref = OC.comoving_distance_mpc(z, 68.0, Om)
        assert abs(cosmo.comoving_distance_mpc(z) - ref) <= 1e-11 * ref
        assert abs(cosmo.luminosity_distance_mpc(z) - (1 + z) * ref) <= 1e-11 * (1 + z) * ref


def test_place_at_redshift_matches_oracle_scalars():
    obs = ops.Observation((0.5, 0.0, 0.0), 40, 40, 1.0, 4000.0, 1.25, 3000, flux_scale=2.0)
    z, arcsec = 0.03, 0.25
    placed = place_at_redshift(obs, z, arcsec)
    zs, s_kpc, fs = OC.observation_scalars(z, arcsec)
    assert placed.z_sys == zs
    assert abs(placed.spaxel_kpc - s_kpc) <= 1e-11 * s_kpc
    assert abs(placed.flux_scale - 2.0 * fs) <= 1e-11 * 2.0 * fs
    assert placed.nx == obs.nx and placed.angles_rad == obs.angles_rad
    with pytest.raises(ValueError):
        place_at_redshift(obs, 0.0, arcsec)
