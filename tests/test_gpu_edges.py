"""Degenerate and maximum-size cases of the forward path against the oracle: every particle in
one spaxel (dozens of work chunks and a long fixed-order combine), a 1x1 grid, a single
telescope bin, ages and metallicities on nodes and beyond the clamps, particles at rest, the
largest PSF/LSF radius, and a batch of the largest number of jobs."""
import math

import numpy as np
import pytest

import oracle as O
from helpers import TIES, WORKERS, assert_cube_in, assert_grads_in, gpu_forward, log
from paper_2412_08265_amd import synth

pytestmark = pytest.mark.gpu

f32 = lambda a: np.asarray(a, dtype=np.float32)


def _particles(n, seed, r=0.4, v=300.0, age=None, met=None):
    rng = np.random.default_rng(seed)
    return synth.Particles(f32(rng.uniform(-r, r, n)), f32(rng.uniform(-r, r, n)),
                           f32(rng.uniform(-1, 1, n)), f32(rng.normal(0, v, n)),
                           f32(rng.normal(0, v, n)), f32(rng.normal(0, v, n)),
                           f32(10 ** rng.uniform(4, 6, n)),
                           f32(rng.uniform(0.1, 13, n) if age is None else age),
                           f32(rng.uniform(-2, 0.3, n) if met is None else met))


def _run(w, tol=1e-5):
    _, g = gpu_forward(w)
    cfg = O.config_from_workload(w)
    fo = O.forward(w.particles, cfg, workers=WORKERS, ties=TIES)
    np.testing.assert_array_equal(g["key"], fo["key"])
    np.testing.assert_array_equal(g["perm"], fo["perm"])
    np.testing.assert_array_equal(g["seg_off"], fo["seg_off"])
    assert_cube_in(g["cube_raw"], fo, "cube_raw", tol, what=f"{w.name} cube_raw")
    assert_cube_in(g["cube"], fo, "cube", tol, what=f"{w.name} cube")
    return g, fo


def test_all_particles_in_one_spaxel():
    """60 000 particles in one 1 kpc spaxel of a 3x3 grid: 30 chunks of <= 2048 particles whose
    partial spectra are combined in chunk order."""
    p = _particles(60_000, 1, r=0.45)
    ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    w = synth.Workload("one-spaxel", p, (0.0, 0.0, 0.0), 3, 3, 1.0, ssp.lam_start, ssp.lam_step,
                       ssp.n_lam, ssp, psf_sigma_spx=0.8, lsf_sigma_A=9.0)
    g, fo = _run(w)
    cnt = np.diff(fo["seg_off"])
    assert cnt[4] == 60_000 and cnt.sum() == 60_000


def test_single_spaxel_grid_and_single_bin():
    p = _particles(3000, 2, r=0.7)
    ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    w = synth.Workload("1x1", p, (30.0, 10.0, 0.0), 1, 1, 1.0, 4000.3, 2.5, 700, ssp,
                       psf_sigma_spx=1.0, lsf_sigma_A=5.0)
    _run(w)
    w = synth.Workload("1-bin", p, (30.0, 10.0, 0.0), 4, 4, 0.5, 5000.7, 3.0, 1, ssp,
                       psf_sigma_spx=1.0)
    _run(w)


def test_ages_and_metallicities_on_nodes_and_beyond_clamps():
    ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    ages = np.concatenate([10.0 ** ssp.log_age_nodes.astype(np.float64),   # on the nodes
                           [0.01, 0.05, 50.0, 13.0, 0.1]])                 # past both clamps
    mets = np.concatenate([ssp.met_nodes.astype(np.float64), [-5.0, 3.0, -2.0, 0.3]])
    n = 4000
    rng = np.random.default_rng(3)
    age = rng.choice(ages, n)
    met = rng.choice(mets, n)
    p = _particles(n, 3, r=2.5, age=age, met=met)
    p = p.replace(vx=f32(np.where(np.arange(n) % 5 == 0, 0.0, p.vx)),
                  vy=f32(np.where(np.arange(n) % 5 == 0, 0.0, p.vy)),
                  vz=f32(np.where(np.arange(n) % 5 == 0, 0.0, p.vz)))   # some at rest
    w = synth.Workload("nodes", p, (45.0, 0.0, 0.0), 6, 6, 1.0, 3640.1, 6.3, 560, ssp,
                       psf_sigma_spx=0.7, lsf_sigma_A=8.0)
    _run(w)


def test_largest_psf_and_lsf_radius():
    """sigma giving radius int(4 sigma + 0.5) = 64 on both the spatial and the spectral axis."""
    p = _particles(20_000, 4, r=20.0)
    ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    sig = 15.9                       # int(4 * 15.9 + 0.5) = 64
    w = synth.Workload("r64", p, (50.0, 0.0, 0.0), 70, 66, 0.6, ssp.lam_start, ssp.lam_step,
                       ssp.n_lam, ssp, psf_sigma_spx=sig, lsf_sigma_A=sig * ssp.lam_step)
    assert int(4 * sig + 0.5) == 64
    _run(w)


def test_batch_of_the_largest_number_of_jobs():
    """64 jobs of different sizes, grids and telescope windows in one call of each entry point:
    every job equals its single-call result bitwise."""
    import torch
    from paper_2412_08265_amd import _lib, ops
    ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    dssp = ops.DeviceSSP.from_grid(ssp)
    rng = np.random.default_rng(9)
    gals, obss = [], []
    for k in range(_lib.RUBIX_MAX_JOBS):
        n = int(rng.integers(0, 3000))
        p = _particles(max(n, 1), 100 + k, r=3.0)
        p = p.subset(slice(0, n))
        gals.append(ops.DeviceGalaxy.from_host(p))
        side = int(rng.integers(1, 12))
        obss.append(ops.Observation((math.radians(rng.uniform(0, 90)), 0.0, 0.0), side, side,
                                    6.0 / side, 3600.0 + float(rng.uniform(0, 100)),
                                    float(rng.uniform(5.0, 9.0)), int(rng.integers(1, 400)),
                                    float(rng.uniform(0, 1.5)), float(rng.uniform(0, 12))))
    bufs = [ops.JobBuffers.allocate(g.n, o) for g, o in zip(gals, obss)]
    jobs = [ops.make_job(g, o, b) for g, o, b in zip(gals, obss, bufs)]
    ws = ops.workspace(ops.rubix_workspace_size(jobs, dssp))
    ops.rubix_rotate_bin(jobs, ws)
    ops.rubix_cube(jobs, dssp, ws)
    ops.rubix_psf_lsf(jobs, [b.cube_raw for b in bufs], [b.cube for b in bufs], ws)
    torch.cuda.synchronize()
    for k in range(0, 64, 7):
        one = ops.Forward(gals[k], obss[k], dssp)
        ref = one()
        torch.cuda.synchronize()
        assert torch.equal(ref.cube, bufs[k].cube), k
        assert torch.equal(ref.perm, bufs[k].perm), k
    log("64-job batch equals single calls")


@pytest.mark.parametrize("n_tel", [61, 62, 63, 247, 248, 249, 993])
def test_wave_and_tile_tails(n_tel):
    """Telescope grids whose last wave ends one bin short of, at and one past a wave's 62 bins,
    at a tile edge (248 bins) and past it; the longest grid also reaches the red end of the SSP
    grid, where waves leave the unchecked path."""
    p = _particles(5000, 40 + n_tel, r=0.9)
    ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    w = synth.Workload(f"tel{n_tel}", p, (20.0, 5.0, 0.0), 6, 5, 0.4, 3700.3, 3.7, n_tel, ssp,
                       psf_sigma_spx=0.9, lsf_sigma_A=4.0)
    log(f"wave/tile tails: n_tel={n_tel}")
    _run(w)


@pytest.mark.parametrize("n_tel", [1, 2, 59, 60, 61, 239, 240, 241, 993])
def test_bin_mean_wave_and_tile_tails(n_tel):
    """Bin-mean resampling on telescope grids of one and two bins, and on grids whose last wave
    ends one bin short of, at and one past a wave's 60 bins, at a tile edge (240 bins) and past
    it: the lanes share bin edges with their neighbours, and the last wave's edges are clamped
    to the band's end. Forward cube and the adjoint's gradients (seeded dL/dC_raw) against the
    oracle."""
    import torch
    from paper_2412_08265_amd import ops
    p = _particles(4000, 70 + n_tel, r=0.9)
    ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    w = synth.Workload(f"binmean-tel{n_tel}", p, (20.0, 5.0, 0.0), 6, 5, 0.4, 3700.3, 3.7, n_tel,
                       ssp, psf_sigma_spx=0.9, lsf_sigma_A=4.0, resample=1)
    log(f"bin-mean wave/tile tails: n_tel={n_tel}")
    _, fo = _run(w)
    cfg = O.config_from_workload(w)
    rng = np.random.default_rng(n_tel)
    G = rng.normal(size=(w.nx * w.ny, w.n_tel)).astype(np.float32)
    fw = ops.Forward(ops.DeviceGalaxy.from_host(w.particles), ops.Observation.from_workload(w),
                     ops.DeviceSSP.from_grid(w.ssp))
    fw()
    out = ops.cube_backward(fw, torch.from_numpy(G).cuda().reshape(w.ny, w.nx, w.n_tel))
    torch.cuda.synchronize()
    ref = O.adjoint(w.particles, cfg, G.astype(np.float64), fo, ties=TIES)
    assert_grads_in({k: out[k].cpu().numpy() for k in ("mass", "age", "met", "vlos")}, ref,
                    ("mass", "age", "met", "vlos"), 2e-5, f"bin-mean tel{n_tel}")


def test_non_finite_particle_values():
    """Non-finite particle values never reach memory out of range, and each has a fixed meaning:
    a position that is not finite leaves the field (keys, perm and seg_off exact against the
    oracle on the same input); a velocity that is not finite contributes nothing; a NaN age or
    [M/H] takes the first node (the cube equals the oracle's with those particles massless or
    below the first node); a NaN mass spoils only its own spaxel."""
    import torch
    n = 3000
    p = _particles(n, 5, r=0.9)
    x, y, vx, vz = p.x.copy(), p.y.copy(), p.vx.copy(), p.vz.copy()
    age, met, mass = p.age.copy(), p.met.copy(), p.mass.copy()
    rng = np.random.default_rng(9)
    idx = rng.permutation(n)
    x[idx[0:10]] = np.nan
    y[idx[10:20]] = np.inf
    vx[idx[20:30]] = np.nan
    vz[idx[30:40]] = -np.inf
    age[idx[40:50]] = np.nan
    met[idx[50:60]] = np.nan
    age[idx[60:65]] = np.inf
    met[idx[65:70]] = -np.inf
    bad = synth.Particles(x, y, p.z, vx, p.vy, vz, mass, age, met)
    ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    w = synth.Workload("non-finite", bad, (30.0, 20.0, 10.0), 8, 7, 0.3, 3650.3, 5.1, 611, ssp,
                       psf_sigma_spx=1.0, lsf_sigma_A=6.0)
    log("non-finite particle values")
    _, g = gpu_forward(w)
    cfg = O.config_from_workload(w)
    fo = O.forward(bad, cfg, with_cube=False)
    np.testing.assert_array_equal(g["key"], fo["key"])
    np.testing.assert_array_equal(g["perm"], fo["perm"])
    np.testing.assert_array_equal(g["seg_off"], fo["seg_off"])
    assert np.all(g["key"][idx[0:20]] == w.nx * w.ny)
    # the same cube from finite inputs: massless particles for non-finite velocities, ages and
    # metallicities below (or above) the grid for NaN (infinite) ones
    moving = np.isfinite(vx) & np.isfinite(vz)
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    fin = synth.Particles(x, y, p.z, f32(np.where(moving, vx, 0.0)), p.vy,
                          f32(np.where(moving, vz, 0.0)), f32(np.where(moving, mass, 0.0)),
                          f32(np.where(np.isnan(age), 1e-6, np.where(np.isinf(age), 1e3, age))),
                          f32(np.where(np.isfinite(met), met, -50.0)))
    ref = O.forward(fin, cfg, ties=TIES)
    assert np.all(np.isfinite(g["cube_raw"]))
    assert_cube_in(g["cube_raw"], ref, "cube_raw", what="non-finite cube_raw")
    assert_cube_in(g["cube"], ref, "cube", what="non-finite cube")
    # a NaN mass: its spaxel's voxels reached by the spectrum are NaN, every other spaxel finite
    i0 = int(np.flatnonzero(fo["key"] < w.nx * w.ny)[0])
    mass2 = mass.copy()
    mass2[i0] = np.nan
    w2 = synth.Workload("nan-mass", synth.Particles(x, y, p.z, vx, p.vy, vz, mass2, age, met),
                        w.angles_deg, w.nx, w.ny, w.spaxel_kpc, w.tel_start, w.tel_step, w.n_tel,
                        ssp)
    _, g2 = gpu_forward(w2)
    raw = g2["cube_raw"].reshape(w.ny * w.nx, w.n_tel)
    s0 = int(fo["key"][i0])
    assert np.isnan(raw[s0]).any()
    others = np.delete(raw, s0, axis=0)
    assert np.all(np.isfinite(others))
    np.testing.assert_array_equal(others, np.delete(g["cube_raw"].reshape(w.ny * w.nx, w.n_tel), s0, axis=0))


@pytest.mark.parametrize("grids,resample", [("linear", 0), ("linear", 1), ("log", 0),
                                             ("log", 1)])
def test_non_finite_velocities_forward_and_adjoint(grids, resample):
    """Particles whose velocity is not finite add nothing and carry no gradient, in every
    resampling mode and grid kind: the cube equals the oracle's with those particles massless
    and at rest, every voxel and gradient is finite, their own gradients are exactly zero, the
    others' gradients and the angle gradients match the oracle's on that finite input."""
    import torch
    from paper_2412_08265_amd import ops
    n = 3000
    p = _particles(n, 15, r=0.9)
    vx, vz, mass = p.vx.copy(), p.vz.copy(), p.mass.copy()
    rng = np.random.default_rng(19)
    idx = rng.permutation(n)
    vx[idx[0:12]] = np.nan
    vz[idx[12:24]] = np.inf
    vz[idx[24:30]] = -np.inf
    bad = synth.Particles(p.x, p.y, p.z, vx, p.vy, vz, mass, p.age, p.met)
    moving = np.isfinite(vx) & np.isfinite(vz)
    fin = synth.Particles(p.x, p.y, p.z, f32(np.where(moving, vx, 0.0)), p.vy,
                          f32(np.where(moving, vz, 0.0)), f32(np.where(moving, mass, 0.0)),
                          p.age, p.met)
    if grids == "log":
        ssp = synth.cached_ssp(8, 5, 3600.0, 2.0e-3, 500, log_lambda=True)
        tel = (3600.0 * math.exp(-3 * 1.7e-3), 1.7e-3, 620)
    else:
        ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
        tel = (3650.3, 5.1, 611)
    w = synth.Workload(f"non-finite-v-{grids}-{resample}", bad, (30.0, 20.0, 10.0), 8, 7, 0.3,
                       tel[0], tel[1], tel[2], ssp, psf_sigma_spx=1.0, lsf_sigma_A=6.0,
                       log_lambda=grids == "log", resample=resample)
    log(f"non-finite velocities: {grids} grids, resample={resample}")
    _, g = gpu_forward(w)
    assert np.all(np.isfinite(g["cube_raw"])) and np.all(np.isfinite(g["cube"]))
    wf = synth.Workload(w.name, fin, w.angles_deg, w.nx, w.ny, w.spaxel_kpc, w.tel_start,
                        w.tel_step, w.n_tel, ssp, w.psf_sigma_spx, w.lsf_sigma_A,
                        log_lambda=w.log_lambda, resample=resample)
    cfg = O.config_from_workload(wf)
    fo = O.forward(fin, cfg, ties=TIES)
    assert_cube_in(g["cube_raw"], fo, "cube_raw", what="non-finite-v cube_raw")
    assert_cube_in(g["cube"], fo, "cube", what="non-finite-v cube")
    # adjoint with a seeded dL/dC_raw
    G = rng.normal(size=(w.nx * w.ny, w.n_tel)).astype(np.float32)
    fw = ops.Forward(ops.DeviceGalaxy.from_host(bad), ops.Observation.from_workload(w),
                     ops.DeviceSSP.from_grid(ssp))
    fw()
    out = ops.cube_backward(fw, torch.from_numpy(G).cuda().reshape(w.ny, w.nx, w.n_tel))
    torch.cuda.synchronize()
    gg = {k: v.cpu().numpy() for k, v in out.items()}
    keys = ("mass", "age", "met", "vlos")
    for k in keys:
        assert np.all(np.isfinite(gg[k])), k
        assert np.all(gg[k][~moving] == 0.0), k
    assert np.all(np.isfinite(gg["angles"]))
    ref = O.adjoint(fin, cfg, G.astype(np.float64), fo, ties=TIES)
    sel = np.flatnonzero(moving)
    assert_grads_in({k: gg[k][sel] for k in keys},
                    {**{k: ref[k][sel] for k in keys},
                     **{f"{k}_{e}": ref[f"{k}_{e}"][sel] for k in keys for e in ("lo", "hi")}},
                    keys, 2e-5, f"non-finite-v {grids} resample={resample}")
    a = np.asarray(gg["angles"])
    err = np.maximum(np.maximum(ref["angles_lo"][:2] - a[:2], a[:2] - ref["angles_hi"][:2]), 0)
    assert err.max() <= 2e-5 * np.abs(ref["angles"][:2]).max()


@pytest.mark.parametrize("ratio", [1.6, 3.0])
def test_telescope_bins_coarser_than_the_ssp_nodes(ratio):
    """Telescope bins wider than the SSP node spacing: no particle's span fits a wave window, so
    every bin gathers its taps directly; the grid runs past both ends of the SSP grid."""
    p = _particles(4000, 70, r=0.9, v=400.0)
    ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    step = ratio * ssp.lam_step
    n_tel = int((ssp.lam_start + ssp.lam_step * (ssp.n_lam - 1) + 40.0 - 3560.0) / step)
    w = synth.Workload(f"coarse-{ratio}", p, (40.0, 15.0, 5.0), 9, 8, 0.25, 3560.0, step, n_tel,
                       ssp, psf_sigma_spx=0.8, lsf_sigma_A=1.5 * step)
    log(f"coarse telescope grid: step {step:.3f} A, {n_tel} bins")
    _run(w)
