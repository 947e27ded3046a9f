"""Parity of the HIP forward path (through the C ABI) with the FP64 oracle on the same seeded
inputs: spaxel keys, permutation and segment offsets bit-exact; vlos bit-exact (FP64 rounded to
FP32 on both sides); cube voxels within 1e-5 of the cube's maximum."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2412_08265_amd import synth
from tests.helpers import (TIES, WORKERS, assert_cube_close, assert_cube_in, gpu_forward, log,
                           oracle_final_window, oracle_rows_parallel, outside)

pytestmark = pytest.mark.gpu


def _check_rotate_bin(w, g, fo=None):
    cfg = O.config_from_workload(w)
    fo = fo or O.forward(w.particles, cfg, with_cube=False)
    np.testing.assert_array_equal(g["key"], fo["key"])
    np.testing.assert_array_equal(g["perm"], fo["perm"])
    np.testing.assert_array_equal(g["seg_off"], fo["seg_off"])
    np.testing.assert_array_equal(g["vlos"], fo["vlos"].astype(np.float32))
    return fo


def _workload(p, nx=12, ny=10, s=0.75, angles=(60.0, 0.0, 0.0), ssp=None, tel=None,
              psf=0.0, lsf=0.0, name="custom"):
    ssp = ssp or synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    tel = tel or (ssp.lam_start, ssp.lam_step, ssp.n_lam)
    return synth.Workload(name, p, angles, nx, ny, s, tel[0], tel[1], tel[2], ssp, psf, lsf)


def test_tiny_forward_matches_oracle():
    w = synth.tiny_workload()
    log("tiny: 1000 particles, 16x16x500")
    _, g = gpu_forward(w)
    cfg = O.config_from_workload(w)
    fo = O.forward(w.particles, cfg, ties=TIES)
    _check_rotate_bin(w, g, fo)
    assert_cube_in(g["cube_raw"], fo, "cube_raw", what="tiny cube_raw")
    assert_cube_in(g["cube"], fo, "cube", what="tiny cube")


@pytest.mark.parametrize("n", [0, 1, 63, 4095, 4096, 4097, 20011])
def test_ragged_particle_counts(n):
    p = synth.make_galaxy(max(n, 1), seed=100 + n).subset(slice(0, n))
    w = _workload(p, tel=(3650.3, 5.1, 611), psf=1.3, lsf=6.0)
    log(f"ragged n={n}")
    _, g = gpu_forward(w)
    cfg = O.config_from_workload(w)
    fo = O.forward(p, cfg, ties=TIES)
    _check_rotate_bin(w, g, fo)
    if n == 0:
        assert np.all(g["cube_raw"] == 0) and np.all(g["cube"] == 0)
    else:
        assert_cube_in(g["cube_raw"], fo, "cube_raw", what=f"n={n} cube_raw")
        assert_cube_in(g["cube"], fo, "cube", what=f"n={n} cube")


def test_edge_particles_and_outside_field():
    """Particles exactly on spaxel edges and on the field border (power-of-two spaxels so the
    edges are exact), plus particles far outside."""
    nx, ny, s = 8, 6, 0.5
    ex = (np.arange(nx + 1) - nx / 2.0) * s
    ey = (np.arange(ny + 1) - ny / 2.0) * s
    xs, ys = np.meshgrid(ex, ey)
    xs, ys = xs.ravel(), ys.ravel()
    xs = np.concatenate([xs, np.nextafter(xs.astype(np.float32), np.float32(-np.inf)), [1e3, -1e3]])
    ys = np.concatenate([ys, np.nextafter(ys.astype(np.float32), np.float32(np.inf)), [0, 0]])
    n = xs.size
    rng = np.random.default_rng(0)
    f = lambda a: np.asarray(a, dtype=np.float32)
    p = synth.Particles(f(xs), f(ys), f(np.zeros(n)), f(rng.normal(0, 100, n)),
                        f(rng.normal(0, 100, n)), f(rng.normal(0, 100, n)),
                        f(10 ** rng.uniform(4, 6, n)), f(rng.uniform(0.1, 13, n)),
                        f(rng.uniform(-2, 0.3, n)))
    w = _workload(p, nx=nx, ny=ny, s=s, angles=(0.0, 0.0, 0.0))
    _, g = gpu_forward(w)
    fo = _check_rotate_bin(w, g)
    assert (fo["key"] == nx * ny).sum() >= nx + ny
    assert_cube_in(g["cube_raw"], O.forward(p, O.config_from_workload(w), ties=TIES), "cube_raw",
                   what="edge cube_raw")


def test_three_pass_sort_large_grid():
    """300 x 300 spaxels: keys need 17 bits, i.e. three 8-bit radix passes."""
    p = synth.make_galaxy(200_000, seed=77)
    ssp = synth.cached_ssp(4, 3, 5000.0, 10.0, 40)
    w = _workload(p, nx=300, ny=300, s=0.1, ssp=ssp)
    log("300x300 grid, 2e5 particles")
    _, g = gpu_forward(w)
    _check_rotate_bin(w, g)


def test_sparse_grid_record_blocks_span_many_spaxels():
    """300 x 300 spaxels of 0.1 kpc over a 1e5-particle galaxy: in the outskirts a block of 1024
    sorted particles spans thousands of spaxels, most of them empty, so the record builder's
    spaxel of each position (from the segment offsets) walks many segment starts per thread."""
    p = synth.make_galaxy(100_000, seed=78)
    w = _workload(p, nx=300, ny=300, s=0.1)
    cfg = O.config_from_workload(w)
    fo = O.forward(p, cfg, ties=TIES)
    n_in = int(fo["seg_off"][-1])
    ks = fo["key"][fo["perm"][:n_in]]
    spans = [int(ks[min(p0 + 1023, n_in - 1)] - ks[p0] + 1) for p0 in range(0, n_in, 1024)]
    assert max(spans) > 4096 and sum(sp > 256 for sp in spans) >= 16, spans
    log(f"sparse 300x300 grid: {n_in} in field, largest block span {max(spans)} spaxels")
    _, g = gpu_forward(w)
    _check_rotate_bin(w, g, fo)
    assert_cube_in(g["cube_raw"], fo, "cube_raw", what="sparse-grid cube_raw")


def test_medium_full_size_matches_oracle():
    """The 1e6-particle workload (50x50x3000, SSP 100x12x3000, PSF 1.5 spx, LSF 2.5 A) in full."""
    w = synth.medium_workload()
    log("medium: GPU forward")
    _, g = gpu_forward(w)
    cfg = O.config_from_workload(w)
    log(f"medium: oracle forward on {WORKERS} workers")
    fo = O.forward(w.particles, cfg, workers=WORKERS, ties=TIES)
    log("medium: compare")
    _check_rotate_bin(w, g, fo)
    assert_cube_in(g["cube_raw"], fo, "cube_raw", what="medium cube_raw")
    assert_cube_in(g["cube"], fo, "cube", what="medium cube")


def _full_size_sampled(w, tag, n_heavy=16, n_rand=256, windows=("blue", "mid", "red"), width=64):
    """Full-size parity on what the oracle can compute in seconds:
      * keys, perm and seg_off in full, bit-exact;
      * C_raw rows of the n_heavy heaviest spaxels, of two spaxels split into exactly 2 work
        chunks and of n_rand random non-empty ones, in full along lambda, within 1e-5 of the
        sampled rows' maximum of the oracle's range (tie bounds);
      * the final cube (after LSF and PSF) of every spaxel on windows of `width` bins (the blue
        end of the band, a seeded interior window and/or the red end), from the oracle's C_raw of
        all spaxels on each window widened by the LSF radius, within 1e-5 of the window's
        maximum;
      * empty spaxels zero and the cube non-negative everywhere."""
    log(f"{tag}: GPU forward")
    _, g = gpu_forward(w)
    cfg = O.config_from_workload(w)
    log(f"{tag}: oracle rotate/bin")
    fo = O.forward(w.particles, cfg, with_cube=False)
    _check_rotate_bin(w, g, fo)
    cnt = np.diff(fo["seg_off"])
    order = np.argsort(-cnt, kind="stable")
    two = np.flatnonzero((cnt > 2048) & (cnt <= 4096))[:2]
    rng = np.random.default_rng(3)
    nonempty = np.flatnonzero(cnt > 0)
    rand = rng.choice(nonempty, min(n_rand, nonempty.size), replace=False)
    spx = list(dict.fromkeys([int(s) for s in np.r_[order[:n_heavy], two, rand]]))
    log(f"{tag}: oracle rows for {len(spx)} spaxels (max count {cnt[spx].max()})")
    ref, lo, hi, nt = oracle_rows_parallel(w.particles, cfg, fo, spx, ties=TIES)
    got = g["cube_raw"][spx]
    scale = np.abs(ref).max()
    err = outside(got, lo, hi).max(axis=1) / scale
    plain = np.abs(got - ref).max(axis=1) / scale
    log(f"{tag}: worst sampled row distance from the oracle's range {err.max():.3e} "
        f"(vs FP64 value {plain.max():.3e}; {nt} tied pairs; scale = sampled max)")
    assert err.max() <= 1e-5
    starts = {"blue": 0, "mid": int(rng.integers(width, w.n_tel - 2 * width)),
              "red": w.n_tel - width}
    for j0 in (starts[k] for k in windows):
        j1 = j0 + width
        log(f"{tag}: oracle final cube of all spaxels on bins {j0}..{j1 - 1}")
        fin, flo, fhi, ft = oracle_final_window(w.particles, cfg, fo, j0, j1, ties=TIES)
        gw = g["cube"][:, j0:j1]
        e = outside(gw, flo, fhi).max() / np.abs(fin).max()
        log(f"{tag}: final cube bins {j0}..{j1 - 1}: max distance from the oracle's range "
            f"{e:.3e} (vs FP64 value {np.abs(gw - fin).max() / np.abs(fin).max():.3e}; "
            f"{ft} tied pairs)")
        assert e <= 1e-5
    # properties at full size: empty spaxels are zero, cube is non-negative (templates > 0)
    assert np.all(g["cube_raw"][cnt == 0] == 0)
    assert g["cube_raw"].min() >= 0


def test_large_full_size_sampled_spaxels():
    """The 1e7-particle workload (150x150x4563) at bin-centre sampling on linear grids."""
    _full_size_sampled(synth.large_workload(), "large")


@pytest.mark.parametrize("variant", ["binmean", "loglam", "binmeanlog"])
def test_large_full_size_sampled_spaxels_variants(variant):
    """The same 1e7-particle galaxy as timed by the bench's other variants: bin-mean resampling
    on linear grids, bin centres on grids uniform in ln(lambda), and bin means on those."""
    w = synth.large_log_workload() if variant in ("loglam", "binmeanlog") else synth.large_workload()
    if variant.startswith("binmean"):
        w.resample = 1
    end = {"binmean": "red", "loglam": "blue", "binmeanlog": "red"}[variant]
    _full_size_sampled(w, f"large {variant}", windows=(end, "mid"))


def test_large_one_kpc_spaxels_stress():
    """The 1e7-particle galaxy on 1-kpc spaxels (150 kpc field): nearly every particle in the
    field and the central spaxel holding ~3.7e5 of them (~180 work chunks combined in one
    spaxel); sampled rows include the heaviest spaxels."""
    w = synth.large_workload(spaxel_kpc=1.0)
    _full_size_sampled(w, "large 1-kpc", n_heavy=4, n_rand=128, windows=("mid",))


def test_deterministic_and_linear_in_mass():
    w = synth.medium_workload(n=200_000)
    _, g1 = gpu_forward(w)
    _, g2 = gpu_forward(w)
    np.testing.assert_array_equal(g1["cube_raw"], g2["cube_raw"])
    np.testing.assert_array_equal(g1["cube"], g2["cube"])
    p2 = w.particles.replace(mass=w.particles.mass.astype(np.float64) * 2.0)
    w2 = synth.Workload(w.name, p2, w.angles_deg, w.nx, w.ny, w.spaxel_kpc, w.tel_start,
                        w.tel_step, w.n_tel, w.ssp, w.psf_sigma_spx, w.lsf_sigma_A)
    _, g3 = gpu_forward(w2)
    np.testing.assert_array_equal(g3["cube_raw"], 2 * g1["cube_raw"])


def test_psf_lsf_on_seeded_random_cube():
    """rubix_psf_lsf alone on a seeded random cube vs the oracle's convolution."""
    import torch
    from paper_2412_08265_amd import ops
    rng = np.random.default_rng(11)
    for (ny, nx, nl, psf, lsf, step) in [(37, 45, 700, 2.0, 2.7, 1.25), (5, 300, 130, 0.7, 0.0, 1.0),
                                         (150, 9, 257, 0.0, 15.0, 1.25), (3, 4, 50, 0.0, 0.0, 1.0)]:
        c = rng.normal(size=(ny, nx, nl)).astype(np.float32)
        obs = ops.Observation((0, 0, 0), nx, ny, 1.0, 5000.0, step, nl, psf, lsf)
        buf = ops.JobBuffers.allocate(0, obs)
        gal = ops.DeviceGalaxy({f: torch.empty(0, dtype=torch.float32, device="cuda")
                                for f in ops.FIELDS})
        job = ops.make_job(gal, obs, buf)
        ws = ops.workspace(ops.rubix_workspace_size([job]))
        cin = torch.from_numpy(c).cuda()
        cout = torch.empty_like(cin)
        ops.rubix_psf_lsf([job], [cin], [cout], ws)
        torch.cuda.synchronize()
        ssp = synth.cached_ssp(3, 3, 5000.0, step, 10)
        cfg = O.OracleConfig((0, 0, 0), nx, ny, 1.0, 5000.0, step, nl, ssp.log_age_nodes,
                             ssp.met_nodes, ssp.lam_start, ssp.lam_step, ssp.flux, psf, lsf)
        ref = O.psf_lsf(c.reshape(ny * nx, nl).astype(np.float64), cfg)
        assert_cube_close(cout.cpu().numpy().reshape(ny * nx, nl), ref, tol=2e-6,
                          what=f"psf/lsf {ny}x{nx}x{nl} psf={psf} lsf={lsf}")


# (ny, nx, n_tel, PSF sigma [spaxels], LSF sigma [bins]): radii int(4 sigma + 0.5) on both sides
# of the fused pass's bounds (PSF 1..8, LSF 0..22), grids smaller than its tiles and its PSF
# radius, and grids of several tiles with ragged x and lambda tails
FUSED_CASES = [(1, 1, 1, 0.3, 0.3), (2, 150, 64, 2.0, 2.16), (7, 17, 65, 1.0, 5.4),
               (7, 17, 65, 1.0, 5.7), (9, 33, 129, 2.1, 1.0), (9, 33, 129, 2.2, 1.0),
               (40, 50, 300, 1.5, 0.0), (23, 16, 640, 0.2, 3.0)]


@pytest.mark.parametrize("ny,nx,nl,psf,lsf_bins", FUSED_CASES)
def test_psf_lsf_fused_pass_bounds_and_tails(ny, nx, nl, psf, lsf_bins):
    """The PSF+LSF operator on a seeded random cube vs the oracle's convolution, for radii inside
    and just outside the range of the fused pass (the three 1-D passes take the others)."""
    import torch
    from paper_2412_08265_amd import ops
    rng = np.random.default_rng(ny * 1000 + nx + nl)
    step = 1.25
    c = rng.normal(size=(ny, nx, nl)).astype(np.float32)
    obs = ops.Observation((0, 0, 0), nx, ny, 1.0, 5000.0, step, nl, psf, lsf_bins * step)
    buf = ops.JobBuffers.allocate(0, obs)
    gal = ops.DeviceGalaxy({f: torch.empty(0, dtype=torch.float32, device="cuda")
                            for f in ops.FIELDS})
    job = ops.make_job(gal, obs, buf)
    ws = ops.workspace(ops.rubix_workspace_size([job]))
    cin = torch.from_numpy(c).cuda()
    cout = torch.full_like(cin, float("nan"))
    log(f"psf/lsf {ny}x{nx}x{nl} psf={psf} lsf={lsf_bins} bins")
    ops.rubix_psf_lsf([job], [cin], [cout], ws)
    torch.cuda.synchronize()
    ssp = synth.cached_ssp(3, 3, 5000.0, step, 10)
    cfg = O.OracleConfig((0, 0, 0), nx, ny, 1.0, 5000.0, step, nl, ssp.log_age_nodes,
                         ssp.met_nodes, ssp.lam_start, ssp.lam_step, ssp.flux, psf,
                         lsf_bins * step)
    ref = O.psf_lsf(c.reshape(ny * nx, nl).astype(np.float64), cfg)
    assert_cube_close(cout.cpu().numpy().reshape(ny * nx, nl), ref, tol=2e-6,
                      what=f"psf/lsf {ny}x{nx}x{nl} psf={psf} lsf={lsf_bins} bins")


def test_batch_equals_single_calls():
    """Jobs batched into one call give bitwise the results of separate calls."""
    import torch
    from paper_2412_08265_amd import ops
    ws_list = [synth.medium_workload(n=30_000 + 7000 * k, seed=50 + k) for k in range(3)]
    ws_list[1] = synth.Workload("b", ws_list[1].particles, (30.0, 10.0, 5.0), 21, 17, 1.7,
                                3700.0, 2.5, 1111, ws_list[1].ssp, 0.0, 4.0)
    ssp = ops.DeviceSSP.from_grid(ws_list[0].ssp)
    singles = [gpu_forward(w)[1] for w in ws_list]
    gals = [ops.DeviceGalaxy.from_host(w.particles) for w in ws_list]
    obss = [ops.Observation.from_workload(w) for w in ws_list]
    bufs = [ops.JobBuffers.allocate(g.n, o) for g, o in zip(gals, obss)]
    jobs = [ops.make_job(g, o, b) for g, o, b in zip(gals, obss, bufs)]
    ws = ops.workspace(ops.rubix_workspace_size(jobs, ssp))
    ops.rubix_rotate_bin(jobs, ws)
    ops.rubix_cube(jobs, ssp, ws)
    ops.rubix_psf_lsf(jobs, [b.cube_raw for b in bufs], [b.cube for b in bufs], ws)
    torch.cuda.synchronize()
    for s, b in zip(singles, bufs):
        np.testing.assert_array_equal(s["perm"], b.perm.cpu().numpy())
        np.testing.assert_array_equal(s["cube_raw"].ravel(), b.cube_raw.cpu().numpy().ravel())
        np.testing.assert_array_equal(s["cube"].ravel(), b.cube.cpu().numpy().ravel())


def test_shifted_line_and_rest_frame_invariants():
    """Single particles: at rest the cube is m * template (identical grids); a narrow line moves
    to lam (1 + v/c); total flux is conserved within the bound the oracle pins."""
    import torch
    ssp = synth.make_line_ssp(5000.0, 0.5, 4000, 6000.0, 0.6)
    f = lambda a: np.asarray(a, dtype=np.float32)
    for v in (0.0, 250.0, -420.0):
        p = synth.Particles(f([0.1]), f([0.1]), f([0]), f([0]), f([0]), f([v]), f([3.0]),
                            f([2.0]), f([-0.5]))
        w = _workload(p, nx=2, ny=2, s=1.0, angles=(0.0, 0.0, 0.0), ssp=ssp)
        _, g = gpu_forward(w)
        spec = g["cube_raw"][g["key"][0]]
        lam = 5000.0 + 0.5 * np.arange(4000)
        expect = 6000.0 * (1 + v / O.C_KMS)
        assert abs(lam[np.argmax(spec)] - expect) <= 0.25 + 1e-6
        if v == 0.0:
            np.testing.assert_allclose(spec, 3.0 * ssp.flux[0, 0].astype(np.float64),
                                       rtol=2e-6, atol=1e-6 * ssp.flux.max() * 3)
        else:
            S = ssp.flux[0, 0].astype(np.float64)
            beta = v / O.C_KMS
            bound = 2 * abs(beta) * S.max() / S.sum() + 4 * beta * beta
            assert abs(spec.sum() - 3.0 * S.sum()) / (3.0 * S.sum()) <= bound + 1e-6


def test_first_ssp_cell_with_window_before_node_zero():
    """Regression: particles in the first SSP cell (youngest age, lowest [M/H]) moving away, on
    identical grids, so that the staged node window of the first bins starts before node 0 of the
    first template row. Enough particles per spaxel for the grouped path and a ragged tail."""
    rng = np.random.default_rng(21)
    n = 4 * 37 + 3
    f = lambda a: np.asarray(a, dtype=np.float32)
    ssp = synth.cached_ssp(8, 5, 3600.0, 7.615230460921844, 500)
    age0 = float(10 ** ssp.log_age_nodes[0])
    p = synth.Particles(f(rng.uniform(-0.4, 0.4, n)), f(rng.uniform(-0.4, 0.4, n)), f(np.zeros(n)),
                        f(np.zeros(n)), f(np.zeros(n)), f(rng.uniform(50, 900, n)),
                        f(10 ** rng.uniform(4, 6, n)),
                        f(np.where(np.arange(n) % 2 == 0, age0, age0 * 1.01)),
                        f(np.where(np.arange(n) % 3 == 0, ssp.met_nodes[0], -1.95)))
    w = _workload(p, nx=2, ny=2, s=0.5, angles=(0.0, 0.0, 0.0), ssp=ssp)
    _, g = gpu_forward(w)
    fo = O.forward(p, O.config_from_workload(w), ties=TIES)
    assert_cube_in(g["cube_raw"], fo, "cube_raw", what="first-cell cube_raw")
    # the blue end is where the missing light showed up
    ref = fo["cube_raw"][:, :64]
    assert np.abs(g["cube_raw"][:, :64] - ref).max() <= 1e-5 * np.abs(fo["cube_raw"]).max()


def test_log_grid_forward_matches_oracle():
    """Both wavelength grids uniform in ln(lambda) (Doppler shift = index shift), telescope grid
    offset from and finer than the SSP grid, systemic redshift, PSF and LSF."""
    w = synth.log_workload()
    log(f"log grids: {w.particles.n} particles, {w.nx}x{w.ny}x{w.n_tel}")
    _, g = gpu_forward(w)
    cfg = O.config_from_workload(w)
    fo = O.forward(w.particles, cfg, workers=WORKERS, ties=TIES)
    _check_rotate_bin(w, g, fo)
    assert_cube_in(g["cube_raw"], fo, "cube_raw", what="log-grid cube_raw")
    assert_cube_in(g["cube"], fo, "cube", what="log-grid cube")


def test_grid_kinds_must_match():
    from paper_2412_08265_amd import _lib, ops
    w = synth.log_workload(n=1000)
    gal = ops.DeviceGalaxy.from_host(w.particles)
    ssp = ops.DeviceSSP.from_grid(w.ssp)
    obs = ops.Observation.from_workload(w)
    obs.log_lambda = False
    obs.lsf_sigma_A = 0.0           # (1.2 A would be 12000 bins of a linear 1e-4 A step)
    with pytest.raises(_lib.RubixError) as e:
        ops.Forward(gal, obs, ssp)()
    assert e.value.code == _lib.RUBIX_EINVAL


def _bin_mean_workload(n=200_000, seed=6):
    """Bin-mean (flux-conserving) resampling on a telescope grid offset from and coarser than
    the SSP grid (1.37 A bins over 1.2671 A nodes), PSF and LSF."""
    p = synth.make_galaxy(n, seed)
    step = (7400.0 - 3600.0) / 2999.0
    ssp = synth.cached_ssp(40, 8, 3600.0, step, 3000)
    return synth.Workload("binmean-2e5", p, (60.0, 0.0, 0.0), 30, 30, 1.0, 3611.3, 1.37, 2700,
                          ssp, psf_sigma_spx=1.0, lsf_sigma_A=2.0, z_sys=0.001, resample=1)


def test_bin_mean_resampling_matches_oracle():
    w = _bin_mean_workload()
    log(f"bin mean: {w.particles.n} particles, {w.nx}x{w.ny}x{w.n_tel}")
    _, g = gpu_forward(w)
    cfg = O.config_from_workload(w)
    fo = O.forward(w.particles, cfg, workers=WORKERS, ties=TIES)
    _check_rotate_bin(w, g, fo)
    assert_cube_in(g["cube_raw"], fo, "cube_raw", what="bin-mean cube_raw")
    assert_cube_in(g["cube"], fo, "cube", what="bin-mean cube")


def test_bin_mean_conserves_flux_and_mixes_with_centre_sampling():
    """Line templates, particles moving at up to 600 km/s: sum_j C_raw[s, j] dlam equals
    sum_i fs m_i dlam_ssp (trapezoid sum of the line) for every spaxel (FP32 accumulation).
    A batch holding a bin-mean job and a bin-centre job gives each job's single-call cube."""
    import torch
    from paper_2412_08265_amd import ops
    rng = np.random.default_rng(12)
    n = 5000
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    p = synth.Particles(f32(rng.uniform(-3, 3, n)), f32(rng.uniform(-3, 3, n)),
                        f32(np.zeros(n)), f32(np.zeros(n)), f32(np.zeros(n)),
                        f32(rng.uniform(-600, 600, n)), f32(10 ** rng.uniform(4, 6, n)),
                        f32(rng.uniform(0.2, 12, n)), f32(rng.uniform(-1.9, 0.2, n)))
    ssp = synth.make_line_ssp(5000.0, 1.0, 2000, 6000.0, 3.0, n_age=3, n_met=3)
    line = ssp.flux[0, 0].astype(np.float64)
    wb = synth.Workload("flux", p, (0.0, 0.0, 0.0), 6, 6, 1.0, 5003.7, 1.3, 1500, ssp,
                        resample=1)
    fw_b, gb = gpu_forward(wb)
    key = gb["key"]
    tot = np.zeros(36)
    np.add.at(tot, key[key < 36], p.mass[key < 36].astype(np.float64))
    expect = tot * np.sum(0.5 * (line[:-1] + line[1:]))
    got = gb["cube_raw"].astype(np.float64).sum(axis=1) * wb.tel_step
    assert np.abs(got - expect).max() <= 1e-5 * expect.max(), np.abs(got - expect).max()
    # mixed batch
    wa = synth.Workload("flux-a", p, (0.0, 0.0, 0.0), 6, 6, 1.0, 5003.7, 1.3, 1500, ssp)
    _, ga = gpu_forward(wa)
    dssp = ops.DeviceSSP.from_grid(ssp)
    gal = ops.DeviceGalaxy.from_host(p)
    bufs, jobs = [], []
    for w in (wb, wa):
        obs = ops.Observation.from_workload(w)
        b = ops.JobBuffers.allocate(gal.n, obs)
        bufs.append(b)
        jobs.append(ops.make_job(gal, obs, b))
    ws = ops.workspace(ops.rubix_workspace_size(jobs, dssp))
    ops.rubix_rotate_bin(jobs, ws)
    ops.rubix_cube(jobs, dssp, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(bufs[0].cube_raw.cpu().numpy().reshape(36, -1), gb["cube_raw"])
    np.testing.assert_array_equal(bufs[1].cube_raw.cpu().numpy().reshape(36, -1), ga["cube_raw"])


@pytest.mark.parametrize("tel_step,n_tel", [(1.0e-4, 3700), (1.9e-4, 1950), (0.55e-4, 6700)])
def test_log_grid_bin_mean_matches_oracle(tel_step, n_tel):
    """Bin-mean resampling on grids uniform in ln(lambda): each segment's integral over rest
    wavelength carries its exponential weight, and each bin is divided by its width. Telescope
    bins finer than, coarser than (several segments per bin) and about half the SSP nodes;
    systemic redshift; the band reaching past the SSP grid's red end."""
    import dataclasses
    w = dataclasses.replace(synth.log_workload(n=60_000), tel_step=tel_step, n_tel=n_tel,
                            resample=1, name=f"binmean-log-{tel_step:g}")
    log(f"log-grid bin mean: {w.nx}x{w.ny}x{w.n_tel}, step {tel_step:g}")
    _, g = gpu_forward(w)
    cfg = O.config_from_workload(w)
    fo = O.forward(w.particles, cfg, workers=WORKERS, ties=TIES)
    _check_rotate_bin(w, g, fo)
    assert_cube_in(g["cube_raw"], fo, "cube_raw", what="log bin-mean cube_raw")
    assert_cube_in(g["cube"], fo, "cube", what="log bin-mean cube")


def test_log_grid_bin_mean_conserves_flux():
    """Line templates on log grids, particles moving at up to 600 km/s: sum_j C_raw[s, j] dlam_j
    equals sum_i fs m_i x the line's integral over wavelength for every spaxel (FP32 sums)."""
    rng = np.random.default_rng(13)
    n = 5000
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    p = synth.Particles(f32(rng.uniform(-3, 3, n)), f32(rng.uniform(-3, 3, n)),
                        f32(np.zeros(n)), f32(np.zeros(n)), f32(np.zeros(n)),
                        f32(rng.uniform(-600, 600, n)), f32(10 ** rng.uniform(4, 6, n)),
                        f32(rng.uniform(0.2, 12, n)), f32(rng.uniform(-1.9, 0.2, n)))
    ssp = synth.make_line_ssp(5000.0, 2.0e-4, 2000, 5600.0, 3.0, n_age=3, n_met=3,
                              log_lambda=True)
    cfg_line = O.OracleConfig((0.0, 0.0, 0.0), 1, 1, 1.0, 5003.7, 2.6e-4, 1500,
                              ssp.log_age_nodes, ssp.met_nodes, ssp.lam_start, ssp.lam_step,
                              ssp.flux, log_lambda=True, resample=1)
    line = ssp.flux[0, 0].astype(np.float64)[None, :]
    integral = O.integral_log_weighted(line, np.array([[0.0]]), np.array([[ssp.n_lam - 1.0]]),
                                       ssp.lam_start, ssp.lam_step)[0, 0]
    w = synth.Workload("flux-log", p, (0.0, 0.0, 0.0), 6, 6, 1.0, 5003.7, 2.6e-4, 1500, ssp,
                       resample=1, log_lambda=True)
    _, g = gpu_forward(w)
    key = g["key"]
    tot = np.zeros(36)
    np.add.at(tot, key[key < 36], p.mass[key < 36].astype(np.float64))
    width = cfg_line.tel_lambda() * 2.0 * math.sinh(0.5 * w.tel_step)
    got = (g["cube_raw"].astype(np.float64) * width[None, :]).sum(axis=1)
    expect = tot * integral
    log(f"log bin-mean flux: max rel err {np.abs(got - expect).max() / expect.max():.2e}")
    assert np.abs(got - expect).max() <= 1e-5 * expect.max()


def test_galaxy_placed_at_redshift_matches_oracle():
    """The medium galaxy placed at z = 0.03 with 0.25 arcsec spaxels (flat LCDM): systemic
    redshift, angular spaxels and 1/(4 pi D_L^2) flux dimming through the whole forward path."""
    import dataclasses
    from paper_2412_08265_amd import ops
    from paper_2412_08265_amd.cosmology import place_at_redshift
    w = synth.medium_workload(n=200_000)
    obs = place_at_redshift(ops.Observation.from_workload(w), 0.03, 0.25)
    w = dataclasses.replace(w, spaxel_kpc=obs.spaxel_kpc, z_sys=obs.z_sys,
                            flux_scale=obs.flux_scale)
    log(f"z = 0.03: spaxel {w.spaxel_kpc:.4f} kpc, flux_scale {w.flux_scale:.4e}")
    _, g = gpu_forward(w)
    cfg = O.config_from_workload(w)
    fo = O.forward(w.particles, cfg, workers=WORKERS, ties=TIES)
    _check_rotate_bin(w, g, fo)
    assert_cube_in(g["cube_raw"], fo, "cube_raw", what="z=0.03 cube_raw")
    assert_cube_in(g["cube"], fo, "cube", what="z=0.03 cube")
