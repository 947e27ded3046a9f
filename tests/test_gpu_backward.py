"""Parity of the hand-written adjoint (rubix_cube_backward and the RubixCube autograd function)
with the FP64 oracle's analytic gradient and with FP64 central finite differences."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2412_08265_amd import synth
from tests.helpers import TIES, WORKERS, assert_grads_in, log, outside

pytestmark = pytest.mark.gpu

GRAD_KEYS = ("mass", "age", "met", "vlos")


def _gpu_grads(w, G_rows):
    """GPU forward (for key/perm/seg_off/vlos) then rubix_cube_backward with dL/dC_raw = G_rows."""
    import torch
    from paper_2412_08265_amd import ops
    gal = ops.DeviceGalaxy.from_host(w.particles)
    ssp = ops.DeviceSSP.from_grid(w.ssp)
    fw = ops.Forward(gal, ops.Observation.from_workload(w), ssp)
    fw()
    G = torch.from_numpy(np.ascontiguousarray(G_rows, dtype=np.float32)).cuda()
    out = ops.cube_backward(fw, G.reshape(w.ny, w.nx, w.n_tel))
    torch.cuda.synchronize()
    return fw, {k: v.cpu().numpy() for k, v in out.items()}


def _compare(gpu, ref, tol, what):
    """Every gradient kind, the angles (phi3 exactly 0) and the velocity gradient within tol of
    the max-norm of the oracle's, measured from the oracle's range of correct values (ref from
    O.adjoint(..., ties=TIES))."""
    assert_grads_in(gpu, ref, GRAD_KEYS, tol, what)
    a, b = np.asarray(gpu["angles"]), np.asarray(ref["angles"])
    lo, hi = ref.get("angles_lo", b), ref.get("angles_hi", b)
    err = outside(a[:2], lo[:2], hi[:2]).max() / np.abs(b[:2]).max()
    log(f"{what} dangles: distance from the oracle's range {err:.3e} "
        f"(vs FP64 value {np.abs(a[:2] - b[:2]).max() / np.abs(b[:2]).max():.3e}); "
        f"gpu phi3 = {a[2]:.3e}")
    assert err <= tol and a[2] == 0.0
    vb = np.asarray(ref["vel"], dtype=np.float64)
    e = outside(gpu["vel"], ref.get("vel_lo", vb), ref.get("vel_hi", vb)).max()
    assert e <= tol * np.abs(vb).max(), (what, "vel", e / np.abs(vb).max())


def _small_workload(n=3000, seed=31):
    p = synth.make_galaxy(n, seed)
    ssp = synth.cached_ssp(12, 6, 3600.0, 3.8, 1000)
    return synth.Workload("grad-small", p, (55.0, 12.0, 20.0), 14, 12, 2.0, 3640.0, 3.1, 1100,
                          ssp, psf_sigma_spx=1.2, lsf_sigma_A=6.0)


def _small_log_workload(n=4000, seed=33):
    p = synth.make_galaxy(n, seed)
    ssp = synth.cached_ssp(12, 6, 3600.0, 3.0e-4, 1000, log_lambda=True)
    return synth.Workload("grad-small-log", p, (55.0, 12.0, 20.0), 14, 12, 2.0, 3620.0, 2.5e-4,
                          1100, ssp, psf_sigma_spx=1.2, lsf_sigma_A=6.0, z_sys=0.003,
                          log_lambda=True)


def test_log_grid_gradient_vs_oracle_and_fd():
    """Adjoint on grids uniform in ln(lambda) (dq/dbeta = -1/((1+beta) dln))."""
    w = _small_log_workload()
    cfg = O.config_from_workload(w)
    fo = O.forward(w.particles, cfg)
    rng = np.random.default_rng(7)
    G = rng.normal(size=(w.nx * w.ny, w.n_tel)).astype(np.float32)
    _, g = _gpu_grads(w, G)
    ref = O.adjoint(w.particles, cfg, G.astype(np.float64), fo, ties=TIES)
    _compare(g, ref, 2e-5, "log-grid seeded-G")
    _fd_check(w, cfg, fo, G.astype(np.float64), g, n_check=30, quadratic=False)


def test_backward_kernel_on_seeded_gradient():
    """dL/dC_raw = a seeded random array, identical on both sides: isolates the adjoint kernels."""
    w = _small_workload()
    cfg = O.config_from_workload(w)
    rng = np.random.default_rng(5)
    G = rng.normal(size=(w.nx * w.ny, w.n_tel)).astype(np.float32)
    _, g = _gpu_grads(w, G)
    ref = O.adjoint(w.particles, cfg, G.astype(np.float64), ties=TIES)
    _compare(g, ref, 2e-5, "seeded-G")


def _edges_workload(n=3000, seed=37):
    """Telescope bins on the SSP nodes, running 5 nodes past both ends of the SSP grid."""
    p = synth.make_galaxy(n, seed)
    ssp = synth.cached_ssp(12, 6, 3600.0, 3.8, 1000)
    return synth.Workload("grad-edges", p, (55.0, 12.0, 20.0), 14, 12, 2.0, 3600.0 - 5 * 3.8,
                          3.8, 1010, ssp, psf_sigma_spx=1.2, lsf_sigma_A=6.0)


def test_seeded_gradient_with_bins_past_both_ends_of_the_ssp_grid():
    """Bins whose rest-frame node lies below the first or above the last SSP node carry no
    gradient; with the telescope grid running past both ends of the SSP grid every particle has
    such bins (redshifted ones more at the blue end, blueshifted ones at the red end). A seeded
    random dL/dC_raw weights them as much as any other bin, so a bin leaking into the dots shows
    at once. Oracle on every particle and FP64 finite differences."""
    w = _edges_workload()
    cfg = O.config_from_workload(w)
    fo = O.forward(w.particles, cfg)
    vl = fo["vlos"]
    assert (vl < 0).sum() > 100 and (vl > 0).sum() > 100
    rng = np.random.default_rng(11)
    G = rng.normal(size=(w.nx * w.ny, w.n_tel)).astype(np.float32)
    _, g = _gpu_grads(w, G)
    ref = O.adjoint(w.particles, cfg, G.astype(np.float64), fo, ties=TIES)
    _compare(g, ref, 2e-5, "edges seeded-G")
    _fd_check(w, cfg, fo, G.astype(np.float64), g, n_check=30, quadratic=False)


def test_seeded_gradient_on_a_coarse_telescope_grid():
    """Telescope bins 1.7 times the SSP node spacing: no particle's span fits a wave window, so
    the adjoint gathers every tap directly. Oracle on every particle and FP64 finite
    differences."""
    p = synth.make_galaxy(3000, 41)
    ssp = synth.cached_ssp(12, 6, 3600.0, 3.8, 1000)
    w = synth.Workload("grad-coarse", p, (55.0, 12.0, 20.0), 14, 12, 2.0, 3700.0, 1.7 * 3.8, 520,
                       ssp, psf_sigma_spx=1.2, lsf_sigma_A=9.0)
    cfg = O.config_from_workload(w)
    fo = O.forward(w.particles, cfg)
    rng = np.random.default_rng(13)
    G = rng.normal(size=(w.nx * w.ny, w.n_tel)).astype(np.float32)
    _, g = _gpu_grads(w, G)
    ref = O.adjoint(w.particles, cfg, G.astype(np.float64), fo, ties=TIES)
    _compare(g, ref, 2e-5, "coarse seeded-G")
    _fd_check(w, cfg, fo, G.astype(np.float64), g, n_check=30, quadratic=False)


@pytest.mark.parametrize("ratio,n_tel,seed", [(1.0, 1010, 43), (2.3, 440, 47), (0.45, 2200, 53)])
def test_bin_mean_seeded_gradient(ratio, n_tel, seed):
    """Adjoint of the bin-mean resampling: the integrals of the corner interpolants over each
    bin's node interval, and for the velocity the Leibniz terms of the moving bin edges (an edge
    clipped to the grid's end gives none). Telescope bins of 1.0, 2.3 (several node segments per
    bin) and 0.45 (bins inside one segment) SSP node spacings, with the band running 5 bins past
    both ends of the SSP grid, so clipped edges of both kinds occur. Oracle on every particle
    and FP64 finite differences."""
    p = synth.make_galaxy(3000, seed)
    ssp = synth.cached_ssp(12, 6, 3600.0, 3.8, 1000)
    step = ratio * 3.8
    w = synth.Workload(f"grad-binmean-{ratio}", p, (55.0, 12.0, 20.0), 14, 12, 2.0,
                       3600.0 - 5 * step, step, n_tel, ssp, psf_sigma_spx=1.2,
                       lsf_sigma_A=6.0, z_sys=0.001, resample=1)
    cfg = O.config_from_workload(w)
    assert cfg.resample == 1
    fo = O.forward(w.particles, cfg)
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(w.nx * w.ny, w.n_tel)).astype(np.float32)
    _, g = _gpu_grads(w, G)
    ref = O.adjoint(w.particles, cfg, G.astype(np.float64), fo, ties=TIES)
    _compare(g, ref, 2e-5, f"bin-mean x{ratio} seeded-G")
    _fd_check(w, cfg, fo, G.astype(np.float64), g, n_check=30, quadratic=False, h_vlos=1e-2,
              h_met=5e-5)


@pytest.mark.parametrize("n", [0, 1, 255, 256, 257, 4097])
def test_ragged_particle_counts_backward(n):
    """Particle counts around the final pass's 256-particle blocks and the adjoint's 16-particle
    work items, and the empty galaxy: gradients against the oracle (all zero for n = 0)."""
    import torch
    from paper_2412_08265_amd import ops
    p = synth.make_galaxy(max(n, 1), seed=300 + n).subset(slice(0, n))
    ssp = synth.cached_ssp(12, 6, 3600.0, 3.8, 1000)
    w = synth.Workload(f"grad-n{n}", p, (55.0, 12.0, 20.0), 14, 12, 2.0, 3640.0, 3.1, 1100, ssp,
                       psf_sigma_spx=1.2, lsf_sigma_A=6.0)
    rng = np.random.default_rng(n)
    G = rng.normal(size=(w.nx * w.ny, w.n_tel)).astype(np.float32)
    _, g = _gpu_grads(w, G)
    if n == 0:
        for k in GRAD_KEYS:
            assert g[k].size == 0
        assert np.all(np.asarray(g["angles"]) == 0.0)
        return
    cfg = O.config_from_workload(w)
    ref = O.adjoint(w.particles, cfg, G.astype(np.float64), ties=TIES)
    assert_grads_in(g, ref, GRAD_KEYS, 2e-5, f"n={n}")
    a, b = np.asarray(g["angles"]), np.asarray(ref["angles"])
    err = outside(a[:2], ref["angles_lo"][:2], ref["angles_hi"][:2]).max()
    assert err <= 2e-5 * max(np.abs(b[:2]).max(), 1e-300) and a[2] == 0.0


@pytest.mark.parametrize("ratio,n_tel,seed", [(1.3, 1300, 61), (2.6, 660, 67), (0.6, 2800, 71)])
def test_log_grid_bin_mean_seeded_gradient(ratio, n_tel, seed):
    """Adjoint of the bin mean on grids uniform in ln(lambda): the corner integrals over rest
    wavelength (divided by the bin widths) and the Leibniz terms Slin lam dln at the moving
    edges. Bins of 1.3, 2.6 and 0.6 SSP steps, the band running past both ends of the SSP grid.
    Oracle on every particle and FP64 finite differences (steps sized against the oracle's
    prefix-sum rounding)."""
    p = synth.make_galaxy(3000, seed)
    ssp = synth.cached_ssp(12, 6, 3600.0, 3.0e-4, 1000, log_lambda=True)
    step = ratio * 3.0e-4
    w = synth.Workload(f"grad-binmean-log-{ratio}", p, (55.0, 12.0, 20.0), 14, 12, 2.0,
                       3600.0 * math.exp(-5 * step), step, n_tel, ssp, psf_sigma_spx=1.2,
                       lsf_sigma_A=6.0, z_sys=0.002, log_lambda=True, resample=1)
    cfg = O.config_from_workload(w)
    fo = O.forward(w.particles, cfg)
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(w.nx * w.ny, w.n_tel)).astype(np.float32)
    _, g = _gpu_grads(w, G)
    ref = O.adjoint(w.particles, cfg, G.astype(np.float64), fo, ties=TIES)
    _compare(g, ref, 2e-5, f"log bin-mean x{ratio} seeded-G")
    _fd_check(w, cfg, fo, G.astype(np.float64), g, n_check=30, quadratic=False, h_vlos=0.03,
              h_met=1e-3, h_age=1e-4, age_rel=True)


def _fd_delta_L(cfg, G, s, dplus, dminus, quadratic=True):
    """L(+) - L(-) when one particle of spaxel s changes its spectrum by d+/d- (FP64).
    For the loss L = |A C - T|^2 / 2 with G = A(A C - T):
    <d+ - d-, G[s]> + (|A d+|^2 - |A d-|^2)/2 with A = Px Py L separable, so
    |A d|^2 = |Px Py e_s|^2 |L d|^2. For the linear functional L = <C, G> (a seeded G that is
    not the gradient of a residual) only the first term (quadratic=False)."""
    if not quadratic:
        return float(np.dot(dplus - dminus, G[s]))
    wl = O.gaussian_weights(cfg.lsf_sigma_bins())
    wp = O.gaussian_weights(cfg.psf_sigma_spx)
    img = np.zeros((cfg.ny, cfg.nx))
    img[s // cfg.nx, s % cfg.nx] = 1.0
    img = O.convolve_axis(O.convolve_axis(img, wp, 0), wp, 1)
    P2 = float(np.sum(img * img))
    Lp = O.convolve_axis(dplus, wl, 0)
    Lm = O.convolve_axis(dminus, wl, 0)
    return float(np.dot(dplus - dminus, G[s])) + 0.5 * P2 * (np.dot(Lp, Lp) - np.dot(Lm, Lm))


def _fd_check(w, cfg, fo, G, gpu, n_check=64, seed=0, quadratic=True, h_vlos=1e-4, h_met=1e-6,
              h_age=1e-6, age_rel=False):
    """FP64 central differences of the oracle's particle spectra against the GPU gradient, on up
    to n_check in-field particles at least 1e-4 away from SSP nodes whose oracle gradients are
    all at least 1e-2 of the sample's largest. h_vlos (km/s) and h_met
    (dex) are the velocity and metallicity steps: the oracle's bin mean is a difference of prefix
    sums over the node grid, whose rounding needs larger steps than bin-centre sampling does (the
    spectrum is linear in [M/H] inside a cell, so any step below the node distance is exact)."""
    p = w.particles
    key, vlos = fo["key"], fo["vlos"]
    la, mz = cfg.log_age_nodes, cfg.met_nodes
    rng = np.random.default_rng(seed)
    cand = rng.permutation(np.flatnonzero(key < cfg.n_spaxels))[:max(4000, 60 * n_check)]
    # particles are chosen by the oracle's gradient (never the GPU's): a GPU gradient wrongly
    # near zero cannot exclude its own particle
    ora = O.adjoint(p, cfg, G, fo, idx=cand)
    ora_at = {int(i): r for r, i in enumerate(cand)}
    maxg = {k: np.abs(ora[k]).max() for k in GRAD_KEYS}
    checked = 0
    worst = {k: 0.0 for k in GRAD_KEYS}
    for i in cand:
        if checked >= n_check:
            break
        m, a, z, v = float(p.mass[i]), float(p.age[i]), float(p.met[i]), float(vlos[i])
        ha = h_age * a if age_rel else h_age       # (a step relative to the age: log10 age)
        # one linear piece on both sides of the step: away from SSP nodes and clamps
        if (np.min(np.abs(la - math.log10(a))) < max(1e-4, 2 * ha / (a * math.log(10)))
                or np.min(np.abs(mz - z)) < max(1e-4, 2 * h_met)):
            continue
        if any(abs(ora[k][ora_at[int(i)]]) < 1e-2 * maxg[k] for k in GRAD_KEYS):
            continue
        one = {f: np.asarray(getattr(p, f)[i:i + 1], dtype=np.float64) for f in p.FIELDS}

        def spec(field=None, val=None, vv=v):
            # FP64 particle (no rounding of the perturbed value back to FP32)
            d = dict(one)
            if field is not None:
                d[field] = np.array([val], dtype=np.float64)
            qq = synth.Particles(**d)
            return O.particle_spectra(qq, np.array([0]), np.array([vv]), cfg)[0]

        base = spec()
        for k, h, mk in (("mass", 1e-6 * m, lambda d: spec("mass", m + d)),
                         ("age", ha, lambda d: spec("age", a + d)),
                         ("met", h_met, lambda d: spec("met", z + d)),
                         ("vlos", h_vlos, lambda d: spec(vv=v + d))):
            dl = _fd_delta_L(cfg, G, int(key[i]), mk(h) - base, mk(-h) - base, quadratic)
            fd = dl / (2 * h)
            rel = abs(gpu[k][i] - fd) / abs(fd)
            worst[k] = max(worst[k], rel)
            assert rel <= 1e-4, (k, i, gpu[k][i], fd)
        checked += 1
    log(f"FD: {checked} particles, worst relative error per parameter {worst}")
    assert checked >= min(n_check, 20)


def _oracle_target(w, workers):
    pt, ang = synth.differentiation_target_params(w.particles)
    cfg_t = O.config_from_workload(w)
    cfg_t.angles_rad = tuple(math.radians(a) for a in ang)
    return O.forward(pt, cfg_t, workers=workers)["cube"].astype(np.float32)


def test_small_loss_gradient_vs_oracle_and_fd():
    w = _small_workload(n=4000, seed=8)
    cfg = O.config_from_workload(w)
    target = _oracle_target(w, 1)
    fo = O.forward(w.particles, cfg)
    G = O.loss_grad_cube(fo["cube"], target, cfg)
    ref = O.adjoint(w.particles, cfg, G, fo, ties=TIES)
    # GPU: the whole loss path on the device (forward, residual, adjoint PSF/LSF, backward)
    import torch
    from paper_2412_08265_amd import ops
    gal = ops.DeviceGalaxy.from_host(w.particles)
    ssp = ops.DeviceSSP.from_grid(w.ssp)
    fw = ops.Forward(gal, ops.Observation.from_workload(w), ssp)
    buf = fw()
    resid = buf.cube - torch.from_numpy(target.reshape(w.ny, w.nx, w.n_tel)).cuda()
    Gd = torch.empty_like(resid)
    ops.rubix_psf_lsf([fw.job], [resid.contiguous()], [Gd], fw.ws)
    out = ops.cube_backward(fw, Gd)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    _compare(g, ref, 1e-4, "small-loss")
    _fd_check(w, cfg, fo, G, g, n_check=40)


def test_autograd_function_matches_direct_calls():
    import torch
    from paper_2412_08265_amd import ops
    w = _small_workload(n=2500, seed=4)
    dev = "cuda"
    t = {f: torch.from_numpy(getattr(w.particles, f)).to(dev) for f in ops.FIELDS}
    for f in ("vx", "vy", "vz", "mass", "age", "met"):
        t[f].requires_grad_(True)
    angles = torch.tensor([math.radians(a) for a in w.angles_deg], dtype=torch.float64,
                          requires_grad=True)
    obs = ops.Observation.from_workload(w)
    ssp = ops.DeviceSSP.from_grid(w.ssp)
    cube = ops.RubixCube.apply(*[t[f] for f in ops.FIELDS], angles, obs, ssp)
    target = torch.zeros_like(cube)
    loss = 0.5 * ((cube - target) ** 2).sum()
    loss.backward()
    # direct path
    gal = ops.DeviceGalaxy.from_host(w.particles)
    fw = ops.Forward(gal, obs, ssp)
    buf = fw()
    G = torch.empty_like(buf.cube)
    ops.rubix_psf_lsf([fw.job], [buf.cube.contiguous()], [G], fw.ws)
    out = ops.cube_backward(fw, G)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(t["mass"].grad.cpu().numpy(), out["mass"].cpu().numpy())
    np.testing.assert_array_equal(t["age"].grad.cpu().numpy(), out["age"].cpu().numpy())
    np.testing.assert_array_equal(t["vz"].grad.cpu().numpy(), out["vel"][2].cpu().numpy())
    np.testing.assert_array_equal(angles.grad.numpy(), out["angles"].cpu().numpy())
    assert t["x"].grad is None


def test_differentiation_workload_full_size():
    """1e6 particles, 50x50x3000 cube, loss against the oracle's cube of perturbed parameters
    (masses +10 %, ages +0.5 Gyr, [M/H] +0.1, inclination +5 deg): GPU gradient vs the oracle's
    analytic gradient (max-norm over 4000 sampled particles, angles) and vs FP64 central finite
    differences on 64 sampled particles."""
    import time
    import torch
    from paper_2412_08265_amd import ops
    w = synth.medium_workload()
    cfg = O.config_from_workload(w)
    log(f"C5: oracle target ({WORKERS} workers)")
    target = _oracle_target(w, WORKERS)
    log("C5: oracle forward")
    fo = O.forward(w.particles, cfg, workers=WORKERS)
    G = O.loss_grad_cube(fo["cube"], target, cfg)
    log("C5: GPU forward + backward")
    gal = ops.DeviceGalaxy.from_host(w.particles)
    ssp = ops.DeviceSSP.from_grid(w.ssp)
    fw = ops.Forward(gal, ops.Observation.from_workload(w), ssp)
    tgt = torch.from_numpy(target.reshape(w.ny, w.nx, w.n_tel)).cuda()
    buf = fw()
    Gd = torch.empty_like(buf.cube)
    ops.rubix_psf_lsf([fw.job], [(buf.cube - tgt).contiguous()], [Gd], fw.ws)
    out = ops.cube_backward(fw, Gd)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    rng = np.random.default_rng(1)
    sub = rng.choice(w.particles.n, 4000, replace=False)
    log("C5: oracle adjoint on 4000 sampled particles")
    ref = O.adjoint(w.particles, cfg, G, fo, idx=sub, ties=TIES)
    gs = {k: g[k][sub] for k in GRAD_KEYS}
    gs["vel"] = g["vel"][:, sub]
    # angles: the full sum needs every particle; compare the oracle's full gradient
    log("C5: oracle adjoint (all particles) for the angle gradient")
    ref_all = O.adjoint(w.particles, cfg, G, fo, chunk=256, workers=WORKERS, ties=TIES)
    gs["angles"] = g["angles"]
    ref["angles"] = ref_all["angles"]
    ref["angles_lo"], ref["angles_hi"] = ref_all["angles_lo"], ref_all["angles_hi"]
    _compare(gs, ref, 1e-4, "C5")
    assert_grads_in(g, ref_all, GRAD_KEYS, 1e-4, "C5 full-vector")
    _fd_check(w, cfg, fo, G, g, n_check=64, seed=2)


def test_bin_mean_adjoint_on_the_differentiation_workload():
    """The bin-mean adjoint at the differentiation workload's size (1e6 particles, 50x50x3000
    cube) with a seeded dL/dC_raw: GPU gradients vs the oracle's on 4000 sampled particles
    (max-norm per parameter) and vs FP64 central differences on 32 of them."""
    import dataclasses
    w = dataclasses.replace(synth.medium_workload(), resample=1)
    cfg = O.config_from_workload(w)
    assert cfg.resample == 1
    log(f"bin-mean C5: oracle keys and velocities ({WORKERS} workers)")
    fo = O.forward(w.particles, cfg, workers=WORKERS, with_cube=False)
    rng = np.random.default_rng(17)
    G = rng.normal(size=(w.nx * w.ny, w.n_tel)).astype(np.float32)
    log("bin-mean C5: GPU forward + backward")
    _, g = _gpu_grads(w, G)
    sub = rng.choice(w.particles.n, 4000, replace=False)
    log("bin-mean C5: oracle adjoint on 4000 sampled particles")
    ref = O.adjoint(w.particles, cfg, G.astype(np.float64), fo, idx=sub, ties=TIES)
    assert_grads_in({k: g[k][sub] for k in GRAD_KEYS}, ref, GRAD_KEYS, 1e-4, "bin-mean C5")
    _fd_check(w, cfg, fo, G.astype(np.float64), g, n_check=32, seed=3, quadratic=False,
              h_vlos=1e-2, h_met=5e-5)


@pytest.mark.parametrize("grids,resample", [("log", 0), ("log", 1), ("linear", 0), ("linear", 1)])
def test_adjoint_on_the_full_size_galaxy(grids, resample):
    """The adjoint that the bench times, at full size (1e7 particles, 150x150x4563, grids linear
    in lambda or uniform in ln(lambda), bin centres and bin means) with a seeded dL/dC_raw: GPU
    gradients vs the oracle's on 4000 sampled particles (max-norm per parameter), and particles
    outside the field get zero."""
    import dataclasses
    base = synth.large_log_workload() if grids == "log" else synth.large_workload()
    w = dataclasses.replace(base, resample=resample)
    cfg = O.config_from_workload(w)
    tag = f"{grids} 1e7 resample={resample}"
    log(f"{tag}: oracle keys and velocities ({WORKERS} workers)")
    fo = O.forward(w.particles, cfg, workers=WORKERS, with_cube=False)
    rng = np.random.default_rng(23)
    G = rng.standard_normal(size=(w.nx * w.ny, w.n_tel), dtype=np.float32)
    log(f"{tag}: GPU forward + backward")
    _, g = _gpu_grads(w, G)
    sub = rng.choice(w.particles.n, 4000, replace=False)
    log(f"{tag}: oracle adjoint on 4000 sampled particles")
    ref = O.adjoint(w.particles, cfg, G.astype(np.float64), fo, idx=sub, ties=TIES)
    assert_grads_in({k: g[k][sub] for k in GRAD_KEYS}, ref, GRAD_KEYS, 1e-4, tag)
    out = np.asarray(fo["key"]) >= w.nx * w.ny
    assert out.any()
    for k in GRAD_KEYS:
        assert np.all(g[k][out] == 0), k
