"""Shared helpers of the GPU tests: run the HIP path through the C ABI and the oracle on the same
seeded inputs. Nothing here computes any part of the forward model."""
import os
import sys
import time

import numpy as np

import oracle as O

WORKERS = min(16, os.cpu_count() or 1)

# Index-error bound of the kernels' node index q = Qi + fl32(Qf - L g): |q - q_exact| <=
# 2^-24 (1.5 + 4 |d|) (d = L g, the Doppler part of q in nodes: the FP32 fraction Qf, the FP32
# factors L and g, one rounding of the fused multiply-add, and v_los rounded to FP32), taken with
# a factor 2 of margin. Pairs within it of a node may fall on either side (the oracle's bounds).
TIES = (2.0 ** -22, 2.0 ** -21)


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)
    sys.stdout.flush()


def gpu_forward(w, device="cuda"):
    """Run rotate/bin -> cube -> PSF/LSF for a synthetic workload; return host numpy arrays."""
    import torch
    from paper_2412_08265_amd import ops
    gal = ops.DeviceGalaxy.from_host(w.particles, device)
    ssp = ops.DeviceSSP.from_grid(w.ssp, device)
    fw = ops.Forward(gal, ops.Observation.from_workload(w), ssp, device)
    buf = fw()
    torch.cuda.synchronize()
    return fw, dict(key=buf.key.cpu().numpy(), perm=buf.perm.cpu().numpy(),
                    seg_off=buf.seg_off.cpu().numpy(), vlos=buf.vlos.cpu().numpy(),
                    cube_raw=buf.cube_raw.cpu().numpy().reshape(w.nx * w.ny, w.n_tel),
                    cube=buf.cube.cpu().numpy().reshape(w.nx * w.ny, w.n_tel))


def assert_cube_close(gpu, ref, tol=1e-5, what="cube"):
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    err = np.abs(np.asarray(gpu, dtype=np.float64) - ref).max()
    log(f"{what}: max|err|/max|ref| = {err / max(scale, 1e-300):.3e} (tol {tol:g})")
    assert scale > 0
    assert err <= tol * scale, (what, err / scale)


def outside(x, lo, hi):
    """Distance of x from the interval [lo, hi] (elementwise, 0 inside)."""
    x = np.asarray(x, dtype=np.float64)
    return np.maximum(np.maximum(np.asarray(lo, dtype=np.float64) - x,
                                 x - np.asarray(hi, dtype=np.float64)), 0.0)


def assert_cube_in(gpu, fo, name="cube_raw", tol=1e-5, what=None):
    """GPU voxels within tol * max|oracle| of the oracle's range of correct values (fo from
    O.forward(..., ties=TIES): the FP64 value, widened where a (particle, bin) pair's node interval
    is decided by rounding); the error against the FP64 value itself is reported beside it."""
    what = what or name
    ref = np.asarray(fo[name], dtype=np.float64)
    lo, hi = fo.get(name + "_lo", ref), fo.get(name + "_hi", ref)
    scale = np.abs(ref).max()
    g = np.asarray(gpu, dtype=np.float64)
    err = outside(g, lo, hi).max() / max(scale, 1e-300)
    plain = np.abs(g - ref).max() / max(scale, 1e-300)
    log(f"{what}: max distance from the oracle's range / max|ref| = {err:.3e} "
        f"(vs FP64 value {plain:.3e}; {fo.get('n_ties', 0)} tied pairs; tol {tol:g})")
    assert scale > 0
    assert err <= tol, (what, err)


def assert_grads_in(gpu, ref, keys, tol, what):
    """Per gradient kind, the GPU values within tol * max|oracle| of the oracle's range (ref from
    O.adjoint(..., ties=TIES)); returns the errors."""
    errs = {}
    for k in keys:
        b = np.asarray(ref[k], dtype=np.float64)
        lo, hi = ref.get(k + "_lo", b), ref.get(k + "_hi", b)
        a = np.asarray(gpu[k], dtype=np.float64)
        scale = np.abs(b).max()
        err = outside(a, lo, hi).max() / scale if scale > 0 else np.abs(a).max()
        plain = np.abs(a - b).max() / scale if scale > 0 else np.abs(a).max()
        log(f"{what} d{k}: max-norm distance from the oracle's range {err:.3e} "
            f"(vs FP64 value {plain:.3e}; {ref.get('n_ties', 0)} tied pairs)")
        assert err <= tol, (what, k, err)
        errs[k] = err
    return errs


def _rows_chunk(p, cfg, fw_or, s, a, b, ties):
    """Oracle C_raw row of spaxel s from its sorted particles a..b (and, with ties, its bounds)."""
    idx = fw_or["perm"][a:b]
    out = np.zeros((3, cfg.n_tel))
    n_tied = 0
    for c0 in range(0, idx.size, 2048):
        sub = idx[c0:c0 + 2048]
        if ties is None:
            out[0] += O.particle_spectra(p, sub, fw_or["vlos"], cfg).sum(0)
            continue
        f, l_, h_, nt = O.particle_spectra_bounds(p, sub, fw_or["vlos"], cfg, ties)
        out[0] += f.sum(0)
        out[1] += l_.sum(0)
        out[2] += h_.sum(0)
        n_tied += nt
    return out, n_tied


def oracle_rows(p, cfg, fw_or, spaxels, ties=None):
    """Oracle C_raw rows for selected spaxels only (using the oracle's own sort). With `ties`
    also the rows' bounds (particle_spectra_bounds) and the tied-pair count:
    returns (rows, lo, hi, n_tied)."""
    res = [_rows_chunk(p, cfg, fw_or, s, int(fw_or["seg_off"][s]), int(fw_or["seg_off"][s + 1]),
                       ties) for s in spaxels]
    rows = np.stack([r[0] for r in res]) if res else np.zeros((0, 3, cfg.n_tel))
    if ties is None:
        return rows[:, 0]
    return rows[:, 0], rows[:, 1], rows[:, 2], sum(r[1] for r in res)


def _rows_task(args):
    s, a, b = args
    st = _ROWS_STATE
    return s, _rows_chunk(st["p"], st["cfg"], st["fw"], s, a, b, st["ties"])


_ROWS_STATE = {}


def oracle_rows_parallel(p, cfg, fw_or, spaxels, workers=WORKERS, ties=None, piece=16384):
    """oracle_rows over forked workers: each spaxel's particles in pieces of at most `piece`
    (heaviest first), the pieces' rows summed per spaxel."""
    import multiprocessing as mp
    _ROWS_STATE.update(p=p, cfg=cfg, fw=fw_or, ties=ties)
    tasks = []
    for s in spaxels:
        a, b = int(fw_or["seg_off"][s]), int(fw_or["seg_off"][s + 1])
        tasks += [(s, c, min(b, c + piece)) for c in range(a, b, piece)]
    tasks.sort(key=lambda t: t[1] - t[2])
    acc = {s: np.zeros((3, cfg.n_tel)) for s in spaxels}
    n_tied = 0
    with O.ForkedPool(mp.get_context("fork"), workers) as pool:
        for s, (rows, nt) in pool.imap_unordered(_rows_task, tasks):
            acc[s] += rows
            n_tied += nt
    _ROWS_STATE.clear()
    out = np.stack([acc[s] for s in spaxels])
    if ties is None:
        return out[:, 0]
    return out[:, 0], out[:, 1], out[:, 2], n_tied


def window_config(cfg, j0, j1, vlos=None):
    """The same observation restricted to telescope bins j0..j1-1 (each bin's value depends only
    on its own centre or edges, so the oracle run on this grid gives exactly those bins). With
    the particles' line-of-sight velocities, the SSP grid is cut to the nodes those bins can reach
    (two nodes of margin; the grid's own ends are kept where they are reached), which leaves every
    value unchanged and saves interpolating the templates at nodes no bin reads."""
    import copy
    c = copy.copy(cfg)
    if cfg.log_lambda:
        c.tel_start = cfg.tel_start * np.exp(cfg.tel_step * j0)
    else:
        c.tel_start = cfg.tel_start + cfg.tel_step * j0
    c.n_tel = j1 - j0
    if vlos is None:
        return c
    v = np.asarray(vlos, dtype=np.float64)
    v = v[np.isfinite(v)]
    if v.size == 0:
        return c
    vv = np.array([v.min(), v.max()])
    if cfg.resample == 1:
        qs = (O.bin_edge_indices_log if cfg.log_lambda else O.bin_edge_indices)(c, vv)
    else:
        qs = (O.doppler_index(c, vv),)
    n = cfg.ssp_flux.shape[2]
    k0 = int(max(0, np.floor(min(q.min() for q in qs)) - 2))
    k1 = int(min(n, np.ceil(max(q.max() for q in qs)) + 3))
    if k1 - k0 < 2:
        k0, k1 = max(0, min(k0, n - 2)), max(2, min(n, max(k1, k0 + 2)))
    if cfg.log_lambda:
        c.ssp_lam_start = cfg.ssp_lam_start * np.exp(cfg.ssp_lam_step * k0)
    else:
        c.ssp_lam_start = cfg.ssp_lam_start + cfg.ssp_lam_step * k0
    c.ssp_flux = cfg.ssp_flux[:, :, k0:k1]
    return c


def oracle_final_window(p, cfg, fo, j0, j1, workers=WORKERS, ties=None):
    """The oracle's final cube (after LSF and PSF) over all spaxels for bins j0..j1-1: C_raw of
    every spaxel on those bins widened by the LSF radius (clipped to the band), then the LSF of the
    full grid and the PSF, cut back to the window. With `ties` returns (cube, lo, hi, n_tied)."""
    wl = O.gaussian_weights(cfg.lsf_sigma_bins())
    wp = O.gaussian_weights(cfg.psf_sigma_spx)
    r = (wl.shape[0] - 1) // 2
    a, b = max(0, j0 - r), min(cfg.n_tel, j1 + r)
    cw = window_config(cfg, a, b, fo["vlos"])
    res = O.cube_raw(p, fo["key"], fo["perm"], fo["seg_off"], fo["vlos"], cw, workers=workers,
                     ties=ties)
    raws = [res] if ties is None else list(res[:3])

    def final(c):
        c = c.reshape(cfg.ny, cfg.nx, b - a)
        c = O.convolve_axis(c, wl, 2)
        c = O.convolve_axis(O.convolve_axis(c, wp, 0), wp, 1)
        return c.reshape(cfg.ny * cfg.nx, b - a)[:, j0 - a:j1 - a]

    outs = [final(c) for c in raws]
    return outs[0] if ties is None else (outs[0], outs[1], outs[2], res[3])
