"""Shared helpers of the GPU tests: run the HIP path through the C ABI and the oracle on the same
seeded inputs. Nothing here computes any part of the forward model."""
import os
import sys
import time

import numpy as np

import oracle as O

WORKERS = min(16, os.cpu_count() or 1)


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


def oracle_rows(p, cfg, fw_or, spaxels):
    """Oracle C_raw rows for selected spaxels only (using the oracle's own sort)."""
    out = np.zeros((len(spaxels), cfg.n_tel))
    for r, s in enumerate(spaxels):
        a, b = int(fw_or["seg_off"][s]), int(fw_or["seg_off"][s + 1])
        idx = fw_or["perm"][a:b]
        for c0 in range(0, idx.size, 2048):
            out[r] += O.particle_spectra(p, idx[c0:c0 + 2048], fw_or["vlos"], cfg).sum(0)
    return out


def _rows_task(args):
    s_list = args
    st = _ROWS_STATE
    return s_list, oracle_rows(st["p"], st["cfg"], st["fw"], s_list)


_ROWS_STATE = {}


def oracle_rows_parallel(p, cfg, fw_or, spaxels, workers=WORKERS):
    """oracle_rows over forked workers (one task per spaxel, heaviest first)."""
    import multiprocessing as mp
    _ROWS_STATE.update(p=p, cfg=cfg, fw=fw_or)
    cnt = np.diff(fw_or["seg_off"])
    order = sorted(spaxels, key=lambda s: -cnt[s])
    tasks = [[s] for s in order]
    res = {}
    with mp.get_context("fork").Pool(workers) as pool:
        for s_list, rows in pool.imap_unordered(_rows_task, tasks):
            for s, row in zip(s_list, rows):
                res[s] = row
    _ROWS_STATE.clear()
    return np.stack([res[s] for s in spaxels])
