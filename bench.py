#!/usr/bin/env python
"""Benchmark of the MI355X datacube forward model.

One step = one pass of the whole forward path over the 1e7-particle workload (80 % exponential
disk + 20 % Hernquist bulge, 150 x 150 spaxels of 0.2 kpc, 4563 telescope bins of 1.25 A from
4700 A, SSP 106 x 12 x 4563, PSF sigma 2 spaxels, LSF sigma 2.7 A): rotate + bin + stable sort,
SSP lookup + Doppler + resampling + spaxel sum, LSF + PSF. Inputs are resident in HBM before the
timed region. Metric: particle x lambda-bins per second into the cube (in-field particles x bins
/ step time).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_VECTOR_TFLOPS = 157.3
CUBE_FLOP_PER_UNIT = 16        # 4 SSP corners x 2 resampling taps x 1 multiply-add (2 FLOP)
# bin mean: per corner the integral of a linear segment over the bin's node interval
# (about 1.5 segments of ~4 FLOP each), 4 corners
BIN_FLOP_PER_UNIT = 24
# template bytes gathered per particle*bin: 4 corner rows x 4 B at 64 staged nodes per 62 bins
CUBE_GATHER_BYTES_PER_UNIT = 16.0 * 64.0 / 62.0
# vector-memory data return of the CUs: 256 CUs x 64 B/clk x 2.4 GHz (the unit the cube kernel's
# template gathers saturate; its counters show it 95 % busy)
PEAK_TD_TBS = 256 * 64 * 2.4e9 / 1e12
ROTBIN_BYTES_PER_PARTICLE = 100  # rotate + key + vlos + two radix passes + offsets (design figure)
PSF_BYTES_PER_VOXEL = 8        # PSF+LSF: the FP32 cube read once and written once


def err(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def source_digest(*names) -> str:
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2412_08265_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(units_kernel: str):
    """HBM bytes per launch of the cube kernel from the committed counter summary, or None when
    the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_cube_disk_bulge_1e7_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_digest") != units_kernel:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_in_full: int, sample_particles: int):
    """The FP64 oracle on a seeded random sample of the same galaxy, scaled to the full workload:
    t = t_particles(sample) * N_in/N_in(sample) + t_psf_lsf(row band) * n_s/rows. It runs in
    forked processes, one per host core available to this job: all of os.cpu_count() up to 16,
    the host share a one-GPU job may use."""
    import numpy as np
    import oracle as O
    host = os.cpu_count() or 1
    cores = min(host, 16)
    cfg = O.config_from_workload(w)
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(w.particles.n, sample_particles, replace=False))
    sub = w.particles.subset(idx)
    t0 = time.perf_counter()
    fo = O.forward(sub, cfg, workers=cores, with_cube=False)
    c = O.cube_raw(sub, fo["key"], fo["perm"], fo["seg_off"], fo["vlos"], cfg, workers=cores)
    t_part = time.perf_counter() - t0
    n_in_s = int(fo["seg_off"][-1])
    # PSF/LSF on a band of 10 y-rows (plus the PSF halo), scaled by rows
    rows = 10
    r = int(4 * w.psf_sigma_spx + 0.5)
    band_cfg = O.OracleConfig(cfg.angles_rad, cfg.nx, rows + 2 * r, cfg.spaxel_kpc,
                              cfg.tel_start, cfg.tel_step, cfg.n_tel, cfg.log_age_nodes,
                              cfg.met_nodes, cfg.ssp_lam_start, cfg.ssp_lam_step, cfg.ssp_flux,
                              cfg.psf_sigma_spx, cfg.lsf_sigma_A, cfg.z_sys, cfg.flux_scale,
                              cfg.log_lambda)
    band = c[: (rows + 2 * r) * cfg.nx]
    t1 = time.perf_counter()
    O.psf_lsf(band, band_cfg)
    t_psf = time.perf_counter() - t1
    t_total = t_part * (n_in_full / max(1, n_in_s)) + t_psf * (cfg.ny / (rows + 2 * r))
    value = n_in_full * cfg.n_tel / t_total
    return {"value": value, "unit": "particle*lambda-bins/s", "cores": cores, "kind": "oracle",
            "host_cpus": host, "cpu_model": cpu_model(),
            "method": ("extrapolated: the particle stage from a random particle sample (time "
                       "scales with in-field particles at fixed bins), the PSF/LSF stage from a "
                       "band of rows (time scales with rows)"),
            "sample": (f"{sample_particles} random particles of the same galaxy ({n_in_s} in "
                       f"field, all {cfg.n_tel} bins, {t_part:.1f} s on {cores} processes) plus "
                       f"PSF/LSF of a {rows + 2 * r}-row band ({t_psf:.1f} s), scaled to "
                       f"{n_in_full} in-field particles and {cfg.ny} rows: {t_total:.0f} s "
                       "for the full step")}


def serve_main(args):
    """Serving report: a Poisson stream of requests (N log-uniform 1e4..5e6, square grids of 20..100
    spaxels over 30 kpc, contiguous windows of 1500..4563 bins of the resident 100 x 12 x 4563 SSP
    grid, inclination uniform in 0..90 deg) through the batched graph executor and through
    one-at-a-time plain launches, at arrival rates doubling until the graph path saturates."""
    import numpy as np
    import torch
    from paper_2412_08265_amd import ops, synth
    from paper_2412_08265_amd.serve import (GraphExecutor, PlainExecutor, Request, Scheduler,
                                            replay_trace)
    grid = synth.serving_ssp()
    dssp = ops.DeviceSSP.from_grid(grid)
    n_req = args.serve_requests
    reqs, n_tot = [], 0
    for i in range(n_req):
        w = synth.serving_request(i, grid)
        reqs.append(Request.from_particles(w.particles, ops.Observation.from_workload(w), rid=i))
        n_tot += w.particles.n
        if (i + 1) % 32 == 0:
            err(f"generated {i + 1}/{n_req} requests ({n_tot:.3g} particles)")
    budget = int(args.serve_budget_gb * 2 ** 30)
    execs = {"graph": (GraphExecutor(dssp, max_jobs=args.serve_slots, lanes=2, mode="native"),
                       args.serve_slots),
             "persistent": (GraphExecutor(dssp, max_jobs=args.serve_slots, lanes=2,
                                          mode="persistent", grid_blocks=2048), args.serve_slots),
             "plain": (PlainExecutor(dssp), 1)}
    execs = {k: v for k, v in execs.items() if k in args.serve_modes.split(",")}
    fps = [execs["plain"][0].footprint(r) for r in reqs] if "plain" in execs else \
        [next(iter(execs.values()))[0].footprint(r) for r in reqs]
    # warm every path (module load, graph upload) on the first requests
    for ex, slots in execs.values():
        sch = Scheduler(ex, budget, max_slots=slots)
        for r in reqs[:4]:
            sch.submit(r)
        sch.drain()
    torch.cuda.synchronize()
    rows = []
    rate = args.serve_rate0
    while True:
        arr = synth.poisson_arrivals(n_req, rate, seed=4)
        row = {"rate_hz": rate}
        for name, (ex, slots) in execs.items():
            sch = Scheduler(ex, budget, max_slots=slots)
            rep = replay_trace(sch, reqs, arr)
            rep.pop("futures")
            row[name] = {k: rep[k] for k in ("p50_ms", "p99_ms", "mean_ms", "cubes_per_s",
                                             "span_s", "batches", "mean_batch", "errors")}
            row[name]["peak_budget_gb"] = rep["peak_budget_bytes"] / 2 ** 30
            del sch, rep
            torch.cuda.synchronize()
            err(f"rate {rate:g}/s {name}: p50 {row[name]['p50_ms']:.1f} ms, p99 "
                f"{row[name]['p99_ms']:.1f} ms, {row[name]['cubes_per_s']:.1f} cubes/s, mean "
                f"batch {row[name]['mean_batch']:.2f}")
        rows.append(row)
        first = next(iter(execs))
        if row[first]["cubes_per_s"] < 0.6 * rate or rate >= args.serve_rate_max:
            break
        rate *= 2
    out = {"metric": "serving latency p50/p99 (ms) and cubes/s (1 GPU)",
           "requests": n_req, "particles_total": n_tot,
           "mean_footprint_mb": float(np.mean(fps)) / 2 ** 20,
           "max_footprint_mb": float(np.max(fps)) / 2 ** 20,
           "budget_gb": args.serve_budget_gb, "max_slots": args.serve_slots, "lanes": 2,
           "modes": {"graph": "native forward graph per lane, exact grids per batch",
                     "persistent": "torch-captured rubix_forward_packed, 2048-block grids",
                     "plain": "one request at a time, plain entry points"},
           "data": "synthetic (seeded request stream, seeds 4000+i)",
           "sweep": rows}
    print(json.dumps(out), flush=True)


def sweep_main(args):
    """Runtime of the forward step against the particle count on one GPU (the one-GPU part of the
    paper's strong-scaling experiment, Sec. 4): the 1e7-particle workload's galaxy generator,
    grids and filters at each N, inputs resident, median of the timed steps. The 6e6 point is the
    particle count of the paper's speed comparison (Sec. 4: 8.58 s on one A100, spaxel and
    wavelength grids not stated), quoted as context."""
    import numpy as np
    import torch
    from paper_2412_08265_amd import ops, synth
    rows = []
    for n in [int(float(x)) for x in args.sweep_n.split(",")]:
        w = synth.large_workload(n=n)
        fw = ops.Forward(ops.DeviceGalaxy.from_host(w.particles), ops.Observation.from_workload(w),
                         ops.DeviceSSP.from_grid(w.ssp))
        for _ in range(args.warmup):
            fw()
        torch.cuda.synchronize()
        n_in = int(fw.buf.seg_off[-1].item())
        ts = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fw()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        rows.append({"particles": n, "in_field": n_in, "ms_per_step": ms,
                     "p90_ms": float(np.percentile(ts, 90)),
                     "particle_lambda_bins_per_s": n_in * w.n_tel / (ms * 1e-3)})
        err(f"N={n}: {ms:.3f} ms per step ({n_in} in field)")
        del fw
        torch.cuda.empty_cache()
    out = {"metric": "forward step time vs particle count (1 GPU)",
           "workload": "disk+bulge galaxy (seed 3) at each N, 150x150 spaxels of 0.2 kpc, 4563 "
                       "bins of 1.25 A from 4700 A, SSP 106x12x4563, PSF 2 spx, LSF 2.7 A",
           "timing": f"HIP events around rotate/bin + cube + PSF/LSF, median of {args.steps} steps "
                     f"after {args.warmup} warm-ups",
           "context": "paper Sec. 4: 6e6 particles in 8.58 s on one A100 (end to end, grids not "
                      "stated) and 123.57 s on a 24-core CPU",
           "data": "synthetic", "sweep": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000, help="particles (default: full 1e7)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true",
                    help="skip timing the gradient pass (reported beside the forward step)")
    ap.add_argument("--cpu-sample", type=int, default=800_000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="after timing, copy 1 GiB device to device once (a known-size kernel "
                         "for calibrating profiler byte counters)")
    ap.add_argument("--variant", choices=("centre", "binmean", "loglam", "binmeanlog"),
                    default="centre",
                    help="resampling reading / grid kind of the forward step: bin-centre sampling "
                         "on linear grids (default, the headline), bin mean (flux conserving), "
                         "grids uniform in ln(lambda), or the bin mean on those grids")
    ap.add_argument("--sweep-n", default=None,
                    help="comma-separated particle counts: print the forward step time against N "
                         "instead of the forward-step line")
    ap.add_argument("--serve", action="store_true",
                    help="print the serving report (request stream, batched graph path vs "
                         "one-at-a-time plain launches) instead of the forward-step line")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-rate0", type=float, default=16.0)
    ap.add_argument("--serve-rate-max", type=float, default=4096.0)
    ap.add_argument("--serve-modes", default="graph,persistent,plain",
                    help="executors to compare (the first one decides when the sweep stops)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the lambda-sharded "
              "design is documented, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        serve_main(args)
        return
    if args.sweep_n:
        sweep_main(args)
        return

    import torch
    from paper_2412_08265_amd import ops, synth

    err(f"generating the 1e7-particle workload ({args.variant})")
    if args.variant in ("loglam", "binmeanlog"):
        w = synth.large_log_workload(n=args.n)
        if args.variant == "binmeanlog":
            w.resample = 1
    else:
        w = synth.large_workload(n=args.n)
        if args.variant == "binmean":
            w.resample = 1
    dev = "cuda"
    gal = ops.DeviceGalaxy.from_host(w.particles, dev)
    ssp = ops.DeviceSSP.from_grid(w.ssp, dev)
    obs = ops.Observation.from_workload(w)
    fw = ops.Forward(gal, obs, ssp, dev)
    torch.cuda.synchronize()
    err(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        fw()
    torch.cuda.synchronize()
    n_in = int(fw.buf.seg_off[-1].item())
    K = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    err(f"timing {K} steps")
    torch.cuda.synchronize()
    ops.rubix_cube_timer_read()                 # drop any earlier pairs
    ops.rubix_cube_timer(True)                  # event pair around k_cube in every timed step
    t0 = time.perf_counter()
    for k in range(K):
        e = evs[k]
        e[0].record()
        fw.rotate_bin()
        e[1].record()
        fw.cube_raw()
        e[2].record()
        fw.psf_lsf()
        e[3].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ops.rubix_cube_timer(False)
    cube_kernel_ms, n_timed = ops.rubix_cube_timer_read()
    assert n_timed == K, (n_timed, K)
    cube_kernel_ms /= K
    ms_step = (t1 - t0) * 1e3 / K
    st = [sum(evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(K)) / K for i in range(3)]
    value = n_in * w.n_tel / (ms_step * 1e-3)
    units = n_in * w.n_tel
    flop_per_unit = BIN_FLOP_PER_UNIT if w.resample else CUBE_FLOP_PER_UNIT
    achieved = flop_per_unit * units / (cube_kernel_ms * 1e-3) / 1e12
    gather_tbs = CUBE_GATHER_BYTES_PER_UNIT * units / (cube_kernel_ms * 1e-3) / 1e12
    digest = source_digest("k_cube.hip", "rubix_internal.h")
    traffic = traffic_from_profile(digest) if args.variant == "centre" else None
    rot_gbs = ROTBIN_BYTES_PER_PARTICLE * w.particles.n / (st[0] * 1e-3) / 1e9
    psf_gbs = PSF_BYTES_PER_VOXEL * w.n_spaxels * w.n_tel / (st[2] * 1e-3) / 1e9
    out = {
        "metric": "particle*lambda-bins/sec into cube (1 GPU)",
        "value": value,
        "unit": "particle*lambda-bins/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded disk+bulge galaxy and SSP grid)",
        "config": {"workload": (f"{w.name}{'' if args.variant == 'centre' else ' ' + args.variant}: "
                                f"{w.particles.n} particles "
                                f"({n_in} in field), {w.nx}x{w.ny} spaxels of {w.spaxel_kpc} kpc, "
                                f"{w.n_tel} bins of {w.tel_step} "
                                f"{'ln(A)' if w.log_lambda else 'A'} from {w.tel_start} A, SSP "
                                f"{w.ssp.n_age}x{w.ssp.n_met}x{w.ssp.n_lam}, PSF {w.psf_sigma_spx} "
                                f"spx, LSF {w.lsf_sigma_A} A"),
                   "particles": w.particles.n, "in_field": n_in, "spaxels": w.n_spaxels,
                   "bins": w.n_tel, "resampling": "bin mean" if w.resample else "bin centre",
                   "grids": "log-lambda" if w.log_lambda else "linear",
                   "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "alu", "kernel": "k_cube_bin" if w.resample else "k_cube",
                     "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
                     "flop_per_unit": flop_per_unit, "units_per_launch": units,
                     "avg_ms": cube_kernel_ms, "source_digest": digest,
                     "timing": "HIP event pair around k_cube on its stream, every timed step"},
        "onchip": None if w.resample else {
            "bound": "vector-memory data return", "kernel": "k_cube", "achieved": gather_tbs,
            "peak": PEAK_TD_TBS, "unit": "TB/s", "frac": gather_tbs / PEAK_TD_TBS,
            "bytes_per_unit": CUBE_GATHER_BYTES_PER_UNIT,
            "what": "template rows gathered through the CUs' load path into the LDS windows"},
        "stages_ms": {"rotate_bin": st[0], "cube": st[1], "psf_lsf": st[2],
                      "k_cube": cube_kernel_ms},
        "stages_hbm": {"rotate_bin_GBs": rot_gbs, "rotate_bin_frac": rot_gbs / PEAK_HBM_GBS,
                       "psf_lsf_GBs": psf_gbs, "psf_lsf_frac": psf_gbs / PEAK_HBM_GBS},
    }
    err(f"step {ms_step:.3f} ms, stages {st}")
    # the noise step beside the step: one read and one write of the cube per call (8 B per voxel)
    noisy = torch.empty_like(fw.buf.cube)
    noisy.copy_(fw.buf.cube)
    spec = [dict(seed=2024, stream=0, gain=1.0, sigma_floor=1e-3)]
    ops.rubix_add_noise([fw.job], spec, [noisy])
    torch.cuda.synchronize()
    n0, n1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n0.record()
    for _ in range(5):
        ops.rubix_add_noise([fw.job], spec, [noisy])
    n1.record()
    torch.cuda.synchronize()
    noise_ms = n0.elapsed_time(n1) / 5
    noise_gbs = 8.0 * w.n_spaxels * w.n_tel / (noise_ms * 1e-3) / 1e9
    out["stages_ms"]["noise"] = noise_ms
    out["stages_hbm"]["noise_GBs"] = noise_gbs
    out["stages_hbm"]["noise_frac"] = noise_gbs / PEAK_HBM_GBS
    del noisy
    err(f"noise {noise_ms:.3f} ms ({noise_gbs:.0f} GB/s)")
    if not args.no_backward:
        # gradient pass beside the forward: adjoint PSF/LSF of a seeded dL/dcube, then the
        # per-particle adjoint (mass, age, [M/H], v_los, velocities, angles)
        gen = torch.Generator(device=dev).manual_seed(7)
        gcube = torch.randn(fw.buf.cube.shape, generator=gen, device=dev)
        graw = torch.empty_like(gcube)

        def backward():
            ops.rubix_psf_lsf([fw.job], [gcube], [graw], fw.ws)
            return ops.cube_backward(fw, graw)

        backward()
        torch.cuda.synchronize()
        b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        nb = 3
        b0.record()
        for _ in range(nb):
            backward()
        b1.record()
        torch.cuda.synchronize()
        out["stages_ms"]["backward"] = b0.elapsed_time(b1) / nb
        err(f"backward {out['stages_ms']['backward']:.3f} ms")
    # achievable HBM rate on this GPU: a 1 GiB device-to-device copy (read + write), quoted beside
    # the 8 TB/s peak
    ca = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        cb.copy_(ca)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * ca.numel() * 4 * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    out["hbm_copy"] = {"GBs": copy_gbs, "frac_of_peak": copy_gbs / PEAK_HBM_GBS,
                       "what": "1 GiB device-to-device copy (torch copy_ kernel), read + write "
                               "bytes / time, 10 repeats"}
    del ca, cb
    err(f"copy {copy_gbs:.0f} GB/s")
    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = {"read": a.numel() * 4, "write": b.numel() * 4}
    if not args.no_cpu_baseline:
        err("cpu baseline (oracle on a sample)")
        out["cpu_baseline"] = cpu_baseline(w, n_in, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
