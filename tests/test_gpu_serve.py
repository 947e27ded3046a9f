"""GPU tests of the serving path: the packed, graph-replayed forward pass gives bitwise the cube of
the plain entry points for every request, alone or in any batch; every graph replay (with other
device work between replays) matches the eager result; a request served through the scheduler
matches the oracle."""
import numpy as np
import pytest
import torch

from helpers import TIES, assert_cube_in, log

import oracle as O
from paper_2412_08265_amd import ops, synth
from paper_2412_08265_amd.serve import (GraphExecutor, PlainExecutor, Rejected, Request,
                                        Scheduler, replay_trace)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssp_grid():
    return synth.serving_ssp()


@pytest.fixture(scope="module")
def dssp(ssp_grid):
    return ops.DeviceSSP.from_grid(ssp_grid)


def _workloads(ssp_grid, ids, n_max=2e5):
    return [synth.serving_request(i, ssp_grid, n_max=n_max, n_min=1e3) for i in ids]


def _requests(ws):
    return [Request.from_particles(w.particles, ops.Observation.from_workload(w), rid=k)
            for k, w in enumerate(ws)]


def _plain_cubes(dssp, reqs):
    ex = PlainExecutor(dssp)
    out = []
    for r in reqs:
        h = ex.launch([r])
        h["done"].synchronize()
        out.append(ex.collect(h)[0].cube.cpu())
    return out


def _graph_batch(ex, reqs):
    h = ex.launch(reqs)
    h["done"].synchronize()
    return [res.cube.cpu() for res in ex.collect(h)]


@pytest.mark.parametrize("mode", ["native", "persistent"])
def test_alone_equals_in_mix_equals_plain(ssp_grid, dssp, mode):
    ws = _workloads(ssp_grid, range(6))
    for w in ws:
        log(f"request {w.name}: n={w.particles.n} grid {w.nx}x{w.ny} n_tel={w.n_tel} "
            f"incl={w.angles_deg[0]:.1f}")
    reqs = _requests(ws)
    plain = _plain_cubes(dssp, reqs)
    ex = GraphExecutor(dssp, max_jobs=8, lanes=1, mode=mode, grid_blocks=1024)
    alone = [_graph_batch(ex, [r])[0] for r in reqs]
    mix = _graph_batch(ex, reqs[::-1])[::-1]
    pair = _graph_batch(ex, [reqs[2], reqs[0]])
    for k in range(len(reqs)):
        assert plain[k].abs().max() > 0
        assert torch.equal(alone[k], plain[k]), k
        assert torch.equal(mix[k], plain[k]), k
    assert torch.equal(pair[0], plain[2]) and torch.equal(pair[1], plain[0])


@pytest.mark.parametrize("mode", ["native", "persistent"])
def test_graph_replays_with_device_work_between(ssp_grid, dssp, mode):
    reqs = _requests(_workloads(ssp_grid, range(10, 14)))
    ref = _plain_cubes(dssp, reqs)
    ex = GraphExecutor(dssp, max_jobs=4, lanes=2, mode=mode, grid_blocks=512)
    junk = torch.randn(1 << 24, device="cuda")
    for rep in range(4):
        got = _graph_batch(ex, reqs if rep % 2 == 0 else reqs[1:])
        want = ref if rep % 2 == 0 else ref[1:]
        for a, b in zip(got, want):
            assert torch.equal(a, b), rep
        # eager work between replays: reductions, a plain forward, a host synchronisation
        s = float(junk.sum()) + float((junk * 2).amax())
        assert np.isfinite(s)
        _plain_cubes(dssp, reqs[:1])
        torch.cuda.synchronize()
        log(f"{mode} replay {rep} matches the eager result")


@pytest.mark.parametrize("mode", ["native", "persistent"])
def test_batch_mixing_bin_centre_and_bin_mean_requests(ssp_grid, dssp, mode):
    """A batch whose jobs alternate between bin-centre sampling and bin means: the packed tables
    launch both cube kernels, each skipping the other kind's jobs; every cube equals the plain
    entry points' bitwise, in the mix and alone."""
    ws = _workloads(ssp_grid, range(20, 24), n_max=1e5)
    for k, w in enumerate(ws):
        w.resample = k % 2
        log(f"request {w.name}: n={w.particles.n} grid {w.nx}x{w.ny} n_tel={w.n_tel} "
            f"resample={w.resample}")
    reqs = _requests(ws)
    plain = _plain_cubes(dssp, reqs)
    ex = GraphExecutor(dssp, max_jobs=4, lanes=1, mode=mode, grid_blocks=1024)
    mix = _graph_batch(ex, reqs)
    alone = [_graph_batch(ex, [r])[0] for r in reqs]
    for k in range(len(reqs)):
        assert plain[k].abs().max() > 0
        assert torch.equal(mix[k], plain[k]), k
        assert torch.equal(alone[k], plain[k]), k


@pytest.mark.parametrize("mode", ["native", "persistent"])
def test_batch_on_log_lambda_grids(mode):
    """An executor on an SSP grid uniform in ln(lambda): requests of different sizes, orientations
    and telescope grids (bins of 0.8 to 2.1 SSP steps), alternating bin centres and bin means;
    every cube equals the plain entry points' bitwise, in the mix and alone."""
    ssp = synth.cached_ssp(40, 8, 3600.0, 1.2e-4, 3000, log_lambda=True)
    dssp_log = ops.DeviceSSP.from_grid(ssp)
    ws = []
    for k, (n, ratio, n_tel, incl) in enumerate([(3000, 1.0, 2900, 30.0), (20000, 1.3, 2000, 60.0),
                                                 (50000, 0.8, 3300, 75.0), (8000, 2.1, 1200, 10.0)]):
        side = 24 + 4 * k
        w = synth.Workload(f"log{k}", synth.make_galaxy(n, 600 + k), (incl, 0.0, 0.0), side, side,
                           30.0 / side, 3600.0 * np.exp((0.37 + 5 * k) * 1.2e-4), 1.2e-4 * ratio,
                           n_tel, ssp, psf_sigma_spx=1.0, lsf_sigma_A=1.2, z_sys=0.002,
                           log_lambda=True)
        w.resample = k % 2
        log(f"request {w.name}: n={n} grid {side}x{side} n_tel={n_tel} ratio={ratio} "
            f"resample={w.resample}")
        ws.append(w)
    reqs = _requests(ws)
    plain = _plain_cubes(dssp_log, reqs)
    ex = GraphExecutor(dssp_log, max_jobs=4, lanes=1, mode=mode, grid_blocks=1024)
    mix = _graph_batch(ex, reqs[::-1])[::-1]
    alone = [_graph_batch(ex, [r])[0] for r in reqs]
    for k in range(len(reqs)):
        assert plain[k].abs().max() > 0
        assert torch.equal(mix[k], plain[k]), k
        assert torch.equal(alone[k], plain[k]), k
    # a request on a linear telescope grid is rejected at submission, before any launch
    lin = synth.serving_request(0, n_max=2e3, n_min=1e3)
    s = Scheduler(ex, budget_bytes=1 << 30, max_slots=2)
    fut = s.submit(Request.from_particles(lin.particles, ops.Observation.from_workload(lin), rid=9))
    with pytest.raises(Rejected, match="linear in lambda but SSP grid uniform in ln"):
        fut.result(timeout=0)


def test_served_bin_mean_request_matches_oracle(ssp_grid, dssp):
    w = synth.serving_request(5, ssp_grid, n_max=3e4, n_min=1e4)
    w.resample = 1
    req = Request.from_particles(w.particles, ops.Observation.from_workload(w), rid=0)
    ex = GraphExecutor(dssp, max_jobs=4, lanes=2)
    s = Scheduler(ex, budget_bytes=8 << 30, max_slots=4)
    fut = s.submit(req)
    s.drain()
    cube = fut.result(timeout=0).cube.cpu().numpy().reshape(w.nx * w.ny, w.n_tel)
    fo = O.forward(w.particles, O.config_from_workload(w), workers=1, ties=TIES)
    assert_cube_in(cube, fo, "cube", what=f"served bin-mean cube ({w.particles.n} particles)")


def test_served_request_matches_oracle(ssp_grid, dssp):
    w = synth.serving_request(3, ssp_grid, n_max=3e4, n_min=1e4)
    req = Request.from_particles(w.particles, ops.Observation.from_workload(w), rid=0)
    ex = GraphExecutor(dssp, max_jobs=4, lanes=2)
    s = Scheduler(ex, budget_bytes=8 << 30, max_slots=4)
    fut = s.submit(req)
    s.drain()
    cube = fut.result(timeout=0).cube.cpu().numpy().reshape(w.nx * w.ny, w.n_tel)
    fo = O.forward(w.particles, O.config_from_workload(w), workers=1, ties=TIES)
    assert_cube_in(cube, fo, "cube", what=f"served cube ({w.particles.n} particles)")


def test_trace_through_scheduler_small_budget(ssp_grid, dssp):
    """A Poisson trace through the graph executor under a budget that admits only a few requests
    at a time: every request completes with the plain path's cube."""
    ws = _workloads(ssp_grid, range(20, 32), n_max=1e5)
    reqs = _requests(ws)
    ref = _plain_cubes(dssp, reqs)
    ex = GraphExecutor(dssp, max_jobs=8, lanes=2)
    budget = 3 * max(ex.footprint(r) for r in reqs)
    s = Scheduler(ex, budget_bytes=budget, max_slots=8)
    arrivals = synth.poisson_arrivals(len(reqs), 2000.0, seed=5)
    rep = replay_trace(s, reqs, arrivals)
    log(f"trace: {rep['batches']} batches, mean size {rep['mean_batch']:.2f}, peak budget use "
        f"{rep['peak_budget_bytes']}/{budget}, p50 {rep['p50_ms']:.2f} ms")
    assert rep["errors"] == 0
    assert rep["peak_budget_bytes"] <= budget
    for k, f in enumerate(rep["futures"]):
        assert torch.equal(f.result(timeout=0).cube.cpu(), ref[k]), k


@pytest.mark.parametrize("mode,req", [("native", 4), ("persistent", 4), ("native", 207),
                                      ("persistent", 207)])
def test_million_particle_request_in_a_mixed_batch(ssp_grid, dssp, mode, req):
    """A large request of the serving trace (request 4: 1.47e6 particles, 29x29 spaxels, 3669
    bins; request 207, the trace's largest: 5.0e6 particles, 67x67 spaxels, 2889 bins) batched
    with four small requests: its cube equals the plain entry points' bitwise alone and in the
    mix; against the oracle, the C_raw rows of its 16 heaviest and 64 random spaxels in full and
    the final cube of every spaxel on 64 interior bins (tie bounds), within 1e-5."""
    from helpers import gpu_forward, oracle_final_window, oracle_rows_parallel, outside
    big = synth.serving_request(req, ssp_grid)
    assert big.particles.n >= 1_000_000
    ws = [big] + _workloads(ssp_grid, range(4))
    for w in ws:
        log(f"request {w.name}: n={w.particles.n} grid {w.nx}x{w.ny} n_tel={w.n_tel}")
    reqs = _requests(ws)
    plain = _plain_cubes(dssp, reqs)
    ex = GraphExecutor(dssp, max_jobs=8, lanes=1, mode=mode, grid_blocks=1024)
    mix = _graph_batch(ex, reqs[::-1])[::-1]
    alone = _graph_batch(ex, reqs[:1])[0]
    for k in range(len(reqs)):
        assert torch.equal(mix[k], plain[k]), k
    assert torch.equal(alone, plain[0])
    if mode != "native":
        return
    # the served cube of the big request against the oracle (the same bytes in both modes)
    cfg = O.config_from_workload(big)
    fo = O.forward(big.particles, cfg, with_cube=False)
    g = plain[0].numpy().reshape(big.nx * big.ny, big.n_tel)
    cnt = np.diff(fo["seg_off"])
    rng = np.random.default_rng(4)
    nonempty = np.flatnonzero(cnt > 0)
    spx = list(dict.fromkeys([int(s) for s in np.r_[np.argsort(-cnt, kind="stable")[:16],
                                                     rng.choice(nonempty, 64, replace=False)]]))
    log(f"big request: oracle C_raw rows of {len(spx)} spaxels (max count {cnt[spx].max()})")
    ref, lo, hi, nt = oracle_rows_parallel(big.particles, cfg, fo, spx, ties=TIES)
    # C_raw from a plain forward of the same request (its final cube equals the served one)
    _, gp = gpu_forward(big)
    assert np.array_equal(gp["cube"], g)
    e = outside(gp["cube_raw"][spx], lo, hi).max() / np.abs(ref).max()
    log(f"big request: sampled C_raw rows within {e:.3e} of the oracle's range ({nt} ties)")
    assert e <= 1e-5
    j0 = int(rng.integers(64, big.n_tel - 128))
    fin, flo, fhi, ft = oracle_final_window(big.particles, cfg, fo, j0, j0 + 64, ties=TIES)
    e = outside(g[:, j0:j0 + 64], flo, fhi).max() / np.abs(fin).max()
    log(f"big request: final cube bins {j0}..{j0 + 63} within {e:.3e} of the oracle's range")
    assert e <= 1e-5


def test_failed_launch_returns_its_lane(ssp_grid, dssp, monkeypatch):
    """A launch that fails after its lane was taken gives the lane back: with one lane, the next
    batch still launches and gives the plain path's cube."""
    reqs = _requests(_workloads(ssp_grid, range(40, 42), n_max=2e4))
    ref = _plain_cubes(dssp, reqs)
    ex = GraphExecutor(dssp, max_jobs=4, lanes=1, mode="native", grid_blocks=256)

    def boom(*a, **k):
        raise RuntimeError("injected launch failure")

    real = ops.rubix_graph_launch
    monkeypatch.setattr(ops, "rubix_graph_launch", boom)
    with pytest.raises(RuntimeError, match="injected"):
        ex.launch(reqs)
    monkeypatch.setattr(ops, "rubix_graph_launch", real)
    got = _graph_batch(ex, reqs)
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
