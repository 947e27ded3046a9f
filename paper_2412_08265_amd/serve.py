"""Continuous-batching server for mock-observation requests.

A request is one galaxy (star particles on the host) plus an Observation. The SSP template grid is
shared by every request and stays resident in device memory. The scheduler admits queued requests
in arrival order into batches, bounded by
  - a device-memory budget: the sum of the footprints (particles, outputs, workspace) of all
    batches in flight never exceeds it; a request whose footprint alone exceeds it is rejected
    when it is submitted;
  - a slot count: at most `max_slots` requests per batch;
and hands each batch to an executor as soon as the executor has a free lane. Arrivals that come
while the device is busy queue up and form the next batch (continuous batching at the granularity
of one forward pass, which is the unit of work of this model).

Failure handling: a batch whose launch or completion fails is split, and its requests are run
again one at a time at the head of the queue, so one bad request fails alone. Requests that wait
longer than `queue_timeout_s` fail with QueueTimeout. The queue is not persisted.

Executors:
  GraphExecutor  the batch's job table is packed on the host (rubix_forward_pack) into the lane's
                 pinned buffer; the lane's forward graph (captured once by the library) copies it
                 to the lane's device table and runs every kernel with the batch's grid, in one
                 graph launch. Particle uploads run on a copy stream, overlapping the kernels of
                 the batch ahead.
  PlainExecutor  one request at a time with the plain entry points rubix_rotate_bin, rubix_cube
                 and rubix_psf_lsf (no batching, no graph): the baseline.
Both give bitwise the same cube for a request (the packed path runs the same kernels over the same
per-job work items), alone or in any batch.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from concurrent.futures import Future
from typing import Any, Callable, Deque, List, Optional, Sequence

import numpy as np
import torch

from . import ops
from ._lib import RubixGrid, RubixJob, RubixLGrid, RubixParticles

FIELDS = ops.FIELDS


class Rejected(RuntimeError):
    """The request can never be served under this scheduler's limits."""


class QueueTimeout(RuntimeError):
    """The request waited in the queue longer than the scheduler's timeout."""


@dataclasses.dataclass
class Request:
    """One mock observation: particles as a [9, n] FP32 host tensor (rows in FIELDS order; pinned
    memory lets the upload overlap compute) and the observation."""
    host: torch.Tensor
    obs: ops.Observation
    rid: int = -1

    @property
    def n(self) -> int:
        return int(self.host.shape[1])

    @classmethod
    def from_particles(cls, p, obs: ops.Observation, rid: int = -1,
                       pin: bool = True) -> "Request":
        """From any object with FP32 arrays x, y, z, vx, vy, vz, mass, age, met."""
        n = len(p.x)
        t = torch.empty((len(FIELDS), n), dtype=torch.float32, pin_memory=pin)
        for k, f in enumerate(FIELDS):
            t[k].copy_(torch.from_numpy(np.ascontiguousarray(getattr(p, f), dtype=np.float32)))
        return cls(t, obs, rid)


@dataclasses.dataclass
class Result:
    rid: int
    cube: torch.Tensor          # [ny, nx, n_tel] FP32, device memory, owned by the caller


@dataclasses.dataclass
class _Entry:
    req: Request
    future: Future
    footprint: int
    arrival: float
    solo: bool = False          # its batch failed: run it alone


@dataclasses.dataclass
class _Batch:
    handle: Any
    entries: List[_Entry]
    footprint: int


class Scheduler:
    """FIFO continuous batching over an executor.

    The executor provides footprint(req) -> bytes, check(req) (raises if it cannot serve the
    request at all), lanes (batches it can hold in flight), launch(requests) -> handle (enqueues
    the work and returns at once), done(handle) -> bool and collect(handle) -> list of Result (in
    request order; raises if the batch failed).
    """

    def __init__(self, executor, budget_bytes: int, max_slots: int = 16,
                 queue_timeout_s: Optional[float] = None,
                 clock: Callable[[], float] = time.perf_counter):
        if max_slots < 1:
            raise ValueError("max_slots must be >= 1")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.timeout = queue_timeout_s
        self.clock = clock
        self.queue: Deque[_Entry] = collections.deque()
        self.inflight: Deque[_Batch] = collections.deque()
        self.used = 0
        self.peak_used = 0
        self.batch_sizes: List[int] = []

    # -- client side ------------------------------------------------------------------------------
    def submit(self, req: Request, arrival: Optional[float] = None) -> Future:
        fut: Future = Future()
        t = self.clock() if arrival is None else arrival
        try:
            self.ex.check(req)
            fp = int(self.ex.footprint(req))
        except Exception as e:                     # noqa: BLE001 (reported through the future)
            fut.set_exception(Rejected(f"request {req.rid}: {e}"))
            return fut
        if fp > self.budget:
            fut.set_exception(Rejected(f"request {req.rid} needs {fp} B of device memory, "
                                       f"more than the whole budget of {self.budget} B"))
            return fut
        self.queue.append(_Entry(req, fut, fp, t))
        return fut

    def busy(self) -> bool:
        return bool(self.queue or self.inflight)

    def poll(self) -> bool:
        """One scheduling round: complete finished batches, expire, admit. Returns True if
        anything changed."""
        changed = self._reap()
        changed |= self._expire()
        changed |= self._admit()
        return changed

    def drain(self, idle_sleep_s: float = 20e-6) -> None:
        while self.busy():
            if not self.poll():
                time.sleep(idle_sleep_s)

    # -- internals --------------------------------------------------------------------------------
    def _reap(self) -> bool:
        changed = False
        while self.inflight and self.ex.done(self.inflight[0].handle):
            b = self.inflight.popleft()
            self.used -= b.footprint
            changed = True
            try:
                results = self.ex.collect(b.handle)
            except Exception as e:                 # noqa: BLE001
                self._failed(b.entries, e)
                continue
            for ent, res in zip(b.entries, results):
                ent.future.set_result(res)
        return changed

    def _expire(self) -> bool:
        if self.timeout is None or not self.queue:
            return False
        now = self.clock()
        keep: Deque[_Entry] = collections.deque()
        changed = False
        for ent in self.queue:
            if now - ent.arrival > self.timeout:
                ent.future.set_exception(QueueTimeout(
                    f"request {ent.req.rid} waited {now - ent.arrival:.3f} s > {self.timeout} s"))
                changed = True
            else:
                keep.append(ent)
        self.queue = keep
        return changed

    def _failed(self, entries: List[_Entry], err: Exception) -> None:
        if len(entries) == 1:
            entries[0].future.set_exception(err)
            return
        for ent in entries:
            ent.solo = True
        self.queue.extendleft(reversed(entries))

    def _admit(self) -> bool:
        changed = False
        while self.queue and len(self.inflight) < self.ex.lanes:
            batch: List[_Entry] = []
            fp = 0
            while self.queue and len(batch) < self.max_slots:
                ent = self.queue[0]
                if ent.solo and batch:
                    break
                if self.used + fp + ent.footprint > self.budget:
                    break                          # FIFO: nobody overtakes the head
                batch.append(self.queue.popleft())
                fp += ent.footprint
                if ent.solo:
                    break
            if not batch:
                break                              # the head waits for memory to come back
            changed = True
            try:
                h = self.ex.launch([e.req for e in batch])
            except Exception as e:                 # noqa: BLE001
                self._failed(batch, e)
                continue
            self.used += fp
            self.peak_used = max(self.peak_used, self.used)
            self.batch_sizes.append(len(batch))
            self.inflight.append(_Batch(h, batch, fp))
        return changed


# --------------------------------------------------------------------------------------------------
# device executors
# --------------------------------------------------------------------------------------------------
def _size_job(req: Request) -> RubixJob:
    o = req.obs
    j = RubixJob()
    j.p = RubixParticles(req.n, *([None] * 9))
    j.grid = RubixGrid(int(o.nx), int(o.ny), float(o.spaxel_kpc))
    j.tel = RubixLGrid(float(o.tel_start), float(o.tel_step), int(o.n_tel), int(o.log_lambda))
    j.psf_sigma_spx, j.lsf_sigma_A = float(o.psf_sigma_spx), float(o.lsf_sigma_A)
    j.resample = int(o.resample)
    return j


def check_grid_kind(ssp: ops.DeviceSSP, req: Request) -> None:
    """A request's telescope grid must be of the executor's SSP grid kind (linear in lambda or
    uniform in ln lambda): the library refuses a launch that mixes them, which would fail the
    whole batch."""
    if bool(req.obs.log_lambda) != ssp.log_lambda:
        kind = ("uniform in ln(lambda)", "linear in lambda")
        raise ValueError(f"telescope grid {kind[not req.obs.log_lambda]} but SSP grid "
                         f"{kind[not ssp.log_lambda]}")


def _al(b: int) -> int:
    return (b + 511) // 512 * 512        # torch's allocator rounds blocks to 512 bytes


def sort_passes(obs: ops.Observation) -> int:
    """Radix passes of the spaxel-key sort (8 bits each over keys 0..nx*ny)."""
    return max(1, (int(obs.nx * obs.ny).bit_length() + 7) // 8)


def psf_radius(obs: ops.Observation) -> int:
    return int(4.0 * obs.psf_sigma_spx + 0.5) if obs.psf_sigma_spx > 0 else 0


class _DeviceExecutorBase:
    def __init__(self, ssp: ops.DeviceSSP, device="cuda"):
        self.ssp = ssp
        self.device = torch.device(device)
        self.compute = torch.cuda.Stream(self.device)      # default priority
        self.copy = torch.cuda.Stream(self.device)

    def footprint(self, req: Request) -> int:
        n, o = req.n, req.obs
        regions = ops.rubix_workspace_size([_size_job(req)]) - ops.rubix_table_bytes(1)
        n_s = o.nx * o.ny
        return (_al(36 * n) + 3 * _al(4 * n) + _al(4 * (n_s + 1)) + 2 * _al(4 * n_s * o.n_tel)
                + _al(regions))

    def _upload(self, reqs: Sequence[Request]):
        """Particle H2D on the copy stream; returns device galaxies and the upload event."""
        gals, hosts = [], []
        with torch.cuda.stream(self.copy):
            for r in reqs:
                d = r.host.to(self.device, non_blocking=True)
                hosts.append(d)
                gals.append(ops.DeviceGalaxy({f: d[k] for k, f in enumerate(FIELDS)}))
        ev = torch.cuda.Event()
        ev.record(self.copy)
        return gals, hosts, ev

    @staticmethod
    def done(h) -> bool:
        return h["done"].query()


class GraphExecutor(_DeviceExecutorBase):
    """Batched forward passes launched as HIP graphs, one graph per lane.

    mode "native" (default): the library's forward graph (rubix_graph_create): each launch copies
      the batch's packed table to the lane's device table and sets every kernel's grid to the
      batch's work-item count, so the kernels run exactly as in the plain entry points.
    mode "persistent": rubix_forward_packed captured once per lane in a torch CUDA graph and
      replayed unchanged; every kernel runs grid_blocks blocks that stride over the work items.
    """

    def __init__(self, ssp: ops.DeviceSSP, max_jobs: int = 16, lanes: int = 2,
                 mode: str = "native", grid_blocks: int = 2048, max_psf_radius: int = 16,
                 max_sort_passes: int = 2, device="cuda"):
        super().__init__(ssp, device)
        if not 1 <= max_jobs <= 64:
            raise ValueError("max_jobs must be in [1, 64]")
        if mode not in ("native", "persistent"):
            raise ValueError(f"unknown graph mode {mode!r}")
        self.mode = mode
        self.max_jobs, self.lanes = max_jobs, lanes
        self.grid_blocks = grid_blocks
        self.max_psf_radius, self.max_sort_passes = max_psf_radius, max_sort_passes
        nb = ops.rubix_table_bytes(max_jobs)
        self._free: Deque[dict] = collections.deque()
        self._graphs: List[int] = []
        self._warm()
        for _ in range(lanes):
            lane = {"dev": torch.empty(nb, dtype=torch.uint8, device=self.device),
                    "host": torch.empty(nb, dtype=torch.uint8, pin_memory=True)}
            if mode == "native":
                lane["graph"] = ops.rubix_graph_create(lane["dev"], max_jobs, max_psf_radius,
                                                       max_sort_passes)
                self._graphs.append(lane["graph"])
            else:
                lane["graph"] = torch.cuda.CUDAGraph()
                torch.cuda.synchronize(self.device)
                with torch.cuda.graph(lane["graph"], stream=self.compute):
                    ops.rubix_forward_packed(lane["dev"], grid_blocks, max_psf_radius,
                                             max_sort_passes)
            self._free.append(lane)

    def close(self) -> None:
        """Release the native graphs (their launches must have completed)."""
        torch.cuda.synchronize(self.device)
        while self._graphs:
            ops.rubix_graph_destroy(self._graphs.pop())

    def __del__(self):
        try:
            if self._graphs:
                self.close()
        except Exception:                         # noqa: BLE001 (interpreter shutdown)
            pass

    def _warm(self) -> None:
        """Run the packed launch sequence once eagerly on a tiny job, so that every kernel's code
        is loaded on the device before the launches are captured."""
        n = 256
        z = torch.zeros((len(FIELDS), n), dtype=torch.float32, device=self.device)
        z[FIELDS.index("age")] = 1.0
        gal = ops.DeviceGalaxy({f: z[k] for k, f in enumerate(FIELDS)})
        ssp = self.ssp
        # a telescope grid of the SSP grid's kind (the library refuses mixed kinds), 64 bins from
        # the SSP grid's 10th node, LSF about one bin wide
        if ssp.log_lambda:
            t0, lsf = ssp.lam_start * math.exp(10 * ssp.lam_step), ssp.lam_start * ssp.lam_step
        else:
            t0, lsf = ssp.lam_start + 10 * ssp.lam_step, ssp.lam_step
        obs = ops.Observation((0.0, 0.0, 0.0), 2, 2, 1.0, t0, ssp.lam_step, 64, psf_sigma_spx=0.5,
                              lsf_sigma_A=lsf, log_lambda=ssp.log_lambda)
        buf = ops.JobBuffers.allocate(n, obs, self.device)
        job = ops.make_job(gal, obs, buf)
        nt = ops.rubix_table_bytes(1)
        ws = ops.workspace(ops.rubix_workspace_size([job], ssp) - nt, self.device)
        host = torch.empty(nt, dtype=torch.uint8, pin_memory=True)
        dev = torch.empty(nt, dtype=torch.uint8, device=self.device)
        ops.rubix_forward_pack([job], ssp, ws, host, self.max_psf_radius, self.max_sort_passes)
        dev.copy_(host)
        ops.rubix_forward_packed(dev, self.grid_blocks, self.max_psf_radius, self.max_sort_passes)
        torch.cuda.synchronize(self.device)

    def check(self, req: Request) -> None:
        check_grid_kind(self.ssp, req)
        if psf_radius(req.obs) > self.max_psf_radius:
            raise ValueError(f"PSF radius {psf_radius(req.obs)} > {self.max_psf_radius}")
        if sort_passes(req.obs) > self.max_sort_passes:
            raise ValueError(f"{req.obs.nx}x{req.obs.ny} spaxels need {sort_passes(req.obs)} "
                             f"sort passes > {self.max_sort_passes}")

    def launch(self, reqs: Sequence[Request]):
        if len(reqs) > self.max_jobs:
            raise ValueError(f"batch of {len(reqs)} > max_jobs {self.max_jobs}")
        if not self._free:
            raise RuntimeError("no free lane")
        gals, hosts, up = self._upload(reqs)
        with torch.cuda.stream(self.compute):
            bufs = [ops.JobBuffers.allocate(g.n, r.obs, self.device) for g, r in zip(gals, reqs)]
            jobs = [ops.make_job(g, r.obs, b) for g, r, b in zip(gals, reqs, bufs)]
            nt = ops.rubix_table_bytes(len(jobs))
            ws = ops.workspace(ops.rubix_workspace_size(jobs, self.ssp) - nt, self.device)
            lane = self._free[0]
            ops.rubix_forward_pack(jobs, self.ssp, ws, lane["host"], self.max_psf_radius,
                                   self.max_sort_passes)
            self._free.popleft()
            try:
                self.compute.wait_event(up)
                for d in hosts:
                    d.record_stream(self.compute)
                if self.mode == "native":
                    ops.rubix_graph_launch(lane["graph"], lane["host"][:nt])
                else:
                    lane["dev"][:nt].copy_(lane["host"][:nt], non_blocking=True)
                    lane["graph"].replay()
            except BaseException:
                # the lane goes back once whatever reached the stream has finished with its
                # buffers, so a failed launch does not lose it
                self.compute.synchronize()
                self._free.append(lane)
                raise
            done = torch.cuda.Event()
            done.record(self.compute)
        return {"lane": lane, "done": done, "bufs": bufs, "hosts": hosts, "ws": ws,
                "rids": [r.rid for r in reqs]}

    def collect(self, h) -> List[Result]:
        self._free.append(h["lane"])
        return [Result(rid, b.cube) for rid, b in zip(h["rids"], h["bufs"])]


class PlainExecutor(_DeviceExecutorBase):
    """One request per launch sequence with the plain entry points (the baseline)."""

    lanes = 1

    def check(self, req: Request) -> None:
        check_grid_kind(self.ssp, req)

    def launch(self, reqs: Sequence[Request]):
        if len(reqs) != 1:
            raise ValueError("PlainExecutor runs one request at a time")
        gals, hosts, up = self._upload(reqs)
        r, g = reqs[0], gals[0]
        with torch.cuda.stream(self.compute):
            buf = ops.JobBuffers.allocate(g.n, r.obs, self.device)
            job = ops.make_job(g, r.obs, buf)
            ws = ops.workspace(ops.rubix_workspace_size([job], self.ssp), self.device)
            self.compute.wait_event(up)
            for d in hosts:
                d.record_stream(self.compute)
            ops.rubix_rotate_bin([job], ws)
            ops.rubix_cube([job], self.ssp, ws)
            ops.rubix_psf_lsf([job], [buf.cube_raw], [buf.cube], ws)
            done = torch.cuda.Event()
            done.record(self.compute)
        return {"done": done, "buf": buf, "hosts": hosts, "ws": ws, "rid": r.rid}

    def collect(self, h) -> List[Result]:
        return [Result(h["rid"], h["buf"].cube)]


# --------------------------------------------------------------------------------------------------
# trace replay
# --------------------------------------------------------------------------------------------------
def replay_trace(sched: Scheduler, requests: Sequence[Request], arrivals_s: Sequence[float],
                 clock: Callable[[], float] = time.perf_counter, poll_sleep_s: float = 20e-6) -> dict:
    """Submit requests[i] at arrivals_s[i] seconds after the start (real time) and run the
    scheduler until every request has finished. Latency = completion - arrival."""
    futs: List[Future] = []
    done_at: List[float] = [math.nan] * len(requests)
    t0 = clock()
    i, n = 0, len(requests)

    def on_done(k):
        return lambda f: done_at.__setitem__(k, clock())

    n_batches0 = len(sched.batch_sizes)
    while i < n or sched.busy():
        now = clock() - t0
        while i < n and arrivals_s[i] <= now:
            f = sched.submit(requests[i], arrival=t0 + arrivals_s[i])
            f.add_done_callback(on_done(i))
            futs.append(f)
            i += 1
        if not sched.poll():
            time.sleep(poll_sleep_s)
    ok = [k for k, f in enumerate(futs) if f.exception() is None]
    lat = np.array([done_at[k] - (t0 + arrivals_s[k]) for k in ok], dtype=np.float64)
    span = max(done_at[k] for k in ok) - t0 if ok else math.nan
    sizes = sched.batch_sizes[n_batches0:]
    return {"requests": n, "errors": n - len(ok),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if ok else math.nan,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if ok else math.nan,
            "mean_ms": float(lat.mean() * 1e3) if ok else math.nan,
            "cubes_per_s": len(ok) / span if ok and span > 0 else math.nan,
            "span_s": span, "batches": len(sizes),
            "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
            "peak_budget_bytes": sched.peak_used, "futures": futs}
