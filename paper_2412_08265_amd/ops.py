"""Python front end of the HIP datacube forward model.

The entry points `rubix_rotate_bin`, `rubix_cube`, `rubix_psf_lsf` and `rubix_cube_backward` carry
the names of the C ABI (include/rubix.h) and only marshal arguments: every step of the forward
model and its adjoint runs in the library's HIP kernels. torch provides device memory (tensors)
and the stream (the current torch stream unless one is given).

Higher-level helpers: `DeviceSSP`, `DeviceGalaxy`, `Observation`, `forward()` (one galaxy through
the whole pipeline) and `RubixCube`, a torch.autograd.Function whose backward is the hand-written
adjoint kernel.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from ctypes import POINTER, byref, c_float, c_size_t, c_void_p
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import RubixGrid, RubixJob, RubixLGrid, RubixParticles, RubixSSP, check, ptr_array

C_KMS = 299792.458


# --------------------------------------------------------------------------------------------------
# device-side inputs
# --------------------------------------------------------------------------------------------------
class DeviceSSP:
    """SSP template grid resident in device memory (flux [n_age][n_met][n_lam] FP32)."""

    def __init__(self, log_age_nodes, met_nodes, lam_start, lam_step, flux, device="cuda",
                 log_lambda=False):
        self.log_age_nodes = np.ascontiguousarray(log_age_nodes, dtype=np.float32)
        self.met_nodes = np.ascontiguousarray(met_nodes, dtype=np.float32)
        flux = np.ascontiguousarray(flux, dtype=np.float32)
        self.flux = torch.from_numpy(flux).to(device)
        self.lam_start, self.lam_step = float(lam_start), float(lam_step)
        self.n_lam = int(flux.shape[2])
        self.log_lambda = bool(log_lambda)
        self.c = RubixSSP(self.log_age_nodes.shape[0], self.met_nodes.shape[0],
                          self.log_age_nodes.ctypes.data_as(POINTER(c_float)),
                          self.met_nodes.ctypes.data_as(POINTER(c_float)),
                          RubixLGrid(self.lam_start, self.lam_step, self.n_lam,
                                     int(self.log_lambda)),
                          self.flux.data_ptr())

    @classmethod
    def from_grid(cls, g, device="cuda") -> "DeviceSSP":
        """From any object with log_age_nodes, met_nodes, lam_start, lam_step, flux (and
        optionally log_lambda)."""
        return cls(g.log_age_nodes, g.met_nodes, g.lam_start, g.lam_step, g.flux, device,
                   getattr(g, "log_lambda", False))


FIELDS = ("x", "y", "z", "vx", "vy", "vz", "mass", "age", "met")


class DeviceGalaxy:
    """Star particles as FP32 device tensors (structure of arrays)."""

    def __init__(self, tensors: Dict[str, torch.Tensor]):
        for f in FIELDS:
            t = tensors[f]
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{f} must be a contiguous float32 device tensor")
            setattr(self, f, t)
        self.n = int(self.x.shape[0])

    @classmethod
    def from_host(cls, p, device="cuda", non_blocking=False) -> "DeviceGalaxy":
        """From any object with FP32 numpy arrays x, y, z, vx, vy, vz, mass, age, met."""
        return cls({f: torch.from_numpy(np.ascontiguousarray(getattr(p, f), dtype=np.float32))
                    .to(device, non_blocking=non_blocking) for f in FIELDS})

    def particles_c(self) -> RubixParticles:
        return RubixParticles(self.n, *[getattr(self, f).data_ptr() for f in FIELDS])


@dataclasses.dataclass
class Observation:
    """Viewing geometry and instrument of one mock observation (the paper's JSON configuration,
    Sec. 3): orientation, spaxel grid, telescope wavelength grid, PSF and LSF."""
    angles_rad: tuple
    nx: int
    ny: int
    spaxel_kpc: float
    tel_start: float
    tel_step: float
    n_tel: int
    psf_sigma_spx: float = 0.0
    lsf_sigma_A: float = 0.0
    z_sys: float = 0.0
    flux_scale: float = 1.0
    log_lambda: bool = False     # telescope bins tel_start * exp(k * tel_step)
    resample: int = 0            # 0 bin-centre sampling, 1 bin mean (flux conserving)

    @classmethod
    def from_workload(cls, w) -> "Observation":
        return cls(tuple(w.angles_rad), w.nx, w.ny, w.spaxel_kpc, w.tel_start, w.tel_step,
                   w.n_tel, w.psf_sigma_spx, w.lsf_sigma_A, w.z_sys, w.flux_scale,
                   bool(getattr(w, "log_lambda", False)), int(getattr(w, "resample", 0)))

    @property
    def n_spaxels(self):
        return self.nx * self.ny


@dataclasses.dataclass
class JobBuffers:
    key: torch.Tensor
    perm: torch.Tensor
    seg_off: torch.Tensor
    vlos: torch.Tensor
    cube_raw: torch.Tensor
    cube: torch.Tensor

    @classmethod
    def allocate(cls, n: int, obs: Observation, device="cuda") -> "JobBuffers":
        shape = (obs.ny, obs.nx, obs.n_tel)
        return cls(torch.empty(n, dtype=torch.int32, device=device),
                   torch.empty(n, dtype=torch.int32, device=device),
                   torch.empty(obs.n_spaxels + 1, dtype=torch.int32, device=device),
                   torch.empty(n, dtype=torch.float32, device=device),
                   torch.empty(shape, dtype=torch.float32, device=device),
                   torch.empty(shape, dtype=torch.float32, device=device))


def make_job(gal: DeviceGalaxy, obs: Observation, buf: JobBuffers) -> RubixJob:
    j = RubixJob()
    j.p = gal.particles_c()
    for k in range(3):
        j.angles_rad[k] = float(obs.angles_rad[k])
    j.grid = RubixGrid(int(obs.nx), int(obs.ny), float(obs.spaxel_kpc))
    j.tel = RubixLGrid(float(obs.tel_start), float(obs.tel_step), int(obs.n_tel),
                       int(obs.log_lambda))
    j.z_sys, j.flux_scale = float(obs.z_sys), float(obs.flux_scale)
    j.psf_sigma_spx, j.lsf_sigma_A = float(obs.psf_sigma_spx), float(obs.lsf_sigma_A)
    j.resample = int(obs.resample)
    j.key, j.perm, j.seg_off = buf.key.data_ptr(), buf.perm.data_ptr(), buf.seg_off.data_ptr()
    j.vlos, j.cube_raw, j.cube = buf.vlos.data_ptr(), buf.cube_raw.data_ptr(), buf.cube.data_ptr()
    return j


def _jobs_array(jobs: Sequence[RubixJob]):
    arr = (RubixJob * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = j
    return arr


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


# --------------------------------------------------------------------------------------------------
# C ABI entry points (same names)
# --------------------------------------------------------------------------------------------------
def rubix_workspace_size(jobs: Sequence[RubixJob], ssp: Optional[DeviceSSP] = None) -> int:
    lib = _lib.load()
    arr = _jobs_array(jobs)
    out = c_size_t(0)
    check(lib.rubix_workspace_size(arr, len(jobs), byref(ssp.c) if ssp else None, byref(out)))
    return int(out.value)


def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    """A device workspace (torch's allocator returns 512-byte aligned blocks)."""
    t = torch.empty(max(256, nbytes), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


def rubix_rotate_bin(jobs, ws: torch.Tensor, stream=None) -> None:
    lib = _lib.load()
    check(lib.rubix_rotate_bin(_jobs_array(jobs), len(jobs), ws.data_ptr(), ws.numel(),
                               _stream(stream)))


def rubix_cube(jobs, ssp: DeviceSSP, ws: torch.Tensor, stream=None) -> None:
    lib = _lib.load()
    check(lib.rubix_cube(_jobs_array(jobs), len(jobs), byref(ssp.c), ws.data_ptr(), ws.numel(),
                         _stream(stream)))


def rubix_psf_lsf(jobs, ins: Sequence[torch.Tensor], outs: Sequence[torch.Tensor],
                  ws: torch.Tensor, stream=None) -> None:
    lib = _lib.load()
    a = ptr_array([t.data_ptr() for t in ins])
    b = ptr_array([t.data_ptr() for t in outs])
    check(lib.rubix_psf_lsf(_jobs_array(jobs), len(jobs), a, b, ws.data_ptr(), ws.numel(),
                            _stream(stream)))


def rubix_psf_lsf_noalloc(jobs, ins: Sequence[torch.Tensor], outs: Sequence[torch.Tensor],
                          stream=None) -> None:
    """rubix_psf_lsf with the library's static scratch instead of a workspace (no allocation)."""
    lib = _lib.load()
    a = ptr_array([t.data_ptr() for t in ins])
    b = ptr_array([t.data_ptr() for t in outs])
    check(lib.rubix_psf_lsf_noalloc(_jobs_array(jobs), len(jobs), a, b, _stream(stream)))


def rubix_cube_backward(jobs, ssp: DeviceSSP, grad_raw, d_mass, d_age, d_met, d_vlos, d_vel,
                        d_angles: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    lib = _lib.load()
    pa = lambda ts: ptr_array([t.data_ptr() for t in ts])
    vel = pa(d_vel) if d_vel is not None else None
    check(lib.rubix_cube_backward(_jobs_array(jobs), len(jobs), byref(ssp.c), pa(grad_raw),
                                  pa(d_mass), pa(d_age), pa(d_met), pa(d_vlos), vel,
                                  d_angles.data_ptr(), ws.data_ptr(), ws.numel(),
                                  _stream(stream)))


def rubix_table_bytes(n_jobs: int) -> int:
    return int(_lib.load().rubix_table_bytes(int(n_jobs)))


def rubix_forward_pack(jobs, ssp: DeviceSSP, ws: torch.Tensor, host_table: torch.Tensor,
                       max_psf_radius: int, max_sort_passes: int) -> None:
    """Write the packed table of a forward batch into host_table (a uint8 CPU tensor)."""
    lib = _lib.load()
    check(lib.rubix_forward_pack(_jobs_array(jobs), len(jobs), byref(ssp.c), ws.data_ptr(),
                                 ws.numel(), host_table.data_ptr(), host_table.numel(),
                                 int(max_psf_radius), int(max_sort_passes)))


def rubix_forward_packed(dev_table: torch.Tensor, grid_blocks: int, max_psf_radius: int,
                         max_sort_passes: int, stream=None) -> None:
    lib = _lib.load()
    check(lib.rubix_forward_packed(dev_table.data_ptr(), int(grid_blocks), int(max_psf_radius),
                                   int(max_sort_passes), _stream(stream)))


def rubix_graph_create(dev_table: torch.Tensor, max_jobs: int, max_psf_radius: int,
                       max_sort_passes: int) -> int:
    """Returns the graph handle (an address); release it with rubix_graph_destroy."""
    lib = _lib.load()
    out = c_void_p(None)
    check(lib.rubix_graph_create(dev_table.data_ptr(), int(max_jobs), int(max_psf_radius),
                                 int(max_sort_passes), byref(out)))
    return int(out.value)


def rubix_graph_launch(graph: int, host_table: torch.Tensor, stream=None) -> None:
    lib = _lib.load()
    check(lib.rubix_graph_launch(graph, host_table.data_ptr(), host_table.numel(),
                                 _stream(stream)))


def rubix_graph_destroy(graph: int) -> None:
    check(_lib.load().rubix_graph_destroy(graph))


def rubix_add_noise(jobs, noise: Sequence[dict], cubes: Sequence[torch.Tensor],
                    stream=None) -> None:
    """noise[k] = dict(seed=..., stream=..., gain=..., sigma_floor=...) for jobs[k]; adds the
    noise to cubes[k] in place."""
    lib = _lib.load()
    arr = (_lib.RubixNoise * len(jobs))()
    for k, p in enumerate(noise):
        arr[k] = _lib.RubixNoise(int(p["seed"]), int(p.get("stream", 0)), 0, float(p["gain"]),
                                 float(p["sigma_floor"]))
    check(lib.rubix_add_noise(_jobs_array(jobs), len(jobs), arr,
                              ptr_array([c.data_ptr() for c in cubes]), _stream(stream)))


def rubix_cube_timer(enable: bool) -> None:
    check(_lib.load().rubix_cube_timer(1 if enable else 0))


def rubix_cube_timer_read():
    """(summed ms, count) of the cube-summation kernel over the timed rubix_cube calls."""
    lib = _lib.load()
    ms, n = ctypes.c_double(0.0), ctypes.c_int(0)
    check(lib.rubix_cube_timer_read(byref(ms), byref(n)))
    return float(ms.value), int(n.value)


# --------------------------------------------------------------------------------------------------
# one galaxy through the pipeline
# --------------------------------------------------------------------------------------------------
class Forward:
    """Reusable forward pass of one galaxy configuration: buffers and workspace are allocated once
    and every call re-runs rotate/bin -> cube -> PSF/LSF on the current stream."""

    def __init__(self, gal: DeviceGalaxy, obs: Observation, ssp: DeviceSSP, device="cuda"):
        self.gal, self.obs, self.ssp = gal, obs, ssp
        self.buf = JobBuffers.allocate(gal.n, obs, device)
        self.job = make_job(gal, obs, self.buf)
        self.ws = workspace(rubix_workspace_size([self.job], ssp), device)

    def rotate_bin(self, stream=None):
        rubix_rotate_bin([self.job], self.ws, stream)

    def cube_raw(self, stream=None):
        rubix_cube([self.job], self.ssp, self.ws, stream)

    def psf_lsf(self, stream=None):
        rubix_psf_lsf([self.job], [self.buf.cube_raw], [self.buf.cube], self.ws, stream)

    def __call__(self, stream=None) -> JobBuffers:
        self.rotate_bin(stream)
        self.cube_raw(stream)
        self.psf_lsf(stream)
        return self.buf


def forward(gal: DeviceGalaxy, obs: Observation, ssp: DeviceSSP) -> JobBuffers:
    return Forward(gal, obs, ssp)()


class RubixCube(torch.autograd.Function):
    """cube = A C_raw(particles, angles) with the hand-written adjoint as backward.

    apply(x, y, z, vx, vy, vz, mass, age, met, angles, obs, ssp):
      particle fields are FP32 device tensors [n]; angles is a float64 CPU tensor [3] (the
      library needs the angles on the host to build the rotation matrix).
    Gradients flow to vx, vy, vz, mass, age, met and angles; positions get none (binning is
    piecewise constant); angle gradients hold the spaxel assignment fixed.
    """

    @staticmethod
    def forward(ctx, x, y, z, vx, vy, vz, mass, age, met, angles, obs: Observation,
                ssp: DeviceSSP):
        ang = tuple(float(a) for a in angles.detach().cpu().double().tolist())
        obs = dataclasses.replace(obs, angles_rad=ang)
        gal = DeviceGalaxy(dict(x=x.detach(), y=y.detach(), z=z.detach(), vx=vx.detach(),
                                vy=vy.detach(), vz=vz.detach(), mass=mass.detach(),
                                age=age.detach(), met=met.detach()))
        fw = Forward(gal, obs, ssp, device=x.device)
        buf = fw()
        ctx.fw = fw
        ctx.angles_device = angles.device
        ctx.angles_dtype = angles.dtype
        return buf.cube.clone()

    @staticmethod
    def backward(ctx, grad_cube):
        fw: Forward = ctx.fw
        g = grad_cube.contiguous()
        G = torch.empty_like(g)
        rubix_psf_lsf([fw.job], [g], [G], fw.ws)            # A is symmetric: A^T = A
        n = fw.gal.n
        dev = g.device
        d = {k: torch.empty(n, dtype=torch.float32, device=dev)
             for k in ("mass", "age", "met", "vlos")}
        d_vel = torch.empty((3, n), dtype=torch.float32, device=dev)
        d_ang = torch.empty(3, dtype=torch.float64, device=dev)
        rubix_cube_backward([fw.job], fw.ssp, [G], [d["mass"]], [d["age"]], [d["met"]],
                            [d["vlos"]], [d_vel], d_ang, fw.ws)
        ga = d_ang.to(ctx.angles_device, ctx.angles_dtype)
        return (None, None, None, d_vel[0], d_vel[1], d_vel[2], d["mass"], d["age"], d["met"],
                ga, None, None)


def cube_backward(fw: Forward, grad_raw: torch.Tensor):
    """Per-particle gradients for dL/dC_raw = grad_raw (after the adjoint PSF/LSF), using the
    buffers of an executed Forward. Returns a dict of device tensors."""
    n = fw.gal.n
    dev = grad_raw.device
    out = {k: torch.empty(n, dtype=torch.float32, device=dev)
           for k in ("mass", "age", "met", "vlos")}
    out["vel"] = torch.empty((3, n), dtype=torch.float32, device=dev)
    out["angles"] = torch.empty(3, dtype=torch.float64, device=dev)
    rubix_cube_backward([fw.job], fw.ssp, [grad_raw.contiguous()], [out["mass"]], [out["age"]],
                        [out["met"]], [out["vlos"]], [out["vel"]], out["angles"], fw.ws)
    return out
