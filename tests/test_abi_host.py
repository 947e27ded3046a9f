"""Host-side tests of the C ABI (no GPU needed): the library loads, exports every entry point the
header declares, sizes workspaces and rejects invalid arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2412_08265_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2412_08265_amd import build
        build.build()
    return _lib.load()


def _declared():
    with open(os.path.join(ROOT, "include", "rubix.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*(rubix_\w+)\s*\(", src, re.M)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"rubix_rotate_bin", "rubix_cube", "rubix_psf_lsf", "rubix_cube_backward",
            "rubix_workspace_size", "rubix_last_error", "rubix_table_bytes",
            "rubix_forward_pack", "rubix_forward_packed", "rubix_graph_create",
            "rubix_graph_launch", "rubix_graph_destroy", "rubix_psf_lsf_noalloc"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert lib.rubix_version().decode().startswith("rubix-mi355x")


def _job(n=100, nx=8, ny=6, tel_n=300):
    from paper_2412_08265_amd import ops
    j = ops.RubixJob()
    j.p.n = n
    fake = 0x1000
    for f in ops.FIELDS:
        setattr(j.p, f, fake)
    j.grid = ops.RubixGrid(nx, ny, 0.5)
    j.tel = ops.RubixLGrid(4000.0, 1.25, tel_n)
    j.flux_scale = 1.0
    j.key = j.perm = j.seg_off = j.vlos = j.cube_raw = j.cube = fake
    return j


def _arr(*jobs):
    from paper_2412_08265_amd import ops
    return (ops.RubixJob * len(jobs))(*jobs)


def _ws_size(lib, jobs, ssp=None):
    out = ctypes.c_size_t(0)
    rc = lib.rubix_workspace_size(_arr(*jobs), len(jobs), ssp, ctypes.byref(out))
    return rc, out.value


def test_workspace_size_grows_with_work(lib):
    rc, a = _ws_size(lib, [_job(1000)])
    assert rc == 0 and a > 0 and a % 256 == 0
    rc, b = _ws_size(lib, [_job(100000)])
    assert rc == 0 and b > a
    rc, c = _ws_size(lib, [_job(1000), _job(100000)])
    assert rc == 0 and c > b


@pytest.mark.parametrize("mut,code", [
    (lambda j: setattr(j.p, "n", -1), -1),
    (lambda j: setattr(j, "grid", type(j.grid)(0, 4, 1.0)), -1),
    (lambda j: setattr(j, "grid", type(j.grid)(4, 4, 0.0)), -1),
    (lambda j: setattr(j, "tel", type(j.tel)(4000.0, -1.0, 10)), -1),
    (lambda j: setattr(j, "tel", type(j.tel)(4000.0, 1.0, 0)), -1),
    (lambda j: setattr(j, "psf_sigma_spx", -0.5), -1),
    (lambda j: setattr(j, "lsf_sigma_A", 1000.0), -4),       # radius > RUBIX_MAX_RADIUS
    (lambda j: setattr(j, "z_sys", -1.0), -1),
    (lambda j: setattr(j.p, "n", 2 ** 31), -4),
])
def test_invalid_jobs_are_rejected(lib, mut, code):
    j = _job()
    mut(j)
    rc, _ = _ws_size(lib, [j])
    assert rc == code
    assert lib.rubix_last_error().decode() != ""


def test_entry_points_validate_before_launch(lib):
    from paper_2412_08265_amd import ops
    j = _job()
    j.p.x = None
    assert lib.rubix_rotate_bin(_arr(j), 1, None, 0, None) == -1
    assert b"position" in lib.rubix_last_error()
    j = _job()
    # workspace missing / misaligned / too small
    assert lib.rubix_rotate_bin(_arr(j), 1, None, 0, None) == -2
    assert lib.rubix_rotate_bin(_arr(j), 1, 0x1001, 1 << 30, None) == -2
    assert lib.rubix_rotate_bin(_arr(j), 1, 0x1000, 16, None) == -2
    assert lib.rubix_rotate_bin(_arr(j), 0, 0x1000, 1 << 30, None) == -1
    too_many = [_job() for _ in range(65)]
    assert lib.rubix_rotate_bin(_arr(*too_many), 65, 0x1000, 1 << 40, None) == -1


def test_noalloc_psf_lsf_rejects_before_device_work(lib):
    """The allocation-free PSF/LSF validates on the host and refuses a batch whose table and
    intermediate cubes exceed its static scratch, before touching a device."""
    from paper_2412_08265_amd import ops
    ins = ops.ptr_array([0x1000])
    outs = ops.ptr_array([0x1000 + (1 << 40)])
    j = _job(nx=8, ny=6, tel_n=300)
    assert lib.rubix_psf_lsf_noalloc(_arr(j), 1, None, outs, None) == -1
    # 4 * 1024 * 1024 * 16 bytes = 64 MiB of intermediate cube alone: one byte too many with the
    # table in front of it
    big = _job(nx=1024, ny=1024, tel_n=16)
    assert lib.rubix_psf_lsf_noalloc(_arr(big), 1, ins, outs, None) == -4
    assert b"scratch" in lib.rubix_last_error()
    over = [_job(nx=512, ny=512, tel_n=16) for _ in range(5)]     # 5 x 16 MiB
    a5 = ops.ptr_array([0x1000 + k * (1 << 32) for k in range(5)])
    b5 = ops.ptr_array([0x1000 + (1 << 40) + k * (1 << 32) for k in range(5)])
    assert lib.rubix_psf_lsf_noalloc(_arr(*over), 5, a5, b5, None) == -4
    # in and out overlapping
    assert lib.rubix_psf_lsf_noalloc(_arr(j), 1, ins, ins, None) == -1


def _ssp_c(la, mz, n_lam=100):
    from paper_2412_08265_amd import ops
    la = np.asarray(la, dtype=np.float32)
    mz = np.asarray(mz, dtype=np.float32)
    s = ops.RubixSSP(la.size, mz.size, la.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                     mz.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                     ops.RubixLGrid(3600.0, 2.0, n_lam), 0x1000)
    return s, (la, mz)


def test_ssp_validation(lib):
    good, keep = _ssp_c([-1, 0, 1], [-2, 0])
    assert _ws_size(lib, [_job()], ctypes.byref(good))[0] == 0
    for la, mz, n in (([-1, 0, 0], [-2, 0], 100), ([0], [-2, 0], 100), ([-1, 0], [0, -2], 100),
                      ([-1, float("nan")], [-2, 0], 100), ([-1, 0], [-2, 0], 1)):
        bad, keep2 = _ssp_c(la, mz, n)
        assert _ws_size(lib, [_job()], ctypes.byref(bad))[0] == -1, (la, mz, n)
    big, keep3 = _ssp_c(np.arange(256) * 0.01, np.arange(64) * 0.01, 200000)
    assert _ws_size(lib, [_job()], ctypes.byref(big))[0] == -4
    # the kernels' 32-bit byte offsets: 2^30 template values are one too many, 2^30 - 16384 fit
    edge, keep4 = _ssp_c(np.arange(256) * 0.01, np.arange(64) * 0.01, 65536)
    assert _ws_size(lib, [_job()], ctypes.byref(edge))[0] == -4
    fits, keep5 = _ssp_c(np.arange(256) * 0.01, np.arange(64) * 0.01, 65535)
    assert _ws_size(lib, [_job()], ctypes.byref(fits))[0] == 0


def test_packed_table_sizes_and_validation(lib):
    """The packed forward path checks its arguments on the host: table sizes, workspace regions,
    the replayed launch's PSF radius and sort passes, the launch shape."""
    from paper_2412_08265_amd import _lib
    t1, t64 = lib.rubix_table_bytes(1), lib.rubix_table_bytes(64)
    assert t1 > 0 and t1 % 256 == 0 and t64 > t1
    assert lib.rubix_table_bytes(0) == 0 and lib.rubix_table_bytes(65) == 0
    ssp, keep = _ssp_c([-1, 0, 1], [-2, 0])
    j = _job(n=1000)
    j.psf_sigma_spx = 2.0                      # radius 8
    rc, full = _ws_size(lib, [j])
    regions = full - t1
    host = (ctypes.c_uint8 * t1)()
    pack = lambda ws, nb, tb, r, p: lib.rubix_forward_pack(_arr(j), 1, ctypes.byref(ssp), ws, nb,
                                                          host, tb, r, p)
    assert pack(0x1000, regions, t1, 8, 1) == _lib.RUBIX_OK
    assert pack(0x1000, regions - 1, t1, 8, 1) == _lib.RUBIX_EWORKSPACE
    assert pack(0x1000, regions, t1 - 1, 8, 1) == _lib.RUBIX_EINVAL
    assert pack(0x1000, regions, t1, 7, 1) == _lib.RUBIX_ERANGE      # PSF radius 8 > 7
    big = _job(n=1000, nx=300, ny=300)          # 90001 keys: 3 radix passes
    rc, fb = _ws_size(lib, [big])
    assert lib.rubix_forward_pack(_arr(big), 1, ctypes.byref(ssp), 0x1000, fb, host, t1, 8,
                                  2) == _lib.RUBIX_ERANGE
    j.cube = None
    assert pack(0x1000, regions, t1, 8, 1) == _lib.RUBIX_EINVAL       # needs the cube output
    for args in ((None, 64, 8, 2), (0x1000, 0, 8, 2), (0x1000, 64, 65, 2), (0x1000, 64, 8, 0),
                 (0x1000, 64, 8, 5)):
        assert lib.rubix_forward_packed(*args, None) == _lib.RUBIX_EINVAL, args


def test_graph_entry_points_validate_before_device_work(lib):
    from paper_2412_08265_amd import _lib
    out = ctypes.c_void_p(1)
    create = lambda *a: lib.rubix_graph_create(*a, ctypes.byref(out))
    assert create(None, 4, 8, 2) == _lib.RUBIX_EINVAL and out.value is None
    assert create(0x1001, 4, 8, 2) == _lib.RUBIX_EINVAL          # misaligned table
    assert create(0x1000, 0, 8, 2) == _lib.RUBIX_EINVAL
    assert create(0x1000, 65, 8, 2) == _lib.RUBIX_EINVAL
    assert create(0x1000, 4, 65, 2) == _lib.RUBIX_EINVAL
    assert create(0x1000, 4, 8, 5) == _lib.RUBIX_EINVAL
    assert lib.rubix_graph_create(0x1000, 4, 8, 2, None) == _lib.RUBIX_EINVAL
    host = (ctypes.c_uint8 * 64)()
    assert lib.rubix_graph_launch(None, host, 64, None) == _lib.RUBIX_EINVAL
    assert lib.rubix_graph_destroy(None) == _lib.RUBIX_OK


def test_wavelength_grid_kinds_are_validated(lib):
    from paper_2412_08265_amd import _lib
    ssp, keep = _ssp_c([-1, 0, 1], [-2, 0])
    j = _job()
    assert _ws_size(lib, [j], ctypes.byref(ssp))[0] == _lib.RUBIX_OK
    ssp.lam.log_spaced = 1                      # log SSP grid, linear telescope grid
    assert _ws_size(lib, [j], ctypes.byref(ssp))[0] == _lib.RUBIX_EINVAL
    assert b"log-spaced" in lib.rubix_last_error()
    j.tel.log_spaced = 1
    assert _ws_size(lib, [j], ctypes.byref(ssp))[0] == _lib.RUBIX_OK
    j.tel.log_spaced = 2
    assert _ws_size(lib, [j])[0] == _lib.RUBIX_EINVAL
    j.tel.log_spaced = 1
    j.tel.start = -5.0                          # ln of a negative start
    assert _ws_size(lib, [j])[0] == _lib.RUBIX_EINVAL


def test_resample_mode_is_validated(lib):
    from paper_2412_08265_amd import _lib, ops
    j = _job()
    j.resample = 1
    assert _ws_size(lib, [j])[0] == _lib.RUBIX_OK
    j.resample = 2
    assert _ws_size(lib, [j])[0] == _lib.RUBIX_EINVAL
    j.resample = 1
    j.tel = ops.RubixLGrid(4000.0, 1.6e-4, 300, 1)    # bin mean on log grids
    assert _ws_size(lib, [j])[0] == _lib.RUBIX_OK
    lssp, keep_l = _ssp_c([-1, 0, 1], [-2, 0])
    lssp.lam = ops.RubixLGrid(3600.0, 1.6e-4, 100, 1)
    assert _ws_size(lib, [j], ctypes.byref(lssp))[0] == _lib.RUBIX_OK
    lssp.lam = ops.RubixLGrid(3600.0, 0.06, 100, 1)    # beyond the step its series admit
    rc = _ws_size(lib, [j], ctypes.byref(lssp))[0]
    assert rc == _lib.RUBIX_EINVAL and b"0.05" in lib.rubix_last_error()
    ptrs = (ctypes.c_void_p * 1)(0x1000)
    # the adjoint applies the same limit before any device work
    rc = lib.rubix_cube_backward(_arr(j), 1, ctypes.byref(lssp), ptrs, ptrs, ptrs, ptrs, ptrs,
                                 None, 0x1000, 0x1000, 1 << 40, None)
    assert rc == _lib.RUBIX_EINVAL and b"0.05" in lib.rubix_last_error()
    j.tel = ops.RubixLGrid(4000.0, 1.25, 300, 0)
    ssp, keep = _ssp_c([-1, 0, 1], [-2, 0])
    # the adjoint validates the mode before any device work
    j.resample = 2
    rc = lib.rubix_cube_backward(_arr(j), 1, ctypes.byref(ssp), ptrs, ptrs, ptrs, ptrs, ptrs,
                                 None, 0x1000, 0x1000, 1 << 40, None)
    assert rc == _lib.RUBIX_EINVAL and b"resample" in lib.rubix_last_error()


def test_product_path_never_touches_the_oracle():
    """The HIP package and its binding import nothing from the oracle (and vice versa)."""
    pkg = os.path.join(ROOT, "paper_2412_08265_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dp, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", src, re.M), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith(".py"):
            src = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2412_08265_amd" not in src, f
