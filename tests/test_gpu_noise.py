"""GPU noise step against the noise oracle: the Philox/Box-Muller deviates and the noisy cube."""
import numpy as np
import pytest

from helpers import gpu_forward, log
from oracle import noise as N
from paper_2412_08265_amd import synth

pytestmark = pytest.mark.gpu


def _job_and_cube(nx, ny, n_tel, values=None):
    import torch
    from paper_2412_08265_amd import ops
    obs = ops.Observation((0.0, 0.0, 0.0), nx, ny, 1.0, 5000.0, 1.0, n_tel)
    buf = ops.JobBuffers.allocate(0, obs)
    job = ops.make_job(ops.DeviceGalaxy({f: torch.zeros(0, device="cuda")
                                         for f in ops.FIELDS}), obs, buf)
    cube = torch.zeros((ny, nx, n_tel), dtype=torch.float32, device="cuda")
    if values is not None:
        cube.copy_(torch.from_numpy(values.reshape(ny, nx, n_tel)))
    return job, cube


def test_noise_deviates_match_oracle():
    """gain 0, floor 1 on a zero cube leaves the deviates themselves: the FP32 rounding of the
    oracle's FP64 values (the two FP64 transcendental implementations may differ in the last
    bit, so one FP32 ulp is allowed)."""
    import torch
    from paper_2412_08265_amd import ops
    nx, ny, nt = 16, 12, 5000
    job, cube = _job_and_cube(nx, ny, nt)
    seed, stream = 0x0123456789ABCDEF, 5
    ops.rubix_add_noise([job], [dict(seed=seed, stream=stream, gain=0.0, sigma_floor=1.0)], [cube])
    torch.cuda.synchronize()
    got = cube.cpu().numpy().ravel()
    ref = N.normals(got.size, seed, stream).astype(np.float32)
    ulp = np.abs(got.view(np.int32).astype(np.int64) - ref.view(np.int32).astype(np.int64))
    log(f"deviates: {got.size}, max ulp diff {ulp.max()}, exact {np.mean(ulp == 0):.6f}")
    assert ulp.max() <= 1 and np.mean(ulp == 0) > 0.999


@pytest.mark.parametrize("nt", [4997, 4998, 4999])
def test_noise_ragged_tail_and_unaligned_cube(nt):
    """Voxel counts that leave 1, 2 or 3 voxels in the last Philox block, on a 16-byte aligned
    cube and on one that starts 4 bytes past an aligned address (the kernel's vector and scalar
    paths): the same deviates as the oracle, voxel for voxel."""
    import torch
    from paper_2412_08265_amd import ops
    nx, ny = 3, 5
    seed, stream = 0xFEEDFACE12345678, 9
    ref = N.normals(nx * ny * nt, seed, stream).astype(np.float32)
    for off in (0, 1):
        job, _ = _job_and_cube(nx, ny, nt)
        store = torch.zeros(nx * ny * nt + 8, dtype=torch.float32, device="cuda")
        cube = store[off:off + nx * ny * nt].view(ny, nx, nt)
        assert (cube.data_ptr() % 16 == 0) == (off == 0)
        ops.rubix_add_noise([job], [dict(seed=seed, stream=stream, gain=0.0, sigma_floor=1.0)],
                            [cube])
        torch.cuda.synchronize()
        got = cube.cpu().numpy().ravel()
        ulp = np.abs(got.view(np.int32).astype(np.int64) - ref.view(np.int32).astype(np.int64))
        log(f"n={got.size} offset {off}: max ulp diff {ulp.max()}")
        assert ulp.max() <= 1 and np.mean(ulp == 0) > 0.999
        # nothing outside the cube is touched
        rest = torch.cat([store[:off], store[off + nx * ny * nt:]])
        assert not torch.any(rest != 0)


def test_noise_on_a_forward_cube_matches_oracle():
    import torch
    from paper_2412_08265_amd import ops
    w = synth.medium_workload(n=100_000)
    fw, g = gpu_forward(w)
    clean = g["cube"].astype(np.float32)
    top = float(np.abs(clean).max())
    p = dict(seed=99, stream=1, gain=top * 1e-4, sigma_floor=top * 1e-3)
    job, cube = _job_and_cube(w.nx, w.ny, w.n_tel, clean)
    ops.rubix_add_noise([job], [p], [cube])
    torch.cuda.synchronize()
    got = cube.cpu().numpy().ravel().astype(np.float64)
    ref = N.add_noise(clean.astype(np.float64).ravel(), p["seed"], p["stream"], p["gain"],
                      p["sigma_floor"])
    err = np.abs(got - ref) / (np.abs(ref) + p["sigma_floor"])
    log(f"noisy cube: max rel err {err.max():.3e}")
    assert err.max() <= 1e-6
    # deterministic in (seed, stream); another stream differs
    job2, c2 = _job_and_cube(w.nx, w.ny, w.n_tel, clean)
    job3, c3 = _job_and_cube(w.nx, w.ny, w.n_tel, clean)
    ops.rubix_add_noise([job2, job3], [p, dict(p, stream=2)], [c2, c3])
    torch.cuda.synchronize()
    assert torch.equal(c2, cube)
    assert not torch.equal(c3, cube)
