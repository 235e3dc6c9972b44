"""The five seeded workloads of the ray caster.

* C0: 64^3 uint16 ellipsoid phantom, 256^2 orthographic view along +z, step
  0.5, no skipping, no early termination (parity / launch-overhead case).
* C1: 512x512x400 int16 CT-like phantom, 1024^2 perspective (60 deg FOV,
  seeded orbit pose), step 0.5, 16^3 block skipping, early termination at
  opacity 0.99 (the throughput workload).
* C2: 1024^3 int16 CT-like phantom (2 GiB) to a 2048^2 perspective view, step
  0.25, same TF and skipping.
* C3: 256^3 fp32 density grid, 64 perspective views of 512^2 on a seeded
  sphere of poses (differentiable rendering).
* C4: 8 resident CT-like volumes of 128^3 .. 512x512x800 and a Poisson stream
  of requests (serving mix).

Each builder returns a plain dict; volumes are NumPy arrays in x-fastest
order (shape (nz, ny, nx)).
"""

from __future__ import annotations

import numpy as np

from .cameras import ortho_axis_camera, orbit_cameras, orbit_directions, orbit_camera
from .phantoms import ct_phantom_i16, density_grid_f32, ellipsoid_phantom_u16
from .tfs import tf0, tf1, tf3


def config_c0():
    vol = ellipsoid_phantom_u16(64, seed=0, count=10)
    cam = ortho_axis_camera(64, 256, 256)
    return dict(
        name="c0_64cube_u16_ortho256",
        volume=vol,
        cameras=[cam],
        tf=tf0(),
        step=0.5,
        ert=0.0,
        use_skip=False,
        block_edge=16,
    )


def config_c1(dims=(512, 512, 400), image=1024, seed_volume=1, seed_pose=2):
    nx, ny, nz = dims
    vol = ct_phantom_i16(nx, ny, nz, seed=seed_volume)
    cams = orbit_cameras((nx, ny, nz), 1, seed_pose, 60.0, image, image)
    return dict(
        name=f"c1_{nx}x{ny}x{nz}_i16_persp{image}",
        volume=vol,
        cameras=cams,
        tf=tf1(),
        step=0.5,
        ert=0.99,
        use_skip=True,
        block_edge=16,
    )


def config_c2(n=1024, image=2048, seed_volume=3, seed_pose=4):
    vol = ct_phantom_i16(n, n, n, seed=seed_volume)
    cams = orbit_cameras((n, n, n), 1, seed_pose, 60.0, image, image)
    return dict(
        name=f"c2_{n}cube_i16_persp{image}",
        volume=vol,
        cameras=cams,
        tf=tf1(),
        step=0.25,
        ert=0.99,
        use_skip=True,
        block_edge=16,
    )


def config_c3(n=256, views=64, image=512, seed_grid=5, seed_pose=6):
    grid = density_grid_f32(n, seed=seed_grid)
    cams = orbit_cameras((n, n, n), views, seed_pose, 60.0, image, image)
    return dict(
        name=f"c3_{n}cube_f32_{views}x{image}",
        volume=grid,
        cameras=cams,
        tf=tf3(),
        step=0.5,
        ert=0.0,
        use_skip=False,
        block_edge=16,
    )


def c3_perturbed_grid(grid: np.ndarray, seed: int = 7, amp: float = 0.05):
    """Starting point of the C3 optimisation: grid + amp * smoothed noise,
    clamped at zero."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    nse = gaussian_filter(rng.standard_normal(grid.shape, dtype=np.float32), 4.0, mode="wrap")
    nse = nse / max(float(np.abs(nse).max()), 1e-12)
    return np.maximum(grid + amp * nse, 0.0).astype(np.float32)


def config_c4_volumes(seed=10, count=8):
    """Sizes of the served volumes: nx, ny ~ U{128..512}, nz ~ U{128..800};
    returns a list of (dims, volume_seed).  Volumes are generated lazily with
    ``ct_phantom_i16(*dims, seed)``."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nx = int(rng.integers(128, 513))
        ny = int(rng.integers(128, 513))
        nz = int(rng.integers(128, 801))
        out.append(((nx, ny, nz), 1000 + seed * 100 + i))
    return out


def c4_arrivals(n_requests, seed=11, rate_hz=200.0, n_volumes=8, sizes=(256, 512, 1024),
                dims_list=None):
    """Open-loop Poisson request stream: exponential gaps of mean 1/rate, each
    request drawing a volume, an image size and an orbit pose."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps)
    vols = rng.integers(0, n_volumes, n_requests)
    size_idx = rng.integers(0, len(sizes), n_requests)
    dirs = rng.standard_normal((n_requests, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    reqs = []
    for i in range(n_requests):
        s = int(sizes[size_idx[i]])
        cam = None
        if dims_list is not None:
            cam = orbit_camera(dims_list[int(vols[i])], dirs[i], 60.0, s, s)
        reqs.append(dict(t=float(t[i]), volume=int(vols[i]), size=s, direction=dirs[i], camera=cam))
    return reqs


def sample_pixels(n_views, width, height, count, seed):
    """``count`` distinct (view, row, col) triples drawn uniformly without
    replacement, as an int64 array of shape (count, 3)."""
    rng = np.random.default_rng(seed)
    total = n_views * width * height
    count = min(count, total)
    flat = rng.choice(total, size=count, replace=False)
    v = flat // (width * height)
    rem = flat % (width * height)
    return np.stack([v, rem // width, rem % width], axis=1).astype(np.int64)


__all__ = [
    "config_c0",
    "config_c1",
    "config_c2",
    "config_c3",
    "c3_perturbed_grid",
    "config_c4_volumes",
    "c4_arrivals",
    "sample_pixels",
    "orbit_directions",
]


# Local-lighting parameter sets (plain numbers; the lighting arithmetic lives
# in the oracle and the GPU library).  Gradient magnitudes are in value units
# per voxel: CT soft-tissue noise gives about 5-10 HU/voxel, bone edges
# hundreds, so grad_min = 20 keeps noise from acting as a surface.
SHADE_CT = dict(ambient=0.25, diffuse=0.7, specular=0.35, shininess=24.0, light=(-0.3, 0.4, -0.87),
                headlight=False, grad_min=20.0)
SHADE_CT_HEADLIGHT = dict(SHADE_CT, headlight=True, light=(0.0, 0.0, 1.0))
SHADE_C0 = dict(ambient=0.3, diffuse=0.6, specular=0.4, shininess=12.0, light=(0.5, -0.5, -0.7071),
                headlight=False, grad_min=50.0)
