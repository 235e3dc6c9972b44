"""Seeded phantom volumes.

Memory order of every volume returned here is x fastest, then y, then z
(NumPy shape ``(nz, ny, nx)``, C-contiguous), one scalar per voxel.
"""

from __future__ import annotations

import numpy as np


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random rotation matrix from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ]
    )


def _box(shape_zyx, centre_xyz, semi_xyz, rot):
    """Grid-clipped bounding box of a rotated ellipsoid as a tuple of z, y, x
    slices, or None when it misses the grid."""
    nz, ny, nx = shape_zyx
    semi = np.asarray(semi_xyz, dtype=np.float64)
    c = np.asarray(centre_xyz, dtype=np.float64)
    half = np.sqrt(((rot * semi[None, :]) ** 2).sum(axis=1))
    lo = np.maximum(np.floor(c - half).astype(np.int64), 0)
    hi = np.minimum(np.ceil(c + half).astype(np.int64) + 1, [nx, ny, nz])
    if np.any(hi <= lo):
        return None
    return (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))


def _quadform(sl, centre_xyz, semi_xyz, rot):
    """sum_i (q_i / a_i)^2 with q = R^T (p - c), evaluated on the voxel centres
    of box ``sl``; <= 1 inside the ellipsoid."""
    c = np.asarray(centre_xyz, dtype=np.float64)
    semi = np.asarray(semi_xyz, dtype=np.float64)
    xs = np.arange(sl[2].start, sl[2].stop, dtype=np.float64) - c[0]
    ys = np.arange(sl[1].start, sl[1].stop, dtype=np.float64) - c[1]
    zs = np.arange(sl[0].start, sl[0].stop, dtype=np.float64) - c[2]
    acc = np.zeros((zs.size, ys.size, xs.size), dtype=np.float64)
    for i in range(3):
        qi = (
            rot[0, i] * xs[None, None, :]
            + rot[1, i] * ys[None, :, None]
            + rot[2, i] * zs[:, None, None]
        )
        acc += (qi / semi[i]) ** 2
    return acc


def ellipsoid_phantom_u16(n: int = 64, seed: int = 0, count: int = 10) -> np.ndarray:
    """Small uint16 phantom: ``count`` random solid ellipsoids on a zero
    background, painted in order (later ones overwrite earlier ones).

    Centres U[0.2n, 0.8n], semi-axes U[0.05n, 0.3n], uniform random rotation,
    integer values U{1..4095} (12-bit CT range)."""
    rng = np.random.default_rng(seed)
    vol = np.zeros((n, n, n), dtype=np.uint16)
    for _ in range(count):
        c = rng.uniform(0.2 * n, 0.8 * n, 3)
        a = rng.uniform(0.05 * n, 0.3 * n, 3)
        rot = _random_rotation(rng)
        val = int(rng.integers(1, 4096))
        sl = _box(vol.shape, c, a, rot)
        if sl is None:
            continue
        vol[sl][_quadform(sl, c, a, rot) <= 1.0] = val
    return vol


def ct_phantom_i16(
    nx: int,
    ny: int,
    nz: int,
    seed: int,
    n_soft: int = 12,
    n_bone: int = 6,
    noise_sigma: float = 10.0,
) -> np.ndarray:
    """CT-like int16 phantom in Hounsfield units.

    * air (-1000 HU) everywhere outside an axis-aligned body ellipsoid centred in
      the box with semi-axes 0.914 x the half-extents (about 40 % of voxels are
      body, 60 % air);
    * body base 40 HU, ``n_soft`` soft-tissue ellipsoids of U[0, 80] HU,
      ``n_bone`` ellipsoidal bone shells 3..8 voxels thick of U[700, 1500] HU;
    * Gaussian noise N(0, ``noise_sigma``) HU added to every body voxel.
    """
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    vol = np.full(shape, -1000, dtype=np.int16)
    centre = np.array([(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
    body_semi = 0.914 * np.array([nx / 2.0, ny / 2.0, nz / 2.0])
    mn = float(min(nx, ny, nz))

    # body ellipsoid, painted slab by slab to bound temporary memory
    xs = (np.arange(nx) - centre[0]) / body_semi[0]
    ys = (np.arange(ny) - centre[1]) / body_semi[1]
    rxy = xs[None, :] ** 2 + ys[:, None] ** 2
    for z in range(nz):
        rz = ((z - centre[2]) / body_semi[2]) ** 2
        m = (rxy + rz) <= 1.0
        if m.any():
            vol[z][m] = 40

    def body_mask(sl):
        zz = (np.arange(sl[0].start, sl[0].stop) - centre[2]) / body_semi[2]
        yy = (np.arange(sl[1].start, sl[1].stop) - centre[1]) / body_semi[1]
        xx = (np.arange(sl[2].start, sl[2].stop) - centre[0]) / body_semi[0]
        return (zz[:, None, None] ** 2 + yy[None, :, None] ** 2 + xx[None, None, :] ** 2) <= 1.0

    for _ in range(n_soft):
        c = centre + rng.uniform(-0.55, 0.55, 3) * body_semi
        a = rng.uniform(0.04, 0.18, 3) * mn
        rot = _random_rotation(rng)
        val = int(rng.integers(0, 81))
        sl = _box(shape, c, a, rot)
        if sl is None:
            continue
        vol[sl][(_quadform(sl, c, a, rot) <= 1.0) & body_mask(sl)] = val

    for _ in range(n_bone):
        c = centre + rng.uniform(-0.4, 0.4, 3) * body_semi
        a = rng.uniform(0.08, 0.25, 3) * mn
        thick = float(rng.integers(3, 9))
        rot = _random_rotation(rng)
        val = int(rng.integers(700, 1501))
        sl = _box(shape, c, a, rot)
        if sl is None:
            continue
        inner = np.maximum(a - thick, 0.5)
        shell = (
            (_quadform(sl, c, a, rot) <= 1.0)
            & (_quadform(sl, c, inner, rot) > 1.0)
            & body_mask(sl)
        )
        vol[sl][shell] = val

    # noise on body voxels, slab by slab
    for z in range(nz):
        rz = ((z - centre[2]) / body_semi[2]) ** 2
        m = (rxy + rz) <= 1.0
        cnt = int(m.sum())
        if cnt == 0:
            continue
        noise = np.rint(rng.standard_normal(cnt, dtype=np.float32) * noise_sigma)
        sl = vol[z]
        sl[m] = np.clip(sl[m].astype(np.float32) + noise, -32768, 32767).astype(np.int16)
    return vol


def density_grid_f32(n: int = 256, seed: int = 5, smooth_sigma: float = 4.0) -> np.ndarray:
    """Differentiable-render density grid: N(0,1) noise smoothed by a Gaussian
    of ``smooth_sigma`` voxels, then d = max(0, s - median) / (max - median), so
    that half of the voxels are exactly zero and the rest lie in (0, 1]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n, n), dtype=np.float32)
    s = gaussian_filter(g, smooth_sigma, mode="wrap").astype(np.float64)
    med = np.median(s)
    d = np.maximum(0.0, s - med) / (s.max() - med)
    return np.ascontiguousarray(d.astype(np.float32))
