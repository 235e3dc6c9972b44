"""Seeded cameras in voxel-index space.

A camera is an eye point and an orthonormal basis (right, up, forward) in the
coordinates where voxel (i, j, k) is centred at (i, j, k).  How pixels map to
rays is part of the method and lives in the renderer and in the oracle, not
here; this module only draws poses.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Camera:
    projection: int  # 0 orthographic, 1 perspective
    eye: np.ndarray
    right: np.ndarray
    up: np.ndarray
    forward: np.ndarray
    fov_y: float = 0.0  # radians, perspective only
    ortho_w: float = 0.0  # image-plane extent in voxels, orthographic only
    ortho_h: float = 0.0
    width: int = 0
    height: int = 0
    meta: dict = field(default_factory=dict)

    def as_tuple(self):
        return (
            int(self.projection),
            tuple(float(x) for x in self.eye),
            tuple(float(x) for x in self.right),
            tuple(float(x) for x in self.up),
            tuple(float(x) for x in self.forward),
            float(self.fov_y),
            float(self.ortho_w),
            float(self.ortho_h),
            int(self.width),
            int(self.height),
        )


def ortho_axis_camera(n: int, width: int, height: int, distance: float = 1000.0) -> Camera:
    """Orthographic view of an n^3 volume along +z: eye above the centre of the
    z = -distance plane, right +x, up -y (so image row j grows with y), image
    plane covering the full n x n face."""
    c = (n - 1) / 2.0
    return Camera(
        projection=0,
        eye=np.array([c, c, -distance]),
        right=np.array([1.0, 0.0, 0.0]),
        up=np.array([0.0, -1.0, 0.0]),
        forward=np.array([0.0, 0.0, 1.0]),
        ortho_w=float(n),
        ortho_h=float(n),
        width=width,
        height=height,
    )


def orbit_directions(count: int, seed: int) -> np.ndarray:
    """``count`` unit vectors uniform on the sphere (normalised Gaussians)."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((count, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def orbit_camera(dims_xyz, u, fov_deg: float, width: int, height: int) -> Camera:
    """Perspective camera on the sphere around the volume centre.

    The eye sits at centre + D u with D = R / sin(fov/2), R = half the box
    diagonal, so the bounding sphere just fills the vertical field of view.
    forward = -u, world up +z (+y when |u_z| > 0.99)."""
    nx, ny, nz = dims_xyz
    centre = np.array([(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
    R = 0.5 * float(np.linalg.norm([nx, ny, nz]))
    half = np.deg2rad(fov_deg) / 2.0
    D = R / np.sin(half)
    u = np.asarray(u, dtype=np.float64)
    u = u / np.linalg.norm(u)
    fwd = -u
    wup = np.array([0.0, 0.0, 1.0]) if abs(u[2]) <= 0.99 else np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, wup)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    up /= np.linalg.norm(up)
    return Camera(
        projection=1,
        eye=centre + D * u,
        right=right,
        up=up,
        forward=fwd,
        fov_y=float(np.deg2rad(fov_deg)),
        width=width,
        height=height,
        meta={"distance": D, "radius": R},
    )


def orbit_cameras(dims_xyz, count: int, seed: int, fov_deg: float, width: int, height: int):
    return [orbit_camera(dims_xyz, u, fov_deg, width, height) for u in orbit_directions(count, seed)]
