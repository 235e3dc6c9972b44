"""Transfer-function tables built from piecewise-linear control points.

A table holds K nodes of (r, g, b, sigma) in fp32; node j belongs to the scalar
value v0 + j (v1 - v0) / (K - 1).  r, g, b are emission colours in [0, 1] and
sigma >= 0 is the extinction per voxel length.  Building the table from
control points is input preparation; how the renderer reads the table between
nodes is part of the method and lives in the renderer and the oracle.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class TransferFunction:
    table: np.ndarray  # (K, 4) float32, rows (r, g, b, sigma)
    v0: float
    v1: float

    @property
    def K(self) -> int:
        return int(self.table.shape[0])


def tf_from_points(points, K: int, v0: float, v1: float) -> TransferFunction:
    """Sample the piecewise-linear function through ``points`` (a list of
    (value, (r, g, b, sigma))) at the K node values."""
    xs = np.array([p[0] for p in points], dtype=np.float64)
    ys = np.array([p[1] for p in points], dtype=np.float64)
    nodes = v0 + np.arange(K, dtype=np.float64) * (v1 - v0) / (K - 1)
    table = np.stack([np.interp(nodes, xs, ys[:, c]) for c in range(4)], axis=1)
    return TransferFunction(np.ascontiguousarray(table.astype(np.float32)), float(v0), float(v1))


# 12-bit phantom TF: value range 0..4080, node pitch 16.
TF0_POINTS = [
    (0.0, (0.0, 0.0, 0.0, 0.0)),
    (512.0, (0.2, 0.4, 1.0, 0.01)),
    (1536.0, (0.2, 1.0, 0.3, 0.05)),
    (2560.0, (1.0, 0.8, 0.2, 0.1)),
    (4080.0, (1.0, 1.0, 1.0, 0.2)),
]

# CT TF in HU: -1024..3056, node pitch 16 HU.  Air and lung are transparent,
# soft tissue faint, bone bright and dense.
TF1_POINTS = [
    (-1024.0, (0.0, 0.0, 0.0, 0.0)),
    (-208.0, (0.0, 0.0, 0.0, 0.0)),
    (-16.0, (0.8, 0.4, 0.3, 0.004)),
    (96.0, (0.9, 0.5, 0.4, 0.008)),
    (304.0, (0.9, 0.6, 0.5, 0.008)),
    (704.0, (1.0, 0.95, 0.85, 0.12)),
    (1504.0, (1.0, 1.0, 1.0, 0.25)),
    (3056.0, (1.0, 1.0, 1.0, 0.25)),
]

# density TF on [0, 1] for the differentiable grid.
TF3_POINTS = [
    (0.0, (0.1, 0.2, 0.9, 0.0)),
    (0.25, (0.2, 0.8, 0.3, 0.05)),
    (0.5, (0.9, 0.7, 0.1, 0.15)),
    (0.75, (1.0, 0.3, 0.2, 0.25)),
    (1.0, (1.0, 1.0, 1.0, 0.3)),
]


def tf0() -> TransferFunction:
    return tf_from_points(TF0_POINTS, 256, 0.0, 4080.0)


def tf1() -> TransferFunction:
    return tf_from_points(TF1_POINTS, 256, -1024.0, 3056.0)


def tf3() -> TransferFunction:
    return tf_from_points(TF3_POINTS, 256, 0.0, 1.0)
