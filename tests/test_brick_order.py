"""The front-to-back brick order of the out-of-core renderer (host logic, no
GPU): along every ray of a camera, the bricks that hold its samples appear in
the order's sequence strictly increasing.  Sample positions come from the
oracle's FP64 ray setup and the lattice definition; a sample's brick is the
block of its clamped cell."""

import math

import numpy as np
import pytest

import oracle
import synth

vr = pytest.importorskip("paper_2005_01442_amd")


def _bricks_along(cam, row, col, dims, step, edge):
    o, d, tin, tout, ns, hit = oracle.ray(cam, row, col, dims, step)
    if not hit:
        return []
    k = max(0, math.floor(tin / step - 0.5))
    while (k + 0.5) * step <= tin:
        k += 1
    nbx, nby = -(-dims[0] // edge), -(-dims[1] // edge)
    out = []
    for _ in range(ns):
        p = o + (k + 0.5) * step * d
        c = [min(max(math.floor(p[a]), 0), dims[a] - 1) // edge for a in range(3)]
        b = c[0] + nbx * (c[1] + nby * c[2])
        if not out or out[-1] != b:
            out.append(b)
        k += 1
    return out


@pytest.mark.parametrize("case", ["outside", "inside", "ortho", "axis"])
def test_every_ray_meets_its_bricks_in_order(case):
    dims, edge, step = (40, 36, 29), 8, 0.5
    if case == "outside":
        cams = synth.orbit_cameras(dims, 3, 71, 60.0, 24, 20)
    elif case == "inside":
        c = synth.orbit_camera(dims, np.array([0.2, -0.4, 0.89]), 90.0, 24, 20)
        c.eye = np.array([17.3, 20.9, 8.2])  # inside the volume, off the brick boundaries
        cams = [c]
    elif case == "ortho":
        c = synth.orbit_camera(dims, np.array([-0.5, 0.3, 0.81]), 60.0, 24, 20)
        c.projection, c.ortho_w, c.ortho_h = 0, 60.0, 50.0
        cams = [c]
    else:
        cams = [synth.ortho_axis_camera(40, 24, 20)]
    checked = 0
    for cam in cams:
        order = vr.vr_brick_order(dims, edge, cam)
        nb = (-(-dims[0] // edge)) * (-(-dims[1] // edge)) * (-(-dims[2] // edge))
        assert sorted(order.tolist()) == list(range(nb))
        rank = np.empty(nb, dtype=np.int64)
        rank[order] = np.arange(nb)
        for row in range(0, 20, 3):
            for col in range(0, 24, 3):
                seq = _bricks_along(cam, row, col, dims, step, edge)
                r = [int(rank[b]) for b in seq]
                assert all(x < y for x, y in zip(r, r[1:])), (case, row, col, seq, r)
                checked += len(seq) > 1
    assert checked > 10
