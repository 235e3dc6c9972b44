"""Pins of the oracle's filter variants (the paper's filter comparison,
Fig. 4 discussion): the interpolating (prefiltered) cubic B-spline, the
Catmull-Rom cubic with its widened skip test, and pre-classification."""

import numpy as np
import pytest
from scipy.linalg import solve_banded

from fractions import Fraction

import oracle
from oracle import brute
import synth


@pytest.mark.parametrize("shape,dtype", [((5, 6, 7), np.float64), ((1, 2, 9), np.float32), ((4, 1, 3), np.uint16),
                                         ((3, 5, 2), np.int16)])
def test_prefiltered_spline_interpolates_every_voxel(oracle_lib, shape, dtype):
    rng = np.random.default_rng(501)
    vol = (rng.normal(0, 500, shape) + (2000 if dtype == np.uint16 else 0)).astype(dtype)
    c = oracle.prefilter(vol)
    nz, ny, nx = shape
    worst = max(abs(oracle.sample(c, (x, y, z)) - float(vol[z, y, x]))
                for z in range(nz) for y in range(ny) for x in range(nx))
    assert worst < 1e-9 * max(1.0, float(np.abs(vol).max()))


def test_prefilter_line_matches_a_banded_solver(oracle_lib):
    """Along one axis the coefficients solve tridiag(1, 4, 1) / 6 with the
    clamped ends (diagonal 5): scipy's banded LU as an independent solver."""
    rng = np.random.default_rng(502)
    for n in (2, 3, 8, 33):
        v = rng.normal(size=n)
        ab = np.zeros((3, n))
        ab[0, 1:] = 1.0
        ab[1, :] = 4.0
        ab[1, 0] = ab[1, -1] = 5.0
        ab[2, :-1] = 1.0
        want = solve_banded((1, 1), ab, 6.0 * v)
        got = oracle.prefilter(v.reshape(1, 1, n))[0, 0]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_prefilter_keeps_constants(oracle_lib):
    vol = np.full((4, 5, 6), 1234, dtype=np.int16)
    np.testing.assert_allclose(oracle.prefilter(vol), 1234.0, rtol=0, atol=1e-10)


# ------------------------------------------------------------ Catmull-Rom --

def test_catmull_rom_weights_match_the_kernel(oracle_lib):
    rng = np.random.default_rng(503)
    for f in list(rng.uniform(0, 1, 100)) + [0.0, 0.5, 0.25]:
        w = oracle.catmull_rom_weights(f)
        for a in range(4):
            assert abs(w[a] - float(brute.catmull_rom_kernel(Fraction(f) + 1 - a))) < 1e-14
        assert abs(w.sum() - 1.0) < 1e-14


def test_catmull_rom_interpolates_and_reproduces_quadratics(oracle_lib):
    rng = np.random.default_rng(504)
    vol = rng.normal(0, 100, (6, 7, 8))
    for z in range(6):
        for y in range(7):
            for x in range(8):
                assert abs(oracle.sample(vol, (x, y, z), filter=1) - vol[z, y, x]) < 1e-11
    z_, y_, x_ = np.meshgrid(np.arange(12.0), np.arange(12.0), np.arange(12.0), indexing="ij")
    q = x_ * x_ - 2.0 * y_ * z_ + 3.0 * z_
    for _ in range(20):
        p = rng.uniform(2.0, 8.99, 3)
        want = p[0] ** 2 - 2 * p[1] * p[2] + 3 * p[2]
        assert abs(oracle.sample(q, p, filter=1) - want) < 1e-10


def test_catmull_rom_overshoot_bound_is_tight(oracle_lib):
    """Samples stay within [lo - w (hi - lo), hi + w (hi - lo)], w = 0.4765625,
    and a checkerboard of the negative taps reaches the bound."""
    rng = np.random.default_rng(505)
    vol = rng.integers(0, 2, (6, 6, 6)).astype(np.float64) * 1000.0
    w = oracle.CATMULL_ROM_WIDEN
    for _ in range(300):
        p = rng.uniform(1.0, 3.999, 3)
        v = oracle.sample(vol, p, filter=1)
        assert -w * 1000.0 - 1e-9 <= v <= 1000.0 + w * 1000.0 + 1e-9
    # taps at offsets -1 and +2 (negative weights at f = 1/2) high, others low,
    # on every axis: the product's negative weights all meet 1000
    chk = np.zeros((4, 4, 4))
    for c in range(4):
        for b in range(4):
            for a in range(4):
                neg = ((a in (0, 3)) + (b in (0, 3)) + (c in (0, 3))) % 2 == 1
                chk[c, b, a] = 1000.0 if neg else 0.0
    assert abs(oracle.sample(chk, (1.5, 1.5, 1.5), filter=1) - (-w * 1000.0)) < 1e-9


def _undershoot_case():
    """Step edges 0 -> 1000 whose Catmull-Rom undershoot reaches values that
    only a TF band below -40 makes visible; the blocks' own ranges [0, 1000]
    never touch that band."""
    vol = np.zeros((16, 16, 32), dtype=np.int16)
    vol[:, :, 16:] = 1000
    vol[:, 8:, :] = np.where(vol[:, 8:, :] == 0, 1000, 0)
    pts = [(-500.0, (0, 0, 0, 0)), (-50.0, (0.2, 0.9, 0.4, 0.8)), (-40.0, (0, 0, 0, 0)), (1500.0, (0, 0, 0, 0))]
    tf = synth.tf_from_points(pts, 201, -500.0, 1500.0)
    cams = synth.orbit_cameras((32, 16, 16), 2, 506, 50.0, 24, 20)
    return vol, tf, cams


def test_catmull_rom_skip_is_lossless_with_widened_ranges(oracle_lib):
    vol, tf, cams = _undershoot_case()
    mm = oracle.blocks(vol, 8)
    full = oracle.render(vol, cams, tf, 0.5, filter=1)
    assert full["rgba"][..., 3].max() > 0.01  # the undershoot band is visible
    skip = oracle.render(vol, cams, tf, 0.5, filter=1, occ=oracle.occupancy(mm, tf, filter=1), edge=8)
    np.testing.assert_array_equal(skip["rgba"], full["rgba"])
    # the B-spline never undershoots: same volume, nothing visible
    assert oracle.render(vol, cams, tf, 0.5)["rgba"].max() == 0.0


# ----------------------------------------------------- pre-classification --

def _ramp_tf(K=9, v0=0.0, v1=4096.0):
    """Extinction linear in the value, constant colour (fp32-exact nodes)."""
    sig = np.arange(K) / 256.0
    table = np.column_stack([np.full(K, 0.75), np.full(K, 0.5), np.full(K, 0.25), sig]).astype(np.float32)
    return synth.TransferFunction(table, v0, v1)


def test_preclassification_equals_post_for_linear_tfs(oracle_lib):
    """A TF linear over the values commutes with the (non-negative, unit-sum)
    B-spline weights: classifying taps then interpolating equals interpolating
    then classifying."""
    vol = synth.ellipsoid_phantom_u16(16, seed=507)
    cams = synth.orbit_cameras((16, 16, 16), 2, 508, 50.0, 12, 12)
    for tf in (_ramp_tf(), synth.TransferFunction(np.tile(np.float32([0.2, 0.6, 0.9, 0.07]), (8, 1)), 0.0, 4095.0)):
        pre = oracle.render(vol, cams, tf, 0.625, filter=2)["rgba"]
        post = oracle.render(vol, cams, tf, 0.625)["rgba"]
        np.testing.assert_allclose(pre, post, rtol=0, atol=1e-12)


def test_preclassification_matches_brute_force(oracle_lib):
    rng = np.random.default_rng(509)
    vol = rng.integers(0, 48, (5, 6, 7)).astype(np.uint16)
    lists = vol.tolist()
    K = 7
    table = rng.uniform(0, 1, (K, 4)).astype(np.float32)
    table[:, 3] *= 0.6
    tf = synth.TransferFunction(table, 0.0, 48.0)
    tt = table.astype(np.float64).tolist()
    cam = synth.orbit_camera((7, 6, 5), np.array([0.5, 0.35, -0.79]), 45.0, 10, 10)
    out = oracle.render(vol, [cam], tf, 0.4375, filter=2)
    import math

    def classified_sample(p):
        fx, fy, fz = (math.floor(c) for c in p)
        acc = [Fraction(0)] * 4
        for z in range(fz - 1, fz + 3):
            for y in range(fy - 1, fy + 3):
                for x in range(fx - 1, fx + 3):
                    v = vol[min(max(z, 0), 4)][min(max(y, 0), 5)][min(max(x, 0), 6)]
                    r, g, b, sg = brute.tf_table_lookup(tt, 0.0, 48.0, float(v))
                    w = (brute.bspline_kernel(Fraction(p[0]) - x) * brute.bspline_kernel(Fraction(p[1]) - y)
                         * brute.bspline_kernel(Fraction(p[2]) - z))
                    acc = [acc[0] + w * Fraction(sg * r), acc[1] + w * Fraction(sg * g), acc[2] + w * Fraction(sg * b),
                           acc[3] + w * Fraction(sg)]
        s = float(acc[3])
        return [float(acc[q]) / s if s > 0 else 0.0 for q in range(3)] + [s]

    checked = 0
    for row in range(2, 8):
        for col in range(2, 8):
            o, d = brute.camera_ray(cam, row, col)
            want, n = brute.composite_ray(lists, o, d, 0.4375, lambda v: (0, 0, 0, 0))
            if n == 0:
                continue
            hit = brute.clip_planes(o, d, (7, 6, 5))
            tin, tout = hit
            k = 0
            while (k + 0.5) * 0.4375 <= tin:
                k += 1
            C, T = [0.0, 0.0, 0.0], 1.0
            while (k + 0.5) * 0.4375 < tout:
                t = (k + 0.5) * 0.4375
                r, g, b, sg = classified_sample([o[c] + t * d[c] for c in range(3)])
                a = 1.0 - math.exp(-sg * 0.4375)
                C = [C[0] + T * a * r, C[1] + T * a * g, C[2] + T * a * b]
                T *= 1.0 - a
                k += 1
            np.testing.assert_allclose(out["rgba"][0, row, col], C + [1.0 - T], rtol=0, atol=1e-11)
            checked += 1
    assert checked >= 16


def test_preclassification_skip_is_lossless_and_differs_from_post(oracle_lib):
    vol = synth.ct_phantom_i16(40, 36, 32, seed=510, n_soft=4, n_bone=3)
    tf = synth.tf1()
    cams = synth.orbit_cameras((40, 36, 32), 2, 511, 55.0, 24, 20)
    mm = oracle.blocks(vol, 8)
    a = oracle.render(vol, cams, tf, 0.5, ert=0.99, filter=2, occ=oracle.occupancy(mm, tf), edge=8)
    b = oracle.render(vol, cams, tf, 0.5, ert=0.99, filter=2)
    np.testing.assert_array_equal(a["rgba"], b["rgba"])
    post = oracle.render(vol, cams, tf, 0.5, ert=0.99)["rgba"]
    assert np.abs(post - b["rgba"]).max() > 1e-3


# -------------------------------------------------------------- trilinear --

def test_trilinear_is_the_eight_tap_formula(oracle_lib):
    rng = np.random.default_rng(512)
    vol = rng.normal(0, 10, (5, 6, 7))
    for _ in range(50):
        p = rng.uniform(-0.5, [6.5, 5.5, 4.5])
        q = [min(max(c, 0.0), n - 1.0) for c, n in zip(p, (7, 6, 5))]
        i = [min(int(np.floor(c)), n - 2) for c, n in zip(q, (7, 6, 5))]
        f = [q[a] - i[a] if q[a] < (7, 6, 5)[a] - 1 else 1.0 for a in range(3)]
        # clamp-to-edge: below the first centre the value is the edge value
        f = [0.0 if p[a] < 0 else f[a] for a in range(3)]
        want = 0.0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    w = (f[0] if dx else 1 - f[0]) * (f[1] if dy else 1 - f[1]) * (f[2] if dz else 1 - f[2])
                    want += w * vol[min(i[2] + dz, 4), min(i[1] + dy, 5), min(i[0] + dx, 6)]
        assert abs(oracle.sample(vol, p, filter=3) - want) < 1e-11, p
    z_, y_, x_ = np.meshgrid(np.arange(8.0), np.arange(8.0), np.arange(8.0), indexing="ij")
    lin = 2 * x_ - y_ + 0.5 * z_
    for _ in range(20):
        p = rng.uniform(0.0, 6.99, 3)
        assert abs(oracle.sample(lin, p, filter=3) - (2 * p[0] - p[1] + 0.5 * p[2])) < 1e-11
