"""Pins of the oracle's local lighting: the analytic gradient of the tricubic
reconstruction and the two-sided Blinn-Phong colour (the paper's Phong
lighting with the gradient computed by the cubic filter, Section 2, the
block-overlap paragraph).

The gradient is checked against closed forms (the cubic B-spline reproduces
linear fields exactly and maps x^2 to x^2 + 1/3, so its gradient is exact for
both), against an exact rational differentiation of the kernel sum, and
against central differences of the separately pinned value.  The lit colour is
checked against closed forms on rays whose samples all share one gradient and
against the brute force."""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
import synth


# --------------------------------------------------------------- gradient --

def test_derivative_weights_match_the_kernel_derivative(oracle_lib):
    """dweights(f)[a] = beta'(f + 1 - a) at dyadic offsets (exact in binary)."""
    for f in [0.0, 0.125, 0.25, 0.5, 0.625, 0.875, 0.96875]:
        d = oracle.dweights(f)
        for a in range(4):
            want = brute.bspline_kernel_deriv(Fraction(f) + 1 - a)
            assert abs(d[a] - float(want)) < 1e-15, (f, a)
        assert abs(d.sum()) < 1e-15


def _field(n, fn, dtype=np.float64):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return fn(x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)).astype(dtype)


def test_gradient_of_linear_field_is_exact(oracle_lib):
    vol = _field(12, lambda x, y, z: 2.0 * x - 3.0 * y + 0.5 * z + 1.0, np.float32)
    rng = np.random.default_rng(301)
    for _ in range(20):
        p = rng.uniform(2.0, 8.99, 3)  # taps inside the grid
        np.testing.assert_allclose(oracle.gradient(vol, p), [2.0, -3.0, 0.5], rtol=0, atol=1e-12)


def test_gradient_of_quadratic_field_is_exact(oracle_lib):
    """B-spline of x^2 samples is x^2 + 1/3: gradient 2p exactly (interior)."""
    vol = _field(12, lambda x, y, z: x * x + 2.0 * y * y - z * z)
    rng = np.random.default_rng(302)
    for _ in range(20):
        p = rng.uniform(2.0, 8.99, 3)
        np.testing.assert_allclose(oracle.gradient(vol, p), [2 * p[0], 4 * p[1], -2 * p[2]], rtol=0, atol=1e-11)


def test_gradient_matches_rational_brute_force(oracle_lib):
    """Random 16-bit volume, points near and beyond the faces (clamped taps)."""
    rng = np.random.default_rng(303)
    vol = rng.integers(-500, 3000, (5, 6, 7)).astype(np.int16)
    lists = vol.tolist()
    pts = [(-0.4, 2.3, 1.7), (6.45, 5.4, 4.45), (3.125, -0.5, 2.75), (0.6, 0.3, 0.2), (2.5, 3.0, 4.0)]
    for p in pts:
        want = [float(x) for x in brute.gradient(lists, p)]
        got = oracle.gradient(vol, p)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-9 * max(1.0, max(abs(w) for w in want)))


def test_gradient_matches_central_differences_of_the_value(oracle_lib):
    rng = np.random.default_rng(304)
    vol = rng.normal(0.0, 1.0, (9, 10, 11))
    h = 1e-5
    for _ in range(12):
        p = rng.uniform(-0.5, 8.5, 3)
        g = oracle.gradient(vol, p)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            fd = (oracle.sample(vol, p + e) - oracle.sample(vol, p - e)) / (2 * h)
            assert abs(fd - g[a]) < 1e-7, (p, a, fd, g[a])


# --------------------------------------------------------------- lighting --

def _constant_tf(c, sigma, K=8, v0=0.0, v1=64.0):
    table = np.tile(np.array([*c, sigma], dtype=np.float32), (K, 1))
    return synth.TransferFunction(table, v0, v1)


def _shade(**kw):
    sh = dict(ambient=0.25, diffuse=0.625, specular=0.5, shininess=8.0, light=(0.0, 0.0, -1.0), headlight=False,
              grad_min=1.0)
    sh.update(kw)
    return sh


def _one_sample_camera(p):
    """A 1x1 orthographic view along +z whose only sample (step 1024) is p."""
    return synth.Camera(projection=0, eye=np.array([p[0], p[1], p[2] - 512.0]), right=np.array([1.0, 0.0, 0.0]),
                        up=np.array([0.0, -1.0, 0.0]), forward=np.array([0.0, 0.0, 1.0]), ortho_w=1.0, ortho_h=1.0,
                        width=1, height=1)


@pytest.mark.parametrize("slope", [2.0, 0.5])
def test_lit_single_sample_closed_form(oracle_lib, slope):
    """Field a z: gradient (0, 0, a), normal (0, 0, -rho) with rho = min(1,
    a / grad_min); headlight: c (ka + kd rho) + ks rho^s; a light at angle
    theta from the normal: c (ka + kd rho cos theta) + ks (rho cos(theta/2))^s."""
    vol = _field(16, lambda x, y, z: slope * z, np.float32)
    c = (0.75, 0.5, 0.25)
    sigma = 1.0 / 2048.0
    tf = _constant_tf(c, sigma, v0=0.0, v1=64.0)
    cam = _one_sample_camera((7.3, 8.1, 7.4))
    alpha = -math.expm1(-sigma * 1024.0)
    rho = min(1.0, slope / 1.0)
    sh = _shade(headlight=True)
    out = oracle.render(vol, [cam], tf, 1024.0, shading=sh)
    assert out["counts"][0, 0, 0, 0] == 1
    lit = [ci * (0.25 + 0.625 * rho) + 0.5 * rho ** 8 for ci in c]
    np.testing.assert_allclose(out["rgba"][0, 0, 0], [alpha * x for x in lit] + [alpha], rtol=0, atol=1e-13)
    theta = 0.7
    sh = _shade(light=(math.sin(theta), 0.0, -math.cos(theta)))
    out = oracle.render(vol, [cam], tf, 1024.0, shading=sh)
    lf = oracle.shade_params(sh)[4:7]
    ct = -lf[2] / np.linalg.norm(lf)  # cos theta of the fp32-rounded light
    lit = [ci * (0.25 + 0.625 * rho * ct) + 0.5 * (rho * math.sqrt((1 + ct) / 2)) ** 8 for ci in c]
    np.testing.assert_allclose(out["rgba"][0, 0, 0], [alpha * x for x in lit] + [alpha], rtol=0, atol=1e-12)


def test_lit_rays_across_the_gradient_closed_form(oracle_lib):
    """Orthographic rays along +x through the field 3 z: every sample has the
    gradient (0, 0, 3), so the lit colour c' is constant along the ray and
    RGBA = (1 - exp(-sigma step N)) (c', 1); headlight: no diffuse, no
    specular; light (0, 0, -1): c (ka + kd) + ks 2^(-s/2)."""
    n = 16
    vol = _field(n, lambda x, y, z: 3.0 * z, np.float32)
    c = (0.5, 0.25, 1.0)
    sigma = 1.0 / 64.0
    tf = _constant_tf(c, sigma, v0=0.0, v1=64.0)
    cam = synth.Camera(projection=0, eye=np.array([-500.0, 7.5, 7.5]), right=np.array([0.0, 1.0, 0.0]),
                       up=np.array([0.0, 0.0, 1.0]), forward=np.array([1.0, 0.0, 0.0]), ortho_w=16.0, ortho_h=16.0,
                       width=16, height=16)
    rows = range(3, 13)  # z = 7.5 - (row - 7.5): taps inside the grid along z
    for sh, lit in [
        (_shade(headlight=True), [0.25 * ci for ci in c]),
        (_shade(), [ci * (0.25 + 0.625) + 0.5 * 2 ** -4 for ci in c]),
    ]:
        out = oracle.render(vol, [cam], tf, 0.5, shading=sh)
        for row in rows:
            for col in (0, 5, 15):
                N = out["counts"][0, row, col, 0]
                assert N == 32
                a = -math.expm1(-sigma * 0.5 * N)
                np.testing.assert_allclose(out["rgba"][0, row, col], [a * x for x in lit] + [a], rtol=0,
                                           atol=1e-12)


def test_lit_render_matches_brute_force(oracle_lib):
    """Random volume, perspective rays, a fixed light, a grad_min inside the
    range of gradient magnitudes, against the rational-gradient brute force."""
    rng = np.random.default_rng(305)
    vol = rng.integers(0, 64, (5, 6, 7)).astype(np.uint16)
    lists = vol.tolist()
    K = 9
    table = rng.uniform(0, 1, (K, 4)).astype(np.float32)
    table[:, 3] *= 0.5
    tf = synth.TransferFunction(table, 0.0, 64.0)
    classify = lambda v: brute.tf_table_lookup(table.astype(np.float64).tolist(), 0.0, 64.0, v)  # noqa: E731
    sh = _shade(light=(0.3, -0.5, 0.8), shininess=5.5, grad_min=12.0)
    shp = oracle.shade_params(sh)
    bsh = (shp[0], shp[1], shp[2], shp[3], tuple(shp[4:7]), False, shp[8])
    pcam = synth.orbit_camera((7, 6, 5), np.array([0.45, -0.3, 0.84]), 45.0, 10, 10)
    out = oracle.render(vol, [pcam], tf, 0.375, shading=sh)
    checked = 0
    for row in range(2, 8):
        for col in range(2, 8):
            want, n = brute.brute_pixel(lists, pcam, row, col, 0.375, classify, shade=bsh)
            np.testing.assert_allclose(out["rgba"][0, row, col], want, rtol=0, atol=1e-10)
            checked += n > 0
    assert checked >= 16
    hsh = _shade(headlight=True, grad_min=12.0)
    hp = oracle.shade_params(hsh)
    out = oracle.render(vol, [pcam], tf, 0.375, shading=hsh)
    for row, col in [(4, 4), (6, 3), (2, 7)]:
        want, n = brute.brute_pixel(lists, pcam, row, col, 0.375, classify,
                                    shade=(hp[0], hp[1], hp[2], hp[3], (0, 0, 0), True, hp[8]))
        assert n > 0
        np.testing.assert_allclose(out["rgba"][0, row, col], want, rtol=0, atol=1e-10)


def test_lighting_leaves_opacity_and_unlit_limit(oracle_lib):
    """Opacity is the unlit one; ka = 1, kd = ks = 0 gives the unlit image."""
    vol = synth.ellipsoid_phantom_u16(16, seed=306)
    tf = synth.tf_from_points(synth.TF0_POINTS, 256, 0.0, 4080.0)
    cam = synth.orbit_camera((16, 16, 16), np.array([0.2, 0.9, 0.3]), 50.0, 12, 12)
    plain = oracle.render(vol, [cam], tf, 0.5)["rgba"]
    lit = oracle.render(vol, [cam], tf, 0.5, shading=_shade())["rgba"]
    np.testing.assert_array_equal(lit[..., 3], plain[..., 3])
    assert np.abs(lit[..., :3] - plain[..., :3]).max() > 1e-3
    same = oracle.render(vol, [cam], tf, 0.5, shading=_shade(ambient=1.0, diffuse=0.0, specular=0.0))["rgba"]
    np.testing.assert_allclose(same, plain, rtol=0, atol=1e-15)
