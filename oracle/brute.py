"""Brute-force ray compositing for tiny volumes, in pure Python.

TEST INFRASTRUCTURE ONLY (used by the ``-m "not gpu"`` pins of the C oracle).

It recomputes a pixel's colour from the definitions alone, with methods chosen
to differ from ``oracle.c``:
  * the B-spline weights come from the cubic B-spline *kernel*
    beta(x) = 2/3 - x^2 + |x|^3/2 for |x| < 1, (2 - |x|)^3/6 for 1 <= |x| < 2,
    evaluated in exact rationals at the tap distances (not from the four
    per-offset polynomials), and the value is the explicit 64-term sum;
  * the ray is clipped by intersecting the six face planes and keeping the hits
    that lie on the box (not by the slab method);
  * the transfer function is evaluated either as an explicit function of the
    value, or by a linear search for the node interval of the table;
  * compositing uses alpha = 1 - exp(-sigma step) and T <- T (1 - alpha);
  * the gradient for local lighting differentiates the kernel sum exactly
    (beta' in rationals), not the per-offset weight polynomials.
Only exp and the square root of the direction normalisation are floating
point; positions are converted exactly to rationals.
"""

from __future__ import annotations

import math
from fractions import Fraction


def bspline_kernel(x: Fraction) -> Fraction:
    ax = abs(x)
    if ax < 1:
        return Fraction(2, 3) - ax * ax + ax * ax * ax / 2
    if ax < 2:
        return (2 - ax) ** 3 / 6
    return Fraction(0)


def reconstruct(vol, p):
    """Exact tricubic B-spline value at p of a volume given as vol[z][y][x]
    (integers or Fractions), clamp-to-edge addressing."""
    nz, ny, nx = len(vol), len(vol[0]), len(vol[0][0])
    px, py, pz = (Fraction(c) for c in p)
    fx, fy, fz = math.floor(px), math.floor(py), math.floor(pz)
    total = Fraction(0)
    for z in range(fz - 1, fz + 3):
        wz = bspline_kernel(pz - z)
        for y in range(fy - 1, fy + 3):
            wy = bspline_kernel(py - y)
            for x in range(fx - 1, fx + 3):
                wx = bspline_kernel(px - x)
                xc = min(max(x, 0), nx - 1)
                yc = min(max(y, 0), ny - 1)
                zc = min(max(z, 0), nz - 1)
                total += wx * wy * wz * Fraction(vol[zc][yc][xc])
    return total


def catmull_rom_kernel(x: Fraction) -> Fraction:
    """Catmull-Rom: 3|x|^3/2 - 5x^2/2 + 1 for |x| < 1, -|x|^3/2 + 5x^2/2 - 4|x| + 2 for 1 <= |x| < 2."""
    ax = abs(x)
    if ax < 1:
        return Fraction(3, 2) * ax ** 3 - Fraction(5, 2) * ax ** 2 + 1
    if ax < 2:
        return -Fraction(1, 2) * ax ** 3 + Fraction(5, 2) * ax ** 2 - 4 * ax + 2
    return Fraction(0)


def bspline_kernel_deriv(x: Fraction) -> Fraction:
    """beta'(x): -2x + 3x|x|/2 for |x| < 1, -sign(x) (2 - |x|)^2 / 2 for 1 <= |x| < 2."""
    ax = abs(x)
    sgn = 1 if x > 0 else (-1 if x < 0 else 0)
    if ax < 1:
        return -2 * x + Fraction(3, 2) * x * ax
    if ax < 2:
        return -sgn * (2 - ax) ** 2 / 2
    return Fraction(0)


def gradient(vol, p):
    """Exact gradient of the tricubic B-spline reconstruction at p (d/dp of
    the 64-term kernel sum), clamp-to-edge addressing; three Fractions."""
    nz, ny, nx = len(vol), len(vol[0]), len(vol[0][0])
    px, py, pz = (Fraction(c) for c in p)
    fx, fy, fz = math.floor(px), math.floor(py), math.floor(pz)
    g = [Fraction(0)] * 3
    for z in range(fz - 1, fz + 3):
        for y in range(fy - 1, fy + 3):
            for x in range(fx - 1, fx + 3):
                v = Fraction(vol[min(max(z, 0), nz - 1)][min(max(y, 0), ny - 1)][min(max(x, 0), nx - 1)])
                kx, ky, kz = bspline_kernel(px - x), bspline_kernel(py - y), bspline_kernel(pz - z)
                g[0] += bspline_kernel_deriv(px - x) * ky * kz * v
                g[1] += kx * bspline_kernel_deriv(py - y) * kz * v
                g[2] += kx * ky * bspline_kernel_deriv(pz - z) * v
    return g


def lit_colour(sh, d, g, c):
    """Blinn-Phong two-sided lighting of colour c (3 floats) at a sample with
    ray direction d and field gradient g; sh = (ka, kd, ks, shininess,
    (lx, ly, lz), headlight, grad_min)."""
    ka, kd, ks, shin, light, headlight, gmin = sh
    eye = [-x for x in d]
    if headlight:
        L = list(eye)
    else:
        ln = math.sqrt(sum(x * x for x in light))
        L = [x / ln for x in light]
    half = [L[k] + eye[k] for k in range(3)]
    hn = math.sqrt(sum(x * x for x in half))
    gn = math.sqrt(sum(float(x) ** 2 for x in g))
    scale = max(gn, gmin)
    normal = [-float(x) / scale for x in g]
    diffuse = abs(sum(normal[k] * L[k] for k in range(3)))
    spec = 0.0 if hn <= 1e-12 else abs(sum(normal[k] * half[k] for k in range(3)) / hn) ** shin
    return [c[k] * (ka + kd * diffuse) + ks * spec for k in range(3)]


def camera_ray(cam, row, col):
    """Pixel centre -> (origin, unit direction) in floats."""
    W, H = cam.width, cam.height
    sx = 2.0 * (col + 0.5) / W - 1.0
    sy = 1.0 - 2.0 * (row + 0.5) / H
    if cam.projection == 1:
        th = math.tan(cam.fov_y / 2.0)
        d = [cam.forward[k] + sx * th * (W / H) * cam.right[k] + sy * th * cam.up[k] for k in range(3)]
        o = [float(cam.eye[k]) for k in range(3)]
    else:
        d = [float(cam.forward[k]) for k in range(3)]
        o = [cam.eye[k] + sx * cam.ortho_w / 2.0 * cam.right[k] + sy * cam.ortho_h / 2.0 * cam.up[k]
             for k in range(3)]
    n = math.sqrt(sum(c * c for c in d))
    return o, [c / n for c in d]


def clip_planes(o, d, dims):
    """Entry/exit parameters from the six face planes of [-1/2, n-1/2]^3."""
    ts = []
    lo = [-0.5] * 3
    hi = [dims[k] - 0.5 for k in range(3)]
    for a in range(3):
        if d[a] == 0:
            continue
        for plane in (lo[a], hi[a]):
            t = (plane - o[a]) / d[a]
            q = [o[k] + t * d[k] for k in range(3)]
            inside = all(lo[k] - 1e-9 <= q[k] <= hi[k] + 1e-9 for k in range(3) if k != a)
            if inside:
                ts.append(t)
    if len(ts) < 2:
        return None
    tin, tout = max(min(ts), 0.0), max(ts)
    if not tout > tin:
        return None
    return tin, tout


def tf_table_lookup(table, v0, v1, v):
    """(r, g, b, sigma) at value v from a K-node table by linear search for
    the node interval; values outside [v0, v1] take the end node."""
    K = len(table)
    h = (v1 - v0) / (K - 1)
    if v <= v0:
        return list(table[0])
    if v >= v1:
        return list(table[K - 1])
    for j in range(K - 1):
        a = v0 + j * h
        b = v0 + (j + 1) * h
        if a <= v < b:
            w = (v - a) / h
            return [(1 - w) * table[j][c] + w * table[j + 1][c] for c in range(4)]
    return list(table[K - 1])


def composite_ray(vol, o, d, step, classify, ert=0.0, shade=None):
    """Front-to-back emission-absorption along one ray; returns (rgba, n_samples).
    ``shade`` (the tuple of ``lit_colour``) lights every sample's colour."""
    dims = (len(vol[0][0]), len(vol[0]), len(vol))
    hit = clip_planes(o, d, dims)
    if hit is None:
        return [0.0, 0.0, 0.0, 0.0], 0
    tin, tout = hit
    C = [0.0, 0.0, 0.0]
    T = 1.0
    # samples at t_k = (k + 1/2) step from the origin, t_in < t_k < t_out
    k = 0
    while (k + 0.5) * step <= tin:
        k += 1
    n = 0
    while (k + 0.5) * step < tout:
        t = (k + 0.5) * step
        p = [o[c] + t * d[c] for c in range(3)]
        v = float(reconstruct(vol, p))
        r, g, b, sigma = classify(v)
        if shade is not None:
            r, g, b = lit_colour(shade, d, gradient(vol, p), (r, g, b))
        alpha = 1.0 - math.exp(-sigma * step)
        C = [C[0] + T * alpha * r, C[1] + T * alpha * g, C[2] + T * alpha * b]
        T = T * (1.0 - alpha)
        n += 1
        k += 1
        if 0.0 < ert < 1.0 and 1.0 - T >= ert:
            break
    return [C[0], C[1], C[2], 1.0 - T], n


def brute_pixel(vol, cam, row, col, step, classify, ert=0.0, shade=None):
    o, d = camera_ray(cam, row, col)
    return composite_ray(vol, o, d, step, classify, ert, shade)
