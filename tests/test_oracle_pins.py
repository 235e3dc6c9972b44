"""Pins of the FP64 oracle against closed forms, invariants and brute force.

None of these compares the oracle with itself: each value comes from the
mathematics (B-spline moments, Beer-Lambert telescoping, clamp worked
examples), from the independent pure-Python brute force in ``oracle/brute.py``,
or from a NumPy re-derivation of the block footprint.
"""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


# ---------------------------------------------------------------- weights --

def test_bspline_weights_worked_values(oracle_lib):
    for row in _read_golden("bspline_weights.txt"):
        f = Fraction(row[0])
        want = [Fraction(x) for x in row[1:]]
        assert sum(want) == 1
        got = oracle.weights(float(f))
        np.testing.assert_allclose(got, [float(x) for x in want], rtol=0, atol=1e-15)


def test_bspline_weights_match_kernel_everywhere(oracle_lib):
    rng = np.random.default_rng(100)
    for f in rng.uniform(0, 1, 200):
        got = oracle.weights(f)
        F = Fraction(float(f))
        want = [brute.bspline_kernel(F + 1), brute.bspline_kernel(F), brute.bspline_kernel(1 - F),
                brute.bspline_kernel(2 - F)]
        np.testing.assert_allclose(got, [float(w) for w in want], rtol=0, atol=1e-15)
        assert np.all(got >= 0)
        assert abs(got.sum() - 1) < 1e-15


# ---------------------------------------------------------- reconstruction --

def _poly_volume(n, fn):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return np.ascontiguousarray(fn(x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)))


@pytest.mark.parametrize(
    "name,field,expect",
    [
        ("constant", lambda x, y, z: 0 * x + 7.25, lambda x, y, z: 7.25),
        ("linear", lambda x, y, z: 3 * x - 2 * y + 0.5 * z + 1, lambda x, y, z: 3 * x - 2 * y + 0.5 * z + 1),
        ("quadratic", lambda x, y, z: x * x, lambda x, y, z: x * x + 1.0 / 3.0),
        ("cubic", lambda x, y, z: x ** 3, lambda x, y, z: x ** 3 + x),
        ("bilinear", lambda x, y, z: x * y, lambda x, y, z: x * y),
        ("quadratic_z", lambda x, y, z: z * z - y, lambda x, y, z: z * z + 1.0 / 3.0 - y),
    ],
)
def test_reconstruction_reproduces_polynomials(oracle_lib, name, field, expect):
    """Interior of the stencil: the cubic B-spline reproduces constants and
    linear fields exactly, maps x^2 to x^2 + 1/3 and x^3 to x^3 + x (its
    second moment is 1/3, odd moments vanish)."""
    n = 12
    vol = _poly_volume(n, field)
    rng = np.random.default_rng(hash(name) % 2**32)
    for p in rng.uniform(1.0, n - 3.0, (40, 3)):
        got = oracle.sample(vol, p)
        want = expect(*p)
        assert abs(got - want) < 1e-9 * max(1.0, abs(want)), (name, p, got, want)


def test_clamp_edge_worked_examples(oracle_lib):
    row = np.arange(4, dtype=np.float64).reshape(1, 1, 4)
    for r in _read_golden("clamp_edge.txt"):
        p = float(Fraction(r[0]))
        want = float(Fraction(r[1]))
        got = oracle.sample(row, (p, 0.0, 0.0))
        assert abs(got - want) < 1e-15, (p, got, want)


def test_reconstruction_matches_rational_brute_force(oracle_lib):
    rng = np.random.default_rng(101)
    vol = rng.integers(-50, 50, (5, 6, 7)).astype(np.int16)
    lists = vol.tolist()
    for p in rng.uniform(-0.5, 6.5, (30, 3)):
        p = np.minimum(p, [6.49, 5.49, 4.49])
        got = oracle.sample(vol, p)
        want = float(brute.reconstruct(lists, p))
        assert abs(got - want) < 1e-12


# ------------------------------------------------------------ Beer-Lambert --

def _constant_tf(c, sigma, K=8, v0=0.0, v1=7.0):
    table = np.tile(np.array([*c, sigma], dtype=np.float32), (K, 1))
    return synth.TransferFunction(table, v0, v1)


def test_beer_lambert_axis_aligned_slab(oracle_lib):
    golden = {r[0]: float(r[1]) for r in _read_golden("beer_lambert.txt")}
    n = 16
    vol = np.full((n, n, n), 3, dtype=np.uint16)
    tf = _constant_tf((0.25, 0.5, 1.0), 1.0 / 16.0)
    cam = synth.ortho_axis_camera(n, 16, 16)
    out = oracle.render(vol, [cam], tf, 0.5)
    rgba = out["rgba"][0]
    assert np.all(out["counts"][0][..., 0] == 32)
    np.testing.assert_allclose(rgba[..., 3], golden["A"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(rgba[..., 0], golden["C_r"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(rgba[..., 1], golden["C_g"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(rgba[..., 2], golden["C_b"], rtol=0, atol=1e-13)


def test_beer_lambert_oblique_rays(oracle_lib):
    """Oblique perspective rays through a homogeneous medium: with every
    segment of full length, T = exp(-sigma0 step n_s) for the lattice count
    n_s of each ray."""
    n = 20
    vol = np.full((n, n, n), 5, dtype=np.int16)
    sigma0 = float(np.float32(0.03))
    tf = _constant_tf((0.5, 0.125, 0.375), sigma0)
    u = np.array([0.3, -0.5, 0.81])
    cam = synth.orbit_camera((n, n, n), u, 50.0, 24, 24)
    step = 0.375
    out = oracle.render(vol, [cam], tf, step)
    ns = out["counts"][0][..., 0]
    assert ns.max() > 0 and (ns == 0).any()
    T = np.exp(-sigma0 * step * ns)
    np.testing.assert_allclose(out["rgba"][0][..., 3], 1 - T, rtol=0, atol=1e-13)
    np.testing.assert_allclose(out["rgba"][0][..., 0], 0.5 * (1 - T), rtol=0, atol=1e-13)
    # lattice count against the definition #{k >= 0 : t_in < (k + 1/2) step < t_out},
    # with t_in/t_out from the face-plane clip of the brute force
    for row, col in [(3, 5), (12, 12), (20, 7), (0, 0)]:
        o, d = brute.camera_ray(cam, row, col)
        hit = brute.clip_planes(o, d, (n, n, n))
        if hit is None:
            assert ns[row, col] == 0
            continue
        k0 = max(math.floor(hit[0] / step - 0.5) + 1, 0)
        k1 = math.ceil(hit[1] / step - 0.5)
        assert ns[row, col] == k1 - k0


# -------------------------------------------------------------- brute force --

def _tiny_volume():
    rng = np.random.default_rng(102)
    return rng.integers(0, 16, (4, 4, 4)).astype(np.uint16)


def _linear_tf():
    # sigma = v / 64, colour constant: node j at value j (v0 = 0, v1 = 15)
    K = 16
    table = np.zeros((K, 4), dtype=np.float32)
    table[:, 0], table[:, 1], table[:, 2] = 0.25, 0.5, 1.0
    table[:, 3] = np.arange(K) / 64.0
    return synth.TransferFunction(table, 0.0, 15.0)


def test_oracle_matches_brute_force_tiny_volume(oracle_lib):
    vol = _tiny_volume()
    lists = vol.tolist()
    tf = _linear_tf()
    classify = lambda v: (0.25, 0.5, 1.0, v / 64.0)  # noqa: E731
    # orthographic rays along +z at pixel centres
    cam = synth.ortho_axis_camera(4, 4, 4)
    out = oracle.render(vol, [cam], tf, 0.5)
    for row in range(4):
        for col in range(4):
            want, n = brute.brute_pixel(lists, cam, row, col, 0.5, classify)
            assert n == out["counts"][0, row, col, 0] == 8
            np.testing.assert_allclose(out["rgba"][0, row, col], want, rtol=0, atol=1e-12)
    # three oblique perspective rays
    pcam = synth.orbit_camera((4, 4, 4), np.array([0.4, 0.7, -0.6]), 40.0, 16, 16)
    pix = [(5, 6), (8, 8), (10, 4)]
    outp = oracle.render(vol, [pcam], tf, 0.3125)
    for row, col in pix:
        want, n = brute.brute_pixel(lists, pcam, row, col, 0.3125, classify)
        assert n == outp["counts"][0, row, col, 0] and n > 0
        np.testing.assert_allclose(outp["rgba"][0, row, col], want, rtol=0, atol=1e-12)


def test_oracle_matches_brute_force_table_tf_and_ert(oracle_lib):
    """A non-linear table (looked up by linear search in the brute force),
    values reaching past both table ends, early termination on."""
    rng = np.random.default_rng(103)
    vol = rng.integers(-200, 1400, (4, 5, 6)).astype(np.int16)
    lists = vol.tolist()
    K = 9
    table = rng.uniform(0, 1, (K, 4)).astype(np.float32)
    table[:, 3] *= 0.9
    tf = synth.TransferFunction(table, 0.0, 1200.0)
    classify = lambda v: brute.tf_table_lookup(table.astype(np.float64).tolist(), 0.0, 1200.0, v)  # noqa: E731
    pcam = synth.orbit_camera((6, 5, 4), np.array([-0.2, 0.5, 0.84]), 45.0, 12, 12)
    out = oracle.render(vol, [pcam], tf, 0.25, ert=0.9)
    checked = 0
    for row in range(0, 12, 3):
        for col in range(0, 12, 2):
            want, n = brute.brute_pixel(lists, pcam, row, col, 0.25, classify, ert=0.9)
            np.testing.assert_allclose(out["rgba"][0, row, col], want, rtol=0, atol=1e-12)
            checked += n > 0
    assert checked > 5


# --------------------------------------------------------- skip and ERT ----

def _small_ct():
    return synth.ct_phantom_i16(48, 40, 36, seed=21, n_soft=4, n_bone=3)


def test_blocks_match_numpy_footprint(oracle_lib):
    vol = _small_ct()
    E = 16
    mm = oracle.blocks(vol, E)
    nz, ny, nx = vol.shape
    for bz in range(mm.shape[0]):
        for by in range(mm.shape[1]):
            for bx in range(mm.shape[2]):
                sl = tuple(
                    slice(max(b * E - 1, 0), min(b * E + E + 1, n - 1) + 1)
                    for b, n in ((bz, nz), (by, ny), (bx, nx))
                )
                sub = vol[sl]
                assert mm[bz, by, bx, 0] == sub.min() and mm[bz, by, bx, 1] == sub.max()


def test_block_footprint_covers_every_tap():
    """Every tap of a sample whose (clamped) cell lies in block b is inside
    b's footprint [bE-1, bE+E+1] (clamped): the property that makes min/max
    skipping conservative."""
    E, n = 16, 37
    rng = np.random.default_rng(104)
    for p in rng.uniform(-0.5, n - 0.5, 2000):
        cell = min(max(math.floor(p), 0), n - 1)
        b = cell // E
        lo, hi = max(b * E - 1, 0), min(b * E + E + 1, n - 1)
        for t in range(math.floor(p) - 1, math.floor(p) + 3):
            tc = min(max(t, 0), n - 1)
            assert lo <= tc <= hi


def test_skip_is_lossless(oracle_lib):
    vol = _small_ct()
    tf = synth.tf1()
    mm = oracle.blocks(vol, 16)
    occ = oracle.occupancy(mm, tf)
    assert 0 < occ.sum() < occ.size
    cams = synth.orbit_cameras((48, 40, 36), 2, 22, 60.0, 40, 40)
    a = oracle.render(vol, cams, tf, 0.5)
    b = oracle.render(vol, cams, tf, 0.5, occ=occ)
    assert np.array_equal(a["rgba"], b["rgba"])
    assert (b["counts"][..., 1] < a["counts"][..., 1]).any()


def test_occupancy_perturbation(oracle_lib):
    """Raising any zero-extinction node inside an empty block's value range
    must flip that block to occupied; an occupied block stays occupied."""
    vol = _small_ct()
    tf = synth.tf1()
    mm = oracle.blocks(vol, 16).reshape(-1, 2)
    occ = oracle.occupancy(mm, tf)
    scale = np.float32(255) / (np.float32(tf.v1) - np.float32(tf.v0))
    empties = np.flatnonzero(occ == 0)
    assert empties.size > 0
    for b in empties[:5]:
        u = (np.float32(mm[b, 0]) - np.float32(tf.v0)) * scale
        j = int(np.floor(u))
        for jj in (j, j + 1):
            t2 = synth.TransferFunction(tf.table.copy(), tf.v0, tf.v1)
            t2.table[jj, 3] = 0.01
            assert oracle.occupancy(mm, t2)[b] == 1
    # the one-node margin on each side of the range is part of the definition
    for b in empties[:5]:
        ulo = (np.float32(mm[b, 0]) - np.float32(tf.v0)) * scale
        uhi = (np.float32(mm[b, 1]) - np.float32(tf.v0)) * scale
        for jj in (int(np.floor(ulo)) - 1, int(np.ceil(uhi)) + 1):
            if 0 <= jj < tf.K:
                t2 = synth.TransferFunction(tf.table.copy(), tf.v0, tf.v1)
                t2.table[jj, 3] = 0.01
                assert oracle.occupancy(mm, t2)[b] == 1
    # a node far above every block's range changes nothing
    t3 = synth.TransferFunction(tf.table.copy(), tf.v0, tf.v1)
    t3.table[250, 3] = 0.0
    assert np.array_equal(oracle.occupancy(mm, t3), occ)


def test_ert_changes_each_channel_by_at_most_one_minus_theta(oracle_lib):
    vol = _small_ct()
    tf = synth.tf1()
    cams = synth.orbit_cameras((48, 40, 36), 2, 23, 60.0, 40, 40)
    theta = 0.9
    a = oracle.render(vol, cams, tf, 0.5)
    b = oracle.render(vol, cams, tf, 0.5, ert=theta)
    diff = np.abs(a["rgba"] - b["rgba"])
    assert diff.max() <= (1 - theta) + 1e-12
    assert (b["counts"][..., 1] < a["counts"][..., 1]).any()
    term = b["rgba"][..., 3] >= theta
    assert term.any()


# --------------------------------------------------------------- gradients --

def _grad_case():
    rng = np.random.default_rng(105)
    from scipy.ndimage import gaussian_filter

    vol = gaussian_filter(rng.standard_normal((9, 10, 11)), 1.5)
    vol = (vol - vol.min()) / (vol.max() - vol.min())
    vol = np.ascontiguousarray(vol.astype(np.float64))
    # node values multiples of 2^-12 so that +-2^-10 is exact in fp32
    K = 12
    table = np.round(rng.uniform(0.05, 0.9, (K, 4)) * 4096) / 4096
    table[:, 3] *= 0.5
    tf = synth.TransferFunction(table.astype(np.float32), -0.1, 1.1)
    cams = synth.orbit_cameras((11, 10, 9), 2, 106, 55.0, 10, 10)
    g = rng.standard_normal((2, 10, 10, 4))
    return vol, tf, cams, g


def _loss(vol, tf, cams, g, step, ert=0.0):
    return float((oracle.render(vol, cams, tf, step, ert=ert)["rgba"] * g).sum())


def _fd_volume(vol, tf, cams, g, step, ijk, h, ert=0.0):
    vp = vol.copy()
    vp[ijk] += h
    vm = vol.copy()
    vm[ijk] -= h
    return (_loss(vp, tf, cams, g, step, ert) - _loss(vm, tf, cams, g, step, ert)) / (2 * h)


def test_grad_volume_matches_central_differences(oracle_lib):
    """Analytic FP64 gradient vs central differences.  A voxel whose
    perturbation moves some sample across a TF node (a kink of the piecewise-
    linear TF, where several subgradients are correct) shows up as FD values
    that disagree between two step sizes; such voxels are re-drawn."""
    vol, tf, cams, g = _grad_case()
    step = 0.4375
    gv, _ = oracle.grad(vol, cams, tf, step, g)
    rng = np.random.default_rng(107)
    scale = max(1.0, abs(gv).max())
    checked = 0
    for _ in range(40):
        ijk = tuple(int(rng.integers(0, s)) for s in vol.shape)
        fd1 = _fd_volume(vol, tf, cams, g, step, ijk, 1e-5)
        fd2 = _fd_volume(vol, tf, cams, g, step, ijk, 4e-6)
        if abs(fd1 - fd2) > 1e-7 * scale:
            continue  # kink inside the FD stencil
        assert abs(fd1 - gv[ijk]) <= 1e-7 * scale, (ijk, fd1, gv[ijk])
        checked += 1
        if checked == 16:
            break
    assert checked >= 12


def test_grad_tf_matches_central_differences(oracle_lib):
    vol, tf, cams, g = _grad_case()
    step = 0.4375
    _, gt = oracle.grad(vol, cams, tf, step, g)
    h = 2.0 ** -10
    for j in range(tf.K):
        for c in range(4):
            tp = synth.TransferFunction(tf.table.copy(), tf.v0, tf.v1)
            tp.table[j, c] += h
            tm = synth.TransferFunction(tf.table.copy(), tf.v0, tf.v1)
            tm.table[j, c] -= h
            fd = (_loss(vol, tp, cams, g, step) - _loss(vol, tm, cams, g, step)) / (2 * h)
            # second-order FD error of the exp in sigma
            assert abs(fd - gt[j, c]) <= 1e-5 * max(1.0, abs(gt).max()), (j, c, fd, gt[j, c])


def test_grad_closed_form_homogeneous_medium(oracle_lib):
    """Constant field sitting exactly on node j: dC/dsigma_j = c L e^{-sigma L},
    dA/dsigma_j = L e^{-sigma L}, dC/dc_j = 1 - e^{-sigma L}, L = n_s step."""
    n = 16
    vol = np.full((n, n, n), 3, dtype=np.uint16)
    sigma, c = 1.0 / 16.0, (0.25, 0.5, 1.0)
    tf = _constant_tf(c, sigma)  # nodes at 0..7, value 3 is node 3
    cam = synth.ortho_axis_camera(n, 4, 4)
    L = 16.0
    e = math.exp(-sigma * L)
    g = np.zeros((1, 4, 4, 4))
    g[0, 1, 2, 0] = 1.0
    _, gt = oracle.grad(vol, [cam], tf, 0.5, g)
    assert abs(gt[3, 3] - c[0] * L * e) < 1e-12
    assert abs(gt[3, 0] - (1 - e)) < 1e-12
    assert np.abs(np.delete(gt, 3, axis=0)).max() < 1e-12
    g = np.zeros((1, 4, 4, 4))
    g[0, 3, 3, 3] = 1.0
    _, gt = oracle.grad(vol, [cam], tf, 0.5, g)
    assert abs(gt[3, 3] - L * e) < 1e-12


def test_grad_with_ert_matches_fd_with_fixed_stop(oracle_lib):
    vol, tf, cams, g = _grad_case()
    tf.table[:, 3] *= 4.0
    step, ert = 0.4375, 0.75
    gv, _ = oracle.grad(vol, cams, tf, step, g, ert=ert)
    assert oracle.render(vol, cams, tf, step, ert=ert)["rgba"][..., 3].max() >= ert
    rng = np.random.default_rng(108)
    h = 1e-6
    base = oracle.render(vol, cams, tf, step, ert=ert)["counts"][..., 1]
    scale = max(1.0, abs(gv).max())
    checked = 0
    for _ in range(40):
        ijk = tuple(int(rng.integers(0, s)) for s in vol.shape)
        vp = vol.copy()
        vp[ijk] += h
        vm = vol.copy()
        vm[ijk] -= h
        # the stopping index must not move for FD to be a derivative
        if not (np.array_equal(oracle.render(vp, cams, tf, step, ert=ert)["counts"][..., 1], base)
                and np.array_equal(oracle.render(vm, cams, tf, step, ert=ert)["counts"][..., 1], base)):
            continue
        fd1 = _fd_volume(vol, tf, cams, g, step, ijk, h, ert)
        fd2 = _fd_volume(vol, tf, cams, g, step, ijk, h / 2, ert)
        if abs(fd1 - fd2) > 1e-6 * scale:
            continue  # kink inside the FD stencil
        assert abs(fd1 - gv[ijk]) <= 1e-6 * scale, (ijk, fd1, gv[ijk])
        checked += 1
        if checked == 12:
            break
    assert checked >= 8


def test_grad_magnitudes_bound_the_gradient(oracle_lib):
    """The magnitude sums (every term of the adjoint sums by its absolute
    value, the suffix-sum difference |T_{k+1} c_k| + |S_k| included) bound the
    gradient element-wise (triangle inequality), equal it where no term can
    cancel (dC/dc of a homogeneous medium: every term positive), do not depend
    on the sign of dL/dRGBA and scale with its magnitude."""
    vol, tf, cams, g = _grad_case()
    step = 0.4375
    gv, gt, mv, mt = oracle.grad(vol, cams, tf, step, g, magnitudes=True)
    assert np.all(mv >= np.abs(gv) * (1 - 1e-12)) and np.all(mt >= np.abs(gt) * (1 - 1e-12))
    assert (mv > np.abs(gv) * (1 + 1e-6)).any()  # cancellation happens somewhere
    gv2, gt2, mv2, mt2 = oracle.grad(vol, cams, tf, step, -2.0 * g, magnitudes=True)
    assert np.allclose(gv2, -2.0 * gv, rtol=1e-12, atol=1e-15) and np.allclose(mv2, 2.0 * mv, rtol=1e-12, atol=1e-15)
    assert np.allclose(mt2, 2.0 * mt, rtol=1e-12, atol=1e-15)
    n = 16
    hv = np.full((n, n, n), 3, dtype=np.uint16)
    htf = _constant_tf((0.25, 0.5, 1.0), 1.0 / 16.0)
    cam = synth.ortho_axis_camera(n, 4, 4)
    gg = np.zeros((1, 4, 4, 4))
    gg[0, 1, 2, 0] = 1.0
    _, ht, _, hm = oracle.grad(hv, [cam], htf, 0.5, gg, magnitudes=True)
    assert abs(hm[3, 0] - ht[3, 0]) <= 1e-12 * abs(ht[3, 0])
