"""Pins of the oracle's pre-integrated classification: the segment table
against closed forms and an independent adaptive quadrature, and the
pre-integrated render against the post-classified render where the two must
agree, against a brute force, and against its own purpose (fewer step-size
artefacts than post-classification at the same step)."""

import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import brute
import synth


def _tf(table, v0=0.0, v1=None):
    table = np.asarray(table, dtype=np.float32)
    return synth.TransferFunction(table, v0, float(table.shape[0] - 1) if v1 is None else v1)


# ------------------------------------------------------------------ table --

def test_table_constant_tf_closed_form(oracle_lib):
    c, sigma, step = (0.25, 0.5, 1.0), 0.3, 0.75
    tab = oracle.preint_table(_tf(np.tile([*c, sigma], (7, 1))), step)
    a = -math.expm1(-float(np.float32(sigma)) * step)
    np.testing.assert_allclose(tab[..., 3], a, rtol=0, atol=1e-10)
    for k in range(3):
        np.testing.assert_allclose(tab[..., k], float(np.float32(c[k])) * a, rtol=0, atol=1e-10)


def test_table_linear_extinction_closed_form(oracle_lib):
    """sigma linear in the node index, colour constant: the optical depth of a
    ramp i -> j is step (sigma_i + sigma_j) / 2 and C = c alpha."""
    K, step = 9, 1.5
    sig = np.arange(K) / 64.0  # exactly linear in fp32
    table = np.column_stack([np.full(K, 0.75), np.full(K, 0.5), np.full(K, 0.25), sig]).astype(np.float32)
    tab = oracle.preint_table(_tf(table), step)
    s32 = table[:, 3].astype(np.float64)
    for i in range(K):
        for j in range(K):
            a = -math.expm1(-step * (s32[i] + s32[j]) / 2)
            assert abs(tab[i, j, 3] - a) < 1e-12
            np.testing.assert_allclose(tab[i, j, :3], table[0, :3].astype(np.float64) * a, rtol=0, atol=1e-10)


def _quad_entry(table, i, j, step):
    """Independent adaptive quadrature (scipy) of the segment integrals."""
    K = table.shape[0]
    tt = table.astype(np.float64)

    def at(u, ch):
        return float(np.interp(u, np.arange(K), tt[:, ch]))

    u = lambda x: i + (j - i) * x / step  # noqa: E731
    pts = sorted({(m - i) * step / (j - i) for m in range(min(i, j) + 1, max(i, j))}) if i != j else []

    def tau(x):
        if x <= 0.0:
            return 0.0
        inner = [p for p in pts if p < x]
        return integrate.quad(lambda y: at(u(y), 3), 0.0, x, points=inner or None, epsabs=1e-14, epsrel=1e-13,
                              limit=200)[0]

    out = []
    for ch in range(3):
        f = lambda x, ch=ch: at(u(x), ch) * at(u(x), 3) * math.exp(-tau(x))  # noqa: E731
        out.append(integrate.quad(f, 0.0, step, points=pts or None, epsabs=1e-13, epsrel=1e-11, limit=200)[0])
    out.append(-math.expm1(-tau(step)))
    return np.array(out)


def test_table_matches_adaptive_quadrature(oracle_lib):
    rng = np.random.default_rng(401)
    K = 6
    table = rng.uniform(0, 1, (K, 4)).astype(np.float32)
    table[:, 3] *= 1.5
    step = 0.875
    tab = oracle.preint_table(_tf(table), step)
    for i, j in [(0, 5), (5, 0), (2, 3), (4, 1), (3, 3), (1, 4)]:
        np.testing.assert_allclose(tab[i, j], _quad_entry(table, i, j, step), rtol=0, atol=1e-9)


def test_table_opacity_is_symmetric_and_diagonal_is_post_classification(oracle_lib):
    tf = synth.tf1()
    tab = oracle.preint_table(tf, 0.5)
    np.testing.assert_allclose(tab[..., 3], tab[..., 3].T, rtol=0, atol=1e-12)
    t = tf.table.astype(np.float64)
    a = -np.expm1(-t[:, 3] * 0.5)
    d = np.arange(t.shape[0])
    np.testing.assert_allclose(tab[d, d, 3], a, rtol=0, atol=1e-15)
    np.testing.assert_allclose(tab[d, d, :3], t[:, :3] * a[:, None], rtol=0, atol=1e-15)
    # colour depends on the direction of the ramp where colour and extinction vary together
    assert np.abs(tab[..., :3] - tab[..., :3].transpose(1, 0, 2)).max() > 1e-4


# ----------------------------------------------------------------- render --

def test_constant_tf_preint_equals_post_classification(oracle_lib):
    """With a constant TF every cell has the post-classified sample's colour
    and opacity: the two renders agree on the same lattice cells."""
    vol = synth.ellipsoid_phantom_u16(16, seed=402)
    tf = _tf(np.tile([0.2, 0.6, 0.9, 0.07], (8, 1)), 0.0, 4095.0)
    cams = synth.orbit_cameras((16, 16, 16), 2, 403, 50.0, 12, 12)
    a = oracle.render_preint(vol, cams, tf, 0.625)
    b = oracle.render(vol, cams, tf, 0.625)
    np.testing.assert_array_equal(a["counts"][..., 0], b["counts"][..., 0])
    np.testing.assert_allclose(a["rgba"], b["rgba"], rtol=0, atol=1e-13)


def _ct(dims=(40, 36, 32), seed=404):
    return synth.ct_phantom_i16(*dims, seed=seed, n_soft=4, n_bone=3)


@pytest.mark.parametrize("step,edge", [(0.5, 8), (2.5, 4)])
def test_preint_skip_is_lossless(oracle_lib, step, edge):
    """A cell is skipped only when no value between its two blocks' ranges
    meets extinction; long cells over small blocks often join an empty and an
    occupied block."""
    vol = _ct()
    tf = synth.tf1()
    cams = synth.orbit_cameras((40, 36, 32), 2, 405, 55.0, 24, 20)
    mm = oracle.blocks(vol, edge)
    a = oracle.render_preint(vol, cams, tf, step, ert=0.99, minmax=mm, edge=edge)
    b = oracle.render_preint(vol, cams, tf, step, ert=0.99)
    np.testing.assert_array_equal(a["rgba"], b["rgba"])
    assert a["counts"][..., 1].sum() < b["counts"][..., 1].sum()


def test_preint_skip_joins_both_blocks(oracle_lib):
    """A cell from an all-air block into a tissue block: its front block alone
    is empty, but the ramp between the two values meets extinction, so the
    cell must be evaluated (air x < 8, tissue x >= 8; rays along +x with
    cell boundaries at x = 3 and 8)."""
    vol = np.full((8, 8, 16), -1000, dtype=np.int16)
    vol[:, :, 8:] = 40
    tf = synth.tf1()
    cam = synth.Camera(projection=0, eye=np.array([-1002.0, 3.5, 3.5]), right=np.array([0.0, 1.0, 0.0]),
                       up=np.array([0.0, 0.0, 1.0]), forward=np.array([1.0, 0.0, 0.0]), ortho_w=8.0, ortho_h=8.0,
                       width=8, height=8)
    mm = oracle.blocks(vol, 4)
    a = oracle.render_preint(vol, [cam], tf, 5.0, minmax=mm, edge=4)
    b = oracle.render_preint(vol, [cam], tf, 5.0)
    np.testing.assert_array_equal(a["rgba"], b["rgba"])
    assert b["rgba"][..., 3].min() > 0.0


def test_preint_render_matches_brute_force(oracle_lib):
    """Rational reconstruction at the cell boundaries, its own clip and an
    independent bilinear lookup of the (separately pinned) table."""
    rng = np.random.default_rng(406)
    vol = rng.integers(0, 48, (5, 6, 7)).astype(np.uint16)
    lists = vol.tolist()
    K = 7
    table = rng.uniform(0, 1, (K, 4)).astype(np.float32)
    table[:, 3] *= 0.6
    tf = _tf(table, 0.0, 48.0)
    step = 0.4375
    tab = oracle.preint_table(tf, step)
    cam = synth.orbit_camera((7, 6, 5), np.array([0.5, 0.35, -0.79]), 45.0, 10, 10)
    out = oracle.render_preint(vol, [cam], tf, step, table=tab)
    scale = (K - 1) / 48.0

    def lookup(uf, ub):
        uf, ub = min(max(uf, 0.0), K - 1.0), min(max(ub, 0.0), K - 1.0)
        i, j = min(int(math.floor(uf)), K - 2), min(int(math.floor(ub)), K - 2)
        a, b = uf - i, ub - j
        return ((1 - a) * (1 - b) * tab[i, j] + a * (1 - b) * tab[i + 1, j] + (1 - a) * b * tab[i, j + 1]
                + a * b * tab[i + 1, j + 1])

    checked = 0
    for row in range(2, 8):
        for col in range(2, 8):
            o, d = brute.camera_ray(cam, row, col)
            hit = brute.clip_planes(o, d, (7, 6, 5))
            want = np.zeros(4)
            if hit is not None:
                tin, tout = hit
                k = 0
                while (k + 0.5) * step <= tin:
                    k += 1
                T, C = 1.0, np.zeros(3)
                while (k + 0.5) * step < tout:
                    vf = float(brute.reconstruct(lists, [o[c] + k * step * d[c] for c in range(3)]))
                    vb = float(brute.reconstruct(lists, [o[c] + (k + 1) * step * d[c] for c in range(3)]))
                    seg = lookup(vf * scale, vb * scale)
                    C += T * seg[:3]
                    T *= 1 - seg[3]
                    k += 1
                want = np.array([*C, 1 - T])
                checked += 1
            np.testing.assert_allclose(out["rgba"][0, row, col], want, rtol=0, atol=1e-11)
    assert checked >= 16


def _psnr(a, b):
    mse = float(np.mean((a - b) ** 2))
    return 10 * math.log10(1.0 / mse)


SPIKE_POINTS = [(-1024.0, (0, 0, 0, 0)), (-16.0, (0, 0, 0, 0)), (0.0, (0.8, 0.3, 0.2, 0.01)),
                (96.0, (0.8, 0.3, 0.2, 0.01)), (112.0, (0, 0, 0, 0)), (336.0, (0, 0, 0, 0)),
                (352.0, (1.0, 0.9, 0.8, 0.6)), (368.0, (0, 0, 0, 0)), (3056.0, (0, 0, 0, 0))]


def test_preint_reduces_step_artefacts(oracle_lib):
    """A TF with a one-node extinction spike (an iso-surface-like feature that
    coarse samples step over): at a coarse step the pre-integrated image is
    much closer to a fine-step reference than the post-classified one (the
    purpose of the tables).  With a smooth TF the midpoint samples win by a
    constant factor; both converge as the step shrinks."""
    vol = _ct((32, 32, 32), seed=407)
    tf = synth.tf_from_points(SPIKE_POINTS, 256, -1024.0, 3056.0)
    cams = synth.orbit_cameras((32, 32, 32), 1, 408, 50.0, 32, 32)
    ref = oracle.render(vol, cams, tf, 1.0 / 16)["rgba"]
    for step in (1.0, 2.0):
        post = oracle.render(vol, cams, tf, step)["rgba"]
        pre = oracle.render_preint(vol, cams, tf, step)["rgba"]
        p_post, p_pre = _psnr(post, ref), _psnr(pre, ref)
        assert p_pre > p_post + 4.0, (step, p_pre, p_post)
    smooth = synth.tf1()
    ref = oracle.render(vol, cams, smooth, 1.0 / 16)["rgba"]
    errs = [_psnr(oracle.render_preint(vol, cams, smooth, st)["rgba"], ref) for st in (0.5, 0.25)]
    assert errs[1] > errs[0] + 9.0 and errs[1] > 75.0, errs
