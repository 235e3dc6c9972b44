"""GPU parity of the filter ablations: the interpolating cubic B-spline
(vr_prefilter_bspline, then the ordinary render of the coefficients) and the
Catmull-Rom filter (vr_params.filter) with its widened skip test.

Bars: coefficients within 1e-5 of the volume's largest magnitude (fp32
elimination against FP64); images within max |dRGBA| <= 2e-4 with the
termination-tie allowance; skipping bit-identical to rendering every sample.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2005_01442_amd as vr  # noqa: E402
from gpu_util import DEV, compare_with_flags, log, upload_tf, upload_volume  # noqa: E402
from test_oracle_filters import _undershoot_case  # noqa: E402

TOL = 2e-4
CR = vr.VR_FILTER_CATMULL_ROM


def _small_ct(dims=(96, 80, 72), seed=71):
    return synth.ct_phantom_i16(*dims, seed=seed, n_soft=6, n_bone=4)


@pytest.mark.parametrize("case", ["u16_odd", "i16_ct", "f32", "thin"])
def test_prefilter_matches_oracle(case):
    vol = {"u16_odd": lambda: synth.ellipsoid_phantom_u16(48, seed=72)[:, :47, :45].copy(),
           "i16_ct": lambda: _small_ct(),
           "f32": lambda: synth.density_grid_f32(40, seed=73),
           "thin": lambda: synth.ellipsoid_phantom_u16(16, seed=74)[:1, :2, :].copy()}[case]()
    c = vr.vr_prefilter_bspline(upload_volume(vol)).tensor.cpu().numpy().astype(np.float64)
    ref = oracle.prefilter(vol)
    d = np.abs(c - ref).max()
    log(f"prefilter {case} {vol.shape}: max |d| = {d:.3e} (max |v| {np.abs(vol).max()})")
    assert d <= 1e-5 * max(1.0, float(np.abs(vol.astype(np.float64)).max()))


def test_interpolating_spline_render_matches_oracle():
    vol = _small_ct()
    dims = (96, 80, 72)
    cams = synth.orbit_cameras(dims, 2, 75, 60.0, 120, 104)
    tf = synth.tf1()
    coef = vr.vr_prefilter_bspline(upload_volume(vol))
    t = upload_tf(tf)
    blocks = vr.vr_build_blocks(coef, 16)
    img = vr.vr_render(coef, blocks, cams, t, 0.5, 0.99, True).cpu().numpy().astype(np.float64)
    ref = oracle.render(oracle.prefilter(vol), cams, tf, 0.5, ert=0.99)
    un, nflag = compare_with_flags(img, ref["rgba"], ref["flags"], 0.99)
    log(f"interpolating spline: max unflagged |dRGBA| = {un:.3e}, flagged {nflag}")
    assert nflag <= 1e-3 * img[..., 0].size + 2


def _cr(vol_np, cams, tf, step, ert=0.0, use_skip=False, vol=None, edge=16, counters=False):
    v = vol if vol is not None else upload_volume(vol_np)
    t = upload_tf(tf)
    b = vr.vr_build_blocks(v, edge) if use_skip else None
    ctr = torch.zeros(4, dtype=torch.int64, device=DEV) if counters else None
    out = vr.vr_render(v, b, cams, t, step, ert, use_skip, counters=ctr, filter=CR)
    torch.cuda.synchronize()
    img = out.cpu().numpy().astype(np.float64)
    return (img, ctr.cpu().numpy()) if counters else img


def test_catmull_rom_c0_full_frame():
    c = synth.config_c0()
    img = _cr(c["volume"], c["cameras"], c["tf"], c["step"])
    ref = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"], filter=1)
    d = np.abs(img - ref["rgba"]).max()
    log(f"catmull-rom c0: max |dRGBA| = {d:.3e}")
    assert d <= TOL


def test_catmull_rom_ct_skip_and_ert():
    vol = _small_ct()
    dims = (96, 80, 72)
    cams = synth.orbit_cameras(dims, 2, 76, 60.0, 120, 104)
    tf = synth.tf1()
    v = upload_volume(vol)
    a, ca = _cr(vol, cams, tf, 0.5, 0.99, True, vol=v, counters=True)
    b, cb = _cr(vol, cams, tf, 0.5, 0.99, False, vol=v, counters=True)
    assert np.array_equal(a, b)
    assert ca[0] < cb[0]
    ref = oracle.render(vol, cams, tf, 0.5, ert=0.99, filter=1)
    un, nflag = compare_with_flags(a, ref["rgba"], ref["flags"], 0.99)
    log(f"catmull-rom ct: max unflagged |dRGBA| = {un:.3e}, flagged {nflag}")
    assert nflag <= 1e-3 * a[..., 0].size + 2


def test_catmull_rom_undershoot_is_not_skipped():
    vol, tf, cams = _undershoot_case()
    v = upload_volume(vol)
    a = _cr(vol, cams, tf, 0.5, use_skip=True, vol=v, edge=8)
    b = _cr(vol, cams, tf, 0.5, use_skip=False, vol=v, edge=8)
    ref = oracle.render(vol, cams, tf, 0.5, filter=1)
    assert np.array_equal(a, b)
    assert a[..., 3].max() > 0.01
    assert np.abs(a - ref["rgba"]).max() <= TOL


def test_catmull_rom_f32_global_path():
    vol = synth.density_grid_f32(48, seed=77)
    tf = synth.tf3()
    cams = synth.orbit_cameras((48, 48, 48), 2, 78, 50.0, 12, 10)
    img, ctr = _cr(vol, cams, tf, 0.5, counters=True)
    ref = oracle.render(vol, cams, tf, 0.5, filter=1)
    assert np.abs(img - ref["rgba"]).max() <= TOL
    assert ctr[3] > 0


def test_catmull_rom_is_rejected_where_unsupported():
    vol = upload_volume(_small_ct((16, 16, 16)))
    t = upload_tf(synth.tf1())
    cams = synth.orbit_cameras((16, 16, 16), 1, 79, 60.0, 8, 8)
    with pytest.raises(vr.VrError, match="VR_E_UNSUPPORTED"):
        vr.vr_render(vol, None, cams, t, 0.5, shading=vr.Shading(), filter=CR)
    with pytest.raises(vr.VrError, match="unknown filter"):
        vr.vr_render(vol, None, cams, t, 0.5, filter=7)


PRE = vr.VR_FILTER_BSPLINE_PRECLASSIFIED


def _pre(vol_np, cams, tf, step, ert=0.0, use_skip=False, vol=None, counters=False):
    v = vol if vol is not None else upload_volume(vol_np)
    t = upload_tf(tf)
    b = vr.vr_build_blocks(v, 16) if use_skip else None
    ctr = torch.zeros(4, dtype=torch.int64, device=DEV) if counters else None
    out = vr.vr_render(v, b, cams, t, step, ert, use_skip, counters=ctr, filter=PRE)
    torch.cuda.synchronize()
    img = out.cpu().numpy().astype(np.float64)
    return (img, ctr.cpu().numpy()) if counters else img


def test_preclassified_ct_skip_and_ert():
    vol = _small_ct()
    dims = (96, 80, 72)
    cams = synth.orbit_cameras(dims, 2, 80, 60.0, 120, 104)
    tf = synth.tf1()
    v = upload_volume(vol)
    a, ca = _pre(vol, cams, tf, 0.5, 0.99, True, vol=v, counters=True)
    b = _pre(vol, cams, tf, 0.5, 0.99, False, vol=v)
    assert np.array_equal(a, b)
    ref = oracle.render(vol, cams, tf, 0.5, ert=0.99, filter=2)
    un, nflag = compare_with_flags(a, ref["rgba"], ref["flags"], 0.99)
    log(f"pre-classified ct: max unflagged |dRGBA| = {un:.3e}, flagged {nflag}")
    assert nflag <= 1e-3 * a[..., 0].size + 2


def test_preclassified_global_path_and_dtypes():
    for vol, tf, dims in [(synth.density_grid_f32(48, seed=81), synth.tf3(), (48, 48, 48)),
                          (synth.ellipsoid_phantom_u16(48, seed=82)[:, :47, :45].copy(), synth.tf0(), (45, 47, 48))]:
        cams = synth.orbit_cameras(dims, 2, 83, 50.0, 12, 10)
        img, ctr = _pre(vol, cams, tf, 0.5, counters=True)
        ref = oracle.render(vol, cams, tf, 0.5, filter=2)
        d = np.abs(img - ref["rgba"]).max()
        log(f"pre-classified {vol.dtype}: max |dRGBA| = {d:.3e}, global-path samples {ctr[3]}")
        assert d <= TOL
        assert ctr[3] > 0



def test_trilinear_ct_skip_and_ert():
    vol = _small_ct()
    dims = (96, 80, 72)
    cams = synth.orbit_cameras(dims, 2, 84, 60.0, 120, 104)
    tf = synth.tf1()
    v = upload_volume(vol)
    t = upload_tf(tf)
    b = vr.vr_build_blocks(v, 16)
    a = vr.vr_render(v, b, cams, t, 0.5, 0.99, True, filter=vr.VR_FILTER_TRILINEAR).cpu().numpy().astype(np.float64)
    n = vr.vr_render(v, None, cams, t, 0.5, 0.99, False, filter=vr.VR_FILTER_TRILINEAR).cpu().numpy().astype(np.float64)
    assert np.array_equal(a, n)
    ref = oracle.render(vol, cams, tf, 0.5, ert=0.99, filter=3)
    un, nflag = compare_with_flags(a, ref["rgba"], ref["flags"], 0.99)
    log(f"trilinear ct: max unflagged |dRGBA| = {un:.3e}, flagged {nflag}")
    assert nflag <= 1e-3 * a[..., 0].size + 2


@pytest.mark.parametrize("mode", ["catmull_rom", "preclassified", "trilinear", "interpolating"])
def test_filters_c1_full_size_sampled_pixels(mode):
    """The 512x512x400 frame in the bench's launch configuration for every
    filter variant; 512 sampled pixels checked against the oracle."""
    c = synth.config_c1()
    v = upload_volume(c["volume"])
    t = upload_tf(c["tf"])
    pix = synth.sample_pixels(1, 1024, 1024, 512, seed=85)
    if mode == "interpolating":
        coef = vr.vr_prefilter_bspline(v)
        img = vr.vr_render(coef, vr.vr_build_blocks(coef, 16), c["cameras"], t, c["step"], c["ert"], True)
        ref = oracle.render(oracle.prefilter(c["volume"]), c["cameras"], c["tf"], c["step"], ert=c["ert"], pixels=pix)
    else:
        f = {"catmull_rom": (CR, 1), "preclassified": (PRE, 2), "trilinear": (vr.VR_FILTER_TRILINEAR, 3)}[mode]
        img = vr.vr_render(v, vr.vr_build_blocks(v, 16), c["cameras"], t, c["step"], c["ert"], True, filter=f[0])
        ref = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"], ert=c["ert"], pixels=pix, filter=f[1])
    torch.cuda.synchronize()
    got = img.cpu().numpy().astype(np.float64)[pix[:, 0], pix[:, 1], pix[:, 2]]
    un, nflag = compare_with_flags(got, ref["rgba"], ref["flags"], c["ert"])
    log(f"c1 {mode}: max unflagged |dRGBA| = {un:.3e}, flagged {nflag}")
    assert nflag <= 4
