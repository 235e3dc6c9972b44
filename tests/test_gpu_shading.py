"""GPU parity of the lit render (vr_render_shaded) against the FP64 oracle.

The lit colour uses the analytic gradient of the cubic reconstruction (same
64 taps, derivative weights) and two-sided Blinn-Phong lighting.  Bar: max
|dRGBA| <= 2e-4, as for the unlit render; pixels where the oracle sees an
early-termination tie may differ by up to 1 - theta more.  Opacity and the
samples evaluated do not depend on lighting: the alpha channel and the
counters must equal the unlit render's bit for bit.
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

TOL = 2e-4


def _lit(vol_np, cams, tf, step, shade, ert=0.0, use_skip=False, vol=None, counters=False):
    v = vol if vol is not None else upload_volume(vol_np)
    t = upload_tf(tf)
    blocks = vr.vr_build_blocks(v, 16) if use_skip else None
    ctr = torch.zeros(4, dtype=torch.int64, device=DEV) if counters else None
    sh = None if shade is None else vr.Shading(**shade)
    out = vr.vr_render(v, blocks, cams, t, step, ert, use_skip, counters=ctr, shading=sh)
    torch.cuda.synchronize()
    img = out.cpu().numpy().astype(np.float64)
    return (img, ctr.cpu().numpy()) if counters else img


def _small_ct(dims=(96, 80, 72), seed=41):
    return synth.ct_phantom_i16(*dims, seed=seed, n_soft=6, n_bone=4)


def test_c0_lit_full_frame_matches_oracle():
    c = synth.config_c0()
    log("lit c0: 64^3 u16 ortho 256^2, fixed light")
    img = _lit(c["volume"], c["cameras"], c["tf"], c["step"], synth.SHADE_C0)
    ref = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"], shading=synth.SHADE_C0)
    d = np.abs(img - ref["rgba"]).max()
    log(f"lit c0 max |dRGBA| = {d:.3e}")
    assert d <= TOL
    plain = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"])["rgba"]
    assert np.abs(ref["rgba"][..., :3] - plain[..., :3]).max() > 0.05  # lighting changes the image


@pytest.mark.parametrize("shade", ["fixed", "headlight"])
def test_ct_lit_perspective_skip_and_ert_match_oracle(shade):
    vol = _small_ct()
    dims = (96, 80, 72)
    cams = synth.orbit_cameras(dims, 2, 42, 60.0, 120, 104)  # ragged: not a multiple of 16
    tf = synth.tf1()
    sh = synth.SHADE_CT if shade == "fixed" else synth.SHADE_CT_HEADLIGHT
    log(f"lit ct 96x80x72 persp 120x104 x2 skip ert=0.99 {shade}")
    img = _lit(vol, cams, tf, 0.5, sh, ert=0.99, use_skip=True)
    ref = oracle.render(vol, cams, tf, 0.5, ert=0.99, shading=sh)
    un, nflag = compare_with_flags(img, ref["rgba"], ref["flags"], 0.99)
    log(f"max unflagged |dRGBA| = {un:.3e}, flagged = {nflag}")
    assert nflag <= 1e-3 * img[..., 0].size + 2


def test_lighting_changes_colour_only():
    """Alpha and the evaluated-sample counters equal the unlit render's."""
    vol = _small_ct()
    cams = synth.orbit_cameras((96, 80, 72), 3, 43, 60.0, 96, 96)
    tf = synth.tf1()
    v = upload_volume(vol)
    a, ca = _lit(vol, cams, tf, 0.5, None, ert=0.99, use_skip=True, vol=v, counters=True)
    b, cb = _lit(vol, cams, tf, 0.5, synth.SHADE_CT, ert=0.99, use_skip=True, vol=v, counters=True)
    assert np.array_equal(a[..., 3], b[..., 3])
    assert np.array_equal(ca[:3], cb[:3])
    assert np.abs(a[..., :3] - b[..., :3]).max() > 0.01


def test_unlit_limit_is_bit_identical():
    """ambient 1, diffuse 0, specular 0 reproduces the unlit image exactly."""
    vol = _small_ct()
    cams = synth.orbit_cameras((96, 80, 72), 2, 44, 60.0, 80, 64)
    tf = synth.tf1()
    v = upload_volume(vol)
    plain = _lit(vol, cams, tf, 0.5, None, ert=0.99, use_skip=True, vol=v)
    same = _lit(vol, cams, tf, 0.5, dict(synth.SHADE_CT, ambient=1.0, diffuse=0.0, specular=0.0), ert=0.99,
                use_skip=True, vol=v)
    assert np.array_equal(plain, same)


@pytest.mark.parametrize("dtype", ["f32", "u16_odd"])
def test_lit_global_path_and_dtypes(dtype):
    """Widely spaced rays (a tiny image over the volume) spread a wavefront's
    stencils wider than an LDS box, so taps come from global memory; f32 grids
    and odd-length u16 rows take the other load forms."""
    if dtype == "f32":
        vol = synth.density_grid_f32(48, seed=45)
        tf = synth.tf3()
        sh = dict(synth.SHADE_C0, grad_min=0.02)
        dims = (48, 48, 48)
    else:
        vol = synth.ellipsoid_phantom_u16(48, seed=46)[:, :47, :45].copy()
        tf = synth.tf0()
        sh = synth.SHADE_C0
        dims = (45, 47, 48)
    cams = synth.orbit_cameras(dims, 2, 47, 50.0, 12, 10) + synth.orbit_cameras(dims, 1, 48, 50.0, 12, 10)
    log(f"lit {dtype} {dims} 12x10 x3")
    img, ctr = _lit(vol, cams, tf, 0.5, sh, counters=True)
    ref = oracle.render(vol, cams, tf, 0.5, shading=sh)
    d = np.abs(img - ref["rgba"]).max()
    log(f"lit {dtype} max |dRGBA| = {d:.3e}, global-path samples {ctr[3]} of {ctr[0]}")
    assert d <= TOL
    assert ctr[3] > 0


def test_lit_c1_full_size_sampled_pixels():
    """The full C1 frame in the bench's launch configuration, lit; a sampled
    pixel set checked against the oracle."""
    c = synth.config_c1()
    log("lit c1: 512x512x400 i16 -> 1024^2, 1024 sampled pixels")
    img = _lit(c["volume"], c["cameras"], c["tf"], c["step"], synth.SHADE_CT, ert=c["ert"], use_skip=True)
    pix = synth.sample_pixels(1, 1024, 1024, 1024, seed=49)
    ref = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"], ert=c["ert"], pixels=pix,
                        shading=synth.SHADE_CT)
    got = img[pix[:, 0], pix[:, 1], pix[:, 2]]
    un, nflag = compare_with_flags(got, ref["rgba"], ref["flags"], c["ert"])
    log(f"lit c1 sampled max unflagged |dRGBA| = {un:.3e}, flagged = {nflag}")
    assert nflag <= 4


def test_invalid_shading_is_rejected():
    vol = upload_volume(_small_ct((16, 16, 16)))
    t = upload_tf(synth.tf1())
    cams = synth.orbit_cameras((16, 16, 16), 1, 50, 60.0, 8, 8)
    for bad, msg in [(dict(shininess=0.5), "shininess"), (dict(grad_min=0.0), "grad_min"),
                     (dict(ambient=-0.1), "ambient"), (dict(headlight=False, light=(0.0, 0.0, 0.0)), "zero length")]:
        sh = vr.Shading(**dict(synth.SHADE_CT, **bad))
        with pytest.raises(vr.VrError, match=msg):
            vr.vr_render(vol, None, cams, t, 0.5, shading=sh)
