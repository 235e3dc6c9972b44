"""GPU parity of pre-integrated classification (vr_preint_build,
vr_render_preint) against the FP64 oracle.

Bars: the fp32 table within 1e-6 of the oracle's FP64 table (both integrate
to ~1e-10; the rest is fp32 rounding); images within max |dRGBA| <= 2e-4 with
the termination-tie allowance of the other render tests; skipping
bit-identical to rendering every cell.
"""

import math

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

SPIKE_POINTS = [(-1024.0, (0, 0, 0, 0)), (-16.0, (0, 0, 0, 0)), (0.0, (0.8, 0.3, 0.2, 0.01)),
                (96.0, (0.8, 0.3, 0.2, 0.01)), (112.0, (0, 0, 0, 0)), (336.0, (0, 0, 0, 0)),
                (352.0, (1.0, 0.9, 0.8, 0.6)), (368.0, (0, 0, 0, 0)), (3056.0, (0, 0, 0, 0))]


def _spike_tf():
    return synth.tf_from_points(SPIKE_POINTS, 256, -1024.0, 3056.0)


def _preint(vol_np, cams, tf, step, ert=0.0, use_skip=False, vol=None, counters=False, edge=16):
    v = vol if vol is not None else upload_volume(vol_np)
    t = upload_tf(tf)
    table = vr.vr_preint_build(t, step)
    blocks = vr.vr_build_blocks(v, edge) if use_skip else None
    ctr = torch.zeros(4, dtype=torch.int64, device=DEV) if counters else None
    out = vr.vr_render_preint(v, blocks, cams, t, table, step, ert, use_skip, counters=ctr)
    torch.cuda.synchronize()
    img = out.cpu().numpy().astype(np.float64)
    return (img, ctr.cpu().numpy()) if counters else img


def _small_ct(dims=(96, 80, 72), seed=51):
    return synth.ct_phantom_i16(*dims, seed=seed, n_soft=6, n_bone=4)


@pytest.mark.parametrize("which,step", [("tf1", 0.5), ("spike", 2.0), ("tf0", 16.0)])
def test_table_matches_oracle(which, step):
    tf = {"tf1": synth.tf1(), "spike": _spike_tf(), "tf0": synth.tf0()}[which]
    t = upload_tf(tf)
    tab = vr.vr_preint_table(vr.vr_preint_build(t, step)).cpu().numpy().astype(np.float64)
    ref = oracle.preint_table(tf, step)
    d = np.abs(tab - ref).max()
    log(f"table {which} step {step}: max |d| = {d:.3e}")
    assert d <= 1e-6


@pytest.mark.parametrize("tfname", ["tf1", "spike"])
def test_ct_preint_perspective_skip_and_ert_match_oracle(tfname):
    vol = _small_ct()
    dims = (96, 80, 72)
    cams = synth.orbit_cameras(dims, 2, 52, 60.0, 120, 104)
    tf = synth.tf1() if tfname == "tf1" else _spike_tf()
    step = 0.5 if tfname == "tf1" else 1.5
    log(f"preint ct 96x80x72 persp 120x104 x2 skip ert=0.99 {tfname} step {step}")
    img = _preint(vol, cams, tf, step, ert=0.99, use_skip=True)
    ref = oracle.render_preint(vol, cams, tf, step, ert=0.99, minmax=oracle.blocks(vol, 16), edge=16)
    un, nflag = compare_with_flags(img, ref["rgba"], ref["flags"], 0.99)
    log(f"max unflagged |dRGBA| = {un:.3e}, flagged = {nflag}")
    assert nflag <= 1e-3 * img[..., 0].size + 2


def test_preint_skip_is_bit_identical_and_counts_cells():
    vol = _small_ct()
    dims = (96, 80, 72)
    cams = synth.orbit_cameras(dims, 3, 53, 60.0, 96, 96)
    tf = synth.tf1()
    v = upload_volume(vol)
    a, ca = _preint(vol, cams, tf, 0.5, ert=0.99, use_skip=False, vol=v, counters=True)
    b, cb = _preint(vol, cams, tf, 0.5, ert=0.99, use_skip=True, vol=v, counters=True)
    assert np.array_equal(a, b)
    assert cb[0] < ca[0]
    assert ca[1] == cb[1] == oracle.lattice(cams, dims, 0.5).sum()


def test_two_block_cell_is_not_skipped():
    """Air x < 8, tissue x >= 8, blocks of 4, cells [3, 8] along +x: the
    front block alone is empty, the cell is not."""
    vol = np.full((8, 8, 16), -1000, dtype=np.int16)
    vol[:, :, 8:] = 40
    tf = synth.tf1()
    cam = synth.Camera(projection=0, eye=np.array([-1002.0, 3.5, 3.5]), right=np.array([0.0, 1.0, 0.0]),
                       up=np.array([0.0, 0.0, 1.0]), forward=np.array([1.0, 0.0, 0.0]), ortho_w=8.0, ortho_h=8.0,
                       width=8, height=8)
    v = upload_volume(vol)
    a = _preint(vol, [cam], tf, 5.0, use_skip=True, vol=v, edge=4)
    b = _preint(vol, [cam], tf, 5.0, use_skip=False, vol=v, edge=4)
    ref = oracle.render_preint(vol, [cam], tf, 5.0)
    assert np.array_equal(a, b)
    assert np.abs(a - ref["rgba"]).max() <= TOL
    assert a[..., 3].min() > 0.0


@pytest.mark.parametrize("dtype", ["u16_ortho", "f32_global", "u16_odd"])
def test_preint_dtypes_and_global_path(dtype):
    if dtype == "u16_ortho":
        c = synth.config_c0()
        vol, cams, tf, step = c["volume"], c["cameras"], c["tf"], 0.75
    elif dtype == "f32_global":
        vol = synth.density_grid_f32(48, seed=54)
        tf = synth.tf3()
        cams = synth.orbit_cameras((48, 48, 48), 2, 55, 50.0, 12, 10)
        step = 0.5
    else:
        vol = synth.ellipsoid_phantom_u16(48, seed=56)[:, :47, :45].copy()
        tf = synth.tf0()
        cams = synth.orbit_cameras((45, 47, 48), 2, 57, 50.0, 40, 36)
        step = 0.625
    log(f"preint {dtype} step {step}")
    img, ctr = _preint(vol, cams, tf, step, counters=True)
    ref = oracle.render_preint(vol, cams, tf, step)
    d = np.abs(img - ref["rgba"]).max()
    log(f"preint {dtype} max |dRGBA| = {d:.3e}, global-path values {ctr[3]}")
    assert d <= TOL
    if dtype == "f32_global":
        assert ctr[3] > 0


def test_preint_c1_full_size_sampled_pixels():
    c = synth.config_c1()
    log("preint c1: 512x512x400 i16 -> 1024^2, 1024 sampled pixels")
    img = _preint(c["volume"], c["cameras"], c["tf"], c["step"], ert=c["ert"], use_skip=True)
    pix = synth.sample_pixels(1, 1024, 1024, 1024, seed=58)
    ref = oracle.render_preint(c["volume"], c["cameras"], c["tf"], c["step"], ert=c["ert"], pixels=pix)
    got = img[pix[:, 0], pix[:, 1], pix[:, 2]]
    un, nflag = compare_with_flags(got, ref["rgba"], ref["flags"], c["ert"])
    log(f"preint c1 sampled max unflagged |dRGBA| = {un:.3e}, flagged = {nflag}")
    assert nflag <= 4


def _psnr(a, b):
    return 10 * math.log10(1.0 / float(np.mean((a - b) ** 2)))


def test_preint_reduces_step_artefacts_on_the_gpu():
    """Spike TF at a coarse step: the pre-integrated image is closer to a
    fine-step post-classified reference than the post-classified one."""
    vol = _small_ct()
    dims = (96, 80, 72)
    cams = synth.orbit_cameras(dims, 1, 59, 60.0, 96, 96)
    tf = _spike_tf()
    v = upload_volume(vol)
    t = upload_tf(tf)
    ref = vr.vr_render(v, None, cams, t, 1.0 / 16).cpu().numpy().astype(np.float64)
    post = vr.vr_render(v, None, cams, t, 2.0).cpu().numpy().astype(np.float64)
    pre = _preint(vol, cams, tf, 2.0, vol=v)
    p_post, p_pre = _psnr(post, ref), _psnr(pre, ref)
    log(f"step 2: PSNR post {p_post:.2f} dB, pre-integrated {p_pre:.2f} dB")
    assert p_pre > p_post + 4.0


def test_table_for_another_step_or_tf_is_rejected():
    v = upload_volume(_small_ct((16, 16, 16)))
    t = upload_tf(synth.tf1())
    cams = synth.orbit_cameras((16, 16, 16), 1, 60, 60.0, 8, 8)
    tab = vr.vr_preint_build(t, 0.5)
    with pytest.raises(vr.VrError, match="another TF or step"):
        vr.vr_render_preint(v, None, cams, t, tab, 0.25)
    t2 = upload_tf(synth.tf1())
    with pytest.raises(vr.VrError, match="another TF or step"):
        vr.vr_render_preint(v, None, cams, t2, tab, 0.5)
