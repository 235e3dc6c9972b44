"""Out-of-core rendering (vr_bricked_*): volumes kept as host bricks, rendered
through a device brick pool in front-to-back passes.

Bar: bit-identical to the in-core vr_render with skipping and blocks of the
brick edge (same samples, same arithmetic, same order; the ray state crosses
passes in fp32 exactly as it stays in registers), for every pool size down to
a single brick; and within 2e-4 of the FP64 oracle.
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
from gpu_util import compare_with_flags, log, upload_tf, upload_volume  # noqa: E402


def _incore(vol_np, cams, tf, step, ert, edge):
    v = upload_volume(vol_np)
    t = upload_tf(tf)
    b = vr.vr_build_blocks(v, edge)
    out = vr.vr_render(v, b, cams, t, step, ert, True)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _bricked(vol_np, cams, tf, step, ert, edge, pool_bricks):
    slot = (((edge + 4) ** 3 * vol_np.dtype.itemsize + 16 + 255) // 256) * 256
    bv = vr.BrickedVolume(vol_np, edge, pool_bricks * slot)
    t = upload_tf(tf)
    out = bv.render(cams, t, step, ert)
    torch.cuda.synchronize()
    return out.cpu().numpy(), bv


def _small_ct(dims=(96, 80, 72), seed=61):
    return synth.ct_phantom_i16(*dims, seed=seed, n_soft=6, n_bone=4)


@pytest.mark.parametrize("edge,pool", [(16, 1), (16, 7), (32, 3), (32, 1000)])
def test_bricked_is_bit_identical_to_incore(edge, pool):
    vol = _small_ct()
    cams = synth.orbit_cameras((96, 80, 72), 3, 62, 60.0, 100, 84)
    tf = synth.tf1()
    log(f"bricked ct 96x80x72 edge {edge} pool {pool} bricks, 3 views")
    want = _incore(vol, cams, tf, 0.5, 0.99, edge)
    got, bv = _bricked(vol, cams, tf, 0.5, 0.99, edge, pool)
    st = bv.stats()
    log(f"passes {st['passes']}, occupied {st['bricks_occupied']}/{st['bricks_total']}, uploads {st['bricks_uploaded']}")
    assert np.array_equal(got, want)
    if pool < st["bricks_occupied"]:
        assert st["passes"] > 3


def test_bricked_matches_oracle_and_reuses_resident_bricks():
    vol = _small_ct()
    cams = synth.orbit_cameras((96, 80, 72), 1, 63, 60.0, 120, 104)
    tf = synth.tf1()
    got, bv = _bricked(vol, cams, tf, 0.5, 0.99, 16, 4096)
    ref = oracle.render(vol, cams, tf, 0.5, ert=0.99)
    un, nflag = compare_with_flags(got.astype(np.float64), ref["rgba"], ref["flags"], 0.99)
    log(f"bricked vs oracle: max unflagged |dRGBA| = {un:.3e}, flagged {nflag}")
    first = bv.stats()["bricks_uploaded"]
    t = upload_tf(tf)
    again = bv.render(cams, t, 0.5, 0.99).cpu().numpy()
    assert np.array_equal(again, got)
    assert bv.stats()["bricks_uploaded"] == first  # everything stayed resident


@pytest.mark.parametrize("dtype", ["u16_odd", "f32", "eye_inside"])
def test_bricked_dtypes_and_cameras(dtype):
    if dtype == "u16_odd":
        vol = synth.ellipsoid_phantom_u16(48, seed=64)[:, :47, :45].copy()
        tf = synth.tf0()
        dims = (45, 47, 48)
        cams = synth.orbit_cameras(dims, 2, 65, 50.0, 40, 36)
    elif dtype == "f32":
        vol = synth.density_grid_f32(48, seed=66)
        tf = synth.tf3()
        dims = (48, 48, 48)
        cams = synth.orbit_cameras(dims, 2, 67, 50.0, 40, 36)
    else:
        vol = _small_ct()
        tf = synth.tf1()
        dims = (96, 80, 72)
        c = synth.orbit_camera(dims, np.array([0.3, -0.2, 0.93]), 100.0, 64, 48)
        c.eye = np.array([40.3, 37.7, 30.1])
        cams = [c]
    want = _incore(vol, cams, tf, 0.5, 0.99, 16)
    got, bv = _bricked(vol, cams, tf, 0.5, 0.99, 16, 5)
    log(f"bricked {dtype}: passes {bv.stats()['passes']}")
    assert np.array_equal(got, want)


def test_bricked_c1_full_size_bit_identical():
    """The 512x512x400 frame through a 64 MiB pool (a fraction of the
    occupied bricks per pass)."""
    c = synth.config_c1()
    log("bricked c1 512x512x400 edge 64, pool 64 MiB")
    want = _incore(c["volume"], c["cameras"], c["tf"], c["step"], c["ert"], 64)
    slot = ((68 ** 3 * 2 + 16 + 255) // 256) * 256
    got, bv = _bricked(c["volume"], c["cameras"], c["tf"], c["step"], c["ert"], 64, (64 << 20) // slot)
    st = bv.stats()
    log(f"c1 bricked: passes {st['passes']}, occupied {st['bricks_occupied']}/{st['bricks_total']}, "
        f"uploaded {st['bytes_uploaded'] / 2**20:.1f} MiB")
    assert st["passes"] >= 2
    assert np.array_equal(got, want)


def test_bricked_validation():
    vol = _small_ct((16, 16, 16))
    with pytest.raises(vr.VrError, match="holds no brick"):
        vr.BrickedVolume(vol, 16, 1000)
    with pytest.raises(vr.VrError, match="power of two"):
        vr.BrickedVolume(vol, 12, 1 << 24)
