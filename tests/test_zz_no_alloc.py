"""The allocation-free render entry point (vr_render_noalloc, through the C
ABI) against vr_render: two calls in a row on one GPU, the second with a
smaller input (the scratch array keeps the first call's contents), each
bit-identical to vr_render and within the oracle's bar on sampled pixels;
sizes beyond the scratch are refused before anything is enqueued."""

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


def _both(vol, blocks, cams, tf, step, ert, skip):
    t = upload_tf(tf)
    W, H = cams[0].width, cams[0].height
    ref = vr.vr_render(vol, blocks, cams, t, step, ert, skip)
    out = torch.full((len(cams), H, W, 4), -7.0, dtype=torch.float32, device=DEV)
    got = vr.vr_render_noalloc(vol, blocks, cams, t, step, ert, skip, out)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_matches_render_on_two_calls_second_smaller():
    c = synth.config_c1()
    log("no-alloc: C1 frame (512x512x400 int16 -> 1024^2, skip + ERT 0.99)")
    v1 = upload_volume(c["volume"])
    b1 = vr.vr_build_blocks(v1, 16)
    got, ref = _both(v1, b1, c["cameras"], c["tf"], c["step"], c["ert"], True)
    assert np.array_equal(got, ref)
    pix = synth.sample_pixels(1, 1024, 1024, 1500, seed=130)
    r = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"], ert=c["ert"], pixels=pix)
    compare_with_flags(got[pix[:, 0], pix[:, 1], pix[:, 2]].astype(np.float64), r["rgba"], r["flags"], c["ert"])
    del v1, b1
    log("no-alloc: second, smaller call (96x80x72 int16, 3 views of 120x104, ragged tiles)")
    vol = synth.ct_phantom_i16(96, 80, 72, seed=131, n_soft=6, n_bone=4)
    v2 = upload_volume(vol)
    b2 = vr.vr_build_blocks(v2, 16)
    cams = synth.orbit_cameras((96, 80, 72), 3, 132, 60.0, 120, 104)
    got, ref = _both(v2, b2, cams, synth.tf1(), 0.5, 0.99, True)
    assert np.array_equal(got, ref)
    r = oracle.render(vol, cams, synth.tf1(), 0.5, ert=0.99)
    compare_with_flags(got.astype(np.float64), r["rgba"], r["flags"], 0.99)
    # and without skipping (no occupancy planes), more views than one launch carries
    cams = synth.orbit_cameras((96, 80, 72), 19, 133, 60.0, 24, 20)
    got, ref = _both(v2, None, cams, synth.tf1(), 0.5, 0.0, False)
    assert np.array_equal(got, ref)
    # two large views in a row: queued launches whose work-queue counters live
    # in the scratch too (each launch's order kernel zeroes them again)
    for seed in (137, 138):
        log(f"no-alloc: queued launch, 1024x768 view (seed {seed})")
        cams = synth.orbit_cameras((96, 80, 72), 1, seed, 60.0, 1024, 768)
        got, ref = _both(v2, b2, cams, synth.tf1(), 0.5, 0.99, True)
        assert np.array_equal(got, ref)
        assert np.all(got[..., 3] >= 0.0)  # every pixel written (the output starts at -7)


def test_noalloc_refuses_sizes_beyond_its_scratch():
    vol = upload_volume(synth.ct_phantom_i16(24, 20, 16, seed=134, n_soft=2, n_bone=1))
    t = upload_tf(synth.tf1())
    big = synth.orbit_cameras((24, 20, 16), 1, 135, 60.0, 8200, 8200)
    out = torch.empty(1, dtype=torch.float32, device=DEV).expand(1)
    with pytest.raises(ValueError):
        vr.vr_render_noalloc(vol, None, big, t, 0.5, 0.0, False, out)
    out = torch.empty((1, 8200, 8200, 4), dtype=torch.float32, device=DEV)
    with pytest.raises(vr.VrError, match="tiles"):
        vr.vr_render_noalloc(vol, None, big, t, 0.5, 0.0, False, out)
    del out
    # 1024 x 1024 x 176 int16 with 4^3 blocks: 2,883,584 blocks > 2,796,192
    huge = upload_volume(np.zeros((176, 1024, 1024), np.int16))
    hb = vr.vr_build_blocks(huge, 4)
    cams = synth.orbit_cameras((1024, 1024, 176), 1, 136, 60.0, 16, 16)
    out = torch.empty((1, 16, 16, 4), dtype=torch.float32, device=DEV)
    with pytest.raises(vr.VrError, match="blocks"):
        vr.vr_render_noalloc(huge, hb, cams, t, 0.5, 0.0, True, out)
    vr.vr_render_noalloc(huge, None, cams, t, 0.5, 0.0, False, out)  # no skipping: no planes needed
    ref = vr.vr_render(huge, None, cams, t, 0.5, 0.0, False)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
