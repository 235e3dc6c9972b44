"""Serving loop on the GPU (through the C ABI): a mix of requests of several
volumes, image sizes and TFs, batched into shared launches, must give every
request the image it gets alone from vr_render (bit-identical); admission,
budget, busy-volume, timeout and shutdown paths behave as documented."""

import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import synth  # noqa: E402
import paper_2005_01442_amd as vr  # noqa: E402
from gpu_util import DEV, log, upload_tf, upload_volume  # noqa: E402


def _volumes():
    vols = [
        synth.ct_phantom_i16(64, 48, 40, seed=60, n_soft=4, n_bone=3),
        synth.ct_phantom_i16(37, 53, 29, seed=61, n_soft=3, n_bone=2),
        synth.ct_phantom_i16(96, 96, 80, seed=62, n_soft=5, n_bone=4),
    ]
    return vols, [upload_volume(v) for v in vols]


def test_mixed_requests_equal_alone_renders():
    vols, dv = _volumes()
    tf1 = synth.tf1()
    tf_b = synth.tf_from_points([(-1024, (0, 0, 0, 0)), (-100, (0.2, 0.3, 0.9, 0.0)), (200, (0.9, 0.4, 0.2, 0.05)),
                                 (3056, (1, 1, 1, 0.3))], 128, -1024.0, 3056.0)
    srv = vr.Server(hbm_budget_bytes=256 << 20, max_inflight=6, max_batch_tiles=48)
    ids = [srv.add_volume(v) for v in dv]
    rng = np.random.default_rng(63)
    reqs = []
    for i in range(24):
        vid = int(rng.integers(0, 3))
        nx, ny, nz = dv[vid].dims
        W, H = [(16, 16), (40, 24), (64, 64), (96, 72), (7, 5)][int(rng.integers(0, 5))]
        cam = synth.orbit_camera((nx, ny, nz), rng.standard_normal(3), 60.0, W, H)
        tf = tf1 if i % 2 == 0 else tf_b
        ert = 0.99 if i % 3 else 0.0
        skip = bool(i % 4)
        t = srv.submit(ids[vid], cam, tf.table, tf.v0, tf.v1, 0.5, ert, skip)
        reqs.append((t, vid, cam, tf, ert, skip))
    for t, vid, cam, tf, ert, skip in reqs:
        got = srv.result(t, cam.height, cam.width).cpu().numpy()
        blocks = vr.vr_build_blocks(dv[vid]) if skip else None
        alone = vr.vr_render(dv[vid], blocks, [cam], upload_tf(tf), 0.5, ert, skip)[0].cpu().numpy()
        assert np.array_equal(got, alone), (t, vid, cam.width, cam.height)
    st = srv.stats()
    log(f"serve stats: {st}")
    assert st["completed"] == 24 and st["launches"] >= 2
    assert st["p99_ms"] >= st["p50_ms"] > 0
    srv.close()


def test_admission_errors_timeout_busy_and_shutdown():
    vols, dv = _volumes()
    tf = synth.tf1()
    img_bytes = 64 * 64 * 16
    srv = vr.Server(hbm_budget_bytes=img_bytes + 64 * 1024, max_inflight=4)
    vid = srv.add_volume(dv[0])
    cam = synth.orbit_camera(dv[0].dims, np.array([0.3, 0.4, 0.8]), 60.0, 64, 64)
    with pytest.raises(vr.VrError, match="VR_E_NOT_FOUND"):
        srv.submit(vid + 7, cam, tf.table, tf.v0, tf.v1, 0.5)
    big = synth.orbit_camera(dv[0].dims, np.array([0.3, 0.4, 0.8]), 60.0, 512, 512)
    with pytest.raises(vr.VrError, match="VR_E_BUDGET"):
        srv.submit(vid, big, tf.table, tf.v0, tf.v1, 0.5)
    a = srv.submit(vid, cam, tf.table, tf.v0, tf.v1, 0.5)
    srv.wait(a)  # A now holds the only image the budget allows
    b = srv.submit(vid, cam, tf.table, tf.v0, tf.v1, 0.5)
    with pytest.raises(vr.VrError, match="VR_E_TIMEOUT"):
        srv.wait(b, timeout_us=2000)
    with pytest.raises(vr.VrError, match="VR_E_BUSY"):
        srv.remove_volume(vid)
    srv.release(a)  # frees the image: B is admitted and completes
    srv.wait(b)
    srv.release(b)
    srv.remove_volume(vid)
    vid = srv.add_volume(dv[1])
    cam1 = synth.orbit_camera(dv[1].dims, np.array([0.3, 0.4, 0.8]), 60.0, 64, 64)
    c = srv.submit(vid, cam1, tf.table, tf.v0, tf.v1, 0.5)
    srv.wait(c)  # holds the budget
    d = srv.submit(vid, cam1, tf.table, tf.v0, tf.v1, 0.5)  # queued behind the budget
    result = {}

    def waiter():
        try:
            srv.wait(d)
            result["status"] = "ok"
        except vr.VrError as e:
            result["status"] = e.status_name

    th = threading.Thread(target=waiter)
    th.start()
    srv.close()
    th.join(timeout=30)
    assert result.get("status") == "VR_E_SHUTDOWN"


def test_request_validation():
    vols, dv = _volumes()
    tf = synth.tf1()
    srv = vr.Server(hbm_budget_bytes=64 << 20, max_inflight=2)
    vid = srv.add_volume(dv[0])
    cam = synth.orbit_camera(dv[0].dims, np.array([0.3, 0.4, 0.8]), 60.0, 16, 16)
    neg = tf.table.copy()
    neg[10, 3] = -1.0
    with pytest.raises(vr.VrError, match="negative extinction"):
        srv.submit(vid, cam, neg, tf.v0, tf.v1, 0.5)
    with pytest.raises(vr.VrError, match="step"):
        srv.submit(vid, cam, tf.table, tf.v0, tf.v1, -1.0)
    srv.close()
