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

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2005_01442_amd as vr  # noqa: E402
from gpu_util import DEV, compare_with_flags, log, upload_tf, upload_volume  # noqa: E402


def _resident_bytes(dims, edge=16, esize=2):
    """Device bytes a served volume is charged: its voxels, its blocks (plain
    and widened ranges, 16 B per block)."""
    nb = 1
    for d in dims:
        nb *= -(-d // edge)
    return dims[0] * dims[1] * dims[2] * esize + 16 * nb


def _occupancy_bytes(dims, edge=16):
    nb = 1
    for d in dims:
        nb *= -(-d // edge)
    return ((nb + 31) // 32 + (nb + 15) // 16) * 4


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
    # room for the volume, one 64^2 request and a little more
    res = _resident_bytes(dv[0].dims) + _occupancy_bytes(dv[0].dims)
    srv = vr.Server(hbm_budget_bytes=res + img_bytes + 8 * 1024, max_inflight=4)
    vid = srv.add_volume(dv[0])
    assert srv.stats()["resident_bytes"] == _resident_bytes(dv[0].dims)
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
    vid = srv.add_volume(dv[0])  # registered again after its removal
    cam1 = synth.orbit_camera(dv[0].dims, np.array([0.3, 0.4, 0.8]), 60.0, 64, 64)
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
    nan = tf.table.copy()
    nan[3, 1] = np.nan
    with pytest.raises(vr.VrError, match="not finite"):
        srv.submit(vid, cam, nan, tf.v0, tf.v1, 0.5)
    srv.close()


def test_budget_counts_volumes_and_never_blocks_the_queue():
    """A 512x512x800 volume is charged to the budget with its blocks: a
    budget of one 1024^2 image plus a margin cannot hold it (VR_E_BUDGET at
    registration, not a time-out later); with room for the volume and one
    request a second request waits for the first's release; a request that
    can never fit next to the volume fails at submit; and a queued request
    that stops fitting because another volume was registered meanwhile
    completes with VR_E_BUDGET instead of blocking the requests behind it."""
    dims = (512, 512, 800)
    vol = synth.ct_phantom_i16(*dims, seed=64, n_soft=6, n_bone=4)
    dvol = upload_volume(vol)
    small = upload_volume(synth.ct_phantom_i16(48, 40, 32, seed=65, n_soft=3, n_bone=2))
    tf = synth.tf1()
    img = 1024 * 1024 * 16
    srv = vr.Server(hbm_budget_bytes=img + (1 << 20), max_inflight=4)
    with pytest.raises(vr.VrError, match="VR_E_BUDGET"):
        srv.add_volume(dvol)
    srv.close()
    need = _resident_bytes(dims) + _occupancy_bytes(dims) + img
    srv = vr.Server(hbm_budget_bytes=need + (64 << 10), max_inflight=4)
    vid = srv.add_volume(dvol)
    cam = synth.orbit_camera(dims, np.array([0.2, -0.5, 0.8]), 60.0, 1024, 1024)
    a = srv.submit(vid, cam, tf.table, tf.v0, tf.v1, 0.5, 0.99, True)
    srv.wait(a)
    b = srv.submit(vid, cam, tf.table, tf.v0, tf.v1, 0.5, 0.99, True)
    with pytest.raises(vr.VrError, match="VR_E_TIMEOUT"):
        srv.wait(b, timeout_us=20000)
    srv.release(a)
    srv.wait(b)
    srv.release(b)
    big = synth.orbit_camera(dims, np.array([0.2, -0.5, 0.8]), 60.0, 1100, 1024)
    with pytest.raises(vr.VrError, match="VR_E_BUDGET"):
        srv.submit(vid, big, tf.table, tf.v0, tf.v1, 0.5, 0.99, True)
    # c (256^2) holds image memory, so d (1024^2) queues; registering a small
    # volume then leaves d no room at all (it needed the whole margin); e,
    # queued behind d, must still complete
    cam_c = synth.orbit_camera(dims, np.array([0.2, -0.5, 0.8]), 60.0, 256, 256)
    c = srv.submit(vid, cam_c, tf.table, tf.v0, tf.v1, 0.5, 0.99, True)
    srv.wait(c)
    d = srv.submit(vid, cam, tf.table, tf.v0, tf.v1, 0.5, 0.99, True)
    with pytest.raises(vr.VrError, match="VR_E_TIMEOUT"):
        srv.wait(d, timeout_us=20000)
    sid = srv.add_volume(small)
    cam_s = synth.orbit_camera(small.dims, np.array([0.3, 0.4, 0.8]), 60.0, 16, 16)
    e = srv.submit(sid, cam_s, tf.table, tf.v0, tf.v1, 0.5, 0.99, True)
    with pytest.raises(vr.VrError, match="VR_E_BUDGET"):
        srv.wait(d, timeout_us=30_000_000)
    srv.release(d)
    srv.wait(e, timeout_us=30_000_000)
    srv.release(e)
    srv.release(c)
    st = srv.stats()
    assert st["hbm_peak"] <= need + (64 << 10)
    srv.close()


def test_c4_mix_matches_alone_renders_and_the_oracle():
    """The serving configuration's volumes (8 C4 phantoms, 128^3 up to
    452x496x688 int16, all resident) with 24 requests of the C4 stream
    (random volume, 256^2 / 512^2 / 1024^2, random orbit pose, TF1, step 0.5,
    early termination at 0.99, skipping) submitted at once so that they share
    launches: every served image equals vr_render of the same request alone
    (bit-identical), and 300 sampled hit pixels of each equal the FP64 oracle
    (2e-4; early-termination ties by the flag rule)."""
    dims = synth.config_c4_volumes(seed=10, count=8)
    host = [synth.ct_phantom_i16(*d, seed=sd) for d, sd in dims]
    dev = [upload_volume(v) for v in host]
    blocks = [vr.vr_build_blocks(v, 16) for v in dev]
    tf = synth.tf1()
    t_dev = upload_tf(tf)
    srv = vr.Server(hbm_budget_bytes=4 << 30, max_inflight=32)
    ids = [srv.add_volume(v) for v in dev]
    reqs = synth.c4_arrivals(24, seed=11, n_volumes=8, dims_list=[d for d, _ in dims])
    log(f"c4 mix: {len(reqs)} requests, sizes {sorted(set(r['size'] for r in reqs))}")
    tickets = [srv.submit(ids[r["volume"]], r["camera"], tf.table, tf.v0, tf.v1, 0.5, 0.99, True) for r in reqs]
    worst, flagged = 0.0, 0
    for q, (t, r) in enumerate(zip(tickets, reqs)):
        cam = r["camera"]
        got = srv.result(t, cam.height, cam.width).cpu().numpy()
        vi = r["volume"]
        alone = vr.vr_render(dev[vi], blocks[vi], [cam], t_dev, 0.5, 0.99, True)[0].cpu().numpy()
        assert np.array_equal(got, alone), (q, vi, cam.width)
        lat = oracle.lattice([cam], dims[vi][0], 0.5)
        pix = synth.sample_pixels(1, cam.width, cam.height, 3000, seed=200 + q)
        pix = pix[lat[0, pix[:, 1], pix[:, 2]] > 0][:300]
        ref = oracle.render(host[vi], [cam], tf, 0.5, ert=0.99, pixels=pix)
        un, nf = compare_with_flags(got[pix[:, 1], pix[:, 2]].astype(np.float64), ref["rgba"], ref["flags"], 0.99)
        worst, flagged = max(worst, un), flagged + nf
    st = srv.stats()
    log(f"c4 mix: max unflagged |dRGBA| vs oracle {worst:.3e}, flagged {flagged}; launches {st['launches']}, "
        f"samples {st['samples']}")
    assert st["completed"] == len(reqs) and st["launches"] >= 2 and st["samples"] > 0
    srv.close()


def test_out_of_core_volumes_served_in_the_mix():
    """Volumes larger than the HBM budget served through the shared brick
    pool: a 256x256x512 int16 host volume (64 MiB) and a 200x180x300 one
    (21 MiB) with a 96 MiB budget and a 24 MiB brick pool (64^3 bricks), next
    to a resident in-core volume; requests on all three submitted at once.
    Every out-of-core image equals vr_render of the same volume in core with
    16^3 skip blocks (bit-identical) and the FP64 oracle on sampled pixels;
    the in-core ones equal their alone renders; the pool is charged once."""
    big = synth.ct_phantom_i16(256, 256, 512, seed=66, n_soft=8, n_bone=5)
    mid = synth.ct_phantom_i16(200, 180, 300, seed=67, n_soft=6, n_bone=4)
    inc = synth.ct_phantom_i16(96, 96, 80, seed=68, n_soft=5, n_bone=4)
    tf = synth.tf1()
    srv = vr.Server(hbm_budget_bytes=96 << 20, max_inflight=8, brick_pool_bytes=24 << 20)
    dinc = upload_volume(inc)
    vid_inc = srv.add_volume(dinc)
    vid_big = srv.add_host_volume(big, 64)
    vid_mid = srv.add_host_volume(mid, 64)
    st = srv.stats()
    assert st["hbm_used"] <= 96 << 20 and st["resident_bytes"] >= 24 << 20
    rng = np.random.default_rng(69)
    reqs = []
    for i in range(12):
        vid, host = [(vid_big, big), (vid_mid, mid), (vid_inc, inc)][i % 3]
        dims = host.shape[::-1]
        W = [48, 96, 130][i % 3]
        cam = synth.orbit_camera(dims, rng.standard_normal(3), 60.0, W, W - 8)
        t = srv.submit(vid, cam, tf.table, tf.v0, tf.v1, 0.5, 0.99 if i % 2 else 0.0, True)
        reqs.append((t, host, cam, 0.99 if i % 2 else 0.0))
    t_dev = upload_tf(tf)
    for q, (t, host, cam, ert) in enumerate(reqs):
        got = srv.result(t, cam.height, cam.width).cpu().numpy()
        dv = upload_volume(host)
        alone = vr.vr_render(dv, vr.vr_build_blocks(dv, 16), [cam], t_dev, 0.5, ert, True)[0].cpu().numpy()
        assert np.array_equal(got, alone), (q, host.shape)
        del dv
        pix = synth.sample_pixels(1, cam.width, cam.height, 150, seed=300 + q)
        ref = oracle.render(host, [cam], tf, 0.5, ert=ert, pixels=pix)
        compare_with_flags(got[pix[:, 1], pix[:, 2]].astype(np.float64), ref["rgba"], ref["flags"],
                           ert if ert else 1.0)
    st = srv.stats()
    log(f"out-of-core serving: {st['completed']} completed, hbm peak {st['hbm_peak'] / 2**20:.1f} MiB")
    assert st["completed"] == 12 and st["hbm_peak"] <= 96 << 20
    srv.remove_volume(vid_big)
    srv.close()
    plain = vr.Server(hbm_budget_bytes=64 << 20)
    with pytest.raises(vr.VrError, match="brick pool"):
        plain.add_host_volume(mid, 64)
    plain.close()
