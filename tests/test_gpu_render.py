"""GPU forward parity: the HIP ray caster (through the C ABI) against the FP64
oracle, element by element, on seeded inputs.

Bar: max |dRGBA| <= 2e-4 (fp32 kernel vs fp64 oracle); pixels where the oracle
sees an early-termination tie (|1 - T - theta| < 1e-5) may differ by up to
1 - theta more.  Integer results (block min/max, occupancy, lattice counts)
must match exactly; skip vs no-skip must be bit-identical.
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
from gpu_util import DEV, compare_with_flags, gpu_render, log, upload_tf, upload_volume  # noqa: E402

TOL = 2e-4


def test_c0_full_frame_matches_oracle():
    c = synth.config_c0()
    log("c0: 64^3 u16 ortho 256^2")
    img, ctr = gpu_render(c["volume"], c["cameras"], c["tf"], c["step"], counters=True)
    ref = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"])
    d = np.abs(img - ref["rgba"]).max()
    log(f"c0 max |dRGBA| = {d:.3e}")
    assert d <= TOL
    assert ctr[1] == ref["counts"][..., 0].sum() == 65536 * 128
    assert ctr[0] == ctr[1]
    assert ctr[2] == 65536


def _small_ct(dims=(96, 80, 72), seed=31):
    return synth.ct_phantom_i16(*dims, seed=seed, n_soft=6, n_bone=4)


@pytest.mark.parametrize("ert", [0.0, 0.99])
def test_ct_perspective_skip_and_ert_match_oracle(ert):
    vol = _small_ct()
    dims = (96, 80, 72)
    cams = synth.orbit_cameras(dims, 3, 32, 60.0, 120, 104)  # ragged: not a multiple of 16
    tf = synth.tf1()
    log(f"ct 96x80x72 persp 120x104 x3 skip ert={ert}")
    img = gpu_render(vol, cams, tf, 0.5, ert=ert, use_skip=True)
    ref = oracle.render(vol, cams, tf, 0.5, ert=ert)
    un, nflag = compare_with_flags(img, ref["rgba"], ref["flags"], ert if ert else 1.0)
    log(f"max unflagged |dRGBA| = {un:.3e}, flagged = {nflag}")
    assert nflag <= 1e-3 * img[..., 0].size + 2


def test_skip_is_bit_identical_to_no_skip():
    vol = _small_ct()
    cams = synth.orbit_cameras((96, 80, 72), 4, 33, 60.0, 96, 96)
    tf = synth.tf1()
    v = upload_volume(vol)
    a, ca = gpu_render(vol, cams, tf, 0.5, ert=0.99, use_skip=False, counters=True, vol=v)
    b, cb = gpu_render(vol, cams, tf, 0.5, ert=0.99, use_skip=True, counters=True, vol=v)
    assert np.array_equal(a, b)
    assert cb[0] < ca[0]  # skipping evaluated fewer samples
    assert ca[1] == cb[1]


def test_lattice_counts_match_oracle_exactly():
    dims = (96, 80, 72)
    cams = synth.orbit_cameras(dims, 5, 34, 60.0, 64, 48) + [synth.ortho_axis_camera(96, 64, 48)]
    vol = _small_ct()
    tf = synth.tf1()
    for step in (0.5, 0.3, 1.7):
        _, ctr = gpu_render(vol, cams, tf, step, counters=True)
        want = oracle.lattice(cams, dims, step)
        assert ctr[1] == want.sum(), (step, ctr[1], want.sum())
        assert ctr[2] == (want > 0).sum()


@pytest.mark.parametrize("dtype", ["u16", "i16", "f32"])
def test_dtypes_and_odd_row_lengths(dtype):
    """Odd nx exercises the unaligned packed-row path; all dtypes."""
    rng = np.random.default_rng(35)
    dims = (37, 29, 23)
    base = synth.ct_phantom_i16(*dims, seed=36, n_soft=3, n_bone=2)
    if dtype == "u16":
        vol = (base.astype(np.int32) + 1024).clip(0, 4095).astype(np.uint16)
        tf = synth.tf_from_points([(v + 1024, c) for v, c in synth.TF1_POINTS], 256, 0.0, 4080.0)
    elif dtype == "i16":
        vol = base
        tf = synth.tf1()
    else:
        vol = (base.astype(np.float32) + rng.standard_normal(base.shape).astype(np.float32))
        tf = synth.tf1()
    cams = synth.orbit_cameras(dims, 2, 37, 55.0, 40, 33)
    cams.append(synth.Camera(0, np.array([18.0, 14.0, -50.0]), np.array([0.8, 0.6, 0.0]),
                             np.array([-0.6, 0.8, 0.0]), np.array([0.0, 0.0, 1.0]), ortho_w=50.0, ortho_h=41.0,
                             width=40, height=33))
    img = gpu_render(vol, cams, tf, 0.4, use_skip=True)
    ref = oracle.render(vol, cams, tf, 0.4)
    d = np.abs(img - ref["rgba"]).max()
    log(f"{dtype}: max |dRGBA| = {d:.3e}")
    assert d <= TOL


def test_blocks_and_occupancy_exact():
    """Block min/max of every dtype, edges 4..64, rows of any length: the
    16-byte-load path (edge 16, x a multiple of 8: 96, 24 whose last block is
    half, 64) and the general one, integer-exact against the oracle."""
    rng = np.random.default_rng(37)
    for dims in ((24, 33, 17), (64, 40, 24), (37, 29, 23), (136, 20, 18)):
        base = synth.ct_phantom_i16(*dims, seed=39, n_soft=3, n_bone=2)
        for vol in (base, (base.astype(np.int32) + 1024).clip(0, 4095).astype(np.uint16),
                    base.astype(np.float32) + rng.standard_normal(base.shape).astype(np.float32)):
            v = upload_volume(vol)
            for edge in (4, 8, 16, 32, 64):
                mm = vr.vr_blocks_minmax(vr.vr_build_blocks(v, edge)).cpu().numpy().astype(np.float64)
                assert np.array_equal(mm, oracle.blocks(vol, edge)), (dims, vol.dtype, edge)
    for dims, edge in (((96, 80, 72), 16), ((37, 29, 23), 8), ((50, 17, 33), 16)):
        vol = synth.ct_phantom_i16(*dims, seed=38, n_soft=4, n_bone=3)
        v = upload_volume(vol)
        b = vr.vr_build_blocks(v, edge)
        mm = vr.vr_blocks_minmax(b).cpu().numpy().astype(np.float64)
        want = oracle.blocks(vol, edge)
        assert np.array_equal(mm, want)
        for tf in (synth.tf1(), synth.tf_from_points([(-1024, (0, 0, 0, 0)), (-900, (1, 1, 1, 0.1)),
                                                     (0, (1, 1, 1, 0.0)), (3056, (1, 1, 1, 0.0))],
                                                    64, -1024.0, 3056.0)):
            occ = vr.vr_block_occupancy(b, upload_tf(tf)).cpu().numpy()
            assert np.array_equal(occ, oracle.occupancy(want, tf))


def test_blocks_streamed_in_z_exact():
    """Grids with at least 1024 (row of blocks, four blocks in z) items take the
    16-bit kernel that streams four blocks in z per workgroup, each footprint
    row read once and added to the one or two blocks holding it: integer-exact
    against the oracle, with a last chunk of three blocks and a last block of
    half height (nz = 1000) and a partial last block in x (nx = 24)."""
    rng = np.random.default_rng(41)
    for dims in ((24, 1040, 1000), (32, 1024, 1024)):
        nx, ny, nz = dims
        base = rng.integers(-1024, 3000, size=(nz, ny, nx)).astype(np.int16)
        # smooth structure plus a few extreme voxels on block boundaries in z
        for z in (15, 16, 17, 31, 32, 33, 991, 999):
            if z < nz:
                base[z, rng.integers(0, ny, 8), rng.integers(0, nx, 8)] = (-32768 if z % 2 else 32767)
        for vol in (base, (base.astype(np.int32) + 32768).astype(np.uint16)):
            log(f"streamed block min/max {dims} {vol.dtype}")
            v = upload_volume(vol)
            mm = vr.vr_blocks_minmax(vr.vr_build_blocks(v, 16)).cpu().numpy().astype(np.float64)
            assert np.array_equal(mm, oracle.blocks(vol, 16)), (dims, vol.dtype)


def test_camera_inside_volume_and_misses():
    vol = _small_ct()
    dims = (96, 80, 72)
    tf = synth.tf1()
    inside = synth.Camera(1, np.array([48.0, 40.0, 30.0]), np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]),
                          np.array([0.0, 0.0, 1.0]), fov_y=np.deg2rad(90.0), width=48, height=40)
    away = synth.Camera(1, np.array([48.0, 40.0, -30.0]), np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]),
                        np.array([0.0, 0.0, -1.0]), fov_y=np.deg2rad(40.0), width=48, height=40)
    for cam in (inside, away):
        img = gpu_render(vol, [cam], tf, 0.5, ert=0.99, use_skip=True)
        ref = oracle.render(vol, [cam], tf, 0.5, ert=0.99)
        compare_with_flags(img, ref["rgba"], ref["flags"], 0.99)
    assert np.all(gpu_render(vol, [away], tf, 0.5) == 0.0)


def test_tiny_volumes_and_single_pixel():
    tf = synth.tf1()
    for dims in ((1, 1, 1), (2, 3, 4), (5, 1, 7)):
        vol = np.arange(np.prod(dims), dtype=np.int16).reshape(dims[::-1]) * 200 - 100
        cams = synth.orbit_cameras(dims, 2, 39, 70.0, 17, 9) + synth.orbit_cameras(dims, 1, 40, 10.0, 1, 1)
        for cam_set in (cams[:2], cams[2:]):
            img = gpu_render(vol, cam_set, tf, 0.25, use_skip=True, block_edge=4)
            ref = oracle.render(vol, cam_set, tf, 0.25)
            assert np.abs(img - ref["rgba"]).max() <= TOL


def test_many_views_span_launches():
    """More views than one launch carries (16) and a view count not a
    multiple of it."""
    vol = _small_ct((48, 40, 36), 41)
    dims = (48, 40, 36)
    cams = synth.orbit_cameras(dims, 19, 42, 60.0, 24, 20)
    tf = synth.tf1()
    img = gpu_render(vol, cams, tf, 0.5, ert=0.95, use_skip=True)
    ref = oracle.render(vol, cams, tf, 0.5, ert=0.95)
    compare_with_flags(img, ref["rgba"], ref["flags"], 0.95)


def test_invalid_arguments_raise_and_enqueue_nothing():
    vol = upload_volume(_small_ct((16, 16, 16), 43))
    t = upload_tf(synth.tf1())
    cam = synth.orbit_cameras((16, 16, 16), 1, 44, 60.0, 8, 8)[0]
    with pytest.raises(vr.VrError, match="VR_E_INVALID_ARG"):
        vr.vr_render(vol, None, [cam], t, 0.0)
    with pytest.raises(vr.VrError, match="VR_E_INVALID_ARG"):
        vr.vr_render(vol, None, [cam], t, 0.5, use_skip=True)  # skip without blocks
    other = vr.vr_build_blocks(upload_volume(_small_ct((16, 16, 16), 45)))
    with pytest.raises(vr.VrError, match="another volume"):
        vr.vr_render(vol, other, [cam], t, 0.5, use_skip=True)
    bad = synth.Camera(1, np.array([np.nan, 0, 0]), cam.right, cam.up, cam.forward, fov_y=1.0, width=8, height=8)
    with pytest.raises(vr.VrError, match="finite"):
        vr.vr_render(vol, None, [bad], t, 0.5)
    t_bad = vr.TF(t.table, 5.0, 5.0)
    with pytest.raises(vr.VrError, match="v1 > v0"):
        vr.vr_render(vol, None, [cam], t_bad, 0.5)


def test_c1_full_frame_counts_and_invariants():
    """The metric configuration at full size (512x512x400 int16 -> 1024^2,
    skip, ERT 0.99) in the launch configuration the benchmark times: every
    pixel against the oracle, lattice counts of every pixel exactly, the
    kernel's evaluated-sample counter (the benchmark's numerator) against the
    oracle's count with the same block skipping, skip and ERT invariants over
    the whole frame."""
    c = synth.config_c1()
    log("c1: building full-size inputs")
    v = upload_volume(c["volume"])
    blocks = vr.vr_build_blocks(v, 16)
    fb0 = vr.fallback_counts()
    img, ctr = gpu_render(None, c["cameras"], c["tf"], c["step"], ert=c["ert"], use_skip=True, counters=True,
                          vol=v, blocks=blocks)
    # the timed path: occupancy planes and workgroup order were built (no fallback)
    assert vr.fallback_counts() == fb0
    noskip = gpu_render(None, c["cameras"], c["tf"], c["step"], ert=c["ert"], use_skip=False, vol=v)
    assert np.array_equal(img, noskip)
    noert = gpu_render(None, c["cameras"], c["tf"], c["step"], ert=0.0, use_skip=True, vol=v, blocks=blocks)
    assert np.abs(noert - img).max() <= (1 - c["ert"]) + 1e-6
    lat = oracle.lattice(c["cameras"], (512, 512, 400), c["step"])
    assert ctr[1] == lat.sum()
    assert ctr[2] == (lat > 0).sum()
    log(f"c1 evaluated={ctr[0]} lattice={ctr[1]} hit={ctr[2]}")
    occ = oracle.occupancy(oracle.blocks(c["volume"], 16), c["tf"])
    ref = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"], ert=c["ert"], occ=occ)
    un, nflag = compare_with_flags(img, ref["rgba"], ref["flags"], c["ert"])
    fl = ref["flags"].astype(bool)
    moved = int((np.abs(img - ref["rgba"]).max(axis=-1)[fl] > TOL).sum())
    log(f"c1 full frame (1024^2): max unflagged |dRGBA| = {un:.3e}, flagged = {nflag}, of which {moved} "
        f"terminated at another sample")
    # the flag window (1e-5 of opacity) is as wide as a soft-tissue step's
    # opacity increment near the threshold (T sigma step = 0.01 x 0.004 x 0.5),
    # so most rays ending in soft tissue are flagged; few actually differ
    assert nflag <= 1e-2 * 1024 * 1024 and moved <= 1e-4 * 1024 * 1024
    # evaluated samples: equal up to the samples of rays whose fp32 and FP64
    # positions fall on different sides of a block face between an occupied
    # and an empty block, and of termination ties (a handful per frame)
    want = int(ref["counts"][..., 1].sum())
    log(f"c1 evaluated samples: kernel {ctr[0]}, oracle {want}, difference {int(ctr[0]) - want} "
        f"({(int(ctr[0]) - want) / want:.2e} relative)")
    assert abs(int(ctr[0]) - want) <= 1e-5 * want
    # the image is not trivially empty or saturated
    assert 0.05 < (img[..., 3] > 0.5).mean() < 0.95


def test_c2_full_size_sampled_pixels():
    """The large configuration (1024^3 int16, 2 GiB, to 2048^2, step 0.25,
    skip, ERT 0.99) in the launch configuration of a full frame: sampled hit
    pixels against the oracle, every pixel's lattice count exactly, skip vs
    no-skip bit-identical over the frame."""
    c = synth.config_c2()
    log("c2: 1024^3 int16 -> 2048^2")
    v = upload_volume(c["volume"])
    blocks = vr.vr_build_blocks(v, 16)
    img, ctr = gpu_render(None, c["cameras"], c["tf"], c["step"], ert=c["ert"], use_skip=True, counters=True,
                          vol=v, blocks=blocks)
    noskip = gpu_render(None, c["cameras"], c["tf"], c["step"], ert=c["ert"], use_skip=False, vol=v)
    assert np.array_equal(img, noskip)
    lat = oracle.lattice(c["cameras"], (1024, 1024, 1024), c["step"])
    assert ctr[1] == lat.sum() and ctr[2] == (lat > 0).sum()
    log(f"c2 evaluated={ctr[0]} lattice={ctr[1]} hit={ctr[2]}")
    pix = synth.sample_pixels(1, 2048, 2048, 4000, seed=47)
    hit_rows = pix[lat[0, pix[:, 1], pix[:, 2]] > 0][:2000]
    ref = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"], ert=c["ert"], pixels=hit_rows)
    got = img[hit_rows[:, 0], hit_rows[:, 1], hit_rows[:, 2]]
    un, nflag = compare_with_flags(got, ref["rgba"], ref["flags"], c["ert"])
    log(f"c2 sampled {len(hit_rows)} hit pixels: max unflagged |dRGBA| = {un:.3e}, flagged = {nflag}")


def test_degenerate_transfer_functions_and_parameters():
    """All-transparent TF (every block empty: the march leaps through the whole
    volume and the image is exactly zero), near-opaque TF with ERT, the
    smallest (K = 2) and largest (K = 1024) tables, a step longer than the
    volume, an ERT threshold just above zero, a camera on a box face."""
    vol = _small_ct((40, 36, 32), 48)
    dims = (40, 36, 32)
    cams = synth.orbit_cameras(dims, 2, 49, 60.0, 32, 24)
    empty = synth.tf_from_points([(-1024, (1, 1, 1, 0)), (3056, (1, 1, 1, 0))], 256, -1024.0, 3056.0)
    img, ctr = gpu_render(vol, cams, empty, 0.5, ert=0.99, use_skip=True, counters=True)
    assert np.all(img == 0.0) and ctr[0] == 0 and ctr[1] > 0
    opaque = synth.tf_from_points([(-1024, (0.2, 0.3, 0.4, 50.0)), (3056, (0.9, 0.1, 0.5, 50.0))], 16,
                                  -1024.0, 3056.0)
    k2 = synth.tf_from_points([(-1024, (0, 0, 0, 0)), (3056, (1, 0.5, 0.25, 0.02))], 2, -1024.0, 3056.0)
    k1024 = synth.tf_from_points(synth.TF1_POINTS, 1024, -1024.0, 3056.0)
    face = synth.Camera(1, np.array([19.5, 17.5, -0.5]), np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]),
                        np.array([0.0, 0.0, 1.0]), fov_y=np.deg2rad(70.0), width=32, height=24)
    cases = [
        (opaque, cams, 0.5, 0.99),
        (k2, cams, 0.5, 0.0),
        (k1024, cams, 0.5, 0.99),
        (synth.tf1(), cams, 200.0, 0.0),
        (opaque, cams, 0.5, 1e-6),
        (synth.tf1(), [face], 0.5, 0.99),
    ]
    for tf, cs, step, ert in cases:
        img = gpu_render(vol, cs, tf, step, ert=ert, use_skip=True)
        ref = oracle.render(vol, cs, tf, step, ert=ert)
        compare_with_flags(img, ref["rgba"], ref["flags"], ert if ert else 1.0)


def test_empty_view_list_is_rejected():
    vol = upload_volume(_small_ct((16, 16, 16), 50))
    t = upload_tf(synth.tf1())
    with pytest.raises(vr.VrError, match="VR_E_INVALID_ARG"):
        vr.vr_render(vol, None, [], t, 0.5)
    with pytest.raises(vr.VrError, match="VR_E_INVALID_ARG"):
        vr.vr_render_backward(vol, None, [], t, 0.5, 0.0, False, torch.zeros(0, device=DEV),
                              torch.zeros(0, device=DEV))


@pytest.mark.parametrize("bad", ["negative", "nan", "inf_colour"])
def test_invalid_tf_gives_nan_and_a_device_status(bad):
    """A device TF with a negative extinction or a non-finite entry cannot be
    checked on the host without waiting: every call that reads it writes NaN
    results and records the fault; vr_device_status reports it once, then
    the device is clean again and a valid TF renders normally."""
    vol_np = _small_ct((24, 20, 18), 51)
    vol = upload_volume(vol_np)
    blocks = vr.vr_build_blocks(vol, 16)
    tf = synth.tf1()
    table = tf.table.copy()
    if bad == "negative":
        table[100, 3] = -0.01
    elif bad == "nan":
        table[7, 3] = np.nan
    else:
        table[200, 0] = np.inf
    t_bad = vr.TF(torch.from_numpy(table).to(DEV), tf.v0, tf.v1)
    cams = synth.orbit_cameras((24, 20, 18), 2, 52, 60.0, 20, 17)
    vr.device_status()  # start clean
    img = vr.vr_render(vol, blocks, cams, t_bad, 0.5, 0.99, True)
    torch.cuda.synchronize()
    assert torch.isnan(img).all()
    with pytest.raises(vr.VrError, match="VR_E_INVALID_ARG"):
        vr.device_status()
    vr.device_status()  # reported once
    occ = vr.vr_block_occupancy(blocks, t_bad)
    torch.cuda.synchronize()
    assert (occ == 1).all()
    grid = upload_volume(vol_np.astype(np.float32))
    gv, gtf = vr.vr_render_backward(grid, None, cams, t_bad, 0.5, 0.0, False, img,
                                    torch.ones_like(img))
    torch.cuda.synchronize()
    assert torch.isnan(gv).all() and torch.isnan(gtf).all()
    with pytest.raises(vr.VrError, match="negative extinction"):
        vr.device_status()
    good = gpu_render(vol_np, cams, tf, 0.5, ert=0.99, use_skip=True, vol=vol, blocks=blocks)
    ref = oracle.render(vol_np, cams, tf, 0.5, ert=0.99)
    compare_with_flags(good, ref["rgba"], ref["flags"], 0.99)
    vr.device_status()


def _islands(dims_xyz, seed, n=7, edge_hugging=True):
    """Zero volume with a few small dense cubes (values 1000-3000), some touching
    the volume's faces: long runs of empty blocks between them, so leaps cross
    cubes of empty blocks (and reach the edge of the block grid)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims_xyz
    vol = np.zeros((nz, ny, nx), np.uint16)
    for i in range(n):
        s = int(rng.integers(3, 9))
        lo = [int(rng.integers(0, d - s)) for d in (nx, ny, nz)]
        if edge_hugging and i < 2:
            lo[i] = 0 if i == 0 else dims_xyz[i] - s
        x, y, z = lo
        vol[z:z + s, y:y + s, x:x + s] = rng.integers(1000, 3000, size=(s, s, s))
    return vol


@pytest.mark.parametrize("edge", [4, 8, 16])
def test_sparse_islands_skip_is_bit_identical(edge):
    """Sparse occupancy: skipping (per-render occupancy bits, leaps across
    cubes of empty blocks) must give exactly the no-skip image."""
    dims = (150, 136, 120)
    vol = _islands(dims, 90 + edge)
    cams = (synth.orbit_cameras(dims, 5, 91, 50.0, 80, 72) + [synth.ortho_axis_camera(150, 80, 72)])
    c = synth.orbit_camera(dims, np.array([0.6, -0.5, 0.62]), 70.0, 80, 72)
    c.eye = np.array([70.2, 60.9, 55.3])  # inside the volume
    cams.append(c)
    tf = synth.tf_from_points([(0, (0, 0, 0, 0)), (600, (0, 0, 0, 0)), (800, (1.0, 0.5, 0.2, 0.05)),
                               (3000, (1, 1, 1, 0.2))], 256, 0.0, 4080.0)
    v = upload_volume(vol)
    log(f"islands {dims} edge {edge}, {len(cams)} views")
    for ert in (0.0, 0.99):
        a, ca = gpu_render(vol, cams, tf, 0.5, ert=ert, use_skip=False, counters=True, vol=v)
        b, cb = gpu_render(vol, cams, tf, 0.5, ert=ert, use_skip=True, counters=True, vol=v, block_edge=edge)
        assert np.array_equal(a, b), f"ert {ert}: max diff {np.abs(a - b).max():.3e}"
        assert cb[0] < ca[0] / 4  # most samples lie in empty blocks
        log(f"ert {ert}: evaluated {cb[0]} of {ca[0]}")


def test_wide_block_grid_falls_back_and_stays_exact():
    """A block grid too wide for the radius kernel's LDS window (and for LDS
    staging of the occupancy bits): leaps fall back to single blocks with the
    bits read from global memory; the image is still exactly the no-skip one."""
    rng = np.random.default_rng(95)
    nx, ny, nz = 8192, 8192, 4
    vol = np.zeros((nz, ny, nx), np.int16)
    for _ in range(40):
        x, y = int(rng.integers(0, nx - 40)), int(rng.integers(0, ny - 40))
        vol[:, y:y + 40, x:x + 40] = rng.integers(200, 1500, size=(nz, 40, 40))
    v = upload_volume(vol)
    cams = [synth.ortho_axis_camera(8192, 96, 96)]
    c = synth.orbit_camera((nx, ny, nz), np.array([0.3, 0.2, 0.93]), 40.0, 96, 96)
    cams.append(c)
    tf = synth.tf1()
    log("wide grid 8192x8192x4 int16, 16^3 blocks (512 x 512 x 1)")
    a, ca = gpu_render(vol, cams, tf, 0.5, ert=0.99, use_skip=False, counters=True, vol=v)
    b, cb = gpu_render(vol, cams, tf, 0.5, ert=0.99, use_skip=True, counters=True, vol=v)
    assert np.array_equal(a, b)
    assert cb[0] <= ca[0]
