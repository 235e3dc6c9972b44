"""GPU adjoint parity: vr_render_backward (through the C ABI) against the
FP64 oracle gradient and against FP64 central differences.

Bar: relative error <= 1e-3, measured as ||g_gpu - g_ref|| / ||g_ref|| and
max |g_gpu - g_ref| / max |g_ref| (fp32 atomics sum in arbitrary order), and
element-wise against m >= |g_ref|, the oracle's sum of the same terms'
magnitudes (the scale of the rounding error of any fp32 evaluation of these
sums; m = |g_ref| where no term cancels):
  * every entry:  |g_gpu - g_ref| <= 1e-3 m + 1e-4 max(m);
  * at least 99.9 % of the grid's non-zero entries (99 % of the TF's, and of
    the grid's at full size, where positions reach |p| of several hundred
    voxels and their fp32 error is tens of times larger): |g_gpu - g_ref| <=
    1e-3 m.
The floor 1e-4 max(m) is there for entries whose terms the fp32 sample
positions move by more than rounding: a tap weight near zero (the far taps
of a stencil, (1 - f)^3 / 6 for f near 1) or a TF segment weight near zero
(a value just past a node) changes by |dw/dp| times the position error
(2^-23 |p| per coordinate), a large relative change of a small term; and a
sample within that error of a TF node takes the other segment's slope (a
kink, where either one-sided derivative is correct).
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
from gpu_util import DEV, log, upload_tf, upload_volume  # noqa: E402

REL = 1e-3


def _rel(a, b):
    na = np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)
    ma = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
    return na, ma


def _check_elementwise(got, ref, mag, what, frac_min=0.999):
    """The element-wise bars of the module docstring; logs the worst ratios."""
    assert np.all(mag >= np.abs(ref) * (1 - 1e-12))
    err = np.abs(got - ref)
    floor = 1e-4 * mag.max()
    outside = err > REL * mag + floor
    nz = mag > 0
    within = (err <= REL * mag)[nz].mean() if nz.any() else 1.0
    ratio = float((err / (REL * mag + floor))[nz].max()) if nz.any() else 0.0
    log(f"{what}: {int(nz.sum())} non-zero entries, {100 * within:.3f} % within 1e-3 m, worst error / "
        f"(1e-3 m + 1e-4 max m) {ratio:.3f}")
    for idx in np.argwhere(outside)[:8]:
        t = tuple(int(i) for i in idx)
        log(f"  {t}: got {got[t]:.9e} ref {ref[t]:.9e} mag {mag[t]:.9e}")
    assert not outside.any(), f"{what}: {int(outside.sum())} entries outside 1e-3 m + 1e-4 max m"
    assert within >= frac_min, f"{what}: only {100 * within:.3f} % of entries within 1e-3 m"


def _case(n=20, views=3, W=24, seed=50):
    grid = synth.density_grid_f32(n, seed=seed, smooth_sigma=2.0)
    tf = synth.tf3()
    cams = synth.orbit_cameras((n, n, n), views, seed + 1, 60.0, W, W)
    g = np.random.default_rng(seed + 2).standard_normal((views, W, W, 4))
    return grid, tf, cams, g


def _gpu_grad(grid, tf, cams, g, step, ert=0.0, use_skip=False, want_volume=True, want_tf=True):
    vol = upload_volume(grid)
    t = upload_tf(tf)
    blocks = vr.vr_build_blocks(vol, 16) if use_skip else None
    out = vr.vr_render(vol, blocks, cams, t, step, ert, use_skip)
    gt = torch.from_numpy(g.astype(np.float32)).to(DEV)
    gv, gtf = vr.vr_render_backward(vol, blocks, cams, t, step, ert, use_skip, out, gt, want_volume, want_tf)
    torch.cuda.synchronize()
    return (None if gv is None else gv.cpu().numpy().astype(np.float64),
            None if gtf is None else gtf.cpu().numpy().astype(np.float64), out)


@pytest.mark.parametrize("ert", [0.0, 0.8])
def test_grad_matches_oracle(ert):
    grid, tf, cams, g = _case()
    if ert:
        tf.table[:, 3] *= 8.0  # opaque enough to terminate
    ref = oracle.render(grid, cams, tf, 0.5, ert=ert)
    g[ref["flags"].astype(bool)] = 0.0
    gv, gtf, _ = _gpu_grad(grid, tf, cams, g, 0.5, ert)
    rv, rt, mv, mt = oracle.grad(grid, cams, tf, 0.5, g, ert=ert, magnitudes=True)
    ev, et = _rel(gv, rv), _rel(gtf, rt)
    log(f"ert={ert}: grid rel {ev[0]:.2e}/{ev[1]:.2e}  tf rel {et[0]:.2e}/{et[1]:.2e}")
    assert max(ev) <= REL and max(et) <= REL
    _check_elementwise(gv, rv, mv, f"ert={ert} grid")
    _check_elementwise(gtf, rt, mt, f"ert={ert} tf", 0.99)


def test_grad_volume_only_with_skipping_matches_oracle():
    """With only the grid gradient requested, empty blocks are skipped (their
    samples have zero extinction slope and zero opacity)."""
    vol = synth.ct_phantom_i16(40, 36, 32, seed=51, n_soft=4, n_bone=3).astype(np.float32)
    tf = synth.tf1()
    cams = synth.orbit_cameras((40, 36, 32), 2, 52, 60.0, 32, 32)
    g = np.random.default_rng(53).standard_normal((2, 32, 32, 4))
    gv, _, _ = _gpu_grad(vol, tf, cams, g, 0.5, 0.99, use_skip=True, want_tf=False)
    rv, _ = oracle.grad(vol, cams, tf, 0.5, g, ert=0.99, want_tf=False)
    e = _rel(gv, rv)
    log(f"skip grid rel {e[0]:.2e}/{e[1]:.2e}")
    assert max(e) <= REL


@pytest.mark.parametrize("W", [8, 11])
def test_grad_narrow_ray_bundle_matches_oracle(W):
    """All rays of a tile inside about one voxel (1 degree field of view): the
    stencils of one wavefront step coincide or overlap, so nearly every pair
    of scatter records applied together shares cells, and the number of
    records per step varies (odd counts included; W = 11 leaves ragged
    tiles)."""
    import dataclasses

    grid, tf, cams, _ = _case(n=16, views=2, W=W, seed=57)
    cams = [dataclasses.replace(c, fov_y=float(np.deg2rad(1.0))) for c in cams]
    g = np.random.default_rng(58).standard_normal((2, W, W, 4))
    gv, gtf, _ = _gpu_grad(grid, tf, cams, g, 0.25)
    rv, rt = oracle.grad(grid, cams, tf, 0.25, g)
    ev, et = _rel(gv, rv), _rel(gtf, rt)
    log(f"narrow bundle W={W}: grid rel {ev[0]:.2e}/{ev[1]:.2e}  tf rel {et[0]:.2e}/{et[1]:.2e}")
    assert np.abs(rv).max() > 0.0
    assert max(ev) <= REL and max(et) <= REL


def test_grad_against_fp64_central_differences():
    """GPU analytic gradient on 32 seeded voxels of the non-zero region
    against central differences of the FP64 oracle render."""
    grid, tf, cams, g = _case(n=16, views=2, W=20, seed=54)
    grid64 = grid.astype(np.float64)
    gv, _, _ = _gpu_grad(grid, tf, cams, g, 0.5, want_tf=False)
    rng = np.random.default_rng(55)
    nz_idx = np.argwhere(grid > 0.05)
    scale = np.abs(gv).max()
    checked = 0
    for i in rng.permutation(len(nz_idx)):
        ijk = tuple(int(x) for x in nz_idx[i])

        def loss(h):
            v = grid64.copy()
            v[ijk] += h
            return float((oracle.render(v, cams, tf, 0.5)["rgba"] * g).sum())

        fd1 = (loss(1e-5) - loss(-1e-5)) / 2e-5
        fd2 = (loss(4e-6) - loss(-4e-6)) / 8e-6
        if abs(fd1 - fd2) > 1e-6 * scale:
            continue  # a TF node inside the FD stencil (kink)
        assert abs(gv[ijk] - fd1) <= REL * scale, (ijk, gv[ijk], fd1)
        checked += 1
        if checked == 32:
            break
    assert checked == 32


def _u16_tf1():
    return synth.tf_from_points([(v + 1024, c) for v, c in synth.TF1_POINTS], 256, 0.0, 4080.0)


@pytest.mark.parametrize("dtype,dims", [("i16", (40, 36, 32)), ("i16", (37, 29, 23)), ("u16", (40, 36, 32)),
                                        ("u16", (37, 29, 23))])
def test_grad_16bit_volumes_match_oracle(dtype, dims):
    """The adjoint of 16-bit volumes (the benchmark's int16 kernel and its
    uint16 twin): even nx takes the prefetched packed-row path, odd nx the
    plain one; skip + early termination at 0.99 in the forward, grid and TF
    gradients, dense dL/dRGBA."""
    base = synth.ct_phantom_i16(*dims, seed=120 + dims[0], n_soft=4, n_bone=3)
    if dtype == "u16":
        vol, tf = (base.astype(np.int32) + 1024).clip(0, 4095).astype(np.uint16), _u16_tf1()
    else:
        vol, tf = base, synth.tf1()
    views, W, H = 2, 32, 28
    cams = synth.orbit_cameras(dims, views, 121, 60.0, W, H)
    g = np.random.default_rng(122).standard_normal((views, H, W, 4))
    ref = oracle.render(vol, cams, tf, 0.5, ert=0.99)
    g[ref["flags"].astype(bool)] = 0.0
    gv, gtf, out = _gpu_grad(vol, tf, cams, g, 0.5, 0.99, use_skip=True)
    un = np.abs(out.cpu().numpy() - ref["rgba"]).max(axis=-1)[~ref["flags"].astype(bool)].max()
    assert un <= 2e-4
    rv, rt, mv, mt = oracle.grad(vol, cams, tf, 0.5, g, ert=0.99, magnitudes=True)
    ev, et = _rel(gv, rv), _rel(gtf, rt)
    log(f"{dtype} {dims}: grid rel {ev[0]:.2e}/{ev[1]:.2e}  tf rel {et[0]:.2e}/{et[1]:.2e}")
    assert np.abs(rv).max() > 0.0
    assert max(ev) <= REL and max(et) <= REL
    _check_elementwise(gv, rv, mv, f"{dtype} {dims} grid")
    _check_elementwise(gtf, rt, mt, f"{dtype} {dims} tf", 0.99)


def test_flat_runs_match_full_evaluation():
    """With the blocks' min/max the adjoint takes the samples of constant empty
    blocks (the air of a CT phantom) without reconstructing them and accounts
    for runs of them at once, also across wavefront leaps: every lattice index
    must still be counted exactly once.  Against the same adjoint without the
    blocks (every sample reconstructed), per view size, orthographic and
    perspective, with and without early termination."""
    dims = (64, 56, 48)
    vol = synth.ct_phantom_i16(*dims, seed=131, n_soft=4, n_bone=3)
    tf = synth.tf1()
    v = upload_volume(vol)
    t = upload_tf(tf)
    blocks = vr.vr_build_blocks(v, 16)
    for ert, cams in ((0.0, [synth.ortho_axis_camera(dims[0], 48, 40)]),
                      (0.99, synth.orbit_cameras(dims, 2, 132, 60.0, 48, 40))):
        out = vr.vr_render(v, None, cams, t, 0.5, ert, False)
        g = torch.from_numpy(np.random.default_rng(133).standard_normal(tuple(out.shape)).astype(np.float32)).to(DEV)
        gv0, gt0 = vr.vr_render_backward(v, None, cams, t, 0.5, ert, False, out, g)
        gv1, gt1 = vr.vr_render_backward(v, blocks, cams, t, 0.5, ert, False, out, g)
        torch.cuda.synchronize()
        gv0, gv1 = gv0.cpu().numpy().astype(np.float64), gv1.cpu().numpy().astype(np.float64)
        gt0, gt1 = gt0.cpu().numpy().astype(np.float64), gt1.cpu().numpy().astype(np.float64)
        # the air's TF segment (its nodes' extinction gradients) is where a
        # miscounted run shows
        u = (-1000.0 - tf.v0) * (tf.table.shape[0] - 1) / (tf.v1 - tf.v0)
        air = [int(np.floor(u)), int(np.floor(u)) + 1]
        assert np.abs(gt0[air, 3]).min() > 0.0
        assert np.abs(gt1[air, 3] - gt0[air, 3]).max() <= 1e-4 * np.abs(gt0[air, 3]).max(), (ert, gt1[air, 3], gt0[air, 3])
        assert _rel(gt1, gt0)[1] <= 1e-4, (ert, _rel(gt1, gt0))
        assert _rel(gv1, gv0)[1] <= 1e-4, (ert, _rel(gv1, gv0))


def test_c1_int16_adjoint_sampled_pixels_match_oracle():
    """The benchmark's fwd+bwd configuration: 512x512x400 int16 to 1024^2,
    skip + early termination at 0.99 in the forward, grid and TF gradients
    (the adjoint then marches every sample), dL/dRGBA non-zero on 3000 seeded
    hit pixels (the FP64 oracle gradient stays cheap)."""
    c = synth.config_c1()
    log("c1 adjoint: 512x512x400 int16 -> 1024^2")
    vol = upload_volume(c["volume"])
    blocks = vr.vr_build_blocks(vol, 16)
    t = upload_tf(c["tf"])
    out = vr.vr_render(vol, blocks, c["cameras"], t, c["step"], c["ert"], True)
    lat = oracle.lattice(c["cameras"], (512, 512, 400), c["step"])
    pix = synth.sample_pixels(1, 1024, 1024, 8000, seed=123)
    pix = pix[lat[0, pix[:, 1], pix[:, 2]] > 0]
    ref = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"], ert=c["ert"], pixels=pix)
    pix = pix[ref["flags"] == 0][:3000]
    g = np.zeros((1, 1024, 1024, 4))
    g[pix[:, 0], pix[:, 1], pix[:, 2]] = np.random.default_rng(124).standard_normal((len(pix), 4))
    gt_dev = torch.from_numpy(g.astype(np.float32)).to(DEV)
    gv, gtf = vr.vr_render_backward(vol, blocks, c["cameras"], t, c["step"], c["ert"], True, out, gt_dev)
    torch.cuda.synchronize()
    gv = gv.cpu().numpy().astype(np.float64)
    gtf = gtf.cpu().numpy().astype(np.float64)
    rv, rt, mv, mt = oracle.grad(c["volume"], c["cameras"], c["tf"], c["step"], g, ert=c["ert"], magnitudes=True)
    ev, et = _rel(gv, rv), _rel(gtf, rt)
    log(f"c1 adjoint ({len(pix)} pixels): grid rel {ev[0]:.2e}/{ev[1]:.2e}  tf rel {et[0]:.2e}/{et[1]:.2e}")
    assert max(ev) <= REL and max(et) <= REL
    _check_elementwise(gv, rv, mv, "c1 grid", 0.99)
    _check_elementwise(gtf, rt, mt, "c1 tf", 0.99)


def test_autograd_function_matches_backward_call():
    grid, tf, cams, g = _case(seed=56)
    t_grid = torch.from_numpy(grid).to(DEV).requires_grad_(True)
    t_tf = torch.from_numpy(tf.table).to(DEV).requires_grad_(True)
    out = vr.VolumeRender.apply(t_grid, t_tf, cams, tf.v0, tf.v1, 0.5, 0.0)
    loss = (out * torch.from_numpy(g.astype(np.float32)).to(DEV)).sum()
    loss.backward()
    gv, gtf, _ = _gpu_grad(grid, tf, cams, g, 0.5)
    assert _rel(t_grid.grad.cpu().numpy().astype(np.float64), gv)[1] <= 1e-5
    assert _rel(t_tf.grad.cpu().numpy().astype(np.float64), gtf)[1] <= 1e-5


def test_c3_full_size_sparse_gradient_matches_oracle():
    """The differentiable workload at full size (256^3 fp32 grid, 64 views of
    512^2) in the benchmark's launch configuration; dL/dRGBA is non-zero on
    3000 seeded pixels so that the FP64 oracle gradient stays cheap."""
    c = synth.config_c3()
    log("c3: 256^3 f32, 64 x 512^2")
    views, W = 64, 512
    g = np.zeros((views, W, W, 4))
    pix = synth.sample_pixels(views, W, W, 3000, seed=57)
    g[pix[:, 0], pix[:, 1], pix[:, 2]] = np.random.default_rng(58).standard_normal((3000, 4))
    gv, gtf, out = _gpu_grad(c["volume"], c["tf"], c["cameras"], g, c["step"])
    rv, rt, mv, mt = oracle.grad(c["volume"], c["cameras"], c["tf"], c["step"], g, magnitudes=True)
    ev, et = _rel(gv, rv), _rel(gtf, rt)
    log(f"c3: grid rel {ev[0]:.2e}/{ev[1]:.2e}  tf rel {et[0]:.2e}/{et[1]:.2e}")
    assert max(ev) <= REL and max(et) <= REL
    _check_elementwise(gv, rv, mv, "c3 grid", 0.99)
    _check_elementwise(gtf, rt, mt, "c3 tf", 0.99)
    # forward images of two views against the oracle on sampled pixels
    sp = synth.sample_pixels(views, W, W, 1500, seed=59)
    ref = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"], pixels=sp)
    got = out.cpu().numpy()[sp[:, 0], sp[:, 1], sp[:, 2]]
    assert np.abs(got - ref["rgba"]).max() <= 2e-4


def _pixels_meeting_box(cam, lo, hi):
    """Conservative (view-local) pixel rectangle of the rays of a perspective
    camera that can meet the axis-aligned box [lo, hi] (camera outside it):
    the projected corners' bounding rectangle, widened by one pixel."""
    corners = np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])],
                       dtype=np.float64)
    d = corners - np.asarray(cam.eye, dtype=np.float64)
    zc = d @ np.asarray(cam.forward, dtype=np.float64)
    assert (zc > 0).all()
    th = np.tan(0.5 * cam.fov_y)
    sx = (d @ np.asarray(cam.right, dtype=np.float64)) / (zc * th * cam.width / cam.height)
    sy = (d @ np.asarray(cam.up, dtype=np.float64)) / (zc * th)
    col = (sx + 1.0) * 0.5 * cam.width - 0.5
    row = (1.0 - sy) * 0.5 * cam.height - 0.5
    c0, c1 = max(int(np.floor(col.min())) - 1, 0), min(int(np.ceil(col.max())) + 1, cam.width - 1)
    r0, r1 = max(int(np.floor(row.min())) - 1, 0), min(int(np.ceil(row.max())) + 1, cam.height - 1)
    if c0 > c1 or r0 > r1:
        return np.zeros((0, 2), np.int64)
    rr, cc = np.meshgrid(np.arange(r0, r1 + 1), np.arange(c0, c1 + 1), indexing="ij")
    return np.stack([rr.ravel(), cc.ravel()], axis=1)


def test_c3_central_differences_on_32_voxels():
    """The differentiable workload at full size (256^3 fp32, 64 views of
    512^2, dense seeded dL/dRGBA): the GPU gradient of 32 seeded voxels of the
    non-zero region against FP64 central differences (h = 1e-4) of the
    oracle's loss, re-rendering only the rays that can meet the voxel's
    4^3 support (other rays provably do not change).  A voxel whose FD values
    at h and h/2 disagree (a sample crossing a TF node: a kink) is re-drawn."""
    c = synth.config_c3()
    grid = c["volume"]
    cams, tf, step = c["cameras"], c["tf"], c["step"]
    views, W = len(cams), cams[0].width
    g = np.random.default_rng(125).standard_normal((views, W, W, 4))
    log("c3 FD: GPU gradient of 256^3 x 64 views")
    gv, _, _ = _gpu_grad(grid, tf, cams, g, step, want_tf=False)
    scale = np.abs(gv).max()
    g64 = grid.astype(np.float64)
    rng = np.random.default_rng(9)
    nz_idx = np.argwhere(grid > 0.05)
    checked, worst = 0, 0.0
    for i in rng.permutation(len(nz_idx))[:200]:
        z, y, x = (int(v) for v in nz_idx[i])
        lo, hi = (x - 2.0, y - 2.0, z - 2.0), (x + 2.0, y + 2.0, z + 2.0)
        pix, wts = [], []
        for v, cam in enumerate(cams):
            p = _pixels_meeting_box(cam, lo, hi)
            if len(p):
                pix.append(np.concatenate([np.full((len(p), 1), v, np.int64), p], axis=1))
        pix = np.concatenate(pix, axis=0)
        gw = g[pix[:, 0], pix[:, 1], pix[:, 2]]

        def loss(h):
            g64[z, y, x] += h
            try:
                return float((oracle.render(g64, cams, tf, step, pixels=pix)["rgba"] * gw).sum())
            finally:
                g64[z, y, x] -= h

        fd1 = (loss(1e-4) - loss(-1e-4)) / 2e-4
        fd2 = (loss(5e-5) - loss(-5e-5)) / 1e-4
        if abs(fd1 - fd2) > 1e-6 * scale:
            continue  # kink inside the FD stencil
        err = abs(gv[z, y, x] - fd1)
        worst = max(worst, err / (REL * abs(fd1) + 1e-5 * scale))
        assert err <= REL * abs(fd1) + 1e-5 * scale, ((x, y, z), gv[z, y, x], fd1)
        checked += 1
        if checked == 32:
            break
    log(f"c3 FD: {checked} voxels, worst error / bound {worst:.3f}")
    assert checked == 32
