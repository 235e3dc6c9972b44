#!/usr/bin/env python3
"""Throughput of the MI355X tricubic ray caster on its headline workload.

Workload (one "step" = one frame of the per-frame hot path): a 512x512x400
int16 CT-like phantom (resident in HBM with its 16^3 block min/max) rendered
to a 1024^2 perspective image, 60 deg FOV, seeded orbit pose, step 0.5 voxel,
tricubic B-spline sampling, TF post-classification, front-to-back
compositing, early termination at opacity 0.99, block empty-space leaping.

Printed as one JSON line:
  value          evaluated samples/s of the forward frame (whole job, wall clock
                 over exactly --steps frames bracketed by device syncs)
  rays_per_s     pixels/s of the same frames
  fwd_bwd        the same frame plus its adjoint (grad w.r.t. the voxels and
                 the TF, loss 0.5 ||image||^2)
  serve          the serving mix: 8 resident volumes, Poisson arrivals at
                 200 req/s, random poses, 256^2 / 512^2 / 1024^2 images;
                 p50/p99 latency (submit -> completion) and rays/s
  roofline       compulsory HBM bytes of one forward launch (the int16 volume
                 read once + the fp32 RGBA image written once) / that launch's
                 median duration (HIP events on the launch stream), against
                 the 8 TB/s HBM peak and against the achievable bandwidth a
                 streaming-read probe measures on this GPU; the HBM-side
                 traffic the PMC counters saw (stored, with its ratio to the
                 compulsory bytes) and the VALU-issue ceiling beside it
  effective_gather  evaluated samples x 64 taps x 2 B per launch / time: the
                 gather rate the taps are served at (LDS boxes and caches
                 serve most of them, so it is not an HBM figure)
  cpu_baseline   the FP64 oracle on the same frame (same skipping and early
                 termination, rays counted over all pixels as on the GPU) on
                 this host's cores, and on one core for a seeded sample
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "samples/s and rays/s (fwd, fwd+bwd) on 512x512x400 at 1024^2; HBM roofline %; p99"
HBM_PEAK_GBS = 8000.0
TAPS_BYTES_I16 = 64 * 2
# MI355X: 256 CUs x 4 SIMDs at 2.4 GHz; one wave64 VALU instruction takes a
# SIMD 4 cycles without packed-FP32 (disabled in this build), so the chip
# issues 256 x 4 x 2.4e9 / 4 wave64 VALU instructions per second
VALU_WAVE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--bwd-steps", type=int, default=5)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="all-core oracle budget (the whole frame if it fits)")
    ap.add_argument("--cpu-single-seconds", type=float, default=8.0, help="single-core oracle budget")
    ap.add_argument("--no-probe", action="store_true", help="skip the achievable-HBM streaming-read probe")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "render_fwd_c1_traffic.json"))
    ap.add_argument("--no-c3", action="store_true", help="skip the differentiable 256^3 x 64-view measurement")
    ap.add_argument("--no-lit", action="store_true", help="skip the lit (local lighting) forward measurement")
    ap.add_argument("--no-preint", action="store_true",
                    help="skip the pre-integrated forward and the step-artefact measurement")
    ap.add_argument("--no-bricked", action="store_true", help="skip the out-of-core (brick pool) measurement")
    ap.add_argument("--no-filters", action="store_true", help="skip the Catmull-Rom / interpolating-spline frames")
    ap.add_argument("--no-c2", action="store_true", help="skip the large 1024^3 -> 2048^2 forward measurement")
    ap.add_argument("--gigavoxel", action="store_true",
                    help="also render a 512x512x5382 int16 volume (the paper's largest CT) out of core through a "
                         "1 GiB pool (about a minute of host-side set-up)")
    return ap.parse_args()


KERNEL_SOURCES = ("render_fwd.hip", "vr_device.h", "vr_internal.h")


def kernel_source_hash():
    """sha256 over the sources of the forward kernel (k_render) and its
    headers; stored PMC traffic is valid only for them."""
    import hashlib

    d = os.path.join(ROOT, "paper_2005_01442_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stats_ms(ev_ms):
    """Median and p99 (nearest rank) of per-step event times."""
    import numpy as np

    a = np.sort(np.asarray(ev_ms, dtype=np.float64))
    return float(np.median(a)), float(a[min(len(a) - 1, int(np.ceil(0.99 * len(a))) - 1)])


def hbm_probe(vr, torch, gib=8, repeats=10):
    """Achievable HBM read bandwidth: a streaming 16-byte-load read of a
    ``gib`` GiB buffer, best of ``repeats`` (HIP events)."""
    nbytes = gib << 30
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    buf.fill_(1)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    vr.vr_probe_stream_read(buf, sink)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(repeats):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        vr.vr_probe_stream_read(buf, sink)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    del buf
    torch.cuda.empty_cache()
    return {"bytes": nbytes, "best_ms": best, "gb_per_s": nbytes / (best * 1e-3) / 1e9, "repeats": repeats,
            "kernel": "k_stream_read (16-byte nontemporal loads, 4 in flight per lane, 8 workgroups per CU)"}


def time_steps(fn, steps, warmup, torch):
    """W untimed steps, then exactly K steps bracketed by device syncs; per
    step HIP events on the current (launch) stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record()
        fn()
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return wall, ev_ms


def cpu_baseline(c, seconds, single_seconds):
    """The FP64 oracle on the C1 frame as the GPU renders it: the same block
    skipping (occupancy from the oracle's own block min/max) and early
    termination; pixels drawn from the whole frame (misses included), so
    rays/s counts all pixels like the GPU figure.  All host cores on the whole
    frame when it fits ``seconds`` (else a seeded sample of that size), then
    one core on a seeded sample of about ``single_seconds``."""
    import numpy as np

    import oracle

    W, H = c["cameras"][0].width, c["cameras"][0].height
    occ = oracle.occupancy(oracle.blocks(c["volume"], 16), c["tf"])
    order = np.random.default_rng(80).permutation(W * H)
    all_threads = oracle.num_threads()

    def run(n, threads):
        q = np.sort(order[:n])
        pix = np.stack([np.zeros(n, np.int64), q // W, q % W], axis=1)
        oracle.set_num_threads(threads)
        try:
            t = time.perf_counter()
            r = oracle.render(c["volume"], c["cameras"], c["tf"], c["step"], ert=c["ert"], occ=occ, pixels=pix)
            return time.perf_counter() - t, int(r["counts"][:, 1].sum())
        finally:
            oracle.set_num_threads(all_threads)

    def measure(threads, budget):
        dt, _ = run(4096, threads)
        n = int(min(W * H, max(4096, 4096 * budget / max(dt, 1e-3))))
        dt, ev = run(n, threads)
        return n, dt, ev

    n, dt, ev = measure(all_threads, seconds)
    n1, dt1, ev1 = measure(1, single_seconds)
    what = "the whole 1024^2 frame" if n == W * H else f"{n} seeded pixels of the 1024^2 frame"
    return dict(
        value=ev / dt,
        unit="samples/s",
        rays_per_s=n / dt,
        seconds=dt,
        cores=all_threads,
        kind="oracle",
        sample=f"{what} (misses included), FP64, the GPU's 16^3 block skipping and early termination at 0.99, "
               f"OpenMP over pixels; {ev} evaluated samples",
        single_core={"value": ev1 / dt1, "unit": "samples/s", "rays_per_s": n1 / dt1, "seconds": dt1, "cores": 1,
                     "sample": f"{n1} seeded pixels of the same frame, one thread; {ev1} evaluated samples"},
    )


def c0_plain(vr, torch, np, synth, args):
    """The plain forward (64^3 uint16, 256^2 orthographic along +z, step 0.5,
    no skipping, no early termination): launch-overhead-sized."""
    c0 = synth.config_c0()
    vol = vr.Volume(torch.from_numpy(c0["volume"].view(np.int16)).cuda(), dtype=vr.VR_U16)
    tf = vr.TF(torch.from_numpy(c0["tf"].table).cuda(), c0["tf"].v0, c0["tf"].v1)
    cams = c0["cameras"]
    out = torch.empty((1, cams[0].height, cams[0].width, 4), dtype=torch.float32, device="cuda")

    def fwd():
        vr.vr_render(vol, None, cams, tf, c0["step"], 0.0, False, out=out)

    wall, ev = time_steps(fwd, args.steps, args.warmup, torch)
    med, p99 = stats_ms(ev)
    samples = 65536 * 128
    return {"workload": "c0_ellipsoids64cube_u16_to_256x256_ortho_step0.5_noskip_noert",
            "ms_per_step": wall / args.steps * 1e3, "kernel_ms_median": med, "kernel_ms_p99": p99,
            "samples_per_s": samples / (wall / args.steps), "rays_per_s": 65536 / (wall / args.steps),
            "evaluated_samples_per_frame": samples}


def differentiable_c3(vr, torch, steps=3):
    """Forward + adjoint of the differentiable workload: 256^3 fp32 density
    grid, 64 views of 512^2, step 0.5, no skipping (the TF gradient needs
    every sample), loss = MSE against renders of a perturbed grid."""
    import synth
    from synth.configs import c3_perturbed_grid

    c = synth.config_c3()
    target_grid = torch.from_numpy(c["volume"]).cuda()
    grid = torch.from_numpy(c3_perturbed_grid(c["volume"])).cuda()
    table = torch.from_numpy(c["tf"].table).cuda()
    tf = vr.TF(table, c["tf"].v0, c["tf"].v1)
    cams = c["cameras"]
    target = vr.vr_render(vr.Volume(target_grid), None, cams, tf, c["step"])
    vol = vr.Volume(grid)
    ctr = torch.zeros(4, dtype=torch.int64, device="cuda")
    vr.vr_render(vol, None, cams, tf, c["step"], counters=ctr)
    torch.cuda.synchronize()
    lattice = int(ctr[1].item())

    def step():
        img = vr.vr_render(vol, None, cams, tf, c["step"])
        g = (img - target) * (2.0 / img.numel())
        return vr.vr_render_backward(vol, None, cams, tf, c["step"], 0.0, False, img, g)

    def fwd():
        vr.vr_render(vol, None, cams, tf, c["step"])

    wall_f, _ = time_steps(fwd, steps, 1, torch)
    wall_fb, _ = time_steps(step, steps, 1, torch)
    rays = len(cams) * cams[0].width * cams[0].height
    return dict(
        workload="c3_density256_f32_64x512x512_step0.5",
        lattice_samples_per_step=lattice,
        fwd_ms=wall_f / steps * 1e3,
        fwd_bwd_ms=wall_fb / steps * 1e3,
        fwd_samples_per_s=lattice / (wall_f / steps),
        fwd_bwd_samples_per_s=lattice / (wall_fb / steps),
        fwd_bwd_rays_per_s=rays / (wall_fb / steps),
        note="all lattice samples evaluated (no skipping: TF gradient requested); loss = MSE vs perturbed-grid renders",
    )


def serve_mix(vr, torch, n_req, n_warm, rate):
    import numpy as np

    import synth

    dims = synth.config_c4_volumes(seed=10, count=8)
    vols = []
    for (nx, ny, nz), seed in dims:
        vols.append(vr.Volume(torch.from_numpy(synth.ct_phantom_i16(nx, ny, nz, seed)).cuda()))
    log(f"serve: {len(vols)} volumes resident ({sum(v.tensor.numel() * 2 for v in vols) / 2**30:.2f} GiB)")
    srv = vr.Server(hbm_budget_bytes=4 << 30, max_inflight=32)
    ids = [srv.add_volume(v) for v in vols]
    tf = synth.tf1()
    total = n_warm + n_req
    reqs = synth.c4_arrivals(total, seed=11, rate_hz=rate, n_volumes=8, dims_list=[d for d, _ in dims])
    tickets = [None] * total
    ready = [threading.Event() for _ in range(total)]
    finished = [threading.Event() for _ in range(total)]
    phase_start = {}
    # 50 seeded requests of the measured phase keep their images for the
    # alone-vs-mix check
    check_idx = set(int(i) for i in np.random.default_rng(81).choice(np.arange(n_warm, total), 50, replace=False))
    kept = {}
    depth = []  # (t, queued, inflight) every 5 ms of the measured phase
    stop_sampling = threading.Event()

    def producer():
        t_base = time.perf_counter()
        for i, r in enumerate(reqs):
            if i == n_warm:
                # warm-up done: wait for it to drain, then reset statistics
                finished[n_warm - 1].wait()
                srv.reset_stats()
                t_base = time.perf_counter() - r["t"]
                phase_start["t"] = time.perf_counter()
            delay = t_base + r["t"] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets[i] = srv.submit(ids[r["volume"]], r["camera"], tf.table, tf.v0, tf.v1, 0.5, 0.99, True)
            ready[i].set()

    done_at = {}

    def consumer():
        for i in range(total):
            ready[i].wait()
            if i in check_idx:
                s = reqs[i]["size"]
                kept[i] = srv.result(tickets[i], s, s)
            else:
                srv.wait(tickets[i])
                srv.release(tickets[i])
            finished[i].set()
        done_at["t"] = time.perf_counter()

    def sampler():
        while not stop_sampling.is_set():
            if "t" in phase_start:
                st_ = srv.stats()
                depth.append((time.perf_counter() - phase_start["t"], int(st_["queued"]), int(st_["inflight"])))
            time.sleep(0.005)

    th_p = threading.Thread(target=producer)
    th_c = threading.Thread(target=consumer)
    th_s = threading.Thread(target=sampler)
    th_p.start()
    th_c.start()
    th_s.start()
    th_p.join()
    th_c.join()
    stop_sampling.set()
    th_s.join()
    st = srv.stats()
    wall = done_at["t"] - phase_start["t"]
    pixels = sum(r["size"] ** 2 for r in reqs[n_warm:])
    srv.close()
    # the kept requests re-rendered alone through vr_render
    blocks = {}
    tf_dev = vr.TF(torch.from_numpy(tf.table).cuda(), tf.v0, tf.v1)
    max_diff, identical = 0.0, 0
    for i, img in kept.items():
        r = reqs[i]
        vi = r["volume"]
        if vi not in blocks:
            blocks[vi] = vr.vr_build_blocks(vols[vi], 16)
        alone = vr.vr_render(vols[vi], blocks[vi], [r["camera"]], tf_dev, 0.5, 0.99, True)[0]
        d = float((alone - img).abs().max().item())
        max_diff = max(max_diff, d)
        identical += int(torch.equal(alone, img))
    q = np.array([d[1] for d in depth]) if depth else np.zeros(1)
    series = []
    for t0 in np.arange(0.0, wall, 0.1):
        w = [d[1] for d in depth if t0 <= d[0] < t0 + 0.1]
        series.append(int(max(w)) if w else 0)
    return dict(
        requests=n_req,
        offered_req_per_s=rate,
        achieved_req_per_s=n_req / wall,
        p50_ms=st["p50_ms"],
        p99_ms=st["p99_ms"],
        mean_ms=st["mean_ms"],
        max_ms=st["max_ms"],
        rays_per_s=pixels / wall,
        rays_per_busy_s=st["rays_per_s"],
        samples_per_s=st["samples"] / wall,
        samples_per_busy_s=st["samples_per_s"],
        evaluated_samples=st["samples"],
        launches=st["launches"],
        hbm_peak_bytes=st["hbm_peak"],
        resident_bytes=st["resident_bytes"],
        queue_depth={"time_mean": st["queued_mean"], "max": st["queued_max"], "p50_sampled": float(np.median(q)),
                     "p99_sampled": float(np.percentile(q, 99)), "max_per_100ms": series,
                     "note": "queued (not yet admitted) requests; time_mean/max from the server, the rest sampled "
                             "every 5 ms"},
        alone_check={"requests": len(kept), "bit_identical": identical, "max_abs_diff": max_diff,
                     "note": "50 seeded requests of the measured phase re-rendered alone with vr_render"},
    )


SPIKE_POINTS = [(-1024.0, (0, 0, 0, 0)), (-16.0, (0, 0, 0, 0)), (0.0, (0.8, 0.3, 0.2, 0.01)),
                (96.0, (0.8, 0.3, 0.2, 0.01)), (112.0, (0, 0, 0, 0)), (336.0, (0, 0, 0, 0)),
                (352.0, (1.0, 0.9, 0.8, 0.6)), (368.0, (0, 0, 0, 0)), (3056.0, (0, 0, 0, 0))]


def _psnr(a, b, np):
    return float(10.0 * np.log10(1.0 / np.mean((a - b) ** 2)))


def _ssim(a, b, np):
    """Mean SSIM over the RGBA channels (Gaussian window sigma 1.5, data range 1)."""
    from scipy.ndimage import gaussian_filter

    c1, c2 = 0.01 ** 2, 0.03 ** 2
    vals = []
    for ch in range(a.shape[-1]):
        x, y = a[..., ch], b[..., ch]
        mx, my = gaussian_filter(x, 1.5), gaussian_filter(y, 1.5)
        sxx = gaussian_filter(x * x, 1.5) - mx * mx
        syy = gaussian_filter(y * y, 1.5) - my * my
        sxy = gaussian_filter(x * y, 1.5) - mx * my
        s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
        vals.append(float(s.mean()))
    return float(np.mean(vals))


def preint_measurements(vr, torch, np, synth, c, vol, blocks, cams, tf, out, args):
    """Pre-integrated C1 frame (TF1, step 0.5, skip, ERT) timed like the
    forward; then the step-artefact metric: a one-node extinction spike TF
    rendered at coarse steps, post-classified and pre-integrated, against a
    post-classified reference at step 1/8 (PSNR and SSIM over RGBA)."""
    W, H = cams[0].width, cams[0].height
    table = vr.vr_preint_build(tf, c["step"])
    ctr = torch.zeros(4, dtype=torch.int64, device="cuda")
    vr.vr_render_preint(vol, blocks, cams, tf, table, c["step"], c["ert"], True, out=out, counters=ctr)
    torch.cuda.synchronize()
    cells = int(ctr[0].item())

    def fwd_pre():
        vr.vr_render_preint(vol, blocks, cams, tf, table, c["step"], c["ert"], True, out=out)

    wall, ev = time_steps(fwd_pre, args.steps, args.warmup, torch)
    ms = wall / args.steps * 1e3
    log(f"fwd pre-integrated: {ms:.3f} ms/frame wall, {float(np.mean(ev)):.3f} ms/launch events")
    t0 = time.perf_counter()
    tbl = vr.vr_preint_build(tf, c["step"])
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    del tbl
    stf = synth.tf_from_points(SPIKE_POINTS, 256, -1024.0, 3056.0)
    spike = vr.TF(torch.from_numpy(stf.table).cuda(), stf.v0, stf.v1)
    ref = vr.vr_render(vol, blocks, cams, spike, 0.125, 0.0, True).cpu().numpy().astype(np.float64)
    artefacts = []
    for st in (1.0, 2.0, 4.0):
        post = vr.vr_render(vol, blocks, cams, spike, st, 0.0, True).cpu().numpy().astype(np.float64)
        tb = vr.vr_preint_build(spike, st)
        pre = vr.vr_render_preint(vol, blocks, cams, spike, tb, st, 0.0, True).cpu().numpy().astype(np.float64)
        row = {"step": st, "psnr_post_db": _psnr(post, ref, np), "psnr_preint_db": _psnr(pre, ref, np),
               "ssim_post": _ssim(post[0], ref[0], np), "ssim_preint": _ssim(pre[0], ref[0], np)}
        log(f"step {st}: PSNR post {row['psnr_post_db']:.2f} dB, pre-integrated {row['psnr_preint_db']:.2f} dB; "
            f"SSIM {row['ssim_post']:.4f} / {row['ssim_preint']:.4f}")
        artefacts.append(row)
    return {
        "ms_per_step": ms,
        "kernel_ms": float(np.mean(ev)),
        "cells_per_s": cells / (wall / args.steps),
        "rays_per_s": W * H / (wall / args.steps),
        "evaluated_cells_per_frame": cells,
        "table_build_ms": build_ms,
        "step_artefacts": {
            "tf": "one-node extinction spike at 352 HU + soft tissue band (K=256)",
            "reference": "post-classified, step 1/8",
            "rows": artefacts,
        },
        "note": "same frame, TF1, step 0.5, skip + ERT 0.99: cells between lattice boundaries, K x K table lookup",
    }


def bricked_measurements(vr, torch, np, c, cams, tf, out, args):
    """The C1 frame rendered out of core: the volume as 64^3-block bricks in
    pinned host memory, a device pool of 64 MiB (a third of the occupied
    bricks: every frame re-streams them over PCIe in front-to-back passes) and
    of 1 GiB (all occupied bricks stay resident after the first frame)."""
    res = {}
    for label, pool in (("pool_64MiB", 64 << 20), ("pool_1GiB", 1 << 30)):
        t0 = time.perf_counter()
        bv = vr.BrickedVolume(c["volume"], 64, pool)
        create_ms = (time.perf_counter() - t0) * 1e3
        bv.render(cams, tf, c["step"], c["ert"], out=out)
        torch.cuda.synchronize()
        s0 = bv.stats()
        steps = max(3, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(steps):
            bv.render(cams, tf, c["step"], c["ert"], out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        s1 = bv.stats()
        up = (s1["bytes_uploaded"] - s0["bytes_uploaded"]) / steps
        res[label] = {
            "ms_per_frame": ms,
            "create_ms": create_ms,
            "passes_per_frame": (s1["passes"] - s0["passes"]) / steps,
            "bricks_occupied": s1["bricks_occupied"],
            "bricks_total": s1["bricks_total"],
            "pool_slots": s1["pool_slots"],
            "bytes_uploaded_per_frame": up,
            "upload_gb_per_s": up / (ms * 1e-3) / 1e9,
        }
        log(f"out of core {label}: {ms:.2f} ms/frame, {res[label]['passes_per_frame']:.1f} passes, "
            f"{up / 2**20:.1f} MiB uploaded per frame")
        del bv
    res["note"] = ("bricks = 64^3 blocks with their cubic-stencil apron (stored as 68^3 voxels); image bit-identical to the "
                   "in-core render with 64^3 skip blocks; frame time includes the occupancy readback, the host's "
                   "pass planning and the host-to-device brick copies")
    return res


def large_forward(vr, torch, np, synth, args):
    """The large forward: 1024^3 int16 (2 GiB, larger than the 256 MB MALL)
    to 2048^2, step 0.25, skip + ERT; effective gather and HBM-side bytes."""
    log("building the 1024^3 int16 phantom")
    c2 = synth.config_c2()
    vol2 = vr.Volume(torch.from_numpy(c2["volume"]).cuda())
    del c2["volume"]
    tf2 = vr.TF(torch.from_numpy(c2["tf"].table).cuda(), c2["tf"].v0, c2["tf"].v1)
    b2 = vr.vr_build_blocks(vol2, 16)
    cams2 = c2["cameras"]
    W2, H2 = cams2[0].width, cams2[0].height
    out2 = torch.empty((1, H2, W2, 4), dtype=torch.float32, device="cuda")
    ctr = torch.zeros(4, dtype=torch.int64, device="cuda")
    vr.vr_render(vol2, b2, cams2, tf2, c2["step"], c2["ert"], True, out=out2, counters=ctr)
    torch.cuda.synchronize()
    ev2 = int(ctr[0].item())

    def fwd2():
        vr.vr_render(vol2, b2, cams2, tf2, c2["step"], c2["ert"], True, out=out2)

    steps = max(3, args.steps // 4)
    wall, ev = time_steps(fwd2, steps, max(1, args.warmup // 2), torch)
    ms = wall / steps * 1e3
    gbs = ev2 * TAPS_BYTES_I16 / (float(np.mean(ev)) * 1e-3) / 1e9
    log(f"c2: {ms:.2f} ms/frame, {ev2 / (wall / steps):.4g} samples/s, {gbs:.0f} GB/s effective")
    res = {
        "workload": "c2_ct1024cube_i16_to_2048x2048_persp60_step0.25_skip16_ert0.99",
        "ms_per_step": ms,
        "kernel_ms": float(np.mean(ev)),
        "samples_per_s": ev2 / (wall / steps),
        "rays_per_s": W2 * H2 / (wall / steps),
        "evaluated_samples_per_frame": ev2,
        "lattice_samples_per_frame": int(ctr[1].item()),
        "effective_gather_gb_per_s": gbs,
        "roofline_frac": gbs / HBM_PEAK_GBS,
    }
    del vol2, b2, out2
    torch.cuda.empty_cache()
    return res


def gigavoxel(vr, torch, synth, c, args):
    """A 512x512x5382 int16 CT phantom (1.41e9 voxels, 2.8 GB) rendered out of
    core to 1024^2 (TF1, step 0.5, ERT 0.99) through a 1 GiB brick pool."""
    dims = (512, 512, 5382)
    log("building the 512x512x5382 int16 phantom")
    t0 = time.perf_counter()
    vol = synth.ct_phantom_i16(*dims, seed=12)
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    bv = vr.BrickedVolume(vol, 64, 1 << 30)
    create_s = time.perf_counter() - t0
    del vol
    tf = vr.TF(torch.from_numpy(c["tf"].table).cuda(), c["tf"].v0, c["tf"].v1)
    cams = synth.orbit_cameras(dims, 1, 13, 60.0, 1024, 1024)
    out = torch.empty((1, 1024, 1024, 4), dtype=torch.float32, device="cuda")
    bv.render(cams, tf, 0.5, 0.99, out=out)
    torch.cuda.synchronize()
    s0 = bv.stats()
    steps = 3
    t0 = time.perf_counter()
    for _ in range(steps):
        bv.render(cams, tf, 0.5, 0.99, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    s1 = bv.stats()
    up = (s1["bytes_uploaded"] - s0["bytes_uploaded"]) / steps
    log(f"gigavoxel out of core: {ms:.1f} ms/frame, {(s1['passes'] - s0['passes']) / steps:.0f} passes, "
        f"{up / 2**30:.2f} GiB uploaded per frame, {s1['bricks_occupied']}/{s1['bricks_total']} bricks occupied")
    res = {
        "volume": list(dims), "volume_bytes": 2 * dims[0] * dims[1] * dims[2], "pool_bytes": 1 << 30,
        "ms_per_frame": ms, "passes_per_frame": (s1["passes"] - s0["passes"]) / steps,
        "bytes_uploaded_per_frame": up, "bricks_occupied": s1["bricks_occupied"], "bricks_total": s1["bricks_total"],
        "phantom_s": gen_s, "create_s": create_s,
    }
    del bv
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(
            f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the renderer runs on a single "
            "MI355X; sharding across GPUs is not implemented)",
            file=sys.stderr,
        )
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_2005_01442_amd as vr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log("building the 512x512x400 int16 phantom")
    c = synth.config_c1()
    cams = c["cameras"]
    W, H = cams[0].width, cams[0].height
    vol = vr.Volume(torch.from_numpy(c["volume"]).cuda())
    tf = vr.TF(torch.from_numpy(c["tf"].table).cuda(), c["tf"].v0, c["tf"].v1)

    # A1: block min/max, once per volume
    for _ in range(2):
        blocks = vr.vr_build_blocks(vol, 16)
    torch.cuda.synchronize()
    wall_b, ev_b = time_steps(lambda: vr.vr_build_blocks(vol, 16), 5, 1, torch)
    blocks = vr.vr_build_blocks(vol, 16)
    out = torch.empty((1, H, W, 4), dtype=torch.float32, device="cuda")

    # evaluated/lattice sample counts of the frame (instrumented run, untimed)
    ctr = torch.zeros(4, dtype=torch.int64, device="cuda")
    vr.vr_render(vol, blocks, cams, tf, c["step"], c["ert"], True, out=out, counters=ctr)
    torch.cuda.synchronize()
    evaluated, lattice_total, hit, unstaged = (int(x) for x in ctr.cpu().numpy()[:4])
    log(f"frame: evaluated {evaluated:.4g} samples, lattice {lattice_total:.4g}, hit rays {hit}, "
        f"unstaged {unstaged / max(evaluated, 1):.3f}")

    def fwd():
        vr.vr_render(vol, blocks, cams, tf, c["step"], c["ert"], True, out=out)

    wall, ev_ms = time_steps(fwd, args.steps, args.warmup, torch)
    ms_per_step = wall / args.steps * 1e3
    kern_ms = float(np.mean(ev_ms))
    kern_med, kern_p99 = stats_ms(ev_ms)
    value = evaluated / (wall / args.steps)
    rays = W * H / (wall / args.steps)
    gather_gbs = evaluated * TAPS_BYTES_I16 / (kern_med * 1e-3) / 1e9
    vol_bytes = 512 * 512 * 400 * 2
    img_bytes = W * H * 16
    compulsory = vol_bytes + img_bytes
    achieved_gbs = compulsory / (kern_med * 1e-3) / 1e9
    log(f"fwd: {ms_per_step:.3f} ms/frame wall, {kern_med:.3f} ms/launch median ({kern_p99:.3f} p99), "
        f"{value:.4g} samples/s, {gather_gbs:.1f} GB/s effective gather")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "c1_ct512x512x400_i16_to_1024x1024_persp60_step0.5_skip16_ert0.99",
            "volume": [512, 512, 400],
            "volume_dtype": "i16",
            "image": [W, H],
            "step": c["step"],
            "ert": c["ert"],
            "block_edge": 16,
            "pose_seed": 2,
            "volume_seed": 1,
        },
        "rays_per_s": rays,
        "evaluated_samples_per_frame": evaluated,
        "lattice_samples_per_frame": lattice_total,
        "hit_rays_per_frame": hit,
        "unstaged_sample_fraction": unstaged / max(evaluated, 1),
        "kernel_ms": kern_ms,
        "kernel_ms_median": kern_med,
        "kernel_ms_p99": kern_p99,
        "block_build_ms": float(np.mean(ev_b)),
    }
    probe = None if args.no_probe else hbm_probe(vr, torch)
    if probe:
        log(f"hbm probe: {probe['gb_per_s']:.0f} GB/s streaming read of {probe['bytes'] >> 30} GiB (best of "
            f"{probe['repeats']})")
    stored, traffic, valu_insts = None, None, None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            if tj.get("kernel_source_sha256") == kernel_source_hash():
                stored = tj
                traffic = tj.get("bytes_per_launch")
                valu_insts = tj.get("sq_insts_valu_per_launch")
        except Exception:
            stored = None
    result["roofline"] = {
        "bound": "hbm",
        "achieved": achieved_gbs,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved_gbs / HBM_PEAK_GBS,
        "traffic": traffic,
        "kernel": "k_render<kI16, unlit, B-spline> (+ k_tile_order, k_occupancy_planes: one vr_render)",
        "bytes_per_launch": compulsory,
        "bytes_definition": f"compulsory: the int16 volume read once ({vol_bytes} B) + the fp32 RGBA image "
                            f"written once ({img_bytes} B); time = median of the {args.steps} timed launches",
        "achievable_gb_per_s": probe["gb_per_s"] if probe else None,
        "frac_of_achievable": achieved_gbs / probe["gb_per_s"] if probe else None,
        "traffic_source": (f"stored: {os.path.relpath(args.traffic_json, ROOT)} (rocprofv3 --pmc FETCH_SIZE, "
                           "WRITE_SIZE per dispatch, scaled by a 1 GiB copy's readings), valid for the hashed "
                           "forward-kernel sources") if traffic else "none stored for the current kernel sources",
        "traffic_over_compulsory": traffic / compulsory if traffic else None,
        "traffic_gb_per_s": traffic / (kern_med * 1e-3) / 1e9 if traffic else None,
    }
    result["effective_gather"] = {
        "bytes_per_launch": evaluated * TAPS_BYTES_I16,
        "gb_per_s": gather_gbs,
        "over_achievable_hbm": gather_gbs / probe["gb_per_s"] if probe else None,
        "over_hbm_peak": gather_gbs / HBM_PEAK_GBS,
        "note": "evaluated samples x 64 taps x 2 B per launch / median launch time: the rate taps are "
                "gathered at; LDS value boxes, L1 and L2 serve most taps, so this is not HBM traffic",
    }
    if valu_insts:
        t_valu = valu_insts / VALU_WAVE_INSTS_PER_S * 1e3
        result["valu_ceiling"] = {
            "sq_insts_valu_per_launch": valu_insts,
            "min_ms_at_full_issue": t_valu,
            "frac": t_valu / kern_med,
            "derivation": "256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 VALU instruction (no packed FP32) "
                          "= 6.144e11 wave instructions/s; SQ_INSTS_VALU of one launch (stored with the traffic)",
        }

    result["c0"] = c0_plain(vr, torch, np, synth, args)
    log(f"c0: {result['c0']['kernel_ms_median'] * 1e3:.1f} us/frame median")

    if not args.no_lit:
        shade = vr.Shading(**synth.SHADE_CT)
        lit_ctr = torch.zeros(4, dtype=torch.int64, device="cuda")
        vr.vr_render(vol, blocks, cams, tf, c["step"], c["ert"], True, out=out, counters=lit_ctr, shading=shade)
        torch.cuda.synchronize()
        lit_eval = int(lit_ctr[0].item())

        def fwd_lit():
            vr.vr_render(vol, blocks, cams, tf, c["step"], c["ert"], True, out=out, shading=shade)

        wall_l, ev_l = time_steps(fwd_lit, args.steps, args.warmup, torch)
        ms_l = wall_l / args.steps * 1e3
        log(f"fwd lit: {ms_l:.3f} ms/frame wall, {float(np.mean(ev_l)):.3f} ms/launch events")
        result["c1_lit"] = {
            "ms_per_step": ms_l,
            "kernel_ms": float(np.mean(ev_l)),
            "samples_per_s": lit_eval / (wall_l / args.steps),
            "rays_per_s": W * H / (wall_l / args.steps),
            "evaluated_samples_per_frame": lit_eval,
            "shading": dict(synth.SHADE_CT),
            "note": "same frame with local lighting: gradient of the cubic reconstruction from the same 64 taps, "
                    "two-sided Blinn-Phong; opacity and samples as the unlit frame",
        }

    if not args.no_preint:
        result["c1_preint"] = preint_measurements(vr, torch, np, synth, c, vol, blocks, cams, tf, out, args)

    if not args.no_filters:
        def fwd_cr():
            vr.vr_render(vol, blocks, cams, tf, c["step"], c["ert"], True, out=out, filter=vr.VR_FILTER_CATMULL_ROM)

        wall_cr, ev_cr = time_steps(fwd_cr, args.steps, args.warmup, torch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        coef = vr.vr_prefilter_bspline(vol)
        torch.cuda.synchronize()
        pre_ms = (time.perf_counter() - t0) * 1e3
        cblocks = vr.vr_build_blocks(coef, 16)

        def fwd_interp():
            vr.vr_render(coef, cblocks, cams, tf, c["step"], c["ert"], True, out=out)

        wall_ip, ev_ip = time_steps(fwd_interp, args.steps, args.warmup, torch)

        def fwd_pre():
            vr.vr_render(vol, blocks, cams, tf, c["step"], c["ert"], True, out=out,
                         filter=vr.VR_FILTER_BSPLINE_PRECLASSIFIED)

        wall_pc, ev_pc = time_steps(fwd_pre, args.steps, args.warmup, torch)
        result["c1_filters"] = {
            "catmull_rom_ms": wall_cr / args.steps * 1e3,
            "interpolating_bspline_ms": wall_ip / args.steps * 1e3,
            "prefilter_ms": pre_ms,
            "preclassified_ms": wall_pc / args.steps * 1e3,
            "note": "same frame; Catmull-Rom with widened block ranges; interpolating cubic B-spline = prefiltered "
                    "fp32 coefficient volume (256 B of taps per sample) rendered with the default filter",
        }
        log(f"filters: Catmull-Rom {wall_cr / args.steps * 1e3:.3f} ms, interpolating B-spline "
            f"{wall_ip / args.steps * 1e3:.3f} ms (+ prefilter {pre_ms:.2f} ms once), pre-classified "
            f"{wall_pc / args.steps * 1e3:.3f} ms")
        del coef, cblocks

    if not args.no_bricked:
        result["c1_out_of_core"] = bricked_measurements(vr, torch, np, c, cams, tf, out, args)

    if not args.no_c2:
        result["c2_large"] = large_forward(vr, torch, np, synth, args)

    if args.gigavoxel:
        result["gigavoxel_out_of_core"] = gigavoxel(vr, torch, synth, c, args)

    if not args.no_bwd:
        gv_holder = {}

        def fwd_bwd():
            img = vr.vr_render(vol, blocks, cams, tf, c["step"], c["ert"], True, out=out)
            gv_holder["g"] = vr.vr_render_backward(vol, blocks, cams, tf, c["step"], c["ert"], True, img, img)

        wall_fb, ev_fb = time_steps(fwd_bwd, args.bwd_steps, 1, torch)
        ms_fb = wall_fb / args.bwd_steps * 1e3
        med_fb, p99_fb = stats_ms(ev_fb)
        result["fwd_bwd"] = {
            "ms_per_step": ms_fb,
            "ms_median": med_fb,
            "ms_p99": p99_fb,
            "samples_per_s": lattice_total / (ms_fb * 1e-3),
            "rays_per_s": W * H / (ms_fb * 1e-3),
            "note": "forward (skip+ERT) + adjoint to grid (fp32) and TF; samples counted as lattice samples "
                    "because the TF gradient disables skipping in the adjoint",
        }
        log(f"fwd+bwd: {ms_fb:.3f} ms/step")
        del gv_holder

    if not args.no_c3:
        log("differentiable 256^3 fp32, 64 views of 512^2")
        result["c3_fwd_bwd"] = differentiable_c3(vr, torch)
        log(f"c3: fwd {result['c3_fwd_bwd']['fwd_ms']:.2f} ms, fwd+bwd {result['c3_fwd_bwd']['fwd_bwd_ms']:.2f} ms")

    if not args.no_serve:
        log("serving mix")
        result["serve"] = serve_mix(vr, torch, args.serve_requests, args.serve_warmup, args.serve_rate)
        result["p99_ms"] = result["serve"]["p99_ms"]
        log(f"serve: p50 {result['serve']['p50_ms']:.2f} ms, p99 {result['serve']['p99_ms']:.2f} ms")

    if not args.no_cpu:
        import oracle

        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(c, args.cpu_seconds, args.cpu_single_seconds)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
