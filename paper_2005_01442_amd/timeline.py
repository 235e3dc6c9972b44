"""Per-wavefront-item timeline of the whole-image kernels on the C1 frame.

A diagnostics build of the library (``libvr_timeline.so``, compiled with
VR_TIMELINE) records for every wavefront item (8x4 rays) of the last forward
(``k_render``) or adjoint (``k_render_bwd``) launch its start and end on the
100 MHz constant clock, its super-tile and its work (see
include/vr_timeline.h).  This script renders the C1 frame (512x512x400 int16
CT phantom -> 1024^2, step 0.5, 16^3 block skipping, early termination at
0.99) with that build and prints a summary: makespan, wave-slot efficiency,
the per-XCD ends (workgroup item i belongs to XCD i mod 8's queue), the
concurrency over time and the last items to finish.

Run it by path (the package must not be imported first, so that it loads the
diagnostics build):

    python3 paper_2005_01442_amd/timeline.py --build          # on the CPU: compile libvr_timeline.so
    python3 paper_2005_01442_amd/timeline.py [--adjoint] [--save out.npy]   # on the GPU
"""

from __future__ import annotations

import argparse
import ctypes
import importlib.util
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TIMELINE_LIB = os.path.join(HERE, "libvr_timeline.so")
TICK_S = 1e-8  # s_memrealtime: 100 MHz


def build_library() -> str:
    spec = importlib.util.spec_from_file_location("_vr_build", os.path.join(HERE, "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b.build(extra=["-DVR_TIMELINE"], out=TIMELINE_LIB)


def summary(rec, slots: int, what: str) -> str:
    import numpy as np

    rec = np.asarray(rec, dtype=np.int64)
    t0 = rec[:, 0].min()
    s, e = rec[:, 0] - t0, rec[:, 1] - t0
    d = e - s
    work = rec[:, 3]
    wg = np.arange(len(rec)) // 4
    xcd = wg % 8
    mk = int(e.max())
    busy = d > 1000  # 10 us: wavefronts that marched samples
    lines = [f"### {what}", ""]
    lines.append(f"wavefronts {len(rec):,}, with work {int(busy.sum()):,}; makespan {mk:,} ticks = {mk * TICK_S * 1e3:.3f} ms")
    lines.append(f"wave slots {slots:,}: mean busy time per slot {d.sum() / slots:,.0f} ticks, slot efficiency "
                 f"{d.sum() / slots / mk * 100:.1f} %")
    if busy.any():
        p = np.percentile(d[busy], [50, 90, 99, 100]).astype(int)
        lines.append(f"durations of wavefronts with work (ticks): median {p[0]:,}, p90 {p[1]:,}, p99 {p[2]:,}, max {p[3]:,}")
    lines.append("")
    lines.append("| XCD | last end (ticks) | busy ticks per slot |")
    lines.append("|---|---|---|")
    for x in range(8):
        m = xcd == x
        lines.append(f"| {x} | {int(e[m].max()):,} | {d[m].sum() / (slots / 8):,.0f} |")
    lines.append("")
    edges = np.linspace(0, mk, 13)
    conc = [int(((s < b1) & (e > b0) & busy).sum()) for b0, b1 in zip(edges[:-1], edges[1:])]
    lines.append("wavefronts with work resident at some time in each twelfth of the launch: " + ", ".join(str(c) for c in conc))
    last = np.argsort(e)[::-1][:5]
    lines.append("last to finish (record, start, duration in ticks, work): " +
                 "; ".join(f"{int(i)}: {int(s[i]):,}, {int(d[i]):,}, {int(work[i]):,}" for i in last))
    lines.append("")
    return "\n".join(lines)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--build", action="store_true", help="compile libvr_timeline.so and exit")
    ap.add_argument("--adjoint", action="store_true", help="also the adjoint (grid + TF gradient) of the frame")
    ap.add_argument("--save", default=None, help="save the records (.npy, forward then adjoint)")
    args = ap.parse_args()
    if args.build:
        print(build_library())
        return 0
    if not os.path.exists(TIMELINE_LIB):
        raise SystemExit(f"{TIMELINE_LIB} is missing: run this script with --build first")
    os.environ["VR_LIBRARY"] = TIMELINE_LIB
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch

    import synth
    import paper_2005_01442_amd as vr
    from paper_2005_01442_amd import _abi

    c = synth.config_c1()
    cams = c["cameras"]
    vol = vr.Volume(torch.from_numpy(c["volume"]).cuda())
    tf = vr.TF(torch.from_numpy(c["tf"].table).cuda(), c["tf"].v0, c["tf"].v1)
    blocks = vr.vr_build_blocks(vol, 16)
    img = torch.empty((1, 1024, 1024, 4), dtype=torch.float32, device="cuda")

    def read(kind):
        buf = np.zeros((1 << 17) * 4, dtype=np.uint64)
        n = ctypes.c_uint64(0)
        _abi.check(_abi.lib().vr_timeline_read(kind, buf.ctypes.data, 1 << 17, ctypes.byref(n)))
        return buf.reshape(-1, 4)[: min(int(n.value), 1 << 17)]

    for _ in range(4):
        vr.vr_render(vol, blocks, cams, tf, c["step"], c["ert"], True, out=img)
    fwd = read(0)
    print(summary(fwd, 256 * 12, "forward, k_render<int16> (C1 frame)"), flush=True)
    out = [fwd]
    if args.adjoint:
        for _ in range(2):
            vr.vr_render_backward(vol, blocks, cams, tf, c["step"], c["ert"], True, img, img)
        bwd = read(1)
        print(summary(bwd, 256 * 8, "adjoint, k_render_bwd<int16> (C1 frame, grid + TF gradient, dL/dRGBA = the image)"),
              flush=True)
        out.append(bwd)
    if args.save:
        np.save(args.save, np.concatenate(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
