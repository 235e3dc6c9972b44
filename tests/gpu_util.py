"""Helpers shared by the GPU tests: upload seeded inputs, compare with the
oracle.  Imported only by tests marked ``gpu``."""

import sys

import numpy as np
import torch

import paper_2005_01442_amd as vr

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def upload_volume(vol_np):
    if vol_np.dtype == np.uint16:
        t = torch.from_numpy(np.ascontiguousarray(vol_np).view(np.int16)).to(DEV)
        return vr.Volume(t, dtype=vr.VR_U16)
    return vr.Volume(torch.from_numpy(np.ascontiguousarray(vol_np)).to(DEV))


def upload_tf(tf):
    return vr.TF(torch.from_numpy(np.ascontiguousarray(tf.table)).to(DEV), tf.v0, tf.v1)


def gpu_render(cfg_vol, cams, tf, step, ert=0.0, use_skip=False, block_edge=16, counters=False, vol=None,
               blocks=None):
    vol = vol if vol is not None else upload_volume(cfg_vol)
    t = upload_tf(tf)
    if use_skip and blocks is None:
        blocks = vr.vr_build_blocks(vol, block_edge)
    ctr = torch.zeros(4, dtype=torch.int64, device=DEV) if counters else None
    out = vr.vr_render(vol, blocks if use_skip else None, cams, t, step, ert, use_skip, counters=ctr)
    torch.cuda.synchronize()
    img = out.cpu().numpy().astype(np.float64)
    return (img, ctr.cpu().numpy()) if counters else img


def compare_with_flags(gpu, ref, flags, theta, tol=2e-4):
    """Unflagged pixels within tol; pixels the oracle flags as termination
    ties within (1 - theta) + tol.  Returns (max unflagged diff, n flagged)."""
    diff = np.abs(gpu - ref).max(axis=-1)
    fl = flags.astype(bool)
    un = diff[~fl]
    assert un.size == 0 or un.max() <= tol, f"max |dRGBA| {un.max():.3e} > {tol} on unflagged pixels"
    if fl.any():
        assert diff[fl].max() <= (1.0 - theta) + tol
    return (float(un.max()) if un.size else 0.0), int(fl.sum())
