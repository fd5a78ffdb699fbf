"""Helpers shared by the GPU parity tests: run the HIP path, map its outputs to
oracle terms, and compare with the oracle's margin-aware alternatives."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_2403_11577_amd import pipeline as pl

ALPHA_T_TOL = 1e-4   # absolute per channel (and on T_final)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_settings():
    return oracle.Settings()


def gpu_render(scene, tile=(16, 16), batch=64, persistent=True, views=None, w2c=None, xi=None, delta=None, roi_y0=0,
               split_len=0, split_fwd=0):
    """Run the batched HIP forward on a scene; returns dict of numpy outputs plus the frame."""
    ds = pl.DeviceScene.from_scene(scene, views=views)
    xi_t = torch.as_tensor(scene.xi if xi is None else xi, dtype=torch.float64, device="cuda")
    dl_t = torch.as_tensor(scene.delta if delta is None else delta, dtype=torch.float64, device="cuda")
    w2c_t = None if w2c is None else torch.as_tensor(np.ascontiguousarray(w2c), dtype=torch.float64, device="cuda")
    st = pl.make_settings(tile=tile, batch=batch, persistent=persistent, roi_y0=roi_y0, split_len=split_len,
                          split_fwd=split_fwd)
    fr = pl.fit_frame(ds, xi_t, dl_t, st, w2c=w2c_t)
    fr.clear_status()
    img, T, last = pl.forward(fr, ds, xi_t, dl_t, w2c=w2c_t)
    torch.cuda.synchronize()
    ns, ni = fr.counts()
    vals = fr.sorted_vals(ni).cpu().numpy().astype(np.int64)
    meta = fr.meta(ns).cpu().numpy()
    lastp = last.cpu().numpy().astype(np.int64)
    gid = np.full(lastp.shape, -1, np.int64)
    m = lastp >= 0
    gid[m] = meta[vals[lastp[m]], 0]
    return dict(img=img.cpu().numpy().astype(np.float64), T=T.cpu().numpy().astype(np.float64),
                last_pos=lastp, last_id=gid, frame=fr, ds=ds, xi=xi_t, delta=dl_t,
                status=fr.status(), slots=ns, inst=ni, w2c=fr.w2c.cpu().numpy())


def use_instance_sort(fr):
    """Switch a frame's plan from the slot-first bin sort to one 64-bit key per instance (always
    allowed), with the sorted-buffer and key-shift fields of that sort; the library checks them."""
    p = fr.plan
    bits = int(p.depth_bits) + int(p.tile_bits)
    rb = int(p.radix_bits)
    passes = (bits + rb - 1) // rb
    ks = -1
    for ps in range(passes - 1):
        s1 = rb * (ps + 1)
        if s1 <= int(p.depth_bits) and bits - s1 <= 32:
            ks = s1
            break
    p.slot_sort, p.sorted_buf, p.key_shift = 0, passes & 1, ks


def compare_images(gpu, orc, tol=ALPHA_T_TOL):
    """Per-pixel comparison with the oracle's alternatives at flagged decisions.

    Returns (n_bad, n_flagged, n_excluded, max_err_unflagged)."""
    img, T, lid = gpu["img"], gpu["T"], gpu["last_id"]
    oimg, oT, olid = orc["img"], orc["T"], orc["last"]
    nflag = orc["nflag"]
    err = np.abs(img - oimg).max(axis=1)
    errT = np.abs(T - oT)
    plain = nflag == 0
    bad = plain & ((err > tol) | (errT > tol) | (lid != olid))
    max_plain = float(err[plain].max()) if plain.any() else 0.0
    flagged = np.argwhere((nflag >= 1) & (nflag <= 2))
    nbad = int(bad.sum())
    for v, y, x in flagged:
        na = int(orc["nalt"][v, y, x])
        ok = False
        for a in range(na):
            alt = orc["alt"][v, y, x, a]
            if (np.abs(img[v, :, y, x] - alt[:3]).max() <= tol and abs(T[v, y, x] - alt[3]) <= tol
                    and lid[v, y, x] == int(alt[4])):
                ok = True
                break
        nbad += 0 if ok else 1
    return nbad, int(flagged.shape[0]), int((nflag > 2).sum()), max_plain


def rel_close(a, b, rtol, floor_frac=1e-2):
    """C19: per tensor ||a-b|| <= rtol ||b|| and per element |a-b| <= rtol max(|b|, floor_frac max|b|)."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    if nb == 0:
        return float(np.abs(a).max()) == 0.0, 0.0
    tens = np.linalg.norm(a - b) / nb
    floor = floor_frac * np.abs(b).max()
    el = (np.abs(a - b) / np.maximum(np.abs(b), floor)).max()
    return bool(tens <= rtol and el <= rtol), float(max(tens, el))
