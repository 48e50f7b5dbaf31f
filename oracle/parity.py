"""Parity checks of GPU results against the FP64 oracle (test infrastructure only).

Images: every channel within `tol` of the oracle.  A pixel that misses is accepted only if the
oracle marked one of its discrete decisions as within the FP32/FP64 margin (cutoff membership,
alpha_min skip, transmittance stop, depth order of two contributors, a cull) and the GPU value
matches one of the results of taking those decisions either way (at most `max_marks` of them;
more is reported as unverified).

Gradients: relative L2 error per parameter group.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np


def check_image(gpu_rgb: np.ndarray, frame, tol: float = 1e-4, xy: Optional[np.ndarray] = None,
                max_marks: int = 4, ref=None, channels: str = "rgb", rel_tol: float = 0.0) -> Dict:
    """gpu_rgb: [C, H, W] (full image) or [n, C] at the pixels xy, C = 3 for channels="rgb" or
    the frame's extra channels for channels="ext".  An element agrees when
    |gpu - oracle| <= tol + rel_tol |oracle|."""
    if ref is None:
        ref = frame.render(xy)
    key, vi = ("rgb", 0) if channels == "rgb" else ("ext", 2)
    nc = 3 if channels == "rgb" else frame.n_ext
    if xy is None:
        g = np.asarray(gpu_rgb, np.float64).reshape(nc, -1).T
        r = ref[key].reshape(nc, -1).T
        marks = ref["n_marks"].reshape(-1)
        W = frame.width
        coords = np.stack([np.arange(g.shape[0]) % W, np.arange(g.shape[0]) // W], 1)
    else:
        g = np.asarray(gpu_rgb, np.float64).reshape(-1, nc)
        r = ref[key]
        marks = ref["n_marks"]
        coords = np.asarray(xy).reshape(-1, 2)
    lim = tol + rel_tol * np.abs(r)
    err = (np.abs(g - r) / lim).max(1) * tol if len(r) else np.zeros(0)
    bad = np.nonzero(err > tol)[0]
    resolved, unverified, failures = 0, 0, []
    for p in bad:
        if marks[p] == 0:
            failures.append((int(coords[p][0]), int(coords[p][1]), float(err[p]), "unmarked"))
            continue
        var = frame.variants(int(coords[p][0]), int(coords[p][1]), max_marks)
        if var is None:
            unverified += 1
            continue
        vv = var[vi]
        if (np.abs(vv - g[p]) <= tol + rel_tol * np.abs(vv)).all(1).any():
            resolved += 1
        else:
            failures.append((int(coords[p][0]), int(coords[p][1]), float(err[p]), "no variant"))
    ok = np.ones(len(err), bool)
    ok[bad] = False
    return dict(n=len(err), max_err=float(err.max()) if len(err) else 0.0,
                max_err_agreeing=float(err[ok].max()) if ok.any() else 0.0,
                n_marked=int((marks > 0).sum()), n_bad=int(len(bad)), n_resolved=resolved,
                n_unverified=unverified, failures=failures[:20], n_failures=len(failures))


def check_counts(gpu_counts: np.ndarray, gpu_rgb: np.ndarray, frame, xy: np.ndarray, ref,
                 tol: float = 1e-4, max_marks: int = 4) -> Dict:
    """Composited-pair counts at the pixels xy ([n, 2]) against the oracle's, exactly.  An
    unmarked pixel must have the oracle's count.  A marked pixel must have the count of one of
    the oracle's variants (its marked decisions taken either way) whose color also agrees with
    the GPU's within tol; with more than max_marks marks it is reported as unverified."""
    gpu_counts = np.asarray(gpu_counts).reshape(-1)
    g = np.asarray(gpu_rgb, np.float64).reshape(-1, 3)
    marks = ref["n_marks"]
    clean = marks == 0
    exact = clean & (gpu_counts == ref["n_contrib"])
    failures = [(int(xy[p][0]), int(xy[p][1]), int(gpu_counts[p]), int(ref["n_contrib"][p]),
                 "unmarked") for p in np.nonzero(clean & ~exact)[0]]
    by_variant, unverified = 0, 0
    for p in np.nonzero(~clean)[0]:
        var = frame.variants(int(xy[p][0]), int(xy[p][1]), max_marks)
        if var is None:
            unverified += 1
            continue
        ok = (np.abs(var[0] - g[p]) <= tol).all(1) & (var[3] == gpu_counts[p])
        if ok.any():
            by_variant += 1
        else:
            failures.append((int(xy[p][0]), int(xy[p][1]), int(gpu_counts[p]),
                             int(ref["n_contrib"][p]), "no variant"))
    n = len(gpu_counts)
    return dict(n=n, n_clean=int(clean.sum()), n_exact=int(exact.sum()), n_by_variant=by_variant,
                n_unverified=unverified, verified_frac=(int(exact.sum()) + by_variant) / max(n, 1),
                failures=failures[:20], n_failures=len(failures))


def grad_rel_errors(gpu: Dict[str, np.ndarray], ref: Dict[str, np.ndarray]) -> Dict[str, float]:
    """Relative L2 error of every group the GPU computed (each must exist in ref)."""
    out = {}
    for k in gpu:
        g = np.asarray(gpu[k], np.float64).reshape(-1)
        r = np.asarray(ref[k], np.float64).reshape(-1)
        nr = np.linalg.norm(r)
        out[k] = float(np.linalg.norm(g - r) / nr) if nr > 0 else float(np.linalg.norm(g))
    return out
