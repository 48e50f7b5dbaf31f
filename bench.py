"""Benchmark: batched forward + backward of the differentiable 4D Gaussian render on one GPU.

A step is one pass of the whole hot path over one batch of views: preprocess (slice, splat,
4DSH color) of every (Gaussian, view), visible compaction, depth sort, key generation, tile
sort, tile ranges, forward raster, backward raster and preprocess backward, with a fixed
synthetic upstream gradient dL/dimage.  The default workload is 300k Gaussians rendered in
16 views (8 ring cameras x 2 times, 1352x1014 and 800x800).  Inputs are resident in HBM
before timing starts.  One JSON line is printed (rank 0).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Mpix/s at 300k 4D Gaussians, 1352x1014; batched vs per-view launch"
PEAK_FP32_VALU = 157.3e12   # MI355X published FP32 vector peak (FLOP/s)
PEAK_HBM = 8.0e12           # MI355X HBM3E (B/s)
# Algorithmic FP32 work per (Gaussian, pixel) pair, counted from the per-pair arithmetic (an
# FMA counts 2).  Every evaluated pair (within the cutoff, visited before the pixel's stop) costs
# the test: offsets 2, quadratic form 7, exp(-d2/2) 2, alpha 1.  A composited pair adds, in the
# forward, transmittance 2, weight 1 and the color FMAs 6 (21 in all); in the backward, the
# transmittance rebuild 2, weight 1, dL/dc 6, g.c 5, g.c - g.R 1, g.R update 2, dL/dalpha 1,
# alpha dL/dalpha 1, opacity partial 2, dL/du and dL/dv 10, conic moments 8 (51 in all).
FLOPS_PER_EVALUATED = 12
FWD_FLOPS_PER_COMPOSITED = 9
BWD_FLOPS_PER_COMPOSITED = 39
# The per-pair figures of the hot-path scope table, charged to every candidate within the
# plain cutoff that a pixel visits before its stop (E_alg, counted on the GPU by a forward that
# bins by the cutoff): about 20 flops + 1 exp forward and 60 flops + 1 exp + 1 rcp backward.
# They charge the full adjoint to candidates that fail alpha_min (which the kernels skip after
# the 12-flop test), so they overstate the work the kernels must do; both are reported.
ALG_FLOPS_FWD = 20
ALG_FLOPS_BWD = 60
WORKLOAD_KEYS = {"0": 0, "1": 1, "2": 2, "2b": "2b", "3": 3, "4": 4}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _code_only(text):
    """C++ source with its comments removed and whitespace runs collapsed, so that an edit to
    a comment leaves the hash of the code unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def raster_source_hash():
    """Hash of the raster kernel's code (comments excluded) that the counter summaries were
    taken with."""
    import hashlib
    h = hashlib.sha256()
    for f in ("k_raster.hip", "g4d_device.h", "g4d_internal.h"):
        text = open(os.path.join(ROOT, "paper_2412_20720_amd", "csrc", f)).read()
        h.update(_code_only(text).encode())
    return h.hexdigest()[:16]


def profiled_traffic(workload_name, settings):
    """HBM bytes per raster_bwd launch from the committed counter summary, if it was taken on
    this workload and launch configuration with the current raster source (else None)."""
    path = os.path.join(ROOT, "profiles", "raster_bwd_w2_traffic.md")
    if workload_name != "w2_300k_16views_mixed" or not os.path.exists(path):
        return None
    lines = open(path).read().splitlines()
    fields = dict(l.split(": ", 1) for l in lines if ": " in l)
    if fields.get("source-hash") != raster_source_hash():
        return None
    key = (f"raster_bwd-traffic-bytes tile={settings.tile_size} batch={settings.lds_batch} "
           f"bwd_px={backward_px(settings)}")
    return int(fields[key]) if key in fields else None


def backward_px(settings):
    """Pixels per lane the backward raster runs with (the library's default when 0)."""
    if settings.bwd_px_per_lane:
        return settings.bwd_px_per_lane
    px = settings.px_per_lane or (1 if settings.tile_size == 8 else 4)
    return 8 if settings.tile_size == 32 and px == 4 else px


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="2", choices=sorted(WORKLOAD_KEYS))
    ap.add_argument("--tile", type=int, default=0, help="tile size (0: autotune)")
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--px", type=int, default=4)
    ap.add_argument("--bwd-px", type=int, default=0, help="backward pixels per lane (0: default)")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=1)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--channels", type=int, default=32, metavar="D",
                    help="also time the render with D feature channels + depth + flow "
                         "(-1: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2412_20720_amd import _binding as B
    from paper_2412_20720_amd import scenes
    from paper_2412_20720_amd.frontend import Renderer

    dev = torch.device("cuda", 0)
    sc = scenes.make_workload(WORKLOAD_KEYS[args.workload])
    log(f"bench: workload {sc.name}: N={sc.n}, {len(sc.views)} views, {sc.pixels / 1e6:.2f} Mpix")
    r = Renderer(0)
    p = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in sc.arrays().items()}
    names = ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh")
    g = r.gaussians(*[p[k] for k in names], sc.sh_degree, sc.t_degree)
    settings = B.default_settings(time_period=sc.time_period, tile_size=args.tile or 16,
                                  lds_batch=args.batch, px_per_lane=args.px,
                                  bwd_px_per_lane=args.bwd_px)
    views = B.make_views(sc.views)
    npix = sc.pixels
    rgb = torch.empty(3 * npix, device=dev)
    T = torch.empty(npix, device=dev)
    dL = torch.from_numpy(np.concatenate([d.reshape(-1) for d in scenes.make_dl_dimage(sc)])).to(dev)
    grads = {k: torch.empty_like(p[k]) for k in names}

    def step():
        r.forward(g, views, settings, rgb, T)
        r.backward(g, views, settings, dL, grads)

    tuned_ms = None
    if args.tile == 0:
        tuned_ms = r.autotune(g, views, settings, dL, rgb, T, grads, reps=2)
        log(f"bench: autotuned tile {settings.tile_size}, LDS batch {settings.lds_batch}, "
            f"pixels/lane {settings.px_per_lane}, backward {backward_px(settings)} ({tuned_ms:.2f} ms)")

    # Work counts of this workload (untimed, counted by the forward kernel itself).
    r.eval_counters(True)
    r.forward(g, views, settings, rgb, T)
    cnt = r.eval_counters(False, npix).cpu().numpy().astype(np.int64)
    stats = r.stats()
    evals = int((cnt & 0xFFFF).sum())
    contrib = int((cnt >> 16).sum())
    log(f"bench: visible {stats['n_visible']}, pairs {stats['n_pairs']}, evaluated pairs {evals}, "
        f"composited pairs {contrib}")
    # E_alg: every candidate within the plain cutoff visited before the stop (the splats are
    # binned by the cutoff for this one untimed forward; the image is the same).
    r.eval_counters(2)
    r.forward(g, views, settings, rgb, T)
    cnt = r.eval_counters(False, npix).cpu().numpy().astype(np.int64)
    e_alg = int((cnt & 0xFFFF).sum())
    if int((cnt >> 16).sum()) != contrib:
        raise RuntimeError("composited pairs differ between the reach and cutoff binnings")
    log(f"bench: candidates within the cutoff up to the stop (E_alg) {e_alg}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # The timed steps record events around the two raster kernels only (the roofline's
    # kernels; each recorded stage idles the GPU briefly between kernels).
    r.profile_mask(["raster_fwd", "raster_bwd"])
    r.profile(True, collect=True, reset=True)   # start stage timing from zero
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    stages = r.profile(False, collect=True, reset=True)
    r.sync()
    value = npix / dt / 1e6
    log(f"bench: batched {dt * 1e3:.3f} ms/step, {value:.1f} Mpix/s")
    timed_ms = {k: v[0] / max(1, v[1]) for k, v in stages.items() if v[1] > 0}
    # Every stage, from a separate (untimed) pass of the same step.
    r.profile_mask(None)
    r.profile(True, collect=True, reset=True)
    for _ in range(max(1, min(args.steps, 5))):
        step()
    stages = r.profile(False, collect=True, reset=True)
    r.sync()
    stage_ms = {k: v[0] / max(1, v[1]) for k, v in stages.items() if v[1] > 0}
    for k, v in stage_ms.items():
        log(f"  {k:15s} {v:8.3f} ms/launch")

    graph = None
    if not args.no_graph:
        # The same step captured once into a hipGraph and replayed (no host sync per step).
        for _ in range(args.warmup):
            r.step(g, views, settings, dL, rgb, T, grads, graph=True, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r.step(g, views, settings, dL, rgb, T, grads, graph=True, check=False)
        torch.cuda.synchronize()
        dg = (time.perf_counter() - t0) / args.steps
        r.sync()
        graph = dict(value=npix / dg / 1e6, ms_per_step=dg * 1e3)
        log(f"bench: graph replay {dg * 1e3:.3f} ms/step, {npix / dg / 1e6:.1f} Mpix/s")

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy calibration {args.copy_calibration} MiB read + written")

    per_view = None
    if not args.no_per_view:
        single = [B.make_views([v]) for v in sc.views]
        offs = np.cumsum([0] + [v["width"] * v["height"] for v in sc.views])

        def step_pv():
            for k, va in enumerate(single):
                a, b = int(offs[k]), int(offs[k + 1])
                r.forward(g, va, settings, rgb[3 * a:3 * b], T[a:b])
                r.backward(g, va, settings, dL[3 * a:3 * b], grads)

        for _ in range(args.warmup):
            step_pv()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step_pv()
        torch.cuda.synchronize()
        dpv = (time.perf_counter() - t0) / args.steps
        per_view = dict(value=npix / dpv / 1e6, ms_per_step=dpv * 1e3,
                        batched_speedup=dpv / dt)
        log(f"bench: per-view {dpv * 1e3:.3f} ms/step, {npix / dpv / 1e6:.1f} Mpix/s")

    chan = None
    if args.channels >= 0:
        chan = channel_step(r, g, views, settings, sc, p, dL, args, npix)
    train = training_step(r, views, settings, sc, p, dL, args, npix)
    sky = sky_step(r, g, views, settings, sc, dL, args, npix)
    compact = compact_forward(r, views, settings, sc, args, npix)

    # Roofline of the dominant kernel (largest time per step), from the live HIP events: the
    # scope table's per-pair figure over E_alg, and beside it the itemised count of the
    # arithmetic each evaluated and composited pair needs.
    dom = max(("raster_fwd", "raster_bwd"), key=lambda k: timed_ms.get(k, 0.0))
    sec = timed_ms[dom] * 1e-3
    per_pair = ALG_FLOPS_BWD if dom == "raster_bwd" else ALG_FLOPS_FWD
    flops_alg = per_pair * e_alg
    per_comp = BWD_FLOPS_PER_COMPOSITED if dom == "raster_bwd" else FWD_FLOPS_PER_COMPOSITED
    flops = FLOPS_PER_EVALUATED * evals + per_comp * contrib
    traffic = profiled_traffic(sc.name, settings) if dom == "raster_bwd" else None
    roofline = dict(kernel=dom, bound="alu", achieved=flops_alg / sec / 1e12,
                    peak=PEAK_FP32_VALU / 1e12, unit="TFLOP/s",
                    frac=flops_alg / sec / PEAK_FP32_VALU, traffic=traffic,
                    units={"e_alg_pairs": e_alg}, flops_per_unit={"pair": per_pair},
                    flops_per_launch=flops_alg, ms_per_launch=timed_ms[dom],
                    itemised=dict(achieved=flops / sec / 1e12, frac=flops / sec / PEAK_FP32_VALU,
                                  units={"evaluated_pairs": evals, "composited_pairs": contrib},
                                  flops_per_unit={"evaluated_pair": FLOPS_PER_EVALUATED,
                                                  "composited_pair_extra": per_comp},
                                  flops_per_launch=flops))

    # Whole-path bound from the raster arithmetic alone at the FP32 VALU peak: the scope
    # table's 80 flops per E_alg pair (forward + backward), and the itemised count.
    bound_s = (ALG_FLOPS_FWD + ALG_FLOPS_BWD) * e_alg / PEAK_FP32_VALU
    bound_i = (2 * FLOPS_PER_EVALUATED * evals +
               (FWD_FLOPS_PER_COMPOSITED + BWD_FLOPS_PER_COMPOSITED) * contrib) / PEAK_FP32_VALU
    alg_bound = dict(mpix_s=npix / bound_s / 1e6, frac=bound_s / dt, e_alg_per_px=e_alg / npix,
                     itemised=dict(mpix_s=npix / bound_i / 1e6, frac=bound_i / dt),
                     evaluated_pairs_per_px=evals / npix, composited_pairs_per_px=contrib / npix)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sc, args.cpu_views)

    out = {
        "metric": METRIC, "value": value, "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": sc.name, "gaussians": sc.n, "views": len(sc.views),
                   "pixels": npix, "sh_degree": sc.sh_degree, "t_degree": sc.t_degree,
                   "tile": settings.tile_size, "lds_batch": settings.lds_batch,
                   "px_per_lane": settings.px_per_lane, "bwd_px_per_lane": backward_px(settings),
                   "autotuned": args.tile == 0},
        "per_view": per_view,
        "graph": graph,
        "roofline": roofline,
        "alg_bound": alg_bound,
        "channels": chan,
        "training_fusion": train,
        "sky": sky,
        "compact": compact,
        "cpu_baseline": cpu,
        "work": {"visible_slots": stats["n_visible"], "pairs": stats["n_pairs"],
                 "e_alg_pairs": e_alg, "evaluated_pairs": evals, "composited_pairs": contrib},
        "stages_ms": stage_ms,
    }
    print(json.dumps(out), flush=True)
    r.close()


def channel_step(r, g, views, settings, sc, p, dL, args, npix):
    """Forward + backward with D normalized gated feature channels, depth and flow (the extra
    channels of the 4D segmentation, depth and flow renders), on the same workload."""
    import torch
    from paper_2412_20720_amd import scenes
    from paper_2412_20720_amd.frontend import Renderer
    dev = p["mean4"].device
    D = args.channels
    feats = torch.from_numpy(scenes.make_features(sc, D)).to(dev) if D else None
    gate = torch.from_numpy(scenes.make_gate(D)).to(dev) if D else None
    ch = Renderer.channels(feats, gate, True, True, 0.05)
    E = D + 3
    rgb = torch.empty(3 * npix, device=dev)
    T = torch.empty(npix, device=dev)
    out = torch.empty(E * npix, device=dev)
    dX = torch.from_numpy(np.concatenate([d.reshape(-1) for d in scenes.make_dl_dchannels(sc, E)])).to(dev)
    grads = {k: torch.empty_like(p[k]) for k in ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh")}
    if D:
        grads["features"] = torch.empty_like(feats)
        grads["gate"] = torch.empty_like(gate)

    def step():
        r.forward_channels(g, views, settings, ch, rgb, T, out)
        r.backward_channels(g, views, settings, ch, dL, dX, grads)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    r.profile_mask(["raster_fwd", "raster_bwd"])
    r.profile(True, collect=True, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    stages = r.profile(False, collect=True, reset=True)
    r.profile_mask(None)
    r.sync()
    st = {k: v[0] / max(1, v[1]) for k, v in stages.items() if v[1] > 0}
    log(f"bench: channels D={D} + depth + flow: {dt * 1e3:.3f} ms/step, {npix / dt / 1e6:.1f} Mpix/s "
        f"(raster_fwd {st.get('raster_fwd', 0):.3f} ms, raster_bwd {st.get('raster_bwd', 0):.3f} ms)")
    return dict(features=D, depth=True, flow=True, flow_dt=0.05, value=npix / dt / 1e6,
                unit="Mpix/s", ms_per_step=dt * 1e3, stages_ms=st)


def training_step(r, views, settings, sc, p, dL, args, npix):
    """The same step with the training-side fusion on: a volume mask (significances U(0, 1),
    threshold 0.1, so about 90% of the Gaussians are kept) and the straight-through mask
    gradient plus the densification statistics written by the backward."""
    import torch
    from paper_2412_20720_amd import scenes
    names = ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh")
    dev = p["mean4"].device
    mask = torch.from_numpy(scenes.make_mask(sc)).to(dev)
    g = r.gaussians(*[p[k] for k in names], sc.sh_degree, sc.t_degree, mask, 0.1)
    rgb = torch.empty(3 * npix, device=dev)
    T = torch.empty(npix, device=dev)
    grads = {k: torch.empty_like(p[k]) for k in names}
    grads["mask"] = torch.empty_like(mask)
    grads["densify"] = torch.empty((sc.n, 3), device=dev)

    def step():
        r.forward(g, views, settings, rgb, T)
        r.backward(g, views, settings, dL, grads)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    r.sync()
    log(f"bench: training fusion (mask 0.1 + densify): {dt * 1e3:.3f} ms/step, "
        f"{npix / dt / 1e6:.1f} Mpix/s")
    return dict(mask_threshold=0.1, kept=float((mask > 0.1).float().mean()), value=npix / dt / 1e6,
                unit="Mpix/s", ms_per_step=dt * 1e3)


def sky_step(r, g, views, settings, sc, dL, args, npix):
    """The step with a learnable 256 x 256 cube-map sky as the background (urban scenes):
    sky lookup, composite, and the cube-map gradient in the backward."""
    import torch
    from paper_2412_20720_amd import scenes
    from paper_2412_20720_amd.frontend import Renderer
    dev = dL.device
    cube = torch.from_numpy(scenes.make_cube(256)).to(dev)
    sk = Renderer.sky(cube)
    rgb = torch.empty(3 * npix, device=dev)
    T = torch.empty(npix, device=dev)
    names = ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh")
    grads = {k: torch.empty((g.n,) + s, device=dev) for k, s in
             zip(names, ((4,), (4,), (4,), (4,), (), (g.t_degree + 1, (g.sh_degree + 1) ** 2, 3)))}
    grads["cube"] = torch.empty_like(cube)

    def step():
        r.forward_sky(g, views, settings, sk, rgb, T)
        r.backward_sky(g, views, settings, sk, dL, grads)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    r.sync()
    log(f"bench: sky (256^2 cube map): {dt * 1e3:.3f} ms/step, {npix / dt / 1e6:.1f} Mpix/s")
    return dict(resolution=256, value=npix / dt / 1e6, unit="Mpix/s", ms_per_step=dt * 1e3)


def compact_forward(r, views, settings, sc, args, npix):
    """Forward-only render of a compact model with the workload's Gaussian count and degrees
    (residual-VQ codebooks, half positions, 8-bit opacity), decoded inside the preprocess,
    against the forward of the same model decoded to full arrays."""
    import torch
    from paper_2412_20720_amd import scenes
    dev = torch.device("cuda", 0)
    c = scenes.make_compact(sc.n, sc.sh_degree, sc.t_degree)
    cd = dict(c)
    for k in ("mean4_h", "scale_idx", "rot_l_idx", "rot_r_idx", "opacity_q", "dc_idx", "rest_idx",
              "scale_cb", "rot_cb", "dc_cb", "rest_cb"):
        a = np.ascontiguousarray(c[k])
        cd[k] = torch.from_numpy(a.view(np.int16) if a.dtype == np.uint16 else a).to(dev)
    d = r.decode_compact(cd)
    g = r.gaussians(*[d[k] for k in ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh")],
                    sc.sh_degree, sc.t_degree)
    rgb = torch.empty(3 * npix, device=dev)
    T = torch.empty(npix, device=dev)
    out = {}
    for name, fwd in (("compact", lambda: r.forward_compact(cd, views, settings, rgb, T)),
                      ("full", lambda: r.forward(g, views, settings, rgb, T))):
        for _ in range(args.warmup):
            fwd()
        torch.cuda.synchronize()
        r.profile_mask(["preprocess"])
        r.profile(True, collect=True, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fwd()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        st = r.profile(False, collect=True, reset=True)
        r.profile_mask(None)
        out[name] = dict(ms=dt * 1e3, mpix_s=npix / dt / 1e6,
                         preprocess_ms=st["preprocess"][0] / max(1, st["preprocess"][1]))
    r.sync()
    log(f"bench: compact forward {out['compact']['ms']:.3f} ms (preprocess "
        f"{out['compact']['preprocess_ms']:.3f} ms), decoded full forward {out['full']['ms']:.3f} ms "
        f"(preprocess {out['full']['preprocess_ms']:.3f} ms)")
    return dict(forward_only=True, **out)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_times(sc, n_views, backward):
    """Seconds and pixels of the FP64 oracle over the first n_views views of sc: the render,
    and with `backward` also its gradient."""
    import oracle
    from paper_2412_20720_amd import scenes
    dls = scenes.make_dl_dimage(sc) if backward else None
    t0 = time.perf_counter()
    px = 0
    for k in range(n_views):
        v = sc.views[k]
        with oracle.Frame(sc.arrays(), sc.sh_degree, sc.t_degree, v,
                          dict(time_period=sc.time_period)) as fr:
            fr.render()
            if backward:
                fr.backward(dls[k])
        px += v["width"] * v["height"]
    return time.perf_counter() - t0, px


def cpu_baseline(sc, n_views):
    """The FP64 oracle, as it stands, on a bounded sample, on all host threads: forward +
    backward of the first n_views views of the benchmark workload (the reported value), and
    forward-only and forward + backward times of the 2k- and 100k-Gaussian workloads and of
    the benchmark workload's first view."""
    import oracle
    from paper_2412_20720_amd import scenes
    dt, px = oracle_times(sc, n_views, True)
    log(f"bench: oracle {px / 1e6:.2f} Mpix fwd+bwd in {dt:.1f} s on {oracle.num_threads()} threads")
    legs = {}
    for name, s_leg, nv in (("w0", scenes.make_workload(0), 1), ("w1", scenes.make_workload(1), 1),
                            (sc.name, sc, 1)):
        t_f, p_f = oracle_times(s_leg, nv, False)
        leg = dict(pixels=p_f, forward_s=t_f, forward_mpix_s=p_f / t_f / 1e6)
        if name != sc.name:
            t_b, _ = oracle_times(s_leg, nv, True)
            leg.update(fwd_bwd_s=t_b, fwd_bwd_mpix_s=p_f / t_b / 1e6)
        else:
            leg.update(fwd_bwd_s=dt * p_f / px, fwd_bwd_mpix_s=px / dt / 1e6)
        legs[name if name != sc.name else f"{sc.name}_view0"] = leg
        log(f"bench: oracle {name}: forward {p_f / t_f / 1e6:.3f} Mpix/s, "
            f"forward + backward {leg['fwd_bwd_mpix_s']:.3f} Mpix/s")
    return dict(value=px / dt / 1e6, unit="Mpix/s", cores=oracle.num_threads(), kind="oracle",
                cpu=cpu_model(),
                sample=f"forward+backward of the first {n_views} view(s) of {sc.name} "
                       f"({px} pixels), FP64, OpenMP", seconds=dt, legs=legs)


if __name__ == "__main__":
    main()
