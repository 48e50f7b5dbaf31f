"""GPU forward parity against the FP64 oracle (Sec. 3.2, eq:4dblending and the slice/splat
steps), through the C ABI.  Image bar: 1e-4 max abs per channel, with the admissible results of
marked FP32/FP64 decisions (see oracle/parity.py)."""
import numpy as np
import pytest

from gpu_util import GpuRun, check_fp32_errors, log, oracle_frame, settings_for
from oracle import parity
from paper_2412_20720_amd import scenes

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def renderer():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_20720_amd.frontend import Renderer
    r = Renderer(0)
    yield r
    r.close()


@pytest.fixture(scope="module")
def w0():
    return scenes.make_workload(0)


@pytest.fixture(scope="module")
def w1():
    return scenes.make_workload(1)


def min_d2_over_rect(mean2d, conic, x0, x1, y0, y1):
    """Minimum of the quadratic form of each conic over the rectangle [x0,x1] x [y0,y1]."""
    u, v = mean2d[:, 0], mean2d[:, 1]
    a, b, c = conic[:, 0], conic[:, 1], conic[:, 2]
    q = lambda dx, dy: a * dx * dx + 2 * b * dx * dy + c * dy * dy
    best = np.where((u >= x0) & (u <= x1) & (v >= y0) & (v <= y1), 0.0, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        for X in (x0, x1):
            dx = X - u
            dy = np.clip(-b * dx / c, y0 - v, y1 - v)
            best = np.minimum(best, q(dx, dy))
        for Y in (y0, y1):
            dy = Y - v
            dx = np.clip(-b * dy / a, x0 - u, x1 - u)
            best = np.minimum(best, q(dx, dy))
    return np.nan_to_num(best, nan=np.inf)


def report(name, rep):
    log(f"{name}: n={rep['n']} max_err={rep['max_err']:.2e} agreeing_max={rep['max_err_agreeing']:.2e}"
        f" marked={rep['n_marked']} bad={rep['n_bad']} resolved={rep['n_resolved']}"
        f" unverified={rep['n_unverified']} failures={rep['n_failures']} {rep['failures'][:3]}")


@pytest.mark.parametrize("marginal_min", [1 / 255, 0.05])
def test_w0_full_image(renderer, w0, marginal_min):
    log(f"w0 full image, marginal_min={marginal_min}")
    run = GpuRun(renderer, w0, marginal_min=marginal_min).forward()
    img, T = run.images()[0], run.transmittance()[0]
    with oracle_frame(w0, w0.views[0], marginal_min=marginal_min) as fr:
        ref = fr.render()
        rep = parity.check_image(img, fr, TOL, ref=ref)
    report("w0", rep)
    assert rep["n_failures"] == 0 and rep["n_unverified"] <= 2
    ok = ref["n_marks"] == 0
    assert np.abs(T - ref["T"])[ok].max() <= TOL


def test_w0_tile_and_batch_do_not_change_the_result(renderer, w0):
    # Tiles and LDS batches only decide which records a wave looks at, never which pass the
    # per-pixel cutoff: images are bit-identical, gradients equal up to atomic summation order.
    dl = scenes.make_dl_dimage(w0)
    imgs, grads = {}, {}
    for tile in (8, 16, 32):
        for batch in (32, 64, 128):
            for px in ((1,) if tile == 8 else (1, 2, 4)):
                log(f"w0 tile {tile} batch {batch} pixels/lane {px}")
                run = GpuRun(renderer, w0, tile_size=tile, lds_batch=batch, px_per_lane=px).forward()
                imgs[tile, batch, px] = run.images()[0]
                grads[tile, batch, px] = run.backward(dl)
    ref_img, ref_g = imgs[16, 64, 1], grads[16, 64, 1]
    for key in imgs:
        assert np.array_equal(imgs[key], ref_img), key
        for k, v in grads[key].items():
            np.testing.assert_allclose(v, ref_g[k], rtol=1e-4, atol=1e-6 * np.abs(ref_g[k]).max())


def test_autotune_picks_a_valid_setting(renderer, w0):
    import torch
    run = GpuRun(renderer, w0)
    dl = torch.from_numpy(scenes.make_dl_dimage(w0)[0].reshape(-1)).to(run.dev)
    grads = {k: torch.empty_like(v) for k, v in run.p.items()}
    ms = renderer.autotune(run.g, run.views, run.settings, dl, run.rgb, run.T, grads, reps=1)
    s = run.settings
    log(f"autotune: tile {s.tile_size} batch {s.lds_batch} pixels/lane {s.px_per_lane} {ms:.3f} ms")
    assert ms > 0 and s.tile_size in (8, 16, 32) and s.lds_batch in (32, 64, 128)
    assert s.px_per_lane in (1, 2, 4) and not (s.tile_size == 8 and s.px_per_lane > 1)
    # cached: a second call returns the same choice
    again = settings_for(w0)
    renderer.autotune(run.g, run.views, again, dl, run.rgb, run.T, grads, reps=1)
    assert (again.tile_size, again.lds_batch, again.px_per_lane) == (s.tile_size, s.lds_batch, s.px_per_lane)
    img = run.forward().images()[0]
    ref = GpuRun(renderer, w0).forward().images()[0]
    assert np.array_equal(img, ref)


def test_w1_records_match_oracle_splats(renderer, w1):
    # K1 stage parity: slice, EWA splat and 4DSH color per Gaussian.
    import torch
    log("w1 records")
    run = GpuRun(renderer, w1)
    rec, tiles = renderer.preprocess(run.g, run.views, run.settings)
    torch.cuda.synchronize()
    rec, tiles = rec.cpu().numpy()[0], tiles.cpu().numpy()[0]
    with oracle_frame(w1, w1.views[0]) as fr:
        sp = fr.splats()
    W, H = w1.views[0]["width"], w1.views[0]["height"]
    # A splat is listed when it survives the culls and can be composited at some pixel centre:
    # the minimum Mahalanobis distance over the image's pixel-centre rectangle lies within the
    # cutoff and within the radius where opacity p_t exp(-d2 / 2) still reaches alpha_min,
    # d2 = 2 ln(opacity p_t / alpha_min).  The GPU widens that radius by 1e-3 relative and
    # 2e-3 absolute: within the widening either outcome is admissible.
    d2min = min_d2_over_rect(sp["mean2d"], sp["conic"], 0.5, W - 0.5, 0.5, H - 0.5)
    gpu_vis = tiles > 0
    log_ratio = np.log(np.maximum(sp["opt"], 1e-300) * 255.0)
    reach = np.minimum(9.0, 2.0 * log_ratio)
    reach_wide = np.minimum(9.0, 2.002 * log_ratio + 2e-3)
    must = (sp["alive"] == 1) & (d2min <= reach * (1 - 1e-4) - 1e-4)
    may = ((sp["alive"] == 1) | (sp["optional"] == 1)) & (d2min <= reach_wide * (1 + 1e-2))
    log(f"visible gpu={gpu_vis.sum()} oracle={must.sum()}..{may.sum()}")
    assert not (must & ~gpu_vis).any() and not (gpu_vis & ~may).any()
    ref_vis = must
    both = np.nonzero(ref_vis & gpu_vis)[0]
    r = rec[both]
    s = sp[both]
    np.testing.assert_allclose(r[:, 0:2], s["mean2d"], atol=2e-3, rtol=0)
    cmax = np.abs(s["conic"]).max(1, keepdims=True)
    assert (np.abs(r[:, 2:5] - s["conic"]) / cmax).max() <= 2e-4
    np.testing.assert_allclose(r[:, 5], s["opt"], rtol=1e-4, atol=1e-7)
    np.testing.assert_allclose(r[:, 6:9], s["color"], atol=2e-5)
    np.testing.assert_allclose(r[:, 11], s["depth"], rtol=2e-6)
    # box half extents: at least sqrt(reach) sigma (3 sigma for splats opaque enough to reach
    # alpha_min beyond the cutoff), at most the widened radius plus 1e-3 relative
    lr = np.log(s["opt"] * 255.0)
    lo_r, hi_r = np.minimum(9.0, 2.0 * lr), np.minimum(9.0, 2.002 * lr + 2e-3)
    assert (hi_r < 9.0).any() and (lo_r == 9.0).any()
    for col, var in ((9, s["cov2d"][:, 0]), (10, s["cov2d"][:, 2])):
        assert (r[:, col] >= np.sqrt(lo_r * var) * (1 - 1e-5)).all()
        assert (r[:, col] <= np.sqrt(hi_r * var) * 1.001).all()


def test_w1_fp32_errors_within_parity_margins(renderer, w1):
    # The oracle marks a decision as admissible either way when its deciding quantity lies
    # within a margin of the threshold.  The margins must cover the GPU's FP32 error in that
    # quantity: measured here on the GPU's records against the oracle's FP64 splats, each at
    # most half its margin (the 300k-Gaussian workload is measured in test_gpu_fullsize).
    check_fp32_errors(renderer, w1, 0, {}, 3000, seed=77)


def test_w1_sampled_pixels(renderer, w1):
    log("w1 sampled pixels")
    run = GpuRun(renderer, w1).forward()
    img = run.images()[0]
    W, H = w1.views[0]["width"], w1.views[0]["height"]
    rng = np.random.default_rng(5)
    xy = np.stack([rng.integers(0, W, 6000), rng.integers(0, H, 6000)], 1)
    # plus two whole tiles and the ragged bottom-right corner tile
    ys, xs = np.mgrid[496:512, 672:688]
    ys2, xs2 = np.mgrid[(H // 16) * 16:H, (W // 16) * 16:W]
    xy = np.concatenate([xy, np.stack([xs.ravel(), ys.ravel()], 1),
                         np.stack([xs2.ravel(), ys2.ravel()], 1)])
    g = img[:, xy[:, 1], xy[:, 0]].T
    with oracle_frame(w1, w1.views[0]) as fr:
        rep = parity.check_image(g, fr, TOL, xy=xy)
    report("w1", rep)
    assert rep["n_failures"] == 0
    assert rep["n_unverified"] <= 0.002 * rep["n"]


def test_batched_views_equal_single_views(renderer, w0):
    # Two views (different cameras, sizes, times) in one call give the same images as two calls.
    v0 = w0.views[0]
    v1 = scenes.pinhole(96, 72, 55.0, scenes.look_at((1.5, 0.5, 2.5), (0, 0, 0)), 0.3, (0.2, 0.1, 0.0))
    both = GpuRun(renderer, w0, views=[v0, v1]).forward().images()
    a = GpuRun(renderer, w0, views=[v0]).forward().images()[0]
    b = GpuRun(renderer, w0, views=[v1]).forward().images()[0]
    assert np.array_equal(both[0], a) and np.array_equal(both[1], b)
    with oracle_frame(w0, v1) as fr:
        rep = parity.check_image(b, fr, TOL)
    report("w0 second view", rep)
    assert rep["n_failures"] == 0


def test_edge_cases(renderer, w0):
    # Ragged image (not a multiple of the tile), empty scene, everything culled in time,
    # everything behind the camera.
    ragged = dict(w0.views[0], width=37, height=29, cx=np.float32(18.5), cy=np.float32(14.5),
                  fx=np.float32(32.0), fy=np.float32(32.0))
    img = GpuRun(renderer, w0, views=[ragged]).forward().images()[0]
    with oracle_frame(w0, ragged) as fr:
        rep = parity.check_image(img, fr, TOL)
    report("ragged", rep)
    assert rep["n_failures"] == 0

    bg = np.array([0.25, 0.5, 0.75], np.float32)
    empty = scenes.subset(w0, np.arange(0))
    empty.views = [dict(w0.views[0], background=bg)]
    run = GpuRun(renderer, empty).forward()
    assert np.all(run.images()[0] == bg[:, None, None]) and np.all(run.transmittance()[0] == 1)

    late = scenes.subset(w0, np.arange(w0.n))
    late.views = [dict(w0.views[0], t=np.float32(50.0), background=bg)]
    run = GpuRun(renderer, late).forward()
    assert np.all(run.images()[0] == bg[:, None, None])
    assert renderer.stats()["n_visible"] == 0

    behind = scenes.subset(w0, np.arange(w0.n))
    behind.views = [dict(w0.views[0], world_to_cam=scenes.look_at((0, 0, 3), (0, 0, 6)), background=bg)]
    run = GpuRun(renderer, behind).forward()
    assert np.all(run.images()[0] == bg[:, None, None])


def test_argument_errors(renderer, w0):
    import ctypes as C
    from paper_2412_20720_amd import _binding as B
    run = GpuRun(renderer, w0)
    bad = settings_for(w0, tile_size=12)
    with pytest.raises(B.G4DError, match="EINVAL"):
        renderer.forward(run.g, run.views, bad, run.rgb, run.T)
    g = B.g4d_gaussians.from_buffer_copy(run.g)
    g.sh_degree = 4
    with pytest.raises(B.G4DError, match="EINVAL"):
        renderer.forward(g, run.views, run.settings, run.rgb, run.T)
    views = [dict(run.views[0], width=0)]
    with pytest.raises(B.G4DError, match="EINVAL"):
        renderer.forward(run.g, views, run.settings, run.rgb, run.T)
    for bad_alpha in (dict(alpha_max=1.0), dict(alpha_min=0.0), dict(alpha_min=0.5, alpha_max=0.4)):
        with pytest.raises(B.G4DError, match="EINVAL"):
            renderer.forward(run.g, run.views, settings_for(w0, **bad_alpha), run.rgb, run.T)


def test_w1_pair_counts_match_oracle(renderer, w1):
    # The counting forward's per-pixel counts: composited pairs equal the oracle's wherever no
    # decision of the pixel lies within the FP32/FP64 margin; evaluated pairs (within the
    # entry's reach) lie between the composited ones and the oracle's pairs within the cutoff.
    log("w1 pair counts")
    run = GpuRun(renderer, w1)
    npix = run.T.numel()
    renderer.eval_counters(True)
    run.forward()
    cnt = renderer.eval_counters(False, npix).cpu().numpy().astype(np.int64)
    W, H = w1.views[0]["width"], w1.views[0]["height"]
    rng = np.random.default_rng(6)
    xy = np.stack([rng.integers(0, W, 4000), rng.integers(0, H, 4000)], 1)
    g = cnt[xy[:, 1] * W + xy[:, 0]]
    evals, contrib = g & 0xFFFF, g >> 16
    rgb = run.images()[0][:, xy[:, 1], xy[:, 0]].T
    with oracle_frame(w1, w1.views[0]) as fr:
        ref = fr.render(xy)
        rep = parity.check_counts(contrib, rgb, fr, xy, ref, TOL)
    marks = ref["n_marks"]
    clean = marks == 0
    log(f"  composited: {contrib.sum()} gpu, {ref['n_contrib'].sum()} oracle; evaluated "
        f"{evals.sum()} gpu, {ref['n_evals'].sum()} oracle within the cutoff; marked {int((~clean).sum())}")
    log(f"  exact counts: {rep['n_exact']} unmarked + {rep['n_by_variant']} marked (a variant's "
        f"count and color) of {rep['n']}, unverified {rep['n_unverified']}, failures "
        f"{rep['n_failures']} {rep['failures'][:3]}")
    # every sampled pixel's count is checked exactly, a marked one against the variant whose
    # color the GPU produced
    assert rep["n_failures"] == 0 and rep["verified_frac"] >= 0.9
    assert np.array_equal(contrib[clean], ref["n_contrib"][clean])
    # a flipped decision moves the count by one (alpha_min) or ends the walk one entry apart
    assert np.all(np.abs(contrib - ref["n_contrib"]) <= 2 * marks)
    assert np.all(contrib <= evals)
    assert np.all(evals[clean] <= ref["n_evals"][clean])
    assert np.all(evals <= ref["n_evals"] + 4 * marks)
    assert evals.sum() < 0.9 * ref["n_evals"].sum()  # the reach drops pixels the cutoff keeps


def test_wide_tile_ids_match_narrow(renderer, w1):
    # Four 1352x1014 views at 8-pixel tiles make 85,852 tiles: the tile ids exceed 16 bits and
    # sort as 32-bit keys; at 32-pixel tiles (5,504 tiles) they sort as 16-bit keys.  The
    # decomposition never changes the image.
    import torch
    views = [w1.views[0]] * 4
    log("w1 x4 views, tile 8 (32-bit keys) against tile 32 (16-bit keys)")
    wide = GpuRun(renderer, w1, views=views, tile_size=8).forward()
    assert renderer.stats()["n_tiles"] == 4 * 169 * 127
    narrow = GpuRun(renderer, w1, views=views, tile_size=32).forward()
    assert torch.equal(wide.rgb, narrow.rgb) and torch.equal(wide.T, narrow.T)


def test_stage_profile_and_mask(renderer, w0):
    # Stage timing records every stage by default; with a mask, only the named stages.
    dl = scenes.make_dl_dimage(w0)
    run = GpuRun(renderer, w0)
    renderer.profile_mask(None)
    renderer.profile(True, collect=True, reset=True)
    run.forward().backward(dl)
    every = renderer.profile(False, collect=True, reset=True)
    log(f"every stage: {every}")
    assert all(n >= 1 for _, n in every.values()), every
    renderer.profile_mask(["raster_bwd"])
    try:
        renderer.profile(True, collect=True, reset=True)
        run.forward().backward(dl)
        only = renderer.profile(False, collect=True, reset=True)
    finally:
        renderer.profile_mask(None)
    log(f"raster_bwd only: {only}")
    assert only["raster_bwd"][1] == 1 and only["raster_bwd"][0] > 0
    assert all(n == 0 for k, (_, n) in only.items() if k != "raster_bwd"), only


def test_pair_buffers_grow_between_calls(renderer, w0):
    # The key generation is queued before the host has read the pair count, into the pair
    # buffers of the previous call; a call with many more pairs grows them and generates the
    # keys again (the overflow flag of the first pass is cleared: sync() would raise).  Images
    # on the used context equal those of a fresh context.
    from paper_2412_20720_amd.frontend import Renderer
    small = scenes.subset(w0, np.arange(200))
    used, fresh = Renderer(0), Renderer(0)
    try:
        img_small = GpuRun(used, small).forward().images()[0]
        n_small = used.stats()["n_pairs"]
        img_full = GpuRun(used, w0).forward().images()[0]
        n_full = used.stats()["n_pairs"]
        again = GpuRun(used, small).forward().images()[0]
        ref_full = GpuRun(fresh, w0).forward().images()[0]
        log(f"pairs: small {n_small}, full {n_full} (fresh {fresh.stats()['n_pairs']})")
        assert n_full > 2 * n_small and n_full == fresh.stats()["n_pairs"]
        assert np.array_equal(img_full, ref_full)
        assert np.array_equal(again, img_small)
    finally:
        used.close()
        fresh.close()
