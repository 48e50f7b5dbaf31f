"""Integer-exact stage check of the binning (the depth-ordered, tile-sorted lists of the
tile-based rasterizer, Sec. 3.2; the depth order of Sec. 3.1's blending): the GPU's sorted
(tile, slot) pairs equal a stable argsort by tile id of the emission order rebuilt from the GPU's
own depth keys (each visible slot in (depth, slot) order, its tiles ascending), every slot has as
many pairs as its tile count, the tile ranges equal a recomputation from the sorted keys, and the
listed tiles of sampled splats are exactly those whose pixel centres fall inside the splat's
reach ellipse, up to a thin band of FP32 rounding at the border.  Run on one 1352x1014 view at
32-pixel tiles, on four views at 8-pixel tiles (more than 2^16 tiles), and on 20 small views, two
of them facing away from the scene, with a Gaussian count that is not a multiple of the 64
Gaussians of a listing mask or the 4,096 slots of a radix workgroup (the depth sort runs per
view)."""
import numpy as np
import pytest

from gpu_util import GpuRun, log
from paper_2412_20720_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def renderer():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_20720_amd.frontend import Renderer
    r = Renderer(0)
    yield r
    r.close()


def tile_grid(views, T):
    base, grids = 0, []
    for v in views:
        tx, ty = -(-int(v["width"]) // T), -(-int(v["height"]) // T)
        grids.append((base, tx, ty))
        base += tx * ty
    return grids, base


@pytest.mark.parametrize("n_views,tile", [(1, 32), (4, 8)])
def test_sorted_pairs_and_ranges_exact(renderer, n_views, tile):
    sc = scenes.make_workload(1)
    views = [sc.views[0]] + [scenes.pinhole(1352, 1014, 50.0,
                                            scenes.look_at((4 * np.sin(a), 0.3, 4 * np.cos(a)),
                                                           (0, 0, 0)), 0.2 + 0.2 * k)
                             for k, a in enumerate((0.7, 2.1, 4.0))][:n_views - 1]
    run = GpuRun(renderer, sc, views=views, tile_size=tile).forward()
    check_lists_exact(renderer, run, sc, views, tile)


def test_many_views_empty_views_ragged_count(renderer):
    sc = scenes.subset(scenes.make_workload(1), np.arange(5000))
    views = []
    for k in range(18):
        a = 2 * np.pi * k / 18
        eye = (4 * np.sin(a), 0.3 + 0.1 * (k % 3), 4 * np.cos(a))
        views.append(scenes.pinhole(320, 240, 60.0, scenes.look_at(eye, (0, 0, 0)), 0.05 * k))
    away = [scenes.pinhole(320, 240, 60.0, scenes.look_at((0, 0, 4), (0, 0, 12)), 0.3),
            scenes.pinhole(320, 240, 60.0, scenes.look_at((4, 0, 0), (12, 0, 0)), 0.6)]
    views.insert(5, away[0])
    views.insert(13, away[1])
    run = GpuRun(renderer, sc, views=views, tile_size=16).forward()
    cnt = check_lists_exact(renderer, run, sc, views, 16)
    per_view = (cnt.reshape(len(views), -1) > 0).sum(1)
    log(f"  listed per view: {per_view.tolist()}")
    assert per_view[5] == 0 and per_view[13] == 0 and (np.delete(per_view, [5, 13]) > 0).all()


def check_lists_exact(renderer, run, sc, views, tile):
    """The checks above on the last forward; returns the tile count per slot."""
    st = renderer.stats()
    tid, slot, ranges = (t.numpy() for t in renderer.pairs())
    n_tiles = st["n_tiles"]
    log(f"{len(views)} view(s), tile {tile}: {st['n_pairs']} pairs, {n_tiles} tiles")
    rec, cnt = renderer.preprocess(run.g, views, run.settings)
    rec = rec.cpu().numpy().reshape(-1, 12)
    cnt = cnt.cpu().numpy().reshape(-1).astype(np.int64)
    N = sc.n
    # every pair is a listed slot; per slot as many pairs as its tile count
    assert len(tid) == st["n_pairs"] == cnt.sum()
    assert np.array_equal(np.bincount(slot, minlength=len(cnt)), cnt)
    assert tid.max() < n_tiles
    # emission order rebuilt from the GPU's own keys: visible slots stably sorted by the float
    # bits of their depth (slot order among ties), each slot's tiles ascending
    vis = np.nonzero(cnt > 0)[0]
    dkey = rec[vis, 11].astype(np.float32).view(np.uint32)
    order = vis[np.argsort(dkey, kind="stable")]
    by_slot = np.lexsort((tid, slot))              # pairs grouped by slot, tiles ascending
    start = np.concatenate([[0], np.cumsum(cnt)])  # group offsets in slot order
    emit = np.concatenate([by_slot[start[s]:start[s + 1]] for s in order])
    expect = emit[np.argsort(tid[emit], kind="stable")]
    assert np.array_equal(tid[expect], tid) and np.array_equal(slot[expect], slot)
    # ranges
    t = np.arange(n_tiles)
    lo, hi = np.searchsorted(tid, t, "left"), np.searchsorted(tid, t, "right")
    want = np.where((hi > lo)[:, None], np.stack([lo, hi], 1), 0)
    assert np.array_equal(ranges, want)
    # tile sets of sampled splats against the reach ellipse, evaluated in FP64 on the GPU's
    # record: every tile with a pixel centre well inside is listed; every listed tile has a
    # centre inside the ellipse widened by the listing's own FP32 margins (1e-3 in d2, 0.01 px
    # along x), or, for a thin tilted ellipse that FP32 cannot resolve, inside its box
    grids, _ = tile_grid(views, tile)
    rng = np.random.default_rng(3)
    alpha_min = 1.0 / 255.0
    n_band = 0
    for s in rng.choice(vis, min(400, len(vis)), replace=False):
        v = s // N
        base, tx, ty = grids[v]
        W, H = int(views[v]["width"]), int(views[v]["height"])
        u, vv, a, b, c, opt = (float(x) for x in rec[s, :6])
        ex, ey = float(rec[s, 9]), float(rec[s, 10])
        r2 = min(9.0, 2.002 * np.log(opt / alpha_min) + 2e-3)
        listed = set(tid[by_slot[start[s]:start[s + 1]]].tolist())
        x0, x1 = max(0, int(np.floor(u - ex)) - tile), min(W - 1, int(np.ceil(u + ex)) + tile)
        y0, y1 = max(0, int(np.floor(vv - ey)) - tile), min(H - 1, int(np.ceil(vv + ey)) + tile)
        ys, xs = np.mgrid[y0:y1 + 1, x0:x1 + 1]
        dy = ys + 0.5 - vv
        q = lambda dx: a * dx * dx + 2 * b * dx * dy + c * dy * dy
        dx = xs + 0.5 - u
        d2 = q(dx)
        d2w = np.minimum(np.minimum(q(dx - 0.011), q(dx + 0.011)), d2)
        tiles_of = base + (ys // tile) * tx + xs // tile
        inside = set(np.unique(tiles_of[d2 <= r2 * (1 - 1e-3)]).tolist())
        if a * c - b * b > 2e-3 * a * c:
            near = d2w <= r2 * 1.0011 * (1 + 1e-4)
        else:
            near = (np.abs(dx) <= ex + 0.011) & (np.abs(dy) <= ey)
        maybe = set(np.unique(tiles_of[near]).tolist())
        assert inside <= listed, (s, sorted(inside - listed)[:5])
        assert listed <= maybe, (s, sorted(listed - maybe)[:5])
        n_band += len(listed - inside)
    log(f"  tile sets of {min(400, len(vis))} splats: {n_band} listed tiles reached only within "
        f"the rounding band")
    return cnt
