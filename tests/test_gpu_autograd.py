"""The autograd functions keep working when several renders share one Renderer before their
backwards (the context holds one forward's state; a backward whose forward is no longer the
last one runs it again first): two renders then one backward of their sum give the sum of the
two separate gradients, for the plain render and for a plain render followed by a sky render."""
import numpy as np
import pytest

from gpu_util import PARAMS, log
from oracle import parity
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


def leaf_params(sc, dev):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev).requires_grad_(True)
            for k, v in sc.arrays().items()}


def test_two_renders_one_backward(renderer):
    import torch
    from paper_2412_20720_amd import _binding as B
    from paper_2412_20720_amd.frontend import render
    sc = scenes.make_workload(0)
    v2 = scenes.pinhole(96, 80, 55.0, scenes.look_at((1.2, 0.4, 2.6), (0, 0, 0)), 0.35)
    s = B.default_settings(time_period=sc.time_period)
    rng = np.random.default_rng(8)
    g1 = torch.from_numpy(rng.normal(size=(3, 128, 128)).astype(np.float32)).to(renderer.device)
    g2 = torch.from_numpy(rng.normal(size=(3, 80, 96)).astype(np.float32)).to(renderer.device)
    kw = dict(sh_degree=sc.sh_degree, t_degree=sc.t_degree, renderer=renderer, settings=s)

    def grads_of(views_and_dl):
        p = leaf_params(sc, renderer.device)
        args = [p[k] for k in PARAMS]
        loss = 0
        for views, dl in views_and_dl:
            imgs, _ = render(*args, views, **kw)
            loss = loss + (imgs[0] * dl).sum()
        loss.backward()
        torch.cuda.synchronize()
        return {k: p[k].grad.cpu().numpy() for k in PARAMS}

    a = grads_of([([sc.views[0]], g1)])
    b = grads_of([([v2], g2)])
    both = grads_of([([sc.views[0]], g1), ([v2], g2)])  # two forwards, then one backward
    errs = parity.grad_rel_errors(both, {k: a[k] + b[k] for k in PARAMS})
    log(f"two renders, one backward: rel diff {errs}")
    assert all(e <= 1e-5 for e in errs.values()), errs


def test_plain_and_sky_render_one_backward(renderer):
    import torch
    from paper_2412_20720_amd import _binding as B
    from paper_2412_20720_amd.frontend import render, render_sky
    sc = scenes.make_workload(0)
    s = B.default_settings(time_period=sc.time_period)
    dev = renderer.device
    cube0 = torch.from_numpy(scenes.make_cube(8)).to(dev)
    rng = np.random.default_rng(9)
    g1 = torch.from_numpy(rng.normal(size=(3, 128, 128)).astype(np.float32)).to(dev)
    g2 = torch.from_numpy(rng.normal(size=(3, 128, 128)).astype(np.float32)).to(dev)
    kw = dict(sh_degree=sc.sh_degree, t_degree=sc.t_degree, renderer=renderer, settings=s)

    def run(plain, sky):
        p = leaf_params(sc, dev)
        cube = cube0.clone().requires_grad_(True)
        args = [p[k] for k in PARAMS]
        loss = 0
        if plain:
            loss = loss + (render(*args, sc.views, **kw)[0][0] * g1).sum()
        if sky:
            loss = loss + (render_sky(*args, cube, sc.views, **kw)[0][0] * g2).sum()
        loss.backward()
        torch.cuda.synchronize()
        out = {k: p[k].grad.cpu().numpy() for k in PARAMS}
        out["cube"] = cube.grad.cpu().numpy() if sky else np.zeros(cube0.shape, np.float32)
        return out

    a, b, both = run(True, False), run(False, True), run(True, True)
    errs = parity.grad_rel_errors(both, {k: a[k] + b[k] for k in a})
    log(f"plain + sky renders, one backward: rel diff {errs}")
    assert all(e <= 1e-5 for e in errs.values()), errs
