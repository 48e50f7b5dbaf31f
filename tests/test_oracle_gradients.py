"""Pin of the oracle's backward: central finite differences of the oracle's own FP64 forward.

The backward is the derivative of the render of eq:4dblending through the slice and splat
steps of Sec. 3.2, with every discrete decision frozen.  Under the smooth settings the only
jumps left are below exp(-12.5) per pixel, so central differences with h = 1e-6 resolve every
parameter.
"""
import math

import numpy as np
import pytest

import oracle

SMOOTH = dict(oracle.SMOOTH_SETTINGS)


def tiny_scene(rng, n=6, sh_degree=1, t_degree=1):
    m4 = np.concatenate([rng.uniform(-0.35, 0.35, (n, 3)), rng.uniform(0.3, 0.7, (n, 1))], 1)
    s4 = np.exp(rng.normal(-2.0, 0.3, (n, 4)))
    s4[:, 3] = np.exp(rng.normal(-1.2, 0.2, n))
    # Unnormalized rotors, so that the gradient passes through the normalization.
    ql = rng.normal(size=(n, 4)) * rng.uniform(0.5, 2.0, (n, 1))
    qr = rng.normal(size=(n, 4)) * rng.uniform(0.5, 2.0, (n, 1))
    op = rng.uniform(0.2, 0.8, n)
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0, 0.15, (n, t_degree + 1, k, 3))
    sh[:, 0, 0, :] = rng.uniform(0.5, 1.5, (n, 3))  # colors stay above the clamp
    return dict(mean4=m4, scale4=s4, rot_l=ql, rot_r=qr, opacity=op, sh=sh)


def view(W=32, H=32, f=36.0, t=0.55):
    return dict(width=W, height=H, fx=f, fy=f, cx=W / 2, cy=H / 2,
                world_to_cam=np.array([[1.0, 0, 0, 0.05], [0, -1, 0, 0.02], [0, 0, -1, 2.2]]),
                t=t, background=np.array([0.2, 0.1, 0.3]))


def loss(arr, sh_degree, t_degree, vw, st, g):
    with oracle.Frame(arr, sh_degree, t_degree, vw, st, exact_f64=True) as fr:
        return float((fr.render()["rgb"] * g).sum())


@pytest.mark.parametrize("seed", [0, 1])
def test_oracle_backward_matches_central_differences(oracle_lib, seed):
    rng = np.random.default_rng(100 + seed)
    arr = tiny_scene(rng)
    vw = view()
    st = dict(SMOOTH, time_period=1.7)
    g = rng.normal(size=(3, vw["height"], vw["width"]))
    with oracle.Frame(arr, 1, 1, vw, st, exact_f64=True) as fr:
        assert fr.splats()["alive"].all()
        grads = fr.backward(g)
    for name in ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh"):
        an = grads[name]
        flat = arr[name].reshape(-1)
        scale = np.abs(an).max()
        assert scale > 0, name
        for j in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[j]))
            plus = {k: v.copy() for k, v in arr.items()}
            minus = {k: v.copy() for k, v in arr.items()}
            plus[name].reshape(-1)[j] += h
            minus[name].reshape(-1)[j] -= h
            fd = (loss(plus, 1, 1, vw, st, g) - loss(minus, 1, 1, vw, st, g)) / (2 * h)
            a = an.reshape(-1)[j]
            assert abs(fd - a) <= 1e-6 * (abs(a) + 1e-2 * scale), (name, j, fd, a)


def test_oracle_backward_default_settings_directional(oracle_lib):
    # Default (non-smooth) settings: along the gradient direction of each group the
    # directional derivative still agrees, because the frozen decisions do not move for a
    # small step.
    rng = np.random.default_rng(7)
    arr = tiny_scene(rng, n=8)
    vw = view()
    st = dict(oracle.DEFAULT_SETTINGS, time_period=1.7)
    g = rng.normal(size=(3, vw["height"], vw["width"]))
    with oracle.Frame(arr, 1, 1, vw, st, exact_f64=True) as fr:
        grads = fr.backward(g)
    for name in ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh"):
        u = grads[name] / np.linalg.norm(grads[name])
        h = 1e-7
        plus = dict(arr, **{name: arr[name] + h * u})
        minus = dict(arr, **{name: arr[name] - h * u})
        fd = (loss(plus, 1, 1, vw, st, g) - loss(minus, 1, 1, vw, st, g)) / (2 * h)
        an = float((grads[name] * u).sum())
        assert abs(fd - an) <= 1e-5 * abs(an), (name, fd, an)
