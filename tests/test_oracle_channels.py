"""Pins of the oracle's extra channels: features, depth and flow composited with the weights of
eq:4dblending.

- Features (Sec. 7, 4D segmentation: the color replaced by the normalized scale-gated
  feature): with unit-norm features equal to the colors, the feature channels are the RGB
  render with a black background (the RGB path is pinned in test_oracle_pins.py); scaling a
  feature does not change it; a zero gate entry zeroes its channel.
- Depth (Sec. 5, the rendered depth of the LiDAR loss): with every Gaussian at depth z0 the
  channel is z0 (1 - T); two Gaussians on the axis give the closed form.
- Flow (Sec. 8.1: the displacement of the conditional mean projected to the image): zero for
  Gaussians whose rotation leaves space and time uncoupled; for a rotation in the (x, t) plane
  the mean moves at Sigma_xt / Sigma_tt (closed form) and the centre pixel shows o times the
  projected displacement.
- Backward: central differences of the oracle's forward for features, gate and (through the
  depth channel) the geometry.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2412_20720_amd import scenes

CF = dict(cutoff_sigma=1e6, alpha_min=0.0, T_min=0.0, alpha_max=1.0, blur=0.0, color_min=-1e30,
          marginal_min=0.0, jacobian_margin=1e6)


def _scene(mean4, scale4, rot_l, rot_r, opacity, dc_rgb):
    n = len(mean4)
    sh = np.zeros((n, 1, 1, 3), np.float64)
    sh[:, 0, 0, :] = (np.asarray(dc_rgb, np.float64) - 0.5) * 2.0 * math.sqrt(math.pi)
    return dict(mean4=np.asarray(mean4, np.float64), scale4=np.asarray(scale4, np.float64),
                rot_l=np.asarray(rot_l, np.float64), rot_r=np.asarray(rot_r, np.float64),
                opacity=np.asarray(opacity, np.float64), sh=sh)


def _view(W, H, f, eye_z, t, bg=(0, 0, 0)):
    E = scenes.look_at((0, 0, eye_z), (0, 0, 0)).astype(np.float64)
    return dict(width=W, height=H, fx=f, fy=f, cx=W / 2, cy=H / 2, world_to_cam=E, t=t,
                background=np.array(bg, float))


def _random_scene(rng, n, colors, t_view=0.5, same_time=False):
    m4 = np.concatenate([rng.uniform(-0.6, 0.6, (n, 3)), rng.uniform(0, 1, (n, 1))], 1)
    if same_time:
        m4[:, 3] = t_view
    s4 = np.exp(rng.normal(-2.5, 0.4, (n, 4)))
    s4[:, 3] = 0.5
    return _scene(m4, s4, rng.normal(size=(n, 4)), rng.normal(size=(n, 4)),
                  rng.uniform(0.05, 0.95, n), colors)


def test_features_equal_rgb_render_of_the_same_vectors(oracle_lib):
    rng = np.random.default_rng(30)
    n = 300
    c = rng.uniform(0.05, 1.0, (n, 3))
    c /= np.linalg.norm(c, axis=1, keepdims=True)  # unit colors
    sc = _random_scene(rng, n, c)
    vw = _view(48, 40, 50.0, 2.5, 0.5)
    feats = c * rng.uniform(0.5, 3.0, (n, 1))  # normalization removes the scale
    with oracle.Frame(sc, 0, 0, vw, {}, exact_f64=True) as fr:
        assert fr.set_channels(feats) == 3
        out = fr.render()
    assert out["n_contrib"].max() > 5
    np.testing.assert_allclose(out["ext"], out["rgb"], atol=1e-12)


def test_feature_gate_and_scale_invariance(oracle_lib):
    rng = np.random.default_rng(31)
    n, D = 200, 5
    sc = _random_scene(rng, n, np.full((n, 3), 0.5))
    vw = _view(40, 32, 45.0, 2.5, 0.5)
    f = rng.normal(size=(n, D))
    gate = rng.uniform(0.1, 1.0, D)
    gate[2] = 0.0
    with oracle.Frame(sc, 0, 0, vw, {}, exact_f64=True) as fr:
        fr.set_channels(f, gate)
        a = fr.render()["ext"]
        fr.set_channels(f * rng.uniform(0.2, 5.0, (n, 1)), gate)
        b = fr.render()["ext"]
        # the gated features of every Gaussian, normalized, then composited by hand
        fr.set_channels(f * gate / np.linalg.norm(f * gate, axis=1, keepdims=True))
        c = fr.render()["ext"]
    assert np.abs(a).max() > 0.1
    assert np.all(a[2] == 0.0)
    np.testing.assert_allclose(a, b, atol=1e-12)
    np.testing.assert_allclose(a, c, atol=1e-12)


def test_depth_channel_of_a_fronto_parallel_layer(oracle_lib):
    # Every sliced mean at world z = 0 (mu_t = t, so the slice does not move it), camera at
    # z = 2.5 looking down -z: every depth is 2.5 and the channel is 2.5 (1 - T).
    rng = np.random.default_rng(32)
    n = 300
    sc = _random_scene(rng, n, np.full((n, 3), 0.5), same_time=True)
    sc["mean4"][:, 2] = 0.0
    vw = _view(48, 40, 50.0, 2.5, 0.5, bg=(0.3, 0.3, 0.3))
    with oracle.Frame(sc, 0, 0, vw, {}, exact_f64=True) as fr:
        assert fr.set_channels(depth=True) == 1
        out = fr.render()
    assert (out["T"] < 0.5).any()
    np.testing.assert_allclose(out["ext"][0], 2.5 * (1.0 - out["T"]), atol=1e-12)


def test_depth_two_gaussian_stack_closed_form(oracle_lib):
    sc = _scene([[0, 0, 0.5, 0.5], [0, 0, -0.5, 0.5]], [[0.1] * 3 + [1.0]] * 2,
                [[1, 0, 0, 0]] * 2, [[1, 0, 0, 0]] * 2, [0.6, 0.7],
                [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    vw = _view(33, 33, 50.0, 3.0, 0.5)
    with oracle.Frame(sc, 0, 0, vw, CF, exact_f64=True) as fr:
        fr.set_channels(depth=True)
        out = fr.render(np.array([[16, 16], [21, 14]]))
    for k, (px, py) in enumerate([(16, 16), (21, 14)]):
        r2 = (px + 0.5 - 16.5) ** 2 + (py + 0.5 - 16.5) ** 2
        a1 = 0.6 * math.exp(-0.5 * r2 / (50 * 0.1 / 2.5) ** 2)
        a2 = 0.7 * math.exp(-0.5 * r2 / (50 * 0.1 / 3.5) ** 2)
        np.testing.assert_allclose(out["ext"][k, 0], a1 * 2.5 + (1 - a1) * a2 * 3.5, atol=1e-12)


def test_flow_is_zero_without_space_time_coupling(oracle_lib):
    rng = np.random.default_rng(33)
    n = 150
    sc = _random_scene(rng, n, np.full((n, 3), 0.5))
    # q_r = (a, b, c, -d) of q_l fixes the time axis: a rotation of space alone
    ql = rng.normal(size=(n, 4))
    sc["rot_l"] = ql
    sc["rot_r"] = ql * np.array([1.0, 1.0, 1.0, -1.0])
    vw = _view(40, 32, 45.0, 2.5, 0.4)
    with oracle.Frame(sc, 0, 0, vw, {}, exact_f64=True) as fr:
        assert fr.set_channels(flow=True, flow_dt=0.1) == 2
        out = fr.render()
    assert out["n_contrib"].max() > 3
    assert np.abs(out["ext"]).max() <= 1e-12


def test_flow_of_a_gaussian_rotated_in_the_xt_plane(oracle_lib):
    # Rotation by 2 th in the (x, t) plane: the conditional mean moves along x at
    # v = Sigma_xt / Sigma_tt, with Sigma_xt = c s (s_x^2 - s_t^2), Sigma_tt = s^2 s_x^2 +
    # c^2 s_t^2 (c, s = cos 2th, sin 2th).  With mu_t = t the mean sits at the origin at t.
    th, dt, o = 0.35, 0.2, 0.8
    s4 = [0.12, 0.12, 0.12, 0.6]
    q = [math.cos(th), 0, 0, math.sin(th)]
    t = 0.5
    sc = _scene([[0, 0, 0, t]], [s4], [q], [q], [o], [[0.5, 0.5, 0.5]])
    vw = _view(33, 33, 60.0, 3.0, t)
    c, s = math.cos(2 * th), math.sin(2 * th)
    v = c * s * (s4[0] ** 2 - s4[3] ** 2) / (s * s * s4[0] ** 2 + c * c * s4[3] ** 2)
    E = vw["world_to_cam"]

    def proj(p):
        x = E[:, :3] @ np.asarray(p, float) + E[:, 3]
        return np.array([vw["fx"] * x[0] / x[2] + vw["cx"], vw["fy"] * x[1] / x[2] + vw["cy"]])

    want = proj([v * dt, 0, 0]) - proj([0, 0, 0])
    assert abs(want[0]) > 0.5
    with oracle.Frame(sc, 0, 0, vw, CF, exact_f64=True) as fr:
        fr.set_channels(depth=True, flow=True, flow_dt=dt)
        out = fr.render(np.array([[16, 16]]))
    # centre pixel: G = 1, p(t) = 1, T = 1 in front, so the weight is o
    np.testing.assert_allclose(out["ext"][0, 0], o * 3.0, atol=1e-12)
    np.testing.assert_allclose(out["ext"][0, 1:], o * want, atol=1e-12)


def _tiny(rng, n=6):
    m4 = np.concatenate([rng.uniform(-0.35, 0.35, (n, 3)), rng.uniform(0.3, 0.7, (n, 1))], 1)
    s4 = np.exp(rng.normal(-2.0, 0.3, (n, 4)))
    s4[:, 3] = np.exp(rng.normal(-1.2, 0.2, n))
    ql = rng.normal(size=(n, 4)) * rng.uniform(0.5, 2.0, (n, 1))
    qr = rng.normal(size=(n, 4)) * rng.uniform(0.5, 2.0, (n, 1))
    sh = rng.normal(0, 0.15, (n, 2, 4, 3))
    sh[:, 0, 0, :] = rng.uniform(0.5, 1.5, (n, 3))
    return dict(mean4=m4, scale4=s4, rot_l=ql, rot_r=qr, opacity=rng.uniform(0.2, 0.8, n), sh=sh)


def _tiny_view(W=32, H=32, f=36.0, t=0.55):
    return dict(width=W, height=H, fx=f, fy=f, cx=W / 2, cy=H / 2,
                world_to_cam=np.array([[1.0, 0, 0, 0.05], [0, -1, 0, 0.02], [0, 0, -1, 2.2]]),
                t=t, background=np.array([0.2, 0.1, 0.3]))


def test_channel_backward_matches_central_differences(oracle_lib):
    rng = np.random.default_rng(34)
    arr = _tiny(rng)
    n, D = 6, 4
    feats = rng.normal(size=(n, D))
    gate = rng.uniform(0.3, 1.0, D)
    vw = _tiny_view()
    st = dict(oracle.SMOOTH_SETTINGS, time_period=1.7)
    E = D + 1 + 2
    g = rng.normal(size=(3, 32, 32))
    gx = rng.normal(size=(E, 32, 32))
    gx_noflow = gx.copy()
    gx_noflow[D + 1:] = 0.0  # flow carries no gradient

    def loss(a, f, gt):
        with oracle.Frame(a, 1, 1, vw, st, exact_f64=True) as fr:
            fr.set_channels(f, gt, depth=True, flow=True, flow_dt=0.05)
            out = fr.render()
        return float((out["rgb"] * g).sum() + (out["ext"] * gx_noflow).sum())

    with oracle.Frame(arr, 1, 1, vw, st, exact_f64=True) as fr:
        assert fr.splats()["alive"].all()
        fr.set_channels(feats, gate, depth=True, flow=True, flow_dt=0.05)
        grads = fr.backward(g, dL_dext=gx)
    checks = [("features", j) for j in range(0, n * D, 3)] + [("gate", j) for j in range(D)]
    checks += [(k, j) for k in ("mean4", "scale4", "rot_l", "rot_r", "opacity") for j in (0, 3, 5)]
    for name, j in checks:
        if name == "features":
            base = feats
        elif name == "gate":
            base = gate
        else:
            base = arr[name]
        h = 1e-6 * max(1.0, abs(base.reshape(-1)[j]))
        vals = []
        for sgn in (1, -1):
            a = {k: v.copy() for k, v in arr.items()}
            f, gt = feats.copy(), gate.copy()
            tgt = f if name == "features" else gt if name == "gate" else a[name]
            tgt.reshape(-1)[j] += sgn * h
            vals.append(loss(a, f, gt))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = grads[name].reshape(-1)[j]
        scale = np.abs(grads[name]).max()
        assert abs(fd - an) <= 1e-6 * (abs(an) + 1e-2 * scale), (name, j, fd, an)


def test_depth_gradient_reaches_the_mean(oracle_lib):
    # dL/d(depth channel) alone (zero image gradient): moving a Gaussian along the view axis
    # changes the depth channel, so its mean receives a gradient along the axis.
    rng = np.random.default_rng(35)
    arr = _tiny(rng)
    vw = _tiny_view()
    st = dict(oracle.SMOOTH_SETTINGS, time_period=1.7)
    with oracle.Frame(arr, 1, 1, vw, st, exact_f64=True) as fr:
        fr.set_channels(depth=True)
        grads = fr.backward(np.zeros((3, 32, 32)), dL_dext=np.ones((1, 32, 32)))
    assert np.abs(grads["mean4"][:, 2]).max() > 0
    assert np.all(grads["sh"] == 0.0)
