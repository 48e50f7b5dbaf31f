"""Pins of the oracle's sky composite (Sec. 5, urban scenes: I = I_gs + (1 - O_gs) M_sky(r), a
cube map queried by the pixel's view direction, consuming the remaining transmittance).

- A constant cube map is a constant background: the composite equals the plain render with
  that background, bit for bit.
- Face choice: with one color per face, every pixel shows the face of the largest |component|
  of its ray, computed here from K^-1 and the camera rotation independently of the oracle.
- Texel placement: a ray through the centre of texel (i, j) of a face (direction from the
  inverse of the published face table) returns that texel exactly.
- The sky adjoint is the transpose of the lookup (dot-product test), and central differences
  of the whole composite agree with the backward for texels and Gaussian parameters.
"""
import math

import numpy as np

import oracle
from paper_2412_20720_amd import scenes

SMOOTH = dict(oracle.SMOOTH_SETTINGS, time_period=1.7)


def _view(W, H, f, eye, target, cx=None, cy=None, t=0.5):
    E = scenes.look_at(eye, target).astype(np.float64)
    return dict(width=W, height=H, fx=f, fy=f, cx=W / 2 if cx is None else cx,
                cy=H / 2 if cy is None else cy, world_to_cam=E, t=t,
                background=np.array([0.2, 0.4, 0.6]))


def _rays(vw):
    H, W = vw["height"], vw["width"]
    ys, xs = np.mgrid[0:H, 0:W]
    d = np.stack([(xs + 0.5 - vw["cx"]) / vw["fx"], (ys + 0.5 - vw["cy"]) / vw["fy"],
                  np.ones((H, W))], -1)
    Rw = np.asarray(vw["world_to_cam"])[:, :3]
    r = d @ Rw  # camera -> world: R^T d
    return r / np.linalg.norm(r, axis=-1, keepdims=True)


def test_constant_cube_map_is_a_constant_background(oracle_lib):
    sc = scenes.make_workload(0)
    vw = dict(sc.views[0], background=np.array([0.3, 0.5, 0.7]))
    cube = np.broadcast_to(np.array([0.3, 0.5, 0.7]), (6, 4, 4, 3)).copy()
    sky, _, _ = oracle.sky(vw, cube, exact_f64=True)
    assert np.all(np.abs(sky - np.array([0.3, 0.5, 0.7])[:, None, None]) <= 1e-15)
    with oracle.Frame(sc.arrays(), 0, 0, vw, {}, exact_f64=True) as fr:
        plain = fr.render()["rgb"]
        fr.set_background(np.broadcast_to(np.array([0.3, 0.5, 0.7])[:, None, None], plain.shape))
        sky_img = fr.render()["rgb"]
    assert np.array_equal(plain, sky_img)


def test_face_choice_by_largest_component(oracle_lib):
    colors = np.arange(18, dtype=np.float64).reshape(6, 3) / 17.0
    cube = np.broadcast_to(colors[:, None, None, :], (6, 3, 3, 3)).copy()
    for eye, target in [((0, 0, 0), (1.0, 0.6, 0.3)), ((0, 0, 0), (-0.4, -1.0, 0.7)),
                        ((0, 0, 0), (0.2, 0.3, -1.0))]:
        vw = _view(64, 48, 20.0, eye, target)  # wide field of view: several faces
        sky, _, near = oracle.sky(vw, cube, exact_f64=True)
        r = _rays(vw)
        ax = np.argmax(np.abs(r), -1)
        sign = np.take_along_axis(r, ax[..., None], -1)[..., 0] < 0
        face = 2 * ax + sign
        want = colors[face].transpose(2, 0, 1)
        ok = near == 0
        assert ok.mean() > 0.99 and len(np.unique(face)) >= 3
        np.testing.assert_allclose(sky[:, ok], want[:, ok], atol=1e-14)


def _texel_dir(face, i, j, R):
    sc, tc = 2 * (i + 0.5) / R - 1, 2 * (j + 0.5) / R - 1
    return {0: (1, -tc, -sc), 1: (-1, -tc, sc), 2: (sc, 1, tc), 3: (sc, -1, -tc),
            4: (sc, -tc, 1), 5: (-sc, -tc, -1)}[face]


def test_ray_through_a_texel_centre_returns_the_texel(oracle_lib):
    rng = np.random.default_rng(50)
    R = 6
    cube = rng.uniform(0, 1, (6, R, R, 3))
    for face in (0, 1, 4, 5):  # side faces: the look-at camera needs a non-vertical axis
        for _ in range(4):
            i, j = rng.integers(0, R, 2)
            d = np.asarray(_texel_dir(face, i, j, R), float)
            vw = _view(9, 7, 30.0, (0, 0, 0), tuple(d), cx=4.5, cy=3.5)  # pixel (4, 3) on axis
            sky, _, near = oracle.sky(vw, cube, exact_f64=True)
            assert near[3, 4] == 0
            np.testing.assert_allclose(sky[:, 3, 4], cube[face, j, i], atol=1e-12)


def test_sky_adjoint_is_the_transpose(oracle_lib):
    rng = np.random.default_rng(51)
    R = 5
    vw = _view(40, 30, 15.0, (0, 0, 0), (0.7, 0.2, 0.5))
    cube = rng.normal(size=(6, R, R, 3))
    dsky = rng.normal(size=(3, 30, 40))
    sky, _, _ = oracle.sky(vw, cube, exact_f64=True)
    adj = oracle.sky_backward(vw, R, dsky, exact_f64=True)
    np.testing.assert_allclose((dsky * sky).sum(), (adj * cube).sum(), rtol=1e-12)


def _tiny(rng, n=6):
    m4 = np.concatenate([rng.uniform(-0.35, 0.35, (n, 3)), rng.uniform(0.3, 0.7, (n, 1))], 1)
    s4 = np.exp(rng.normal(-2.0, 0.3, (n, 4)))
    s4[:, 3] = np.exp(rng.normal(-1.2, 0.2, n))
    ql = rng.normal(size=(n, 4)) * rng.uniform(0.5, 2.0, (n, 1))
    qr = rng.normal(size=(n, 4)) * rng.uniform(0.5, 2.0, (n, 1))
    sh = rng.normal(0, 0.15, (n, 2, 4, 3))
    sh[:, 0, 0, :] = rng.uniform(0.5, 1.5, (n, 3))
    return dict(mean4=m4, scale4=s4, rot_l=ql, rot_r=qr, opacity=rng.uniform(0.2, 0.8, n), sh=sh)


def test_sky_composite_backward_matches_central_differences(oracle_lib):
    rng = np.random.default_rng(52)
    arr = _tiny(rng)
    R = 4
    cube = rng.uniform(0, 1, (6, R, R, 3))
    vw = dict(width=32, height=32, fx=36.0, fy=36.0, cx=16.0, cy=16.0,
              world_to_cam=np.array([[1.0, 0, 0, 0.05], [0, -1, 0, 0.02], [0, 0, -1, 2.2]]),
              t=0.55, background=np.zeros(3))
    g = rng.normal(size=(3, 32, 32))

    def loss(a, cb):
        sky, _, _ = oracle.sky(vw, cb, exact_f64=True)
        with oracle.Frame(a, 1, 1, vw, SMOOTH, exact_f64=True) as fr:
            fr.set_background(sky)
            return float((fr.render()["rgb"] * g).sum())

    sky, _, _ = oracle.sky(vw, cube, exact_f64=True)
    with oracle.Frame(arr, 1, 1, vw, SMOOTH, exact_f64=True) as fr:
        fr.set_background(sky)
        out = fr.render()
        grads = fr.backward(g)
    d_cube = oracle.sky_backward(vw, R, g * out["T"][None], exact_f64=True)
    h = 1e-6
    hit = np.argwhere(np.abs(d_cube) > 0)
    assert len(hit) > 10
    for idx in hit[rng.choice(len(hit), 6, replace=False)]:
        cp, cm = cube.copy(), cube.copy()
        cp[tuple(idx)] += h
        cm[tuple(idx)] -= h
        fd = (loss(arr, cp) - loss(arr, cm)) / (2 * h)
        assert abs(fd - d_cube[tuple(idx)]) <= 1e-6 * (abs(fd) + 1e-2), (idx, fd)
    for name in ("mean4", "opacity", "scale4"):
        scale = np.abs(grads[name]).max()
        for j in (0, 3):
            a = {k: v.copy() for k, v in arr.items()}
            b = {k: v.copy() for k, v in arr.items()}
            a[name].reshape(-1)[j] += h
            b[name].reshape(-1)[j] -= h
            fd = (loss(a, cube) - loss(b, cube)) / (2 * h)
            an = grads[name].reshape(-1)[j]
            assert abs(fd - an) <= 1e-6 * (abs(an) + 1e-2 * scale), (name, j, fd, an)
