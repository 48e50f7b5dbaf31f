"""Seeded synthetic 4D Gaussian scenes and cameras.

This module only draws inputs: Gaussian parameter arrays, pinhole cameras and upstream image
gradients.  It holds none of the render's arithmetic, so both the GPU library and the CPU oracle
can be fed from it without sharing any of the method.

Parameter layout (structure of arrays, float32, row-major), following the 4D Gaussian
representation of Sec. 3.2 (mean (x, y, z, t), diagonal 4D scale, left/right rotors) and the
4D spherindrical-harmonic color:

    mean4   [N, 4]                       (mu_x, mu_y, mu_z, mu_t)
    scale4  [N, 4]                       activated (positive) scales (s_x, s_y, s_z, s_t)
    rot_l   [N, 4]                       left rotor  (a, b, c, d), need not be unit length
    rot_r   [N, 4]                       right rotor (p, q, r, s), need not be unit length
    opacity [N]                          activated opacity in (0, 1)
    sh      [N, t_degree+1, (sh_degree+1)^2, 3]   coefficient k[n, l*l+l+m, channel]

A view is a dict with width, height, fx, fy, cx, cy, world_to_cam (3x4 [R|tau], OpenCV axes:
x right, y down, z forward), t and background (3,).

Every workload draws from ``numpy.random.default_rng(1000 + index)`` in a fixed order:
mu_xyz, mu_t, log s_xyz, log s_t, q_l, q_r, opacity logits, SH DC, SH rest, then per-workload
extras, then cameras and times, then one dL/dimage per view.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List

import numpy as np

__all__ = ["Scene", "WORKLOADS", "make_workload", "make_dl_dimage", "look_at", "pinhole",
           "ring_views", "random_scene", "subset", "stress_variant"]

# Constant of the degree-0 real spherical harmonic, 1 / (2 sqrt(pi)); used only to store an
# RGB draw as the DC coefficient that reproduces it.
_Y00 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Scene:
    mean4: np.ndarray
    scale4: np.ndarray
    rot_l: np.ndarray
    rot_r: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int
    t_degree: int
    time_period: float
    views: List[Dict]
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.mean4.shape[0])

    def arrays(self):
        return dict(mean4=self.mean4, scale4=self.scale4, rot_l=self.rot_l, rot_r=self.rot_r,
                    opacity=self.opacity, sh=self.sh)

    @property
    def pixels(self) -> int:
        return int(sum(v["width"] * v["height"] for v in self.views))


def look_at(eye, target, up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """World-to-camera [R|tau] (3x4) for a camera at ``eye`` looking at ``target``.

    Rows of R are (right, down, forward): forward f = normalize(target - eye),
    right r = normalize(f x up), down d = f x r; tau = -R eye.
    """
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    return np.concatenate([R, (-R @ eye)[:, None]], axis=1).astype(np.float32)


def pinhole(width: int, height: int, fov_deg: float, world_to_cam, t: float,
            background=(0.0, 0.0, 0.0)) -> Dict:
    """Pinhole view with horizontal field of view ``fov_deg`` and centred principal point."""
    f = width / (2.0 * math.tan(math.radians(fov_deg) / 2.0))
    return dict(width=int(width), height=int(height), fx=np.float32(f), fy=np.float32(f),
                cx=np.float32(width / 2.0), cy=np.float32(height / 2.0),
                world_to_cam=np.asarray(world_to_cam, np.float32).reshape(3, 4),
                t=np.float32(t), background=np.asarray(background, np.float32).reshape(3))


def _unit_rows(x: np.ndarray) -> np.ndarray:
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def random_scene(rng: np.random.Generator, n: int, *, box=((-1, 1), (-1, 1), (-1, 1)),
                 t_range=(0.0, 1.0), log_s=(-3.0, 0.5), log_st=(-2.0, 0.5),
                 sh_degree=0, t_degree=0, rgb_dc=True):
    """Draw the Gaussian parameter arrays in the fixed order (see module docstring)."""
    lo = np.array([b[0] for b in box], np.float64)
    hi = np.array([b[1] for b in box], np.float64)
    mu_xyz = rng.uniform(lo, hi, size=(n, 3))
    mu_t = rng.uniform(t_range[0], t_range[1], size=n)
    log_sxyz = rng.normal(log_s[0], log_s[1], size=(n, 3))
    log_st = rng.normal(log_st[0], log_st[1], size=n)
    q_l = _unit_rows(rng.normal(size=(n, 4)))
    q_r = _unit_rows(rng.normal(size=(n, 4)))
    logit = rng.normal(size=n)
    n_sh = (sh_degree + 1) ** 2
    sh = np.zeros((n, t_degree + 1, n_sh, 3), np.float64)
    if rgb_dc:
        sh[:, 0, 0, :] = (rng.uniform(0.0, 1.0, size=(n, 3)) - 0.5) / _Y00
    else:
        sh[:, 0, 0, :] = rng.uniform(0.0, 1.0, size=(n, 3))
    n_rest = (t_degree + 1) * n_sh - 1
    if n_rest > 0:
        rest = rng.normal(0.0, 0.1, size=(n, n_rest, 3))
        flat = sh.reshape(n, (t_degree + 1) * n_sh, 3)
        flat[:, 1:, :] = rest
        sh = flat.reshape(sh.shape)
    mean4 = np.concatenate([mu_xyz, mu_t[:, None]], axis=1)
    scale4 = np.exp(np.concatenate([log_sxyz, log_st[:, None]], axis=1))
    opacity = 1.0 / (1.0 + np.exp(-logit))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(mean4=f32(mean4), scale4=f32(scale4), rot_l=f32(q_l), rot_r=f32(q_r),
                opacity=f32(opacity), sh=f32(sh))


def ring_views(angles, times, sizes, fov_deg=50.0, radius=4.0, background=(0.0, 0.0, 0.0)):
    views = []
    for a, t, (w, h) in zip(angles, times, sizes):
        eye = (radius * math.sin(a), 0.0, radius * math.cos(a))
        views.append(pinhole(w, h, fov_deg, look_at(eye, (0.0, 0.0, 0.0)), t, background))
    return views


def _w0(rng):
    """2,000 Gaussians in [-1,1]^3 x [0,1], degree-0 RGB, one 128x128 view at t = 0.5."""
    p = random_scene(rng, 2000)
    views = [pinhole(128, 128, 60.0, look_at((0, 0, 3), (0, 0, 0)), 0.5)]
    return Scene(**p, sh_degree=0, t_degree=0, time_period=1.0, views=views)


def _cfg1_params(rng, n):
    return random_scene(rng, n, box=((-2, 2),) * 3, sh_degree=3, t_degree=1, rgb_dc=False)


def _w1(rng):
    """100k Gaussians in [-2,2]^3, SH degree 3 x Fourier degree 1, one 1352x1014 view."""
    p = _cfg1_params(rng, 100_000)
    t = float(rng.uniform(0.0, 1.0))
    views = [pinhole(1352, 1014, 50.0, look_at((0, 0, 4), (0, 0, 0)), t)]
    return Scene(**p, sh_degree=3, t_degree=1, time_period=1.0, views=views)


def _w2(rng, mixed=True):
    """300k Gaussians, 8 ring cameras x 2 timestamps; even cameras 1352x1014, odd 800x800."""
    p = _cfg1_params(rng, 300_000)
    angles, times, sizes = [], [], []
    for t in (0.25, 0.75):
        for k in range(8):
            angles.append(2.0 * math.pi * k / 8.0)
            times.append(t)
            sizes.append((1352, 1014) if (k % 2 == 0 or not mixed) else (800, 800))
    views = ring_views(angles, times, sizes)
    return Scene(**p, sh_degree=3, t_degree=1, time_period=1.0, views=views)


def _w3(rng):
    """500k Gaussians over t in [0,10] with short temporal support, 32 random ring views."""
    p = random_scene(rng, 500_000, box=((-2, 2),) * 3, t_range=(0.0, 10.0), log_st=(-1.0, 0.7),
                     sh_degree=3, t_degree=1, rgb_dc=False)
    angles = rng.uniform(0.0, 2.0 * math.pi, size=32)
    times = rng.uniform(0.0, 10.0, size=32)
    views = ring_views(angles, times, [(1352, 1014)] * 32)
    return Scene(**p, sh_degree=3, t_degree=1, time_period=10.0, views=views)


def _w4(rng):
    """2M Gaussians in a 40x6x40 box over t in [0,20]; 30% near-static; 8 forward-moving views."""
    n = 2_000_000
    p = random_scene(rng, n, box=((-20, 20), (-3, 3), (-20, 20)), t_range=(0.0, 20.0),
                     log_s=(-2.5, 0.8), log_st=(-1.0, 0.7), sh_degree=3, t_degree=1,
                     rgb_dc=False)
    static = rng.uniform(size=n) < 0.3
    log_st_static = rng.uniform(math.log(20.0), math.log(100.0), size=n)
    ql = p["rot_l"]
    # Right rotor (a, b, c, -d) of the left rotor (a, b, c, d): the product of the two
    # isoclinic matrices then fixes the time axis (block-diagonal covariance).
    qr_static = ql * np.array([1, 1, 1, -1], np.float32)
    p["rot_r"] = np.where(static[:, None], qr_static, p["rot_r"]).astype(np.float32)
    st = np.where(static, np.exp(log_st_static), p["scale4"][:, 3])
    p["scale4"][:, 3] = st.astype(np.float32)
    views = []
    for k in range(8):
        eye = (0.0, 0.0, -18.0 + 4.0 * k)
        views.append(pinhole(1920, 1280, 70.0, look_at(eye, (eye[0], eye[1], eye[2] + 1.0)),
                             20.0 * (k + 0.5) / 8.0))
    return Scene(**p, sh_degree=3, t_degree=1, time_period=20.0, views=views)


WORKLOADS = {
    0: ("w0_2k_128px", _w0),
    1: ("w1_100k_1352x1014", _w1),
    2: ("w2_300k_16views_mixed", lambda r: _w2(r, True)),
    "2b": ("w2b_300k_16views_1352x1014", lambda r: _w2(r, False)),
    3: ("w3_500k_32views_t10", _w3),
    4: ("w4_2M_8views_1920x1280", _w4),
}


def make_workload(index) -> Scene:
    """Build workload ``index`` (0..4 or "2b") from its fixed seed."""
    name, fn = WORKLOADS[index]
    seed_index = 2 if index == "2b" else int(index)
    rng = np.random.default_rng(1000 + seed_index)
    scene = fn(rng)
    scene.name = name
    return scene


def make_dl_dimage(scene: Scene, seed: int = 7) -> List[np.ndarray]:
    """Upstream dL/dimage ~ N(0,1) per view, planar [3, H, W] float32."""
    rng = np.random.default_rng(seed)
    return [rng.normal(size=(3, v["height"], v["width"])).astype(np.float32) for v in scene.views]


def make_features(scene: Scene, dim: int = 32, seed: int = 11) -> np.ndarray:
    """Per-Gaussian feature vectors f ~ N(0, 1), [N, dim] float32 (the segmentation features
    are learned; D = 32 as in the paper's segmentation experiments)."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=(scene.n, dim)).astype(np.float32)


def make_gate(dim: int = 32, seed: int = 12) -> np.ndarray:
    """A scale gate S(s) in [0, 1]^dim, float32."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, dim).astype(np.float32)


def make_dl_dchannels(scene: Scene, n_channels: int, seed: int = 13) -> List[np.ndarray]:
    """Upstream dL/d(extra channels) ~ N(0,1) per view, planar [E, H, W] float32."""
    rng = np.random.default_rng(seed)
    return [rng.normal(size=(n_channels, v["height"], v["width"])).astype(np.float32)
            for v in scene.views]


def make_mask(scene: Scene, seed: int = 14) -> np.ndarray:
    """Volume-mask significances M ~ U(0, 1) per Gaussian, float32."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, scene.n).astype(np.float32)


def make_cube(resolution: int = 16, seed: int = 15) -> np.ndarray:
    """A sky cube map [6, R, R, 3] ~ U(0, 1), float32 (the urban sky model is learned)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, (6, resolution, resolution, 3)).astype(np.float32)


def make_compact(n: int, sh_degree: int = 3, t_degree: int = 1, extent: float = 2.0,
                 seed: int = 16) -> Dict[str, np.ndarray]:
    """A synthetic compact model with the layout of the compact 4DGS (residual VQ codebooks
    of 6 x 64 for the log-scale, the rotors and the direct color component, 8 x 256 for the
    rest of the 4DSH; half-precision positions; 8-bit min-max opacity).  The first codebook
    of each model carries the bulk of the value and the others small residuals, so that the
    decoded parameters follow the distributions of the workloads above."""
    rng = np.random.default_rng(seed)
    K = (t_degree + 1) * (sh_degree + 1) ** 2 * 3

    def cb(shape, first, rest):
        c = rng.normal(0.0, rest, shape)
        c[0] = first(shape[1:])
        return c.astype(np.float32)

    y00 = 0.28209479177387814
    m4 = np.concatenate([rng.uniform(-extent, extent, (n, 3)), rng.uniform(0.0, 1.0, (n, 1))], 1)
    return dict(
        n=n, sh_degree=sh_degree, t_degree=t_degree,
        mean4_h=m4.astype(np.float16).view(np.uint16),
        scale_idx=rng.integers(0, 64, (n, 6), dtype=np.uint8),
        rot_l_idx=rng.integers(0, 64, (n, 6), dtype=np.uint8),
        rot_r_idx=rng.integers(0, 64, (n, 6), dtype=np.uint8),
        opacity_q=rng.integers(0, 256, n, dtype=np.uint8), op_lo=np.float32(0.02),
        op_hi=np.float32(0.98),
        dc_idx=rng.integers(0, 64, (n, 6), dtype=np.uint8),
        rest_idx=rng.integers(0, 256, (n, 8), dtype=np.uint8),
        scale_cb=cb((6, 64, 4), lambda s: np.stack([rng.normal(-3.0, 0.5, s[0])] * 3 +
                                                   [rng.normal(-2.0, 0.5, s[0])], 1), 0.05),
        rot_cb=cb((6, 64, 4), lambda s: rng.normal(0.0, 1.0, s), 0.1),
        dc_cb=cb((6, 64, 3), lambda s: (rng.uniform(0.0, 1.0, s) - 0.5) / y00, 0.05),
        rest_cb=cb((8, 256, K - 3), lambda s: rng.normal(0.0, 0.1, s), 0.02),
    )


def subset(scene: Scene, idx) -> Scene:
    """Scene restricted to the Gaussians ``idx`` (same views)."""
    idx = np.asarray(idx)
    return Scene(mean4=scene.mean4[idx].copy(), scale4=scene.scale4[idx].copy(),
                 rot_l=scene.rot_l[idx].copy(), rot_r=scene.rot_r[idx].copy(),
                 opacity=scene.opacity[idx].copy(), sh=scene.sh[idx].copy(),
                 sh_degree=scene.sh_degree, t_degree=scene.t_degree,
                 time_period=scene.time_period, views=list(scene.views), name=scene.name)


def stress_variant(scene: Scene, seed: int = 17, opacity=(0.95, 1.0),
                   rotor_scale=(0.3, 3.0)) -> Scene:
    """The scene with opacities redrawn ~U(opacity) (None keeps them) and every rotor row
    multiplied by its own factor ~U(rotor_scale) (None keeps them unit).  High opacities make
    o p(t) reach the alpha_max clamp; non-unit rotors exercise the normalization inside the
    render.  Draw order: opacities, then the left and right rotor factors."""
    rng = np.random.default_rng(seed)
    out = subset(scene, np.arange(scene.n))
    out.name = scene.name + "_stress"
    if opacity is not None:
        out.opacity = rng.uniform(opacity[0], opacity[1], scene.n).astype(np.float32)
    if rotor_scale is not None:
        fl = rng.uniform(rotor_scale[0], rotor_scale[1], (scene.n, 1))
        fr = rng.uniform(rotor_scale[0], rotor_scale[1], (scene.n, 1))
        out.rot_l = (scene.rot_l * fl).astype(np.float32)
        out.rot_r = (scene.rot_r * fr).astype(np.float32)
    return out
