"""ctypes binding of the FP64 CPU oracle (``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it; the GPU library never does.  Inputs are the float32 arrays of
``paper_2412_20720_amd.scenes`` promoted to float64, so input rounding is not counted as error.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC_PATH = os.path.join(HERE, "oracle.cpp")
# G4D_ORACLE_LIB points the binding at another build of oracle.cpp (the mutation test uses it
# to load copies with planted mistakes).
LIB_OVERRIDE = os.environ.get("G4D_ORACLE_LIB")
LIB_PATH = LIB_OVERRIDE or os.path.join(HERE, "liboracle.so")

# Renderer settings (readings of the paper where it is silent; see the oracle header) and the
# parity margins within which a discrete decision is marked as legitimately ambiguous between
# FP32 and FP64.  Each margin is set from the FP32 error of its deciding quantity as measured
# on the GPU against this oracle (tests check that every measured error stays within half its
# margin): camera depth 1.9e-7 relative to max(1, z), so two depths differ by at most 3.8e-7
# and margin_depth is 2e-6; d2 6.0e-5 relative, margin_d2 2e-4; alpha, whose relative error is
# about half the absolute error of d2 (up to 9 margin_d2 / 2 = 9e-4 at the cutoff), margin_alpha
# 1e-3; the final transmittance 6.2e-6 relative, margin_T 1e-4; culls (p(t) and the near
# plane) margin_cull 1e-4.
DEFAULT_SETTINGS: Dict[str, float] = dict(
    near_z=0.2, marginal_min=1.0 / 255.0, cutoff_sigma=3.0, blur=0.3, jacobian_margin=0.15,
    alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4, color_offset=0.5, color_min=0.0,
    time_period=1.0,
    margin_d2=2e-4, margin_alpha=1e-3, margin_T=1e-4, margin_depth=2e-6, margin_cull=1e-4,
)

# Smooth settings for finite differences: the jumps left are at most exp(-12.5) per pixel.
SMOOTH_SETTINGS = dict(DEFAULT_SETTINGS, cutoff_sigma=5.0, alpha_min=1e-6, T_min=1e-8,
                       marginal_min=1e-8)


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with g++ (-O2, OpenMP)."""
    tmp = f"{LIB_PATH}.tmp{os.getpid()}"  # one per process: parallel test workers may build
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC_PATH]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Gaussians(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32), ("t_degree", C.c_int32),
                ("mean4", C.POINTER(C.c_double)), ("scale4", C.POINTER(C.c_double)),
                ("rot_l", C.POINTER(C.c_double)), ("rot_r", C.POINTER(C.c_double)),
                ("opacity", C.POINTER(C.c_double)), ("sh", C.POINTER(C.c_double)),
                ("mask", C.POINTER(C.c_double)), ("mask_threshold", C.c_double)]


class _View(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("world_to_cam", C.c_double * 12), ("t", C.c_double),
                ("background", C.c_double * 3)]


_SETTING_NAMES = ["near_z", "marginal_min", "cutoff_sigma", "blur", "jacobian_margin",
                  "alpha_min", "alpha_max", "T_min", "color_offset", "color_min", "time_period",
                  "margin_d2", "margin_alpha", "margin_T", "margin_depth", "margin_cull"]


class _Settings(C.Structure):
    _fields_ = [(k, C.c_double) for k in _SETTING_NAMES]


class _Grads(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_double)) for k in
                ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh", "mask", "densify")]


class _Channels(C.Structure):
    _fields_ = [("n_features", C.c_int32), ("features", C.POINTER(C.c_double)),
                ("gate", C.POINTER(C.c_double)), ("depth", C.c_int32), ("flow", C.c_int32),
                ("flow_dt", C.c_double)]


SPLAT_DTYPE = np.dtype([("alive", np.int32), ("optional", np.int32), ("depth", np.float64),
                        ("mean2d", np.float64, 2), ("cov2d", np.float64, 3),
                        ("conic", np.float64, 3), ("p_t", np.float64), ("opt", np.float64),
                        ("color", np.float64, 3), ("mean3", np.float64, 3),
                        ("cov3", np.float64, 6)])

_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not LIB_OVERRIDE and (not os.path.exists(LIB_PATH) or
                                 os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH)):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_rotation.argtypes = [dp, dp, dp]
        L.orc_slice.argtypes = [dp, dp, dp, dp, C.c_double, dp, dp, dp, dp]
        L.orc_legendre.argtypes = [C.c_int, C.c_int, C.c_double]
        L.orc_legendre.restype = C.c_double
        L.orc_sh_basis.argtypes = [C.c_int, dp, dp]
        L.orc_frame_new.argtypes = [C.POINTER(_Gaussians), C.POINTER(_View),
                                    C.POINTER(_Settings), C.c_int]
        L.orc_frame_new.restype = C.c_void_p
        L.orc_frame_free.argtypes = [C.c_void_p]
        L.orc_frame_splats.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_frame_set_channels.argtypes = [C.c_void_p, C.POINTER(_Channels)]
        L.orc_frame_set_channels.restype = C.c_int
        L.orc_frame_render.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_frame_variants.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_frame_backward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(_Grads),
                                         C.c_void_p, C.c_void_p]
        L.orc_frame_backward_splat.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_decode_compact.argtypes = [C.c_int, C.c_int, C.c_int] + [C.c_void_p] * 5 + \
            [C.c_double, C.c_double] + [C.c_void_p] * 12
        L.orc_sky.argtypes = [C.POINTER(_View), dp, C.c_int, C.c_double, dp, dp, C.c_void_p]
        L.orc_sky_backward.argtypes = [C.POINTER(_View), C.c_int, dp, dp]
        L.orc_frame_set_background.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32), dtype=np.float64)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def rotation(q_l, q_r) -> np.ndarray:
    """4x4 rotation L(q_l/|q_l|) R(q_r/|q_r|) (float64 inputs taken as given)."""
    ql = np.ascontiguousarray(q_l, np.float64)
    qr = np.ascontiguousarray(q_r, np.float64)
    R = np.zeros(16)
    lib().orc_rotation(_dp(ql), _dp(qr), _dp(R))
    return R.reshape(4, 4)


def slice_gaussian(mean4, scale4, q_l, q_r, t):
    """(Sigma4, conditional mean, conditional covariance, p(t)) in float64."""
    args = [np.ascontiguousarray(x, np.float64) for x in (mean4, scale4, q_l, q_r)]
    cov4, mu, cov3, pt = np.zeros(16), np.zeros(3), np.zeros(9), np.zeros(1)
    lib().orc_slice(*[_dp(a) for a in args], float(t), _dp(cov4), _dp(mu), _dp(cov3), _dp(pt))
    return cov4.reshape(4, 4), mu, cov3.reshape(3, 3), float(pt[0])


def legendre(l: int, m: int, x: float) -> float:
    return float(lib().orc_legendre(l, m, float(x)))


def sh_basis(deg: int, direction) -> np.ndarray:
    d = np.ascontiguousarray(direction, np.float64)
    Y = np.zeros((deg + 1) ** 2)
    lib().orc_sh_basis(deg, _dp(d), _dp(Y))
    return Y


def _make_view(view: Dict, exact_f64: bool) -> "_View":
    conv_s = (lambda x: float(x)) if exact_f64 else (lambda x: float(np.float32(x)))
    return _View(int(view["width"]), int(view["height"]), conv_s(view["fx"]), conv_s(view["fy"]),
                 conv_s(view["cx"]), conv_s(view["cy"]),
                 (C.c_double * 12)(*[conv_s(x) for x in np.asarray(view["world_to_cam"]).ravel()]),
                 conv_s(view["t"]),
                 (C.c_double * 3)(*[conv_s(x) for x in np.asarray(view["background"]).ravel()]))


def decode_compact(c: Dict) -> Dict[str, np.ndarray]:
    """Full float64 parameters of a compact model (see ``scenes.make_compact``): mean4, scale4,
    rot_l, rot_r, opacity, sh [n, t+1, (s+1)^2, 3]."""
    n, ds, dt = int(c["n"]), int(c["sh_degree"]), int(c["t_degree"])
    K = (dt + 1) * (ds + 1) ** 2 * 3
    u8 = lambda k: np.ascontiguousarray(c[k], np.uint8)
    cb = lambda k: np.ascontiguousarray(np.asarray(c[k], np.float32), np.float64)
    out = dict(mean4=np.zeros((n, 4)), scale4=np.zeros((n, 4)), rot_l=np.zeros((n, 4)),
               rot_r=np.zeros((n, 4)), opacity=np.zeros(n), sh=np.zeros((n, dt + 1, (ds + 1) ** 2, 3)))
    keep = [np.ascontiguousarray(c["mean4_h"], np.uint16), u8("scale_idx"), u8("rot_l_idx"),
            u8("rot_r_idx"), u8("opacity_q"), u8("dc_idx"), u8("rest_idx"), cb("scale_cb"),
            cb("rot_cb"), cb("dc_cb"), cb("rest_cb")]
    assert keep[-1].shape == (8, 256, K - 3)
    lib().orc_decode_compact(
        n, ds, dt, *[a.ctypes.data for a in keep[:5]],
        float(np.float32(c["op_lo"])), float(np.float32(c["op_hi"])),
        *[a.ctypes.data for a in keep[5:]], *[out[k].ctypes.data for k in
                                              ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh")])
    return out


def sky(view: Dict, cube: np.ndarray, margin: float = 1e-5, exact_f64: bool = False):
    """Cube-map sky of a view: (sky [3, H, W], alt [3, H, W], near [H, W]); alt is the lookup
    on the other face where the face choice is within `margin` of a tie (else equal to sky)."""
    v = _make_view(view, exact_f64)
    R = int(cube.shape[1])
    cb = np.ascontiguousarray(cube, np.float64) if exact_f64 else _f64(cube)
    H, W = v.height, v.width
    out, alt = np.zeros((H, W, 3)), np.zeros((H, W, 3))
    near = np.zeros((H, W), np.int32)
    lib().orc_sky(C.byref(v), _dp(cb), R, float(margin), _dp(out), _dp(alt), near.ctypes.data)
    return out.transpose(2, 0, 1).copy(), alt.transpose(2, 0, 1).copy(), near


def sky_backward(view: Dict, R: int, dsky: np.ndarray, exact_f64: bool = False) -> np.ndarray:
    """Adjoint of `sky`: gradient [6, R, R, 3] of <dsky [3, H, W], sky image> w.r.t. the cube."""
    v = _make_view(view, exact_f64)
    d = np.ascontiguousarray(np.asarray(dsky, np.float64).transpose(1, 2, 0))
    out = np.zeros((6, R, R, 3))
    lib().orc_sky_backward(C.byref(v), int(R), _dp(d), _dp(out))
    return out


class Frame:
    """All Gaussians of a scene preprocessed in FP64 for one view."""

    def __init__(self, arrays: Dict[str, np.ndarray], sh_degree: int, t_degree: int, view: Dict,
                 settings: Optional[Dict[str, float]] = None, use_bins: bool = True,
                 exact_f64: bool = False, mask: Optional[np.ndarray] = None,
                 mask_threshold: float = 0.0):
        st = dict(DEFAULT_SETTINGS)
        if settings:
            st.update(settings)
        conv = (lambda a: np.ascontiguousarray(a, np.float64)) if exact_f64 else _f64
        self._arrays = {k: conv(arrays[k]) for k in
                        ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh")}
        self.n = int(self._arrays["mean4"].shape[0])
        self.sh_degree, self.t_degree = int(sh_degree), int(t_degree)
        assert self._arrays["sh"].size == self.n * (t_degree + 1) * (sh_degree + 1) ** 2 * 3
        self.view = view
        self.width, self.height = int(view["width"]), int(view["height"])
        # Volume mask: significance M per Gaussian, kept when M > threshold.
        self._mask = None if mask is None else conv(mask)
        thr = float(mask_threshold) if exact_f64 else float(np.float32(mask_threshold))
        g = _Gaussians(self.n, self.sh_degree, self.t_degree,
                       *[_dp(self._arrays[k]) for k in
                         ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh")],
                       None if self._mask is None else _dp(self._mask), thr)
        conv_s = (lambda x: float(x)) if exact_f64 else (lambda x: float(np.float32(x)))
        v = _View(self.width, self.height, conv_s(view["fx"]), conv_s(view["fy"]),
                  conv_s(view["cx"]), conv_s(view["cy"]),
                  (C.c_double * 12)(*[conv_s(x) for x in np.asarray(view["world_to_cam"]).ravel()]),
                  conv_s(view["t"]),
                  (C.c_double * 3)(*[conv_s(x) for x in np.asarray(view["background"]).ravel()]))
        # Thresholds reach the GPU as float32; the oracle takes the same rounded values.
        s = _Settings(*[float(st[k]) if (exact_f64 or k.startswith("margin_"))
                        else float(np.float32(st[k])) for k in _SETTING_NAMES])
        self.settings = st
        self._conv = conv
        self.n_ext = self.n_features = 0
        self.depth = self.flow = False
        self._h = lib().orc_frame_new(C.byref(g), C.byref(v), C.byref(s), int(use_bins))

    def set_background(self, bg: Optional[np.ndarray]) -> None:
        """Per-pixel background [3, H, W] (float64, e.g. a sky image) instead of the view's
        constant; None restores the constant."""
        if bg is None:
            self._bg = None
            lib().orc_frame_set_background(self._h, None)
            return
        self._bg = np.ascontiguousarray(np.asarray(bg, np.float64).transpose(1, 2, 0))
        lib().orc_frame_set_background(self._h, self._bg.ctypes.data)

    def set_channels(self, features: Optional[np.ndarray] = None, gate=None, depth: bool = False,
                     flow: bool = False, flow_dt: float = 0.0) -> int:
        """Attach extra channels (features [n, D] gated by `gate` [D] and normalized, depth,
        flow over `flow_dt`); returns their number E = D + depth + 2 flow."""
        D = 0 if features is None else int(np.asarray(features).shape[1])
        self._features = self._conv(features) if D else None
        self._gate = self._conv(gate) if (D and gate is not None) else None
        dt = float(flow_dt) if self._conv is not _f64 else float(np.float32(flow_dt))
        ch = _Channels(D, _dp(self._features) if D else None,
                       _dp(self._gate) if self._gate is not None else None, int(depth),
                       int(flow), dt)
        self.n_ext = int(lib().orc_frame_set_channels(self._h, C.byref(ch)))
        self.n_features, self.depth, self.flow = D, bool(depth), bool(flow)
        return self.n_ext

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_frame_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def splats(self) -> np.ndarray:
        out = np.zeros(self.n, SPLAT_DTYPE)
        lib().orc_frame_splats(self._h, out.ctypes.data)
        return out

    def render(self, xy: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
        """Render the listed pixels (int (x, y) pairs) or, with xy=None, the whole image."""
        if xy is None:
            n = self.width * self.height
            xyp = None
        else:
            xyp = np.ascontiguousarray(xy, np.int32).reshape(-1, 2)
            n = xyp.shape[0]
        rgb = np.zeros((n, 3))
        T = np.zeros(n)
        nc = np.zeros(n, np.int32)
        nm = np.zeros(n, np.int32)
        ne = np.zeros(n, np.int64)
        E = self.n_ext
        ext = np.zeros((n, E))
        lib().orc_frame_render(self._h, n, None if xyp is None else xyp.ctypes.data,
                               rgb.ctypes.data, T.ctypes.data, nc.ctypes.data, nm.ctypes.data,
                               ne.ctypes.data, ext.ctypes.data if E else None)
        out = dict(rgb=rgb, T=T, n_contrib=nc, n_marks=nm, n_evals=ne)
        if E:
            out["ext"] = ext
        if xy is None:
            H, W = self.height, self.width
            out = dict(rgb=rgb.reshape(H, W, 3).transpose(2, 0, 1).copy(), T=T.reshape(H, W),
                       n_contrib=nc.reshape(H, W), n_marks=nm.reshape(H, W),
                       n_evals=ne.reshape(H, W))
            if E:
                out["ext"] = ext.reshape(H, W, E).transpose(2, 0, 1).copy()
        return out

    def variants(self, x: int, y: int, max_marks: int = 4):
        """All admissible (rgb, T, extra channels, composited count) of pixel (x, y), or None
        if it has too many marked decisions."""
        cap = 1 << max_marks
        rgb = np.zeros((cap, 3))
        T = np.zeros(cap)
        ext = np.zeros((cap, self.n_ext))
        nc = np.zeros(cap, np.int32)
        nv = lib().orc_frame_variants(self._h, int(x), int(y), max_marks, cap, rgb.ctypes.data,
                                      T.ctypes.data, ext.ctypes.data if self.n_ext else None,
                                      nc.ctypes.data)
        if nv < 0:
            return None
        return rgb[:nv], T[:nv], ext[:nv], nc[:nv]

    def backward(self, dL_drgb: np.ndarray, grads: Optional[Dict[str, np.ndarray]] = None,
                 dL_dext: Optional[np.ndarray] = None):
        """Accumulate d(<dL_drgb, image> + <dL_dext, extra channels>)/d(params) into ``grads``
        (float64; created if None).  With features attached, ``grads`` also receives
        "features" [n, D] and "gate" [D].  The flow channels of dL_dext are ignored.  "densify"
        [n] accumulates |dL/d mean2d| of this view; with a mask, "mask" [n] the
        straight-through dL/dM."""
        if grads is None:
            grads = {k: np.zeros_like(a) for k, a in self._arrays.items()}
        grads.setdefault("densify", np.zeros(self.n))
        if self._mask is not None:
            grads.setdefault("mask", np.zeros(self.n))
        if self.n_features:
            grads.setdefault("features", np.zeros((self.n, self.n_features)))
            grads.setdefault("gate", np.zeros(self.n_features))
        g = np.ascontiguousarray(dL_drgb, np.float64).reshape(3, self.height, self.width)
        gx = None
        if dL_dext is not None and self.n_ext:
            gx = np.ascontiguousarray(dL_dext, np.float64).reshape(self.n_ext, self.height,
                                                                    self.width)
        gs = _Grads(*[_dp(grads[k]) for k in ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh")],
                    _dp(grads["mask"]) if self._mask is not None else None,
                    _dp(grads["densify"]))
        lib().orc_frame_backward(self._h, g.ctypes.data, None if gx is None else gx.ctypes.data,
                                 C.byref(gs),
                                 grads["features"].ctypes.data if self.n_features else None,
                                 grads["gate"].ctypes.data if self.n_features else None)
        return grads

    def backward_splat(self, dL_drgb: np.ndarray) -> np.ndarray:
        """Per-Gaussian gradient of (u, v, conic a, b, c, opacity*p_t, r, g, b): [n, 9]."""
        g = np.ascontiguousarray(dL_drgb, np.float64).reshape(3, self.height, self.width)
        out = np.zeros((self.n, 9))
        lib().orc_frame_backward_splat(self._h, g.ctypes.data, out.ctypes.data)
        return out


def render_scene_view(scene, view_index: int = 0, settings=None, xy=None, use_bins=True):
    """Convenience: oracle render of one view of a ``scenes.Scene``."""
    st = dict(settings or {})
    st.setdefault("time_period", scene.time_period)
    with Frame(scene.arrays(), scene.sh_degree, scene.t_degree, scene.views[view_index], st,
               use_bins=use_bins) as f:
        return f.render(xy)
