"""PyTorch front end: a Renderer owning a g4d context and a torch.autograd.Function.

PyTorch provides device memory and the stream; every step of the render runs in the HIP
kernels of libg4d.so.  Activations (exp for scales, sigmoid for opacity) stay in PyTorch; the
library sees activated scales and opacity and raw rotors.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Optional, Sequence

import torch

from . import _binding as B

PARAM_NAMES = ("mean4", "scale4", "rot_l", "rot_r", "opacity", "sh")


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Renderer:
    """One g4d context on one GPU.  The context keeps the state of its last forward for the
    matching backward (the library reports G4D_ESTATE for any other).  The autograd functions
    below accept several renders on one Renderer before their backwards: a backward whose
    forward is no longer the context's last one runs that forward again first (the forward is
    deterministic, so its state is the one the outputs came from)."""

    def __init__(self, device: int | torch.device = 0):
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if dev.type != "cuda":
            raise ValueError("Renderer needs a GPU device")
        self.device = dev
        self._ctx = C.c_void_p()
        B.check(B.lib().g4d_create(C.byref(self._ctx), dev.index or 0))

    def close(self) -> None:
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            B.lib().g4d_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- marshalling ---------------------------------------------------------------------
    def gaussians(self, mean4, scale4, rot_l, rot_r, opacity, sh, sh_degree: int,
                  t_degree: int, mask: Optional[torch.Tensor] = None,
                  mask_threshold: float = 0.0) -> B.g4d_gaussians:
        """Parameter pointers for the ABI; `mask` [N] is the optional volume-mask
        significance (kept where mask > mask_threshold)."""
        n = int(mean4.shape[0])
        k = (sh_degree + 1) ** 2
        want = {"mean4": (n, 4), "scale4": (n, 4), "rot_l": (n, 4), "rot_r": (n, 4),
                "opacity": (n,), "sh": (n, t_degree + 1, k, 3)}
        for name, t in zip(PARAM_NAMES, (mean4, scale4, rot_l, rot_r, opacity, sh)):
            if t.dtype != torch.float32 or t.device != self.device or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 tensor on {self.device}")
            if tuple(t.shape) != want[name]:
                raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {want[name]}")
        if mask is not None and (mask.dtype != torch.float32 or mask.device != self.device or
                                 not mask.is_contiguous() or tuple(mask.shape) != (n,)):
            raise ValueError(f"mask must be a contiguous float32 [{n}] tensor on {self.device}")
        return B.g4d_gaussians(n, sh_degree, t_degree, mean4.data_ptr(), scale4.data_ptr(),
                               rot_l.data_ptr(), rot_r.data_ptr(), opacity.data_ptr(),
                               sh.data_ptr(), None if mask is None else mask.data_ptr(),
                               float(mask_threshold))

    @staticmethod
    def pixel_count(views) -> int:
        return sum(int(v["width"]) * int(v["height"]) for v in views)

    @staticmethod
    def pixel_count_array(views) -> int:
        """Pixels of a g4d_view array (or of a list of view dicts)."""
        if isinstance(views, C.Array):
            return sum(int(v.width) * int(v.height) for v in views)
        return Renderer.pixel_count(views)

    def pairs(self):
        """Sorted (tile id, slot) pairs and tile ranges of the last forward, as int64 CPU
        tensors: (tile_ids [n_pairs], slots [n_pairs], ranges [n_tiles, 2])."""
        st = self.stats()
        n, nt = st["n_pairs"], st["n_tiles"]
        tid = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        slots = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        ranges = torch.empty((max(nt, 1), 2), dtype=torch.int32, device=self.device)
        B.check(B.lib().g4d_get_pairs(self._ctx, tid.data_ptr(), slots.data_ptr(),
                                      ranges.data_ptr(), _stream_handle(self.device)), self._ctx)
        torch.cuda.synchronize(self.device)
        u32 = lambda t: t.cpu().to(torch.int64) & 0xFFFFFFFF
        return u32(tid[:n]), u32(slots[:n]), u32(ranges[:nt])

    # -- entry points ----------------------------------------------------------------------
    def forward(self, g: B.g4d_gaussians, views, settings: B.g4d_settings, out_rgb: torch.Tensor,
                out_T: Optional[torch.Tensor]) -> None:
        va = views if isinstance(views, C.Array) else B.make_views(views)
        st = _stream_handle(self.device)
        B.check(B.lib().g4d_render_forward(self._ctx, C.byref(g), va, len(va), C.byref(settings),
                                           out_rgb.data_ptr(),
                                           None if out_T is None else out_T.data_ptr(), st),
                self._ctx)

    def backward(self, g: B.g4d_gaussians, views, settings: B.g4d_settings, dL: torch.Tensor,
                 grads: Dict[str, torch.Tensor]) -> None:
        va = views if isinstance(views, C.Array) else B.make_views(views)
        st = _stream_handle(self.device)
        gr = B.g4d_grads(*[grads[k].data_ptr() if grads.get(k) is not None else None
                           for k in PARAM_NAMES + ("mask", "densify")])
        B.check(B.lib().g4d_render_backward(self._ctx, C.byref(g), va, len(va), C.byref(settings),
                                            dL.data_ptr(), C.byref(gr), st), self._ctx)

    @staticmethod
    def channels(features: Optional[torch.Tensor] = None, gate: Optional[torch.Tensor] = None,
                 depth: bool = False, flow: bool = False, flow_dt: float = 0.0) -> B.g4d_channels:
        """Extra-channel spec: features [N, D] (float32, contiguous, on the device) gated by
        `gate` [D] and normalized, then depth, then the two flow channels."""
        D = 0 if features is None else int(features.shape[1])
        return B.g4d_channels(D, None if features is None else features.data_ptr(),
                              None if gate is None else gate.data_ptr(), int(depth), int(flow),
                              float(flow_dt))

    def forward_channels(self, g: B.g4d_gaussians, views, settings: B.g4d_settings,
                         ch: B.g4d_channels, out_rgb: torch.Tensor, out_T: Optional[torch.Tensor],
                         out_ch: torch.Tensor) -> None:
        va = views if isinstance(views, C.Array) else B.make_views(views)
        B.check(B.lib().g4d_render_channels_forward(
            self._ctx, C.byref(g), va, len(va), C.byref(settings), C.byref(ch), out_rgb.data_ptr(),
            None if out_T is None else out_T.data_ptr(), out_ch.data_ptr(),
            _stream_handle(self.device)), self._ctx)

    def backward_channels(self, g: B.g4d_gaussians, views, settings: B.g4d_settings,
                          ch: B.g4d_channels, dL: torch.Tensor, dL_ch: Optional[torch.Tensor],
                          grads: Dict[str, torch.Tensor]) -> None:
        """grads: the parameter groups plus "features" [N, D] and "gate" [D] (optional)."""
        va = views if isinstance(views, C.Array) else B.make_views(views)
        gr = B.g4d_grads(*[grads[k].data_ptr() if grads.get(k) is not None else None
                           for k in PARAM_NAMES + ("mask", "densify")])
        df, dg = grads.get("features"), grads.get("gate")
        B.check(B.lib().g4d_render_channels_backward(
            self._ctx, C.byref(g), va, len(va), C.byref(settings), C.byref(ch), dL.data_ptr(),
            None if dL_ch is None else dL_ch.data_ptr(), C.byref(gr),
            None if df is None else df.data_ptr(), None if dg is None else dg.data_ptr(),
            _stream_handle(self.device)), self._ctx)

    @staticmethod
    def sky(cube: torch.Tensor) -> B.g4d_sky:
        """Sky spec of a cube map [6, R, R, 3] (float32, contiguous, on the device)."""
        if cube.dim() != 4 or cube.shape[0] != 6 or cube.shape[1] != cube.shape[2] or \
                cube.shape[3] != 3 or cube.dtype != torch.float32 or not cube.is_contiguous():
            raise ValueError("cube must be a contiguous float32 [6, R, R, 3] tensor")
        return B.g4d_sky(cube.data_ptr(), int(cube.shape[1]))

    def forward_sky(self, g: B.g4d_gaussians, views, settings: B.g4d_settings, sky: B.g4d_sky,
                    out_rgb: torch.Tensor, out_T: Optional[torch.Tensor]) -> None:
        va = views if isinstance(views, C.Array) else B.make_views(views)
        B.check(B.lib().g4d_render_sky_forward(
            self._ctx, C.byref(g), va, len(va), C.byref(settings), C.byref(sky), out_rgb.data_ptr(),
            None if out_T is None else out_T.data_ptr(), _stream_handle(self.device)), self._ctx)

    def backward_sky(self, g: B.g4d_gaussians, views, settings: B.g4d_settings, sky: B.g4d_sky,
                     dL: torch.Tensor, grads: Dict[str, torch.Tensor]) -> None:
        """grads: the parameter groups (optional mask/densify) and "cube" [6, R, R, 3]."""
        va = views if isinstance(views, C.Array) else B.make_views(views)
        gr = B.g4d_grads(*[grads[k].data_ptr() if grads.get(k) is not None else None
                           for k in PARAM_NAMES + ("mask", "densify")])
        dc = grads.get("cube")
        B.check(B.lib().g4d_render_sky_backward(
            self._ctx, C.byref(g), va, len(va), C.byref(settings), C.byref(sky), dL.data_ptr(),
            C.byref(gr), None if dc is None else dc.data_ptr(), _stream_handle(self.device)),
            self._ctx)

    # -- compact models ------------------------------------------------------------------
    _COMPACT_ARRAYS = ("mean4_h", "scale_idx", "rot_l_idx", "rot_r_idx", "opacity_q", "dc_idx",
                       "rest_idx", "scale_cb", "rot_cb", "dc_cb", "rest_cb")

    def compact(self, c: Dict) -> B.g4d_compact:
        """ABI view of a compact model: a dict with n, sh_degree, t_degree, op_lo, op_hi and
        the device tensors mean4_h (int16 bit patterns of halves) [N, 4], uint8 index arrays
        [N, 6] / [N, 8] and float32 codebooks (see include/g4d.h)."""
        for k in self._COMPACT_ARRAYS:
            t = c[k]
            if t.device != self.device or not t.is_contiguous():
                raise ValueError(f"{k} must be a contiguous tensor on {self.device}")
        p = {k: c[k].data_ptr() for k in self._COMPACT_ARRAYS}
        return B.g4d_compact(int(c["n"]), int(c["sh_degree"]), int(c["t_degree"]), p["mean4_h"],
                             p["scale_idx"], p["rot_l_idx"], p["rot_r_idx"], p["opacity_q"],
                             p["dc_idx"], p["rest_idx"], float(c["op_lo"]), float(c["op_hi"]),
                             p["scale_cb"], p["rot_cb"], p["dc_cb"], p["rest_cb"])

    def decode_compact(self, c: Dict) -> Dict[str, torch.Tensor]:
        """Full float32 parameters of a compact model, on the device."""
        n, ds, dt = int(c["n"]), int(c["sh_degree"]), int(c["t_degree"])
        out = {"mean4": torch.empty((n, 4), device=self.device),
               "scale4": torch.empty((n, 4), device=self.device),
               "rot_l": torch.empty((n, 4), device=self.device),
               "rot_r": torch.empty((n, 4), device=self.device),
               "opacity": torch.empty(n, device=self.device),
               "sh": torch.empty((n, dt + 1, (ds + 1) ** 2, 3), device=self.device)}
        cc = self.compact(c)
        B.check(B.lib().g4d_decode_compact(self._ctx, C.byref(cc),
                                           *[out[k].data_ptr() for k in PARAM_NAMES],
                                           _stream_handle(self.device)), self._ctx)
        return out

    def forward_compact(self, c: Dict, views, settings: B.g4d_settings, out_rgb: torch.Tensor,
                        out_T: Optional[torch.Tensor]) -> None:
        va = views if isinstance(views, C.Array) else B.make_views(views)
        cc = self.compact(c)
        B.check(B.lib().g4d_render_compact_forward(
            self._ctx, C.byref(cc), va, len(va), C.byref(settings), out_rgb.data_ptr(),
            None if out_T is None else out_T.data_ptr(), _stream_handle(self.device)), self._ctx)

    def step(self, g: B.g4d_gaussians, views, settings: B.g4d_settings, dL: torch.Tensor,
             out_rgb: torch.Tensor, out_T: Optional[torch.Tensor],
             grads: Dict[str, torch.Tensor], graph: bool = True, check: bool = True) -> bool:
        """Forward + backward in one call; with graph=True a captured hipGraph is replayed.

        A replay sorts into pair buffers of fixed capacity.  With check=True (the default) the
        call waits for the replay and reads the device status; if the pairs outgrew the
        capacity (parameters moved since the capture), the library drops the graph and this
        call redoes the step eagerly, so the outputs are always valid, and the next graph call
        captures again with a larger capacity.  With check=False nothing waits: call sync()
        before using the outputs.  Returns False when the step had to be redone."""
        va = views if isinstance(views, C.Array) else B.make_views(views)
        gr = B.g4d_grads(*[grads[k].data_ptr() for k in PARAM_NAMES])
        args = (self._ctx, C.byref(g), va, len(va), C.byref(settings), dL.data_ptr(),
                out_rgb.data_ptr(), None if out_T is None else out_T.data_ptr(), C.byref(gr))
        st = _stream_handle(self.device)
        B.check(B.lib().g4d_render_step(*args, B.G4D_STEP_GRAPH if graph else 0, st), self._ctx)
        if not (graph and check):
            return True
        try:
            self.sync()
            return True
        except B.G4DError as e:
            if e.status != B.G4D_ECAPACITY:
                raise
        B.check(B.lib().g4d_render_step(*args, 0, st), self._ctx)
        return False

    def preprocess(self, g: B.g4d_gaussians, views, settings: B.g4d_settings):
        va = views if isinstance(views, C.Array) else B.make_views(views)
        rec = torch.empty((len(va), g.n, B.G4D_RECORD_FLOATS), device=self.device)
        tiles = torch.empty((len(va), g.n), dtype=torch.int32, device=self.device)
        B.check(B.lib().g4d_preprocess(self._ctx, C.byref(g), va, len(va), C.byref(settings),
                                       rec.data_ptr(), tiles.data_ptr(),
                                       _stream_handle(self.device)), self._ctx)
        return rec, tiles

    def sync(self) -> None:
        B.check(B.lib().g4d_sync_status(self._ctx, _stream_handle(self.device)), self._ctx)

    def stats(self) -> Dict[str, int]:
        s = B.g4d_stats()
        B.check(B.lib().g4d_get_stats(self._ctx, C.byref(s), _stream_handle(self.device)),
                self._ctx)
        return {k: int(getattr(s, k)) for k, _ in B.g4d_stats._fields_}

    def eval_counters(self, enable: bool, n_pixels: Optional[int] = None):
        out = None
        if n_pixels is not None:
            out = torch.empty(n_pixels, dtype=torch.int32, device=self.device)
        B.check(B.lib().g4d_eval_counters(self._ctx, int(enable),
                                          None if out is None else out.data_ptr(),
                                          _stream_handle(self.device)), self._ctx)
        return out


    def autotune(self, g: B.g4d_gaussians, views, settings: B.g4d_settings, dL: torch.Tensor,
                 out_rgb: torch.Tensor, out_T: Optional[torch.Tensor],
                 grads: Dict[str, torch.Tensor], reps: int = 2) -> float:
        """Pick tile size, LDS batch and pixels per lane in place in ``settings``; returns the
        chosen forward + backward time in ms."""
        va = views if isinstance(views, C.Array) else B.make_views(views)
        gr = B.g4d_grads(*[grads[k].data_ptr() for k in PARAM_NAMES])
        ms = C.c_double()
        B.check(B.lib().g4d_autotune(self._ctx, C.byref(g), va, len(va), C.byref(settings),
                                     dL.data_ptr(), out_rgb.data_ptr(),
                                     None if out_T is None else out_T.data_ptr(), C.byref(gr),
                                     int(reps), C.byref(ms), _stream_handle(self.device)),
                self._ctx)
        return ms.value

    def profile_mask(self, stages=None) -> None:
        """Record only the named stages while profiling (None: every stage)."""
        if stages is None:
            mask = 0xFFFFFFFF
        else:
            names = _stage_names()
            mask = 0
            for s in stages:
                mask |= 1 << names.index(s)
        B.check(B.lib().g4d_profile_mask(self._ctx, mask), self._ctx)

    def profile(self, enable: bool, collect: bool = True, reset: bool = True):
        """Stage timing (HIP events on the call's stream): returns {stage: (ms, launches)}."""
        # room for more stages than the header declares, so that a library built with more
        # stages cannot write past the arrays
        ms = (C.c_double * 64)()
        n = (C.c_int64 * 64)()
        B.check(B.lib().g4d_profile(self._ctx, int(enable), ms if collect else None,
                                    n if collect else None, int(reset)), self._ctx)
        if not collect:
            return None
        return {name: (ms[k], n[k]) for k, name in enumerate(_stage_names())}


def _stage_names():
    """The library's stage names, in index order (it names no stage past the last)."""
    names = []
    while len(names) < 64:
        name = B.lib().g4d_stage_name(len(names)).decode()
        if not name:
            break
        names.append(name)
    return names


def _after_forward(r: Renderer, forward, backward, views) -> None:
    """Run `backward`; if the context's saved forward is another one (G4D_ESTATE), run
    `forward` (into scratch outputs) again first."""
    try:
        backward()
        return
    except B.G4DError as e:
        if e.status != B.G4D_ESTATE:
            raise
    npix = Renderer.pixel_count_array(views)
    forward(torch.empty(3 * npix, device=r.device), torch.empty(npix, device=r.device))
    backward()


class _Render4D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer: Renderer, views, settings, sh_degree, t_degree, mask_threshold,
                densify_out, mean4, scale4, rot_l, rot_r, opacity, sh, mask):
        g = renderer.gaussians(mean4, scale4, rot_l, rot_r, opacity, sh, sh_degree, t_degree,
                               mask, mask_threshold)
        va = B.make_views(views)
        npix = Renderer.pixel_count(views)
        rgb = torch.empty(3 * npix, device=renderer.device)
        T = torch.empty(npix, device=renderer.device)
        renderer.forward(g, va, settings, rgb, T)
        ctx.renderer, ctx.views, ctx.settings = renderer, va, settings
        ctx.degrees = (sh_degree, t_degree)
        ctx.mask_threshold, ctx.densify_out = mask_threshold, densify_out
        ctx.save_for_backward(mean4, scale4, rot_l, rot_r, opacity, sh, mask)
        ctx.mark_non_differentiable(T)
        return rgb, T

    @staticmethod
    def backward(ctx, d_rgb, d_T):
        *params, mask = ctx.saved_tensors
        r: Renderer = ctx.renderer
        g = r.gaussians(*params, *ctx.degrees, mask, ctx.mask_threshold)
        grads = {k: torch.empty_like(p) for k, p in zip(PARAM_NAMES, params)}
        if mask is not None:
            grads["mask"] = torch.empty_like(mask)
        if ctx.densify_out is not None:
            grads["densify"] = ctx.densify_out
        _after_forward(r, lambda rgb, T: r.forward(g, ctx.views, ctx.settings, rgb, T),
                       lambda: r.backward(g, ctx.views, ctx.settings, d_rgb.contiguous(), grads),
                       ctx.views)
        return ((None,) * 7 + tuple(grads[k] for k in PARAM_NAMES) + (grads.get("mask"),))


class _RenderChannels(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer: Renderer, views, settings, sh_degree, t_degree, depth, flow,
                flow_dt, mean4, scale4, rot_l, rot_r, opacity, sh, features, gate):
        g = renderer.gaussians(mean4, scale4, rot_l, rot_r, opacity, sh, sh_degree, t_degree)
        va = B.make_views(views)
        npix = Renderer.pixel_count(views)
        ch = Renderer.channels(features, gate, depth, flow, flow_dt)
        E = ch.n_features + int(depth) + 2 * int(flow)
        rgb = torch.empty(3 * npix, device=renderer.device)
        T = torch.empty(npix, device=renderer.device)
        out = torch.empty(E * npix, device=renderer.device)
        renderer.forward_channels(g, va, settings, ch, rgb, T, out)
        ctx.renderer, ctx.views, ctx.settings = renderer, va, settings
        ctx.degrees = (sh_degree, t_degree)
        ctx.spec = (depth, flow, flow_dt)
        ctx.save_for_backward(mean4, scale4, rot_l, rot_r, opacity, sh, features, gate)
        ctx.mark_non_differentiable(T)
        return rgb, T, out

    @staticmethod
    def backward(ctx, d_rgb, d_T, d_ch):
        *params, features, gate = ctx.saved_tensors
        r: Renderer = ctx.renderer
        g = r.gaussians(*params, *ctx.degrees)
        ch = Renderer.channels(features, gate, *ctx.spec)
        grads = {k: torch.empty_like(p) for k, p in zip(PARAM_NAMES, params)}
        if features is not None:
            grads["features"] = torch.empty_like(features)
            if gate is not None:
                grads["gate"] = torch.empty_like(gate)
        E = ch.n_features + int(ctx.spec[0]) + 2 * int(ctx.spec[1])
        npix = Renderer.pixel_count_array(ctx.views)

        def refwd(rgb, T):
            r.forward_channels(g, ctx.views, ctx.settings, ch, rgb, T,
                               torch.empty(E * npix, device=r.device))

        _after_forward(r, refwd,
                       lambda: r.backward_channels(g, ctx.views, ctx.settings, ch,
                                                   d_rgb.contiguous(),
                                                   None if d_ch is None else d_ch.contiguous(),
                                                   grads),
                       ctx.views)
        return ((None,) * 8 + tuple(grads[k] for k in PARAM_NAMES) +
                (grads.get("features"), grads.get("gate")))


class _RenderSky(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer: Renderer, views, settings, sh_degree, t_degree, mean4, scale4,
                rot_l, rot_r, opacity, sh, cube):
        g = renderer.gaussians(mean4, scale4, rot_l, rot_r, opacity, sh, sh_degree, t_degree)
        va = B.make_views(views)
        npix = Renderer.pixel_count(views)
        rgb = torch.empty(3 * npix, device=renderer.device)
        T = torch.empty(npix, device=renderer.device)
        renderer.forward_sky(g, va, settings, Renderer.sky(cube), rgb, T)
        ctx.renderer, ctx.views, ctx.settings = renderer, va, settings
        ctx.degrees = (sh_degree, t_degree)
        ctx.save_for_backward(mean4, scale4, rot_l, rot_r, opacity, sh, cube)
        ctx.mark_non_differentiable(T)
        return rgb, T

    @staticmethod
    def backward(ctx, d_rgb, d_T):
        *params, cube = ctx.saved_tensors
        r: Renderer = ctx.renderer
        g = r.gaussians(*params, *ctx.degrees)
        grads = {k: torch.empty_like(p) for k, p in zip(PARAM_NAMES, params)}
        grads["cube"] = torch.empty_like(cube)
        sky = Renderer.sky(cube)
        _after_forward(r, lambda rgb, T: r.forward_sky(g, ctx.views, ctx.settings, sky, rgb, T),
                       lambda: r.backward_sky(g, ctx.views, ctx.settings, sky, d_rgb.contiguous(),
                                              grads),
                       ctx.views)
        return (None,) * 5 + tuple(grads[k] for k in PARAM_NAMES) + (grads["cube"],)


def split_views(flat: torch.Tensor, views, channels: int) -> List[torch.Tensor]:
    out, off = [], 0
    for v in views:
        h, w = int(v["height"]), int(v["width"])
        out.append(flat[off:off + channels * h * w].view(channels, h, w))
        off += channels * h * w
    return out


def render(mean4, scale4, rot_l, rot_r, opacity, sh, views: Sequence[dict], *, sh_degree: int,
           t_degree: int, renderer: Renderer, settings: Optional[B.g4d_settings] = None,
           mask: Optional[torch.Tensor] = None, mask_threshold: float = 0.0,
           densify_out: Optional[torch.Tensor] = None):
    """Differentiable render of all ``views`` in one batch.

    ``mask`` [N] is the optional volume-mask significance (activated; kept where above
    ``mask_threshold``, straight-through gradient).  ``densify_out`` [N, 3] receives the
    densification statistics of the backward (sum over views of |dL/d mean2d|, |dL/d mu_t|,
    number of views).  Returns (images, transmittances): lists of [3, H, W] and [H, W] tensors.
    """
    s = settings if settings is not None else B.default_settings()
    rgb, T = _Render4D.apply(renderer, list(views), s, sh_degree, t_degree, mask_threshold,
                             densify_out, mean4, scale4, rot_l, rot_r, opacity, sh,
                             None if mask is None else mask.contiguous())
    return split_views(rgb, views, 3), [t[0] for t in split_views(T, views, 1)]


def render_channels(mean4, scale4, rot_l, rot_r, opacity, sh, views: Sequence[dict], *,
                    sh_degree: int, t_degree: int, renderer: Renderer,
                    features: Optional[torch.Tensor] = None, gate: Optional[torch.Tensor] = None,
                    depth: bool = False, flow: bool = False, flow_dt: float = 0.0,
                    settings: Optional[B.g4d_settings] = None):
    """Differentiable render with extra channels (normalized gated features, depth, flow).

    Returns (images, transmittances, channels): per view [3, H, W], [H, W] and [E, H, W] with
    E = D + depth + 2 flow (features first).  Gradients reach the parameters, the features and
    the gate; the flow channels carry none.
    """
    s = settings if settings is not None else B.default_settings()
    if features is not None:
        features = features.contiguous()
    if gate is not None:
        gate = gate.contiguous()
    E = (0 if features is None else int(features.shape[1])) + int(depth) + 2 * int(flow)
    rgb, T, ch = _RenderChannels.apply(renderer, list(views), s, sh_degree, t_degree, depth, flow,
                                       flow_dt, mean4, scale4, rot_l, rot_r, opacity, sh,
                                       features, gate)
    return (split_views(rgb, views, 3), [t[0] for t in split_views(T, views, 1)],
            split_views(ch, views, E))


def render_sky(mean4, scale4, rot_l, rot_r, opacity, sh, cube, views: Sequence[dict], *,
               sh_degree: int, t_degree: int, renderer: Renderer,
               settings: Optional[B.g4d_settings] = None):
    """Differentiable render with a learnable cube-map sky [6, R, R, 3] as every pixel's
    background (urban scenes).  Returns (images, transmittances) per view; gradients reach the
    parameters and the cube map."""
    s = settings if settings is not None else B.default_settings()
    rgb, T = _RenderSky.apply(renderer, list(views), s, sh_degree, t_degree, mean4, scale4,
                              rot_l, rot_r, opacity, sh, cube.contiguous())
    return split_views(rgb, views, 3), [t[0] for t in split_views(T, views, 1)]
