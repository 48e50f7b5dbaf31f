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
    """One g4d context on one GPU.  A backward must follow its own forward before the next
    forward on the same Renderer (the library reports G4D_ESTATE otherwise)."""

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
                  t_degree: int) -> B.g4d_gaussians:
        n = int(mean4.shape[0])
        k = (sh_degree + 1) ** 2
        want = {"mean4": (n, 4), "scale4": (n, 4), "rot_l": (n, 4), "rot_r": (n, 4),
                "opacity": (n,), "sh": (n, t_degree + 1, k, 3)}
        for name, t in zip(PARAM_NAMES, (mean4, scale4, rot_l, rot_r, opacity, sh)):
            if t.dtype != torch.float32 or t.device != self.device or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 tensor on {self.device}")
            if tuple(t.shape) != want[name]:
                raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {want[name]}")
        return B.g4d_gaussians(n, sh_degree, t_degree, mean4.data_ptr(), scale4.data_ptr(),
                               rot_l.data_ptr(), rot_r.data_ptr(), opacity.data_ptr(),
                               sh.data_ptr())

    @staticmethod
    def pixel_count(views) -> int:
        return sum(int(v["width"]) * int(v["height"]) for v in views)

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
                           for k in PARAM_NAMES])
        B.check(B.lib().g4d_render_backward(self._ctx, C.byref(g), va, len(va), C.byref(settings),
                                            dL.data_ptr(), C.byref(gr), st), self._ctx)

    def step(self, g: B.g4d_gaussians, views, settings: B.g4d_settings, dL: torch.Tensor,
             out_rgb: torch.Tensor, out_T: Optional[torch.Tensor],
             grads: Dict[str, torch.Tensor], graph: bool = True) -> None:
        """Forward + backward in one call; with graph=True a captured hipGraph is replayed."""
        va = views if isinstance(views, C.Array) else B.make_views(views)
        gr = B.g4d_grads(*[grads[k].data_ptr() for k in PARAM_NAMES])
        B.check(B.lib().g4d_render_step(self._ctx, C.byref(g), va, len(va), C.byref(settings),
                                        dL.data_ptr(), out_rgb.data_ptr(),
                                        None if out_T is None else out_T.data_ptr(), C.byref(gr),
                                        B.G4D_STEP_GRAPH if graph else 0,
                                        _stream_handle(self.device)), self._ctx)

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

    def profile(self, enable: bool, collect: bool = True, reset: bool = True):
        """Stage timing (HIP events on the call's stream): returns {stage: (ms, launches)}."""
        ms = (C.c_double * B.G4D_NUM_STAGES)()
        n = (C.c_int64 * B.G4D_NUM_STAGES)()
        B.check(B.lib().g4d_profile(self._ctx, int(enable), ms if collect else None,
                                    n if collect else None, int(reset)), self._ctx)
        if not collect:
            return None
        return {B.lib().g4d_stage_name(k).decode(): (ms[k], n[k]) for k in range(B.G4D_NUM_STAGES)}


class _Render4D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer: Renderer, views, settings, sh_degree, t_degree, mean4, scale4,
                rot_l, rot_r, opacity, sh):
        g = renderer.gaussians(mean4, scale4, rot_l, rot_r, opacity, sh, sh_degree, t_degree)
        va = B.make_views(views)
        npix = Renderer.pixel_count(views)
        rgb = torch.empty(3 * npix, device=renderer.device)
        T = torch.empty(npix, device=renderer.device)
        renderer.forward(g, va, settings, rgb, T)
        ctx.renderer, ctx.views, ctx.settings = renderer, va, settings
        ctx.degrees = (sh_degree, t_degree)
        ctx.save_for_backward(mean4, scale4, rot_l, rot_r, opacity, sh)
        ctx.mark_non_differentiable(T)
        return rgb, T

    @staticmethod
    def backward(ctx, d_rgb, d_T):
        params = ctx.saved_tensors
        r: Renderer = ctx.renderer
        g = r.gaussians(*params, *ctx.degrees)
        grads = {k: torch.empty_like(p) for k, p in zip(PARAM_NAMES, params)}
        r.backward(g, ctx.views, ctx.settings, d_rgb.contiguous(), grads)
        return (None, None, None, None, None) + tuple(grads[k] for k in PARAM_NAMES)


def split_views(flat: torch.Tensor, views, channels: int) -> List[torch.Tensor]:
    out, off = [], 0
    for v in views:
        h, w = int(v["height"]), int(v["width"])
        out.append(flat[off:off + channels * h * w].view(channels, h, w))
        off += channels * h * w
    return out


def render(mean4, scale4, rot_l, rot_r, opacity, sh, views: Sequence[dict], *, sh_degree: int,
           t_degree: int, renderer: Renderer, settings: Optional[B.g4d_settings] = None):
    """Differentiable render of all ``views`` in one batch.

    Returns (images, transmittances): lists of [3, H, W] and [H, W] tensors, one per view.
    """
    s = settings if settings is not None else B.default_settings()
    rgb, T = _Render4D.apply(renderer, list(views), s, sh_degree, t_degree, mean4, scale4, rot_l,
                             rot_r, opacity, sh)
    return split_views(rgb, views, 3), [t[0] for t in split_views(T, views, 1)]
