"""Differentiable render of native 4D Gaussians on AMD Instinct MI355X (gfx950).

The render (arXiv 2412.20720, Sec. 3.2) and its backward run in the HIP kernels of libg4d.so;
this package only marshals arguments.  Importing it loads nothing: the library is opened on
first use and a missing build raises RuntimeError.
"""
import importlib

__all__ = ["render", "Renderer", "default_settings"]


def __getattr__(name):
    if name in ("render", "Renderer"):
        return getattr(importlib.import_module(".frontend", __name__), name)
    if name == "default_settings":
        return importlib.import_module("._binding", __name__).default_settings
    raise AttributeError(name)
