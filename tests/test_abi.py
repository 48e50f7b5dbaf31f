"""CPU checks of the C ABI: the library loads, exports every function include/g4d.h declares,
the ctypes structures have the C layout, and host-side argument checks need no GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "g4d.h")


@pytest.fixture(scope="module")
def B():
    from paper_2412_20720_amd import _binding, build
    if not os.path.exists(_binding.LIB_PATH):
        build.build()
    _binding.lib()
    return _binding


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:g4d_status|const char \*)\s*(g4d_\w+)\(", text, re.M)))


def test_header_declares_the_binding_names(B):
    assert declared_functions() == sorted(B.EXPORTED)


def test_library_exports_every_declared_symbol(B):
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(B.lib(), name)


def test_struct_layouts_match_c(B, tmp_path):
    src = tmp_path / "sizes.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "g4d.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(g4d_gaussians),"
        " sizeof(g4d_grads), sizeof(g4d_view), sizeof(g4d_settings), sizeof(g4d_stats),"
        " offsetof(g4d_view, t), offsetof(g4d_settings, tile_size));return 0;}\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(B.g4d_gaussians), C.sizeof(B.g4d_grads), C.sizeof(B.g4d_view),
            C.sizeof(B.g4d_settings), C.sizeof(B.g4d_stats), B.g4d_view.t.offset,
            B.g4d_settings.tile_size.offset]
    assert got == want


def test_default_settings(B):
    s = B.default_settings()
    assert s.tile_size == 16 and s.lds_batch == 0 and s.px_per_lane == 0 and s.bwd_px_per_lane == 0
    assert abs(s.marginal_min - 1 / 255) < 1e-9 and abs(s.alpha_min - 1 / 255) < 1e-9
    assert abs(s.alpha_max - 0.99) < 1e-7 and abs(s.T_min - 1e-4) < 1e-10
    assert abs(s.cutoff_sigma - 3.0) < 1e-7 and abs(s.blur - 0.3) < 1e-7
    assert B.lib().g4d_default_settings(None) == B.G4D_EINVAL


def test_null_arguments_are_rejected_without_a_gpu(B):
    L = B.lib()
    s = B.default_settings()
    assert L.g4d_render_forward(None, None, None, 1, C.byref(s), None, None, None) == B.G4D_EINVAL
    assert L.g4d_render_backward(None, None, None, 1, C.byref(s), None, None, None) == B.G4D_EINVAL
    assert L.g4d_preprocess(None, None, None, 1, C.byref(s), None, None, None) == B.G4D_EINVAL
    assert L.g4d_sync_status(None, None) == B.G4D_EINVAL
    assert L.g4d_get_stats(None, None, None) == B.G4D_EINVAL
    assert L.g4d_eval_counters(None, 0, None, None) == B.G4D_EINVAL
    assert L.g4d_destroy(None) == B.G4D_EINVAL
    assert L.g4d_create(None, 0) == B.G4D_EINVAL
    assert L.g4d_last_error(None) == b"null context"


def test_create_without_gpu_fails_cleanly(B):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = C.c_void_p(1234)
    assert B.lib().g4d_create(C.byref(ctx), 0) == B.G4D_EHIP
    assert not ctx.value


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2412_20720_amd import _binding
    monkeypatch.setattr(_binding, "_lib", None)
    monkeypatch.setattr(_binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _binding.lib()
