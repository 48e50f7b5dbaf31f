"""Pins of the oracle's compact-4DGS decode (Sec. 4.2 parameter compression; codebook sizes of
Sec. 8.3): half-precision positions against numpy's float16 for every bit pattern; residual VQ
with one-hot codebooks (one nonzero codeword) giving that codeword exactly where it is selected
and zero (scale: exp(0) = 1) elsewhere, which fixes the codebook layout, the index of each
codebook and the log-space scale; the SH direct component first and the rest in order; opacity
min-max quantization at its ends and a rational point."""
import numpy as np

import oracle
from paper_2412_20720_amd import scenes


def test_half_positions_for_every_bit_pattern(oracle_lib):
    bits = np.arange(65536, dtype=np.uint16)
    n = 65536 // 4
    c = scenes.make_compact(n, sh_degree=0, t_degree=0)
    c["mean4_h"] = bits.reshape(n, 4)
    got = oracle.decode_compact(c)["mean4"].reshape(-1)
    want = bits.view(np.float16).astype(np.float64)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], want[~nan])


def test_residual_vq_one_hot_codebooks(oracle_lib):
    rng = np.random.default_rng(60)
    n = 400
    c = scenes.make_compact(n, sh_degree=1, t_degree=1)
    K = 2 * 4 * 3
    for name, ncb, nent, dim in (("scale_cb", 6, 64, 4), ("rot_cb", 6, 64, 4), ("dc_cb", 6, 64, 3),
                                 ("rest_cb", 8, 256, K - 3)):
        for _ in range(3):
            k, e = int(rng.integers(0, ncb)), int(rng.integers(0, nent))
            vec = rng.normal(size=dim).astype(np.float32)
            cc = dict(c)
            for other in ("scale_cb", "rot_cb", "dc_cb", "rest_cb"):
                cc[other] = np.zeros_like(c[other])
            cc[name] = np.zeros_like(c[name])
            cc[name][k, e] = vec
            d = oracle.decode_compact(cc)
            v64 = vec.astype(np.float64)
            if name == "scale_cb":
                sel = c["scale_idx"][:, k] == e
                np.testing.assert_allclose(d["scale4"][sel], np.exp(v64)[None].repeat(sel.sum(), 0),
                                           rtol=1e-15)
                assert np.all(d["scale4"][~sel] == 1.0)
            elif name == "rot_cb":
                for q, idx in (("rot_l", "rot_l_idx"), ("rot_r", "rot_r_idx")):
                    sel = c[idx][:, k] == e
                    assert np.array_equal(d[q][sel], np.tile(v64, (sel.sum(), 1)))
                    assert np.all(d[q][~sel] == 0.0)
            elif name == "dc_cb":
                sel = c["dc_idx"][:, k] == e
                flat = d["sh"].reshape(n, -1)
                assert np.array_equal(flat[sel, :3], np.tile(v64, (sel.sum(), 1)))
                assert np.all(flat[~sel, :3] == 0.0) and np.all(flat[:, 3:] == 0.0)
            else:
                sel = c["rest_idx"][:, k] == e
                flat = d["sh"].reshape(n, -1)
                assert np.array_equal(flat[sel, 3:], np.tile(v64, (sel.sum(), 1)))
                assert np.all(flat[~sel, 3:] == 0.0) and np.all(flat[:, :3] == 0.0)


def test_opacity_min_max_quantization(oracle_lib):
    c = scenes.make_compact(4, sh_degree=0, t_degree=0)
    c["opacity_q"] = np.array([0, 255, 51, 102], np.uint8)
    c["op_lo"], c["op_hi"] = np.float32(0.25), np.float32(0.75)
    o = oracle.decode_compact(c)["opacity"]
    np.testing.assert_allclose(o, [0.25, 0.75, 0.35, 0.45], rtol=1e-15)
