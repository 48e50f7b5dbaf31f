"""The pins catch plausible mistakes: each case plants one slip in a copy of the oracle source
(on the CPU), builds it, and runs the pin tests against it in a subprocess; at least one pin
must fail.  This checks the pins, not the GPU library."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")
PINS = [os.path.join(ROOT, "tests", "test_oracle_pins.py"),
        os.path.join(ROOT, "tests", "test_oracle_branches.py"),
        os.path.join(ROOT, "tests", "test_oracle_gradients.py"),
        os.path.join(ROOT, "tests", "test_oracle_channels.py"),
        os.path.join(ROOT, "tests", "test_oracle_training.py"),
        os.path.join(ROOT, "tests", "test_oracle_sky.py"),
        os.path.join(ROOT, "tests", "test_oracle_compact.py")]

# (name, exact text in oracle.cpp, replacement)
MUTATIONS = [
    ("left rotor sign", "L[1][2] = -d;", "L[1][2] = d;"),
    ("right rotor sign", "R[1][2] = s;", "R[1][2] = -s;"),
    ("rotor not normalized", "out[i] = q[i] / n;", "out[i] = q[i];"),
    ("slice mean sign", "mu_c[i] = mean4[i] + Sig[i][3]", "mu_c[i] = mean4[i] - Sig[i][3]"),
    ("slice covariance term dropped",
     "cov_c[i][j] = Sig[i][j] - Sig[i][3] * Sig[3][j] / Sig[3][3];", "cov_c[i][j] = Sig[i][j];"),
    ("marginal variance squared", "p_t = exp(-0.5 * dt * dt / Sig[3][3]);",
     "p_t = exp(-0.5 * dt * dt / (Sig[3][3] * Sig[3][3]));"),
    ("Jacobian sign", "J[0][2] = -vw.fx * tx / x[2];", "J[0][2] = vw.fx * tx / x[2];"),
    ("J W transposed",
     "T[i][j] = J[i][0] * E[0 * 4 + j] + J[i][1] * E[1 * 4 + j] + J[i][2] * E[2 * 4 + j];",
     "T[i][j] = J[i][0] * E[j * 4 + 0] + J[i][1] * E[j * 4 + 1] + J[i][2] * E[j * 4 + 2];"),
    ("blur dropped", "sp.cov2d[0] = C2[0][0] + st.blur;", "sp.cov2d[0] = C2[0][0];"),
    ("principal point swapped", "sp.u = vw.fx * x[0] / x[2] + vw.cx;", "sp.u = vw.fx * x[0] / x[2] + vw.cy;"),
    ("SH normalization", "std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI)", "std::sqrt((2.0 * l) / (4.0 * M_PI)"),
    ("SH m<0 uses cosine", "y = std::sqrt(2.0) * K * P * sin((double)am * phi);",
     "y = std::sqrt(2.0) * K * P * cos((double)am * phi);"),
    ("Fourier period", "cos(2.0 * M_PI * (double)n * dts / st.time_period)",
     "cos(M_PI * (double)n * dts / st.time_period)"),
    ("color offset dropped", "S acc = S(st.color_offset);", "S acc = S(0.0);"),
    ("transmittance dropped", "C[ch] += T * alpha * s.col[ch];", "C[ch] += alpha * s.col[ch];"),
    ("no stop", "    if (stop) break;\n", "\n"),
    ("back-to-front order", "if (a.depth != b.depth) return a.depth < b.depth;",
     "if (a.depth != b.depth) return a.depth > b.depth;"),
    ("background dropped", "res.rgb[ch] = C[ch] + T * bg[ch];", "res.rgb[ch] = C[ch];"),
    ("backward color-behind recursion",
     "R[ch] = ct.alpha * s.col[ch] + (1.0 - ct.alpha) * R[ch];", "R[ch] = s.col[ch];"),
    ("backward conic term sign", "a[3] += dalpha * ct.alpha * (-dx * dy);",
     "a[3] += dalpha * ct.alpha * (dx * dy);"),
    ("extra channels without transmittance",
     "res.ext[c] += T * alpha * f.ext[(size_t)cd.idx * f.E + c];",
     "res.ext[c] += alpha * f.ext[(size_t)cd.idx * f.E + c];"),
    ("features not normalized", "e[c] = nrm > 0.0 ? f.gate[c] * f.features[(size_t)i * f.D + c] / nrm : 0.0;",
     "e[c] = f.gate[c] * f.features[(size_t)i * f.D + c];"),
    ("flow over the wrong time", "slice<double>(Sig, m4, f.vw.t + dt, mu[1], cov, pt);",
     "slice<double>(Sig, m4, f.vw.t + 0.5 * dt, mu[1], cov, pt);"),
    ("extra channels behind not updated", "Rx[c] = ct.alpha * e[c] + (1.0 - ct.alpha) * Rx[c];",
     "Rx[c] = e[c];"),
    ("feature gradient without the projection", "const double ds = (gf[c] - fh[c] * dot) / nrm;",
     "const double ds = gf[c] / nrm;"),
    ("mask gradient without the opacity term", "double gm = o * grad[16];", "double gm = 0.0;"),
    ("densify statistic of u only", "out.densify[i] += std::sqrt(q[0] * q[0] + q[1] * q[1]);",
     "out.densify[i] += std::fabs(q[0]);"),
    ("sky face table sign", "    sc = z >= 0 ? x : -x;", "    sc = z >= 0 ? -x : x;"),
    ("sky bilinear weights swapped", "const double wx[2] = {1.0 - ax, ax}, wy[2] = {1.0 - ay, ay};",
     "const double wx[2] = {ax, 1.0 - ax}, wy[2] = {1.0 - ay, ay};"),
    ("backward ignores the per-pixel background", "  double R[3] = {bg[0], bg[1], bg[2]};",
     "  double R[3] = {f.vw.background[0], f.vw.background[1], f.vw.background[2]};"),
    ("compact scale not exponentiated", "scale4[4 * i + k] = std::exp(ls);",
     "scale4[4 * i + k] = ls;"),
    ("compact right rotor with the left indices",
     "qr += rot_cb[(c * 64 + rot_r_idx[6 * i + c]) * 4 + k];",
     "qr += rot_cb[(c * 64 + rot_l_idx[6 * i + c]) * 4 + k];"),
    ("half exponent bias", "v = std::ldexp((double)(m + 1024), e - 25);",
     "v = std::ldexp((double)(m + 1024), e - 24);"),
    ("mask threshold inclusive", "if (f.g.mask && !(f.g.mask[i] > f.g.mask_threshold)) {",
     "if (f.g.mask && !(f.g.mask[i] > f.g.mask_threshold + 0.2)) {"),
    ("alpha_max clamp removed", "const double alpha = std::min(st.alpha_max, raw);",
     "const double alpha = raw;"),
    ("backward ignores the alpha clamp", "    if (!ct.clamped) {", "    if (true) {"),
    ("alpha_min skip removed", "bool skip = alpha < st.alpha_min;", "bool skip = false;"),
    ("view direction from the unsliced mean", "for (int j = 0; j < 3; ++j) d[j] = sp.mean3[j] - Cc[j];",
     "for (int j = 0; j < 3; ++j) d[j] = mean4[j] - Cc[j];"),
    ("view direction reversed", "for (int j = 0; j < 3; ++j) d[j] = sp.mean3[j] - Cc[j];",
     "for (int j = 0; j < 3; ++j) d[j] = Cc[j] - sp.mean3[j];"),
    ("camera centre taken as -tau",
     "Cc[j] = -(E[0 * 4 + j] * E[3] + E[1 * 4 + j] * E[7] + E[2 * 4 + j] * E[11]);",
     "Cc[j] = -E[4 * j + 3];"),
    ("Jacobian x clamp removed", "const S tx = clamp_val(S(x[0] / x[2]), xlo, xhi);",
     "const S tx = S(x[0] / x[2]);"),
    ("Jacobian y clamp removed", "const S ty = clamp_val(S(x[1] / x[2]), ylo, yhi);",
     "const S ty = S(x[1] / x[2]);"),
    ("Jacobian y clamp bound from the width", "yhi = ((1.0 + m) * vw.height - vw.cy) / vw.fy;",
     "yhi = ((1.0 + m) * vw.width - vw.cy) / vw.fy;"),
    ("Jacobian lower x bound sign", "const double xlo = (-m * vw.width - vw.cx) / vw.fx",
     "const double xlo = (-m * vw.width + vw.cx) / vw.fx"),
    ("near-plane cull removed", "  if (!(z > st.near_z)) cull = true;\n", "\n"),
    ("marginal cull removed", "  if (!(pt >= st.marginal_min)) cull = true;\n", "\n"),
    ("color clamp removed", "if (val(acc) < st.color_min) {", "if (false) {"),
    ("backward ignores the color clamp", "if (!sp.color_clamped[ch]) gsh[", "if (true) gsh["),
    ("non-finite Gaussians kept", "    if (!finite) {\n      f.splats[i].alive", "    if (false) {\n      f.splats[i].alive"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique or missing: {old!r}"
    mutated = tmp_path / "oracle_mut.cpp"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                    str(mutated)], check=True)
    env = dict(os.environ, G4D_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin failed for planted mistake '{name}'"
