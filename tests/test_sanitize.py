"""Host code under the address and undefined-behaviour sanitizers (CPU only).

- The host-side argument checks of the C ABI (csrc/g4d_checks.cpp, plain C++ that the library
  also builds) are compiled with g++ -fsanitize=address,undefined together with a driver
  (tests/sanitize_checks.cpp) that feeds them valid and invalid arguments and random bit
  patterns; any sanitizer report aborts the driver.
- The FP64 oracle is compiled the same way and its pin tests run against that build in a
  child process with the sanitizer runtime preloaded.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_20720_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
PIN_FILES = ["test_oracle_pins.py", "test_oracle_branches.py", "test_oracle_gradients.py",
             "test_oracle_channels.py", "test_oracle_sky.py", "test_oracle_compact.py",
             "test_oracle_training.py"]


def _libasan():
    path = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("the host compiler has no address-sanitizer runtime")
    return path


def test_host_argument_checks_under_sanitizers(tmp_path):
    _libasan()
    exe = str(tmp_path / "checks")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", *SAN, "-I", os.path.join(ROOT, "include"),
                    "-I", CSRC, os.path.join(ROOT, "tests", "sanitize_checks.cpp"),
                    os.path.join(CSRC, "g4d_checks.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=dict(os.environ, **ENV),
                       timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "checks ok" in r.stdout


def test_oracle_pins_under_sanitizers(tmp_path):
    libasan = _libasan()
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", *SAN,
                    "-o", lib, os.path.join(ROOT, "oracle", "oracle.cpp")], check=True)
    env = dict(os.environ, **ENV, G4D_ORACLE_LIB=lib, LD_PRELOAD=libasan, OMP_NUM_THREADS="4")
    files = [os.path.join(ROOT, "tests", f) for f in PIN_FILES]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-m", "not gpu",
                        "-p", "no:cacheprovider", *files], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    tail = r.stdout[-3000:] + r.stderr[-4000:]
    assert r.returncode == 0, tail
    assert " passed" in r.stdout, tail
