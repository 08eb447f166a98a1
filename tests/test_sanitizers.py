"""Host-side sanitizer runs (no GPU needed).

* The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer runs its own pin
  tests (every oracle function on grids from 1 x 2 up, edges and pins included).
* The library built with AddressSanitizer on its host code (the device code is compiled as
  usual) runs the C-ABI tests: argument validation, plan sizing, status strings and layouts.

Each run is a subprocess with the sanitizer runtime preloaded; a report aborts it with a
non-zero status and the report in its output."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2403_12820_amd", "csrc")


def _run_pytest(files, env_extra):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *files], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "Sanitizer" not in out, out[-4000:]
    return out


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    tests = [os.path.join("tests", t) for t in ("test_oracle_pins.py", "test_oracle_bf16.py", "test_oracle_pressure.py",
                                                "test_oracle_sphere.py", "test_oracle_pair_cell.py")]
    out = _run_pytest(tests, {"LD_PRELOAD": asan, "PECNN_ORACLE_LIB": lib})
    assert "passed" in out


def test_host_runtime_under_address_sanitizer(tmp_path):
    rts = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    hipcc = "/opt/rocm/bin/hipcc"
    if not rts or not os.path.exists(hipcc):
        pytest.skip("hipcc or its AddressSanitizer runtime is not installed")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-mllvm", "-amdgpu-mfma-vgpr-form=1", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"),
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    procs = [(subprocess.Popen([hipcc, *flags, "-c", s, "-o", str(tmp_path / (os.path.basename(s) + ".o"))],
                               stdout=subprocess.PIPE, stderr=subprocess.STDOUT), s) for s in srcs]
    for p, s in procs:
        out = p.communicate()[0]
        assert p.returncode == 0, (s, out[-2000:])
    lib = str(tmp_path / "libpecnn.so")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                           "-o", lib, *[str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs],
                           "-lrocprofiler-sdk-roctx"])
    out = _run_pytest([os.path.join("tests", "test_abi.py")], {"LD_PRELOAD": rts[-1], "PECNN_LIB": lib})
    assert "passed" in out
