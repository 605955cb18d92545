"""The host code under the sanitizers, on the CPU.

Builds and runs three programs under ``tests/native/``:
 - ``serve_core_test.cpp``: the serving loop's decisions (admission by HBM
   budget, queue limit, deadlines, continuous batching, release, propagation
   of launcher failures, a multi-threaded run) with a fake clock and a mock
   launcher, under AddressSanitizer + UBSan and, with the ROCm LLVM clang, under
   ThreadSanitizer (GCC's runtime does not see the condition-variable waits
   libstdc++ makes with pthread_cond_clockwait and reports false races);
 - ``host_fuzz.cpp``: geometry validation, launch planning, workspace and
   output checks and the tuning-table reader on random and hostile arguments,
   every accepted plan checked against the invariants the kernels rely on;
 - ``oracle_san.c``: every oracle entry point, its rejected arguments and a few
   identities.
No GPU and no HIP: the planner, the serving core and the oracle are plain
C/C++.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2311_00482_amd", "csrc")
INC = os.path.join(ROOT, "include")
SAN = ["-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-g", "-O1"]
CLANG = "/opt/rocm/llvm/bin/clang++"


def _build(tmp_path, name, cmd):
    out = str(tmp_path / name)
    r = subprocess.run(cmd + ["-o", out], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, f"build of {name} failed:\n{r.stderr[-4000:]}"
    return out


def _run(exe, *args, timeout=300):
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=timeout, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "all ok" in r.stdout
    assert "runtime error" not in out and "WARNING: ThreadSanitizer" not in out, out[-6000:]
    return r.stdout


def test_serve_core_asan_ubsan(tmp_path):
    exe = _build(tmp_path, "serve_core_test",
                 ["g++", "-std=c++17", "-Wall", "-Wextra", "-pthread", *SAN, f"-I{INC}",
                  os.path.join(NATIVE, "serve_core_test.cpp"),
                  os.path.join(CSRC, "serve_core.cpp")])
    out = _run(exe)
    for case in ("budget_admission_and_release", "deadline_expiry", "upload_failure_propagates",
                 "launch_failure_propagates", "continuous_batching", "threads"):
        assert f"ok {case}" in out


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm LLVM clang++ not installed")
def test_serve_core_tsan(tmp_path):
    exe = _build(tmp_path, "serve_core_tsan",
                 [CLANG, "-std=c++17", "-pthread", "-fsanitize=thread", "-g", "-O1",
                  f"-I{INC}", os.path.join(NATIVE, "serve_core_test.cpp"),
                  os.path.join(CSRC, "serve_core.cpp")])
    _run(exe)


def test_planner_and_tuning_fuzz_asan_ubsan(tmp_path):
    exe = _build(tmp_path, "host_fuzz",
                 ["g++", "-std=c++17", "-Wall", "-Wextra", "-pthread", *SAN, f"-I{INC}",
                  os.path.join(NATIVE, "host_fuzz.cpp"), os.path.join(CSRC, "plan.cpp"),
                  os.path.join(CSRC, "tune.cpp")])
    out = _run(exe, "100000", str(tmp_path))
    assert "ok plans" in out and "ok tune" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_oracle_asan_ubsan(tmp_path):
    exe = _build(tmp_path, "oracle_san",
                 ["gcc", "-std=gnu11", "-Wall", "-Wno-unknown-pragmas", *SAN,
                  os.path.join(NATIVE, "oracle_san.c"), "-lm"])
    _run(exe)


def test_tune_cache_environment(tmp_path):
    """PWBF_TUNE_CACHE: a shape stored in one process is planned in the next."""
    exe = _build(tmp_path, "tune_env_test",
                 ["g++", "-std=c++17", "-Wall", "-pthread", *SAN, f"-I{INC}",
                  os.path.join(NATIVE, "tune_env_test.cpp"), os.path.join(CSRC, "plan.cpp"),
                  os.path.join(CSRC, "tune.cpp")])
    cache = tmp_path / "shapes.json"
    env = dict(os.environ, PWBF_TUNE_CACHE=str(cache), PWBF_DEBUG="1")
    r = subprocess.run([exe, "store"], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0 and "all ok" in r.stdout, r.stderr
    assert "default shape" in r.stderr and "tuned shape cpw 2 lz 4 wz 2 wx 4" in r.stderr
    assert cache.exists() and "[2, 4, 2, 4, 0]" in cache.read_text()
    r = subprocess.run([exe, "load"], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0 and "all ok" in r.stdout, r.stderr
    assert "tune cache" in r.stderr and "1 shapes" in r.stderr
    # without the variable the stored shape is not seen, and nothing is printed
    env.pop("PWBF_TUNE_CACHE")
    env.pop("PWBF_DEBUG")
    r = subprocess.run([exe, "load"], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode != 0 and "pwbf:" not in r.stderr


def test_debug_environment_reports_errors_and_plans():
    """PWBF_DEBUG=1 through the built library: plans and errors go to stderr."""
    code = (
        "import ctypes\n"
        "from paper_2311_00482_amd import _abi\n"
        "from paper_2311_00482_amd.api import GeometryArg\n"
        "from synth import config_c1\n"
        "L = _abi.lib()\n"
        "g = GeometryArg(config_c1())\n"
        "info = _abi.PlanInfo()\n"
        "assert L.pwbf_describe_plan(g.ref, _abi.DAS, -1, None, ctypes.byref(info)) == 0\n"
        "g.s.n_angles = 0\n"
        "assert L.pwbf_describe_plan(g.ref, _abi.DAS, -1, None, ctypes.byref(info)) == -1\n")
    env = dict(os.environ, PWBF_DEBUG="1", PYTHONPATH=ROOT)
    r = subprocess.run(["python", "-c", code], capture_output=True, text=True, timeout=300,
                       env=env, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "pwbf: plan mode 0" in r.stderr and " shape cpw " in r.stderr
    assert "pwbf: error -1: n_angles 0 outside" in r.stderr
