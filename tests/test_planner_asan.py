"""The planner's host code under AddressSanitizer: tests/asan_planner_driver.cpp, linked against the library's
objects with api.cpp (validation, planning, shapes, baselines, description) rebuilt with -fsanitize=address on
its host side only.  Runs on the CPU (host-only plans and argument checks); an ASan report or a wrong status
fails the test."""

import importlib.util
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_0909_0001_amd")
OUT = os.path.join(ROOT, "_build", "asan")


def _build_module():
    spec = importlib.util.spec_from_file_location("_omni_build_asan", os.path.join(PKG, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:
        raise AssertionError(f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}")
    return r


def test_planner_host_code_under_asan():
    b = _build_module()
    try:
        hipcc = b.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    os.makedirs(b.BUILD, exist_ok=True)
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(os.path.join(b.CSRC, f) for f in os.listdir(b.CSRC) if f.endswith((".hip", ".cpp")))
    objs = [b._compile(s, incremental=True) for s in srcs if not s.endswith("api.cpp")]
    asan = ["-g", "-O1", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address"]
    api_obj = os.path.join(OUT, "api_asan.o")
    _run([hipcc, *b.COMMON, *asan, "-c", os.path.join(b.CSRC, "api.cpp"), "-o", api_obj])
    drv_obj = os.path.join(OUT, "driver.o")
    _run([hipcc, "-std=c++17", *asan, "-I", os.path.join(ROOT, "include"), "-x", "c++", "-c",
          os.path.join(ROOT, "tests", "asan_planner_driver.cpp"), "-o", drv_obj])
    exe = os.path.join(OUT, "planner_driver")
    _run([hipcc, f"--offload-arch={b.ARCH}", *asan, drv_obj, api_obj, *objs, "-L/opt/rocm/lib",
          "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "planner host checks passed" in r.stdout
