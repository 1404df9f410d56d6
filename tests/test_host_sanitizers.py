"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

* The library: every source compiled with the sanitizers on its host side only
  (device code unchanged and never run), linked with clang++, and driven by
  tests/sanitize/host_calls.c through the host-side parts of the C ABI: plan
  and workspace layout over every width, storage type, form, primitive, NDFD
  setting and view count, tuning candidates, buffer views, size queries and
  the argument validation of every entry point.
* The FP64 oracle's C code (oracle/raster.c) built with the same sanitizers
  and run, in a child interpreter that preloads the sanitizer runtime, over
  small scenes that reach every branch: Gaussians with fusion, opacity-aware
  binning, the NDFD branch with its gradient, and surfels with fusion and NDFD.

Any sanitizer finding aborts the child with a report, which fails the test.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2505_19154_amd import build as hip_build  # noqa: E402

CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN_ENV = dict(ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=87")

needs_rocm = pytest.mark.skipif(not (os.path.exists(CLANG) and shutil.which(hip_build.hipcc())),
                                reason="ROCm clang/hipcc not found")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:   # (no traceback: it would print the child's environment)
        pytest.fail(f"exit {r.returncode}: {' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-8000:]}", pytrace=False)
    return r


@needs_rocm
def test_library_host_code_under_asan_ubsan(tmp_path):
    # sanitizers on the host side of every translation unit; the device side
    # is compiled as usual (it is embedded, never launched here)
    host_san = ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
                "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    flags = [f for f in hip_build.compile_flags() if f != "-O3"] + ["-O1"] + host_san

    def one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        _run([hip_build.hipcc(), "-c", os.path.join(hip_build.CSRC, src), "-o", obj] + flags)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(one, hip_build.SOURCES))
    lib = str(tmp_path / "libfhgs_san.so")
    rocm_lib = "/opt/rocm/lib"
    _run([CLANGXX, "-shared", "-fPIC", "-fsanitize=address,undefined", "-o", lib] + objs +
         [f"-L{rocm_lib}", "-lamdhip64", f"-Wl,-rpath,{rocm_lib}"])
    drv_obj = str(tmp_path / "host_calls.o")
    _run([CLANG, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", f"-I{hip_build.INCLUDE}", "-I/opt/rocm/include",
          "-c", os.path.join(ROOT, "tests", "sanitize", "host_calls.c"), "-o", drv_obj])
    exe = str(tmp_path / "host_calls")
    _run([CLANGXX, "-fsanitize=address,undefined", "-o", exe, drv_obj, lib, f"-L{rocm_lib}", "-lamdhip64",
          f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{rocm_lib}"])
    r = _run([exe], env=dict(os.environ, **SAN_ENV), timeout=600)
    assert "host calls:" in r.stdout, r.stdout


ORACLE_SCRIPT = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle.raster as R
R.build = lambda force=False: sys.argv[2]   # the sanitized build of raster.c
import scenegen
from oracle import pipeline

cams = [scenegen.look_at_camera(p, w, h) for p, w, h in (((0, -4, 0), 40, 36), ((2.5, -3, 1.0), 52, 20))]
d = 8
for prim in ("gaussian", "surfel"):
    g = scenegen.make_gaussians(160, 1.2, 2, d, seed=5, feat_dtype="bf16")
    if prim == "surfel":
        g["scales"] = (np.asarray(g["scales"]) * 3.0).astype(np.float32)
    rules = ("box", "opacity") if prim == "gaussian" else ("surfel",)
    for rule in rules:
        vts = [dict(scenegen.make_view_tensors(i, c.npix, d, with_dT=True)) for i, c in enumerate(cams)]
        o = pipeline.run(g, cams, vts, fusion=True, want_Fmag=True, want_dfeat=True, bin_rule=rule)
        assert all(np.isfinite(v["C"]).all() for v in o["views"])
        rng = np.random.default_rng(3)
        for vt, c in zip(vts, cams):
            vt["gt"] = rng.normal(size=(c.npix, d))
            vt["ndfd_a"] = rng.normal(size=c.npix)
            vt["ndfd_b"] = rng.normal(size=c.npix)
        o = pipeline.run(g, cams, vts, bin_rule=rule, ndfd=dict(lam=0.5, k=20.0))
        assert all(np.isfinite(v["Lcf"]).all() for v in o["views"])
        print(prim, rule, "ok", flush=True)
print("oracle under sanitizers: ok")
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_c_code_under_asan_ubsan(tmp_path):
    import oracle.raster as R
    lib = str(tmp_path / "liboracle_san.so")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
          "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          R._SRC, "-o", lib, "-lm"])
    asan_rt = _run(["gcc", "-print-file-name=libasan.so"]).stdout.strip()
    assert os.path.isabs(asan_rt), "gcc does not ship a shared AddressSanitizer runtime"
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=asan_rt, OMP_NUM_THREADS="2")
    r = _run([sys.executable, "-c", ORACLE_SCRIPT, ROOT, lib], env=env, timeout=900, cwd=ROOT)
    assert "oracle under sanitizers: ok" in r.stdout, r.stdout
