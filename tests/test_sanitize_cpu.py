"""Host code and the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only, no GPU call).

- oracle/oracle.c with tests/sanitize/oracle_driver.c (gcc): every entry point
  on tables of several shapes and storage formats, non-finite positions,
  argument errors and rounding edge cases.
- The library's host sources (layout and sizes, the host packer for every
  storage type, frequency selection, network and Jastrow layouts, plan
  workspace sizes and task lists, the tuning-cache parser) built with the
  sanitizers on the host side only, linked with the library's other objects,
  and driven by tests/sanitize/host_driver.cpp.

Each driver checks its own results and exits 0; a sanitizer report aborts it
(recovery off), so the test passes only on a clean run.
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_02645_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
# host sources instrumented here; every other object comes from the library build
HOST_SOURCES = ["spline_host.cpp", "plan_host.cpp", "vgh_host.cpp", "mlp_host.cpp", "spectrum_host.cpp", "jastrow.hip"]
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


def _clean(r):
    text = r.stdout + r.stderr
    return "runtime error" not in text and "AddressSanitizer" not in text and "LeakSanitizer" not in text


def test_oracle_under_sanitizers():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_driver")
        _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-fopenmp", "-o", exe, os.path.join(ROOT, "oracle", "oracle.c"),
              os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm"])
        r = subprocess.run([exe], capture_output=True, text=True, env=dict(os.environ, OMP_NUM_THREADS="2"))
        print(r.stdout, r.stderr[-2000:])
        assert r.returncode == 0 and _clean(r)


def test_library_host_code_under_sanitizers():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not available")
    from paper_1708_02645_amd import build as hipbuild

    objs = glob.glob(os.path.join(hipbuild.BUILD, "*.o"))
    if len(objs) < len(hipbuild.sources()):
        hipbuild.build()
        objs = glob.glob(os.path.join(hipbuild.BUILD, "*.o"))
    keep = [o for o in objs if os.path.basename(o)[:-2] not in HOST_SOURCES]
    with tempfile.TemporaryDirectory() as d:
        def compile_one(src):
            out = os.path.join(d, src + ".o")
            _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=" + hipbuild.ARCH] + SAN_HOST +
                 ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", out])
            return out

        with cf.ThreadPoolExecutor(6) as ex:
            san = list(ex.map(compile_one, HOST_SOURCES))
        drv = os.path.join(d, "host_driver.o")
        _run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-c", os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), "-o", drv])
        exe = os.path.join(d, "host_driver")
        _run([CLANG, "-fsanitize=address,undefined", "-o", exe, drv] + san + keep +
             ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
        # leak checking off: the HIP runtime's own start-up allocations live
        # until exit
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
        env.pop("QMCSPLINE_TUNE_CACHE", None)
        r = subprocess.run([exe, d], capture_output=True, text=True, env=env)
        print(r.stdout, r.stderr[-2000:])
        assert r.returncode == 0 and _clean(r)
