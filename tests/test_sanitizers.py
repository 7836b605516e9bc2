"""Host sanitizer builds (CPU only): the oracle and the library's host runtime
built with AddressSanitizer and UndefinedBehaviorSanitizer (recovery off) and
driven through every entry point by tests/sanitize/*_driver.*; any invalid
access, leak or undefined operation fails the run. Two checks that the
sanitizers are live: a copy of the oracle with a planted out-of-bounds write
must be caught, and so must a canary program built with the library's host
flags."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_DIR = os.path.join(ROOT, "tests", "sanitize")
ORACLE_SRC = os.path.join(ROOT, "oracle", "bpsf_oracle.c")
CSRC = os.path.join(ROOT, "paper_2507_00254_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2507_00254_amd", "_build")
CLANGXX = "/opt/rocm/llvm/bin/clang++"

# sanitizer flags: for gcc and clang++ as they are, for the HIP compiler
# behind -Xarch_host (host code only; no device code is built with them)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, env=ENV, **kw)


def _oracle_driver(src, out_dir):
    exe = os.path.join(out_dir, "oracle_driver")
    r = _run(["gcc", "-std=c11", "-g", "-O1", *SAN, "-ffp-contract=off", "-DREAL=double", "-DSUFFIX=_f64",
              os.path.join(SAN_DIR, "oracle_driver.c"), src, "-o", exe, "-lm", "-lpthread"])
    assert r.returncode == 0, r.stderr
    return exe


def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        r = _run([_oracle_driver(ORACLE_SRC, d)], timeout=300)
        assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_sanitizer_catches_a_planted_oracle_overflow():
    """The flip counts allocated one entry short: the first write to the last
    bit's count must stop the run."""
    src = open(ORACLE_SRC).read()
    old = "w->flips = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));"
    assert src.count(old) == 1
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "planted.c")
        with open(path, "w") as f:
            f.write(src.replace(old, "w->flips = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 1 ? N - 1 : 1));"))
        r = _run([_oracle_driver(path, d)], timeout=300)
        assert r.returncode != 0 and "AddressSanitizer" in r.stderr


@pytest.fixture(scope="module")
def hip_tools():
    if not shutil.which("hipcc") or not os.path.exists(CLANGXX):
        pytest.skip("no HIP toolchain")
    if not all(os.path.exists(os.path.join(BUILD, f"{u}.o")) for u in ("bpsf_kernels", "bpsf_wide", "bpsf_sparse")):
        from paper_2507_00254_amd import build
        build.build()
    return True


def test_runtime_under_sanitizers(hip_tools):
    """The host runtime (code loading, the sparse family's layout, parameter
    and argument checks, server set-up) built with host-side sanitizers, linked with the library's kernel
    objects and driven without a device: every entry point's rejection path,
    and a load that stops at the first device call when no GPU is present."""
    with tempfile.TemporaryDirectory() as d:
        objs, procs = [], []
        for unit in ("bpsf_api", "bpsf_server", "bpsf_sparse_layout"):
            obj = os.path.join(d, unit + ".o")
            procs.append(subprocess.Popen(
                ["hipcc", "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                 "-Xclang", "-packed-fp32-ops", *HOST_SAN, "-fPIC", "-c", os.path.join(CSRC, unit + ".hip"),
                 "-o", obj], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
            objs.append(obj)
        for p in procs:
            _, err = p.communicate(timeout=600)
            assert p.returncode == 0, err
        drv = os.path.join(d, "drv.o")
        r = _run([CLANGXX, "-std=c++17", "-O1", "-g", *SAN, "-c", os.path.join(SAN_DIR, "abi_driver.cpp"), "-o", drv])
        assert r.returncode == 0, r.stderr
        exe = os.path.join(d, "abi_driver")
        kernels = [os.path.join(BUILD, f"{u}.o") for u in ("bpsf_kernels", "bpsf_wide", "bpsf_sparse")]
        r = _run(["hipcc", "--offload-arch=gfx950", *HOST_SAN, drv, *objs, *kernels, "-o", exe])
        assert r.returncode == 0, r.stderr
        r = _run([exe], timeout=300)
        assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_sanitizer_catches_a_canary_with_the_runtime_flags(hip_tools):
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "canary.cpp")
        with open(src, "w") as f:
            f.write("#include <stdlib.h>\nint main(int argc, char**) { int* a = (int*)malloc(4 * sizeof(int));\n"
                    "  int r = a[argc + 3]; free(a); return r & 1; }\n")
        exe = os.path.join(d, "canary")
        r = _run(["hipcc", "-std=c++17", "-O0", "-g", "--offload-arch=gfx950", *HOST_SAN, "-x", "hip", src, "-o", exe])
        assert r.returncode == 0, r.stderr
        r = _run([exe], timeout=60)
        assert r.returncode != 0 and "AddressSanitizer" in r.stderr
