"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the CPU oracle and
of the host side of the C ABI, each run once on the CPU.

The oracle is built with gcc together with ``tests/sanitize/oracle_san.c``,
which calls every oracle entry point on small and degenerate inputs.  The
library's HIP sources are built with hipcc for gfx950 with the sanitizers on
the host code only (each ``-fsanitize`` flag behind ``-Xarch_host``; the
device code is untouched) and linked with ``tests/sanitize/abi_san.cpp``,
which exercises the paths that run without a GPU: workspace sizing, the
launch-configuration table, tuning-file parsing, trap constants and every
entry point's argument checks.  A sanitizer report aborts the driver with a
non-zero status.  Builds are cached under ``tests/sanitize/_build`` by a hash
of their sources and flags.
"""
import concurrent.futures as cf
import glob
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(SAN, "_build")
CSRC = os.path.join(ROOT, "paper_2106_11143_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _digest(paths, flags):
    h = hashlib.sha256(" ".join(flags).encode())
    for p in sorted(paths):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _drop_stale(prefix, keep):
    """Removes the cached builds of earlier sources (prefix*), keeping `keep`."""
    for old in glob.glob(os.path.join(OUT, prefix + "*")):
        if old != keep:
            shutil.rmtree(old, ignore_errors=True) if os.path.isdir(old) else os.remove(old)


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:
        raise AssertionError(f"{' '.join(cmd[:3])} ... failed ({r.returncode}):\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}")
    return r


def test_oracle_under_asan_ubsan():
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    os.makedirs(OUT, exist_ok=True)
    src = os.path.join(SAN, "oracle_san.c")
    deps = [src] + glob.glob(os.path.join(ROOT, "oracle", "*.c"))
    flags = ["-std=c11", "-g", "-O1", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    exe = os.path.join(OUT, f"oracle_san_{_digest(deps, flags)}")
    if not os.path.exists(exe):
        _drop_stale("oracle_san_", exe)
        _run(["gcc", *flags, src, "-o", exe, "-lm"])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="3"))
    assert "oracle_san ok" in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]


def test_host_abi_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    drv = os.path.join(SAN, "abi_san.cpp")
    deps = srcs + glob.glob(os.path.join(CSRC, "*.hpp")) + [drv, os.path.join(ROOT, "include", "coulomb.h")]
    cflags = ["--offload-arch=gfx950", "-O1", "-std=c++17", "-fno-omit-frame-pointer",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", *HOST_SAN]
    key = _digest(deps, cflags)
    exe = os.path.join(OUT, f"abi_san_{key}")
    if not os.path.exists(exe):
        _drop_stale("abi_san_", exe)
        _drop_stale("obj_", "")
        objdir = os.path.join(OUT, f"obj_{key}")
        os.makedirs(objdir, exist_ok=True)
        jobs = [(s, os.path.join(objdir, os.path.basename(s) + ".o")) for s in srcs + [drv]]
        with cf.ThreadPoolExecutor(min(len(jobs), os.cpu_count() or 2)) as ex:
            list(ex.map(lambda so: _run([HIPCC, *cflags, "-c", so[0], "-o", so[1]]), jobs))
        _run([HIPCC, "--offload-arch=gfx950", *HOST_SAN, *[o for _, o in jobs], "-o", exe])
        shutil.rmtree(objdir, ignore_errors=True)
    # the HIP runtime keeps allocations of its own to the end of the process:
    # leak detection would report those, not ours
    env = dict(ENV, ASAN_OPTIONS="halt_on_error=1:detect_leaks=0")
    r = _run([exe, str(tmp_path)], env=env)
    assert "abi_san ok" in r.stdout, r.stdout[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
