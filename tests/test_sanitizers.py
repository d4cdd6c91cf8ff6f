"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The oracle (plain C) is rebuilt with gcc's sanitizers and its pins are run again against that
build.  libka's host translation units are rebuilt with hipcc, the sanitizers applied to the
host compilation only (device code is never instrumented), linked with ordinary device
objects, and the host-logic tests are run again against that library.  Each run is a child
pytest process with the sanitizer runtime preloaded; any report fails it.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _child_pytest(test_args, env_extra, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    # -s: a sanitizer report goes to the child's stderr even when it aborts inside a test
    cmd = [sys.executable, "-m", "pytest", *test_args, "-q", "-s", "-x", "-p", "no:cacheprovider", "-m", "not gpu"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out, out[-2000:]


def test_oracle_pins_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run([gcc, "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    os.path.join(ROOT, "oracle", "ka_oracle.c"), "-o", lib], check=True)
    runtimes = [subprocess.run([gcc, f"-print-file-name={name}"], capture_output=True, text=True,
                               check=True).stdout.strip() for name in ("libasan.so", "libubsan.so")]
    _child_pytest(["tests/test_oracle_rule.py", "tests/test_oracle_graphs.py", "tests/test_oracle_dynamics.py",
                   "tests/test_oracle_random_sequential.py",
                   "-k", "not rocrand"],     # that pin compiles and runs a probe of its own
                  {"LD_PRELOAD": ":".join(runtimes), "KA_ORACLE_LIB": lib,
                   "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                   "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}, timeout=1200)


def test_host_library_under_sanitizers(tmp_path):
    from paper_1710_05155_amd import build as kb
    hipcc = kb._hipcc()
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's AddressSanitizer runtime not found")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in kb.COMMON if f != "-O3"] + ["-O1", "-g"]
    objs = []
    for src in kb.SOURCES:
        stem = os.path.splitext(src)[0]
        path = os.path.join(kb.CSRC, src)
        obj = str(tmp_path / (stem + ".o"))
        if src.endswith(".cpp"):
            subprocess.run([hipcc, *flags, *kb.DEVICE, *san, "-c", path, "-o", obj], check=True)
        else:
            # device code: the ordinary build's object when it is newer than every source
            built = os.path.join(kb.PKG, "_build", stem + ".o")
            newest = max(os.path.getmtime(f) for f in glob.glob(os.path.join(kb.CSRC, "*")))
            if os.path.exists(built) and os.path.getmtime(built) >= newest:
                obj = built
            else:
                subprocess.run([hipcc, *kb.COMMON, *kb.DEVICE, "-c", path, "-o", obj], check=True)
        objs.append(obj)
    lib = str(tmp_path / "libka_san.so")
    subprocess.run([hipcc, *kb.DEVICE, "-shared", "-fPIC", *objs, "-pthread", *san, "-shared-libsan",
                    "-o", lib], check=True)
    _child_pytest(["tests/test_library_cpu.py", "-k", "not missing_library"],
                  {"LD_PRELOAD": rt[-1], "KA_LIB": lib,
                   "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                   "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}, timeout=1200)
