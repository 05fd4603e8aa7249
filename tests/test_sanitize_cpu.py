"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code,
run on the CPU (no GPU, no device code instrumented):

- the oracle (oracle.c, built with gcc and both sanitizers) under the whole
  oracle pin suite;
- the library's host runtime (runtime.cpp, serve.cpp: argument checks, the
  status and message paths, the autotune table's parser and writer, the
  allocator hooks), built with hipcc and both sanitizers on the host side
  only, under the host-side ABI and tune-table tests.

Each runs in a child process with the sanitizer runtime preloaded, and must
finish with no sanitizer report."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1412_1127_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87"}


def _run_child(tests, extra_env):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(extra_env)
    env["PYTHONPATH"] = ROOT + os.pathsep + os.path.join(ROOT, "tests")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "--noconftest", "-p", "no:cacheprovider", "-m", "not gpu",
           *[os.path.join(ROOT, "tests", t) for t in tests]]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=900, cwd=ROOT)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    libasan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not gcc or not os.path.isabs(libasan):
        pytest.skip("gcc with AddressSanitizer is not available")
    so = str(tmp_path / "liboracle_san.so")
    subprocess.check_call([gcc, "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-shared", "-fPIC", "-o", so,
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    out = _run_child(["test_oracle_pins.py"], {"LD_PRELOAD": libasan, "ACCX_ORACLE_LIB": so})
    assert " passed" in out


def _clang_asan_runtime():
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    if os.path.isabs(p) and os.path.exists(p):
        return p
    base = "/opt/rocm/lib/llvm/lib/clang"
    for v in sorted(os.listdir(base)) if os.path.isdir(base) else []:
        q = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(q):
            return q
    return None


def test_host_runtime_under_asan_ubsan(tmp_path):
    import importlib.util
    spec = importlib.util.spec_from_file_location("_accx_build", os.path.join(ROOT, "paper_1412_1127_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    rt = _clang_asan_runtime()
    if not os.path.exists(HIPCC) or not rt:
        pytest.skip("hipcc with AddressSanitizer is not available")
    host = ["runtime.cpp", "serve.cpp"]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xarch_host", "-g"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [HIPCC, *b.COMMON, *(san if src in host else []), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(b.SOURCES))) as ex:
        objs = list(ex.map(compile_one, b.SOURCES))
    so = str(tmp_path / "libaccx_san.so")
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "--offload-arch=" + b.ARCH, "-o", so, *objs])
    out = _run_child(["test_abi_cpu.py", "test_tune_cpu.py"], {"LD_PRELOAD": rt, "ACCX_LIB": so})
    assert " passed" in out
