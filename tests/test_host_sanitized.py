"""The library's host code is clean under AddressSanitizer and
UndefinedBehaviorSanitizer: its host-side sources (argument checks, key
schedule, batch planner, serving engine with its worker thread, host
pipeline) are built on the CPU into a host-only library with the sanitizers
on the host pass only and the kernel launchers stubbed
(tests/sanitizer_stubs.cpp).  The CPU tests of the C ABI and of the serving
engine's policy then run against that build in a child process with the
sanitizer runtime preloaded; any report aborts the child.  A second build
with ThreadSanitizer runs the serving engine's CPU tests (a worker thread
beside the submitting, polling and releasing thread) the same way."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1902_05234_amd", "csrc")
HOST_SOURCES = [os.path.join(CSRC, f) for f in ("aes_abi.cpp", "aes_serve.cpp", "aes_pipe.cpp")] + [
    os.path.join(ROOT, "tests", "sanitizer_stubs.cpp")]
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _runtime(name):
    found = sorted(glob.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.%s-x86_64.so" % name))
    return found[-1] if found else None


def _build_host_library(tmp_path, flags, name, sources=HOST_SOURCES):
    from paper_1902_05234_amd import build
    objs = []
    for src in sources:
        obj = str(tmp_path / (os.path.splitext(os.path.basename(src))[0] + ".o"))
        cmd = [build.hipcc(), "-std=c++17", "-fPIC", "-O1", "-g", "-x", "hip", "--cuda-host-only", *flags,
               "-I" + build.INCLUDE, "-I" + CSRC, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    lib = str(tmp_path / name)
    r = subprocess.run([build.hipcc(), "-shared", "-fPIC", *objs, "-o", lib], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return lib


def _run_child(tmp_path, lib, runtime, options, test_args):
    logs = str(tmp_path / "report")  # the runtimes write here: the child's own stderr is captured by its pytest
    env = dict(os.environ, AESGPU_LIBRARY=lib, LD_PRELOAD=runtime)
    for var, opts in options.items():
        env[var] = opts + ":log_path=" + logs
    out = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                          *test_args], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    report = "".join(open(f).read() for f in sorted(glob.glob(logs + "*")))
    return out, report


def _run_tests(tmp_path, lib, runtime, options, test_files):
    out, report = _run_child(tmp_path, lib, runtime, options,
                             [os.path.join(ROOT, "tests", f) for f in test_files])
    assert out.returncode == 0 and not report, report[:4000] or (out.stdout[-3000:], out.stderr[-3000:])
    assert " passed" in out.stdout


def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    runtime = _runtime("asan")
    if runtime is None:
        pytest.skip("no clang AddressSanitizer runtime in the ROCm toolchain")
    lib = _build_host_library(tmp_path, SANITIZE, "libaesgpu_host_asan.so")
    _run_tests(tmp_path, lib, runtime,
               {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"},
               ("test_host_abi.py", "test_native_serve.py"))


def test_serving_engine_under_thread_sanitizer(tmp_path):
    runtime = _runtime("tsan")
    if runtime is None:
        pytest.skip("no clang ThreadSanitizer runtime in the ROCm toolchain")
    lib = _build_host_library(tmp_path, ["-Xarch_host", "-fsanitize=thread"], "libaesgpu_host_tsan.so")
    _run_tests(tmp_path, lib, runtime, {"TSAN_OPTIONS": "halt_on_error=1"}, ("test_native_serve.py",))


def test_address_sanitizer_reports_a_planted_planner_overflow(tmp_path):
    """The harness above can fail: a copy of the C ABI whose batch planner
    writes each item one slot further on runs past the end of the item array
    the binding allocated, and the report names the planner."""
    runtime = _runtime("asan")
    if runtime is None:
        pytest.skip("no clang AddressSanitizer runtime in the ROCm toolchain")
    src = open(os.path.join(CSRC, "aes_abi.cpp")).read()
    good = "aes_work_item& it = items[m.decrypt ? id++ : ie++];"
    assert src.count(good) == 1
    planted = tmp_path / "aes_abi.cpp"
    planted.write_text(src.replace(good, "aes_work_item& it = items[(m.decrypt ? id++ : ie++) + 1];"))
    sources = [str(planted)] + [f for f in HOST_SOURCES if not f.endswith("aes_abi.cpp")]
    lib = _build_host_library(tmp_path, SANITIZE, "libaesgpu_planted.so", sources)
    out, report = _run_child(tmp_path, lib, runtime,
                             {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                              "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"},
                             [os.path.join(ROOT, "tests", "test_host_abi.py"), "-k", "batch_plan_covers"])
    assert out.returncode != 0
    assert "heap-buffer-overflow" in report and "aes_batch_plan" in report, report[:3000]
