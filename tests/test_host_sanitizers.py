"""The library's host code and the oracle's C routines under the compiler's
sanitizers (CPU only).  tests/native/host_sanitize.cpp drives the host-side
entry points -- handles and argument errors, the greedy grouping and the
analytic planner, placed layouts, remap descriptors, the host backend's
sections, reductions and remaps, the trainer's scratch-size check -- and is
built twice with the library's host C++ sources: with AddressSanitizer and
UndefinedBehaviorSanitizer (every check), and with ThreadSanitizer (many
small jobs through the host backend's thread pool).  The HIP sources' objects
come from the library's own build, uninstrumented (nothing is launched)."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1407_4859_amd", "csrc")
ROCM = "/opt/rocm"
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
HOST_CPP = ["layout.cpp", "abi.cpp", "plan.cpp", "costmodel.cpp", "tune.cpp", "host.cpp"]
HIP = ["remap.hip", "section.hip", "mlp.hip", "probe.hip"]

pytestmark = pytest.mark.skipif(not os.path.exists(CLANGXX),
                                reason="ROCm's clang is needed for the sanitizer builds")


def _hip_object(src):
    """The library build's object of a HIP source (built first when missing)."""
    from paper_1407_4859_amd import build as B
    obj = os.path.join(B.BUILD, os.path.splitext(src)[0] + ".o")
    if not os.path.exists(obj):
        B.build()
    return obj


def _build(tmp, kind):
    """Objects and the driver for one sanitizer kind ('address' or 'thread')."""
    san = ["address", "undefined"] if kind == "address" else ["thread"]
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fPIC", "-ffp-contract=off", "-pthread"]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    cxx_san = ["-fsanitize=" + ",".join(san)]
    if kind == "address":
        cxx_san.append("-fno-sanitize-recover=undefined")
    jobs = []
    for src in HOST_CPP:
        jobs.append([CLANGXX, "-x", "c++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", ROCM + "/include",
                     *flags, *cxx_san, *inc, "-c", os.path.join(CSRC, src), "-o", os.path.join(tmp, src + ".o")])
    jobs.append([CLANG, "-x", "c", "-std=c11", *flags, *cxx_san, "-c", os.path.join(ROOT, "oracle", "adha_oracle.c"),
                 "-o", os.path.join(tmp, "oracle.o")])
    jobs.append([CLANGXX, "-x", "c++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", ROCM + "/include", *flags,
                 *cxx_san, *inc, "-c", os.path.join(ROOT, "tests", "native", "host_sanitize.cpp"), "-o",
                 os.path.join(tmp, "driver.o")])

    def run(cmd):
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, " ".join(cmd) + "\n" + r.stderr[-4000:]

    with ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:
        list(ex.map(run, jobs))
    exe = os.path.join(tmp, "host_sanitize_" + kind)
    objs = ([os.path.join(tmp, s + ".o") for s in HOST_CPP] + [_hip_object(s) for s in HIP] +
            [os.path.join(tmp, "oracle.o"), os.path.join(tmp, "driver.o")])
    run([CLANGXX, *cxx_san, "-pthread", "-o", exe, *objs, "-L", ROCM + "/lib", "-lamdhip64",
         "-Wl,-rpath," + ROCM + "/lib"])
    return exe


def _run(exe, mode, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([exe, mode], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "host checks passed" in r.stdout


def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = _build(str(tmp_path), "address")
    # leaks are checked too; halt on the first report
    _run(exe, "all", {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1:abort_on_error=0",
                      "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})


def test_host_thread_pool_under_thread_sanitizer(tmp_path):
    exe = _build(str(tmp_path), "thread")
    _run(exe, "pool", {"TSAN_OPTIONS": "halt_on_error=1:exitcode=66"})
