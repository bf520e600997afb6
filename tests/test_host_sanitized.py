"""libgap's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library's host side (handle lifecycle, stream fork and join, graph
capture, drop and re-capture, launch-shape changes, timing, diagnostics,
state loading, the allocator callbacks) is compiled with hipcc with the
sanitizers on the host pass only, and linked against a strict stand-in for
the HIP runtime (``host_harness/hip_stub.cpp``) instead of the real one: no
kernel runs, device memory is host memory, and every stream, event, graph,
graph exec and allocation is tracked so that misuse is reported where it
happens.  ``host_harness/replay.cpp`` drives the C ABI through the batched
launch-shape sweep (shape set -> graph dropped -> captured again, 24 cycles,
with the store parity flipping) and the other host paths.

The second test plants the former capture of the two-stream step (the
photon side forked onto the second stream inside a capture) in a copy of
the source and checks that the harness reports its fault: the capture ends
with the photon branch not joined back, and the next call waits on an event
recorded inside the ended capture, whose graph is already destroyed.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_harness")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no ROCm toolchain")


def _build(tmp, src_dir):
    lib_o = os.path.join(tmp, "gap.o")
    # sanitizers on the host pass only (the device code is built as usual)
    cmd = [HIPCC, "-c", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"), os.path.join(src_dir, "gap.hip"), "-o", lib_o]
    subprocess.run(cmd, check=True, capture_output=True)
    objs = [lib_o]
    for name in ("hip_stub.cpp", "replay.cpp"):
        o = os.path.join(tmp, name + ".o")
        subprocess.run([CLANG, "-c", "-g", "-O1", "-std=c++17", "-Wno-unused-value", *SAN, "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, name),
                        "-o", o], check=True, capture_output=True)
        objs.append(o)
    exe = os.path.join(tmp, "replay")
    subprocess.run([CLANG, *SAN, *objs, "-o", exe], check=True, capture_output=True)
    return exe


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)


def test_host_code_is_clean_under_sanitizers(tmp_path):
    exe = _build(str(tmp_path), os.path.join(ROOT, "paper_2608_21920_amd", "csrc"))
    r = _run(exe)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "REPLAY OK" in r.stdout
    assert "left: 0 allocations, 0 streams, 0 events, 0 graphs, 0 execs" in r.stdout


def test_harness_catches_the_former_two_stream_capture(tmp_path):
    src = os.path.join(str(tmp_path), "src")
    shutil.copytree(os.path.join(ROOT, "paper_2608_21920_amd", "csrc"), src)
    path = os.path.join(src, "gap.hip")
    text = open(path).read()
    line = "  const bool two = !g->capturing;"
    assert text.count(line) == 1
    open(path, "w").write(text.replace(line, "  const bool two = true;"))
    exe = _build(str(tmp_path), src)
    r = _run(exe)
    assert r.returncode != 0
    assert "HIPSTUB ERROR: capture ends with a forked stream not joined back" in r.stderr, r.stderr[-3000:]


def test_oracle_is_clean_under_sanitizers(tmp_path):
    """The FP64 oracle through every path (QED with sub-cycling, tracked
    photons, conversion, injection, merge, filter, periodic box, event record
    and replay, state loading) under ASan, UBSan and the leak checker."""
    exe = os.path.join(str(tmp_path), "odrive")
    subprocess.run(["gcc", "-g", "-O1", "-std=c11", *SAN, os.path.join(HERE, "oracle_drive.c"), "-o", exe, "-lm"],
                   check=True, capture_output=True)
    r = _run(exe)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ORACLE OK" in r.stdout
