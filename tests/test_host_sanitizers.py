"""The host code of the C ABI built with AddressSanitizer and
UndefinedBehaviorSanitizer (host pass only: -Xarch_host before every
-fsanitize=) and driven on the CPU through its host-only paths
(tests/host_sanitize/driver.cpp: parameter derivation and validation over
seeded random, extreme and invalid parameter sets, buffer sizes, argument
checks of every entry point).  The kernel launchers are stubs
(tests/host_sanitize/launch_stubs.hip) that those paths never reach."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
COMMON = ["-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert res.returncode == 0, (" ".join(cmd), res.stdout[-3000:], res.stderr[-3000:])
    return res


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_host_paths_under_asan_and_ubsan(tmp_path):
    here = os.path.join(ROOT, "tests", "host_sanitize")
    capi = os.path.join(ROOT, "paper_2206_00366_amd", "csrc", "rmrt_capi.cpp")
    objs = []
    for src, lang in ((capi, "hip"), (os.path.join(here, "launch_stubs.hip"), "hip"),
                      (os.path.join(here, "driver.cpp"), "c++")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, *COMMON, *SAN, "-x", lang, "-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "host_sanitize")
    _run([HIPCC, "--offload-arch=gfx950", *SAN, *objs, "-o", exe])
    # the host code is instrumented: the objects call into both runtimes
    syms = _run(["nm", objs[0]]).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = _run([exe], env=env)
    assert res.stdout.startswith("ok"), res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-3000:]
    shutil.rmtree(tmp_path, ignore_errors=True)
