"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU:

* the C oracle, built with gcc -fsanitize=address,undefined, driven through
  every exported routine (tests/sanitize/oracle_driver.c);
* the host runtimes of libch.so (ch_host.cpp, dp_host.cpp), built with the
  sanitizers on the host pass (kernel launchers stubbed out), driven
  through the argument-validation paths of both C ABIs
  (tests/sanitize/host_driver.cpp).

Any sanitizer report aborts the program (no recovery), so the test passes
only on a clean run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

pytestmark = pytest.mark.slow


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-o", exe, os.path.join(SAN, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "ch_oracle.c"), "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "oracle driver: ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_runtime_under_sanitizers(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    # the device pass stays uninstrumented (ch_host.cpp holds a device array)
    common = ["-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-I" + os.path.join(ROOT, "include")]
    objs = []
    for src in ("paper_1911_03386_amd/csrc/ch_host.cpp", "paper_1911_03386_amd/csrc/dp_host.cpp",
                "tests/sanitize/launcher_stubs.cpp", "tests/sanitize/host_driver.cpp"):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, *common, *san, "-c", os.path.join(ROOT, src), "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "host_san")
    _run([HIPCC, "--offload-arch=gfx950", *san, "-o", exe, *objs])
    r = _run([exe], env=ENV, timeout=300)
    assert "host driver: ok" in r.stdout
