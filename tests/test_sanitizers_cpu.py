"""The C oracle and the C graph generators built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code) and driven over every function,
generator family, dirty rows and degenerate inputs (tests/sanitize_driver.c);
the request scheduler's device-free path is driven under the same sanitizers
through the C-ABI (tests/sanitize_server.cpp, host-only build of the library
sources it needs)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    _run(["gcc", "-std=c11", *SAN, os.path.join(HERE, "sanitize_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
          os.path.join(ROOT, "graphgen", "graphgen.c"), "-o", exe, "-lm", "-lpthread"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([exe], env=env)
    assert "ok" in r.stdout


def _asan_library_objects():
    """Every library source compiled for gfx950 with the host code under
    AddressSanitizer and UndefinedBehaviorSanitizer (device code as usual),
    cached in _build/ under a hash of the sources and headers."""
    import concurrent.futures as cf
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2509_19703_amd", "csrc")
    srcs = sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.cpp")))
    deps = srcs + sorted(glob.glob(os.path.join(csrc, "*.h")) + glob.glob(os.path.join(ROOT, "include", "*.h")))
    h = hashlib.sha256()
    for f in deps:
        with open(f, "rb") as fh:
            h.update(fh.read())
    out = os.path.join(ROOT, "_build", "asan_" + h.hexdigest()[:16])
    os.makedirs(out, exist_ok=True)
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]

    def compile_one(src):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        if not os.path.exists(obj):
            _run([hipcc, "-x", "hip", "-std=c++17", "-O1", "-g", "-fPIC", "--offload-arch=gfx950", *host_san,
                  "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
                  "-c", src, "-o", obj + ".tmp"], timeout=900)
            os.replace(obj + ".tmp", obj)
        return obj

    with cf.ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:
        objs = list(ex.map(compile_one, srcs))
    return hipcc, host_san, objs, out


@pytest.mark.slow
@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_scheduler_without_device_under_asan_ubsan(tmp_path):
    hipcc, host_san, objs, out = _asan_library_objects()
    drv = str(tmp_path / "sanitize_server.o")
    _run([hipcc, "-x", "hip", "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", *host_san, "-I",
          os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "sanitize_server.cpp"), "-o", drv])
    exe = str(tmp_path / "sanitize_server")
    _run([hipcc, "--offload-arch=gfx950", *host_san, drv, *objs, "-o", exe, "-lpthread"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([exe], env=env, timeout=300)
    assert "ok" in r.stdout
