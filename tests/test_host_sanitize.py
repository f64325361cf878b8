"""Host code of the library under AddressSanitizer / UndefinedBehaviorSanitizer
(no GPU): tests/host_sanitize/driver.cpp drives validation and preprocessing
through proxsdp_workspace_size on valid and malformed problems.  The device
code is built without sanitizers (each -fsanitize flag applies to the host
pass only)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_preprocessing_is_clean_under_sanitizers():
    tmp = tempfile.mkdtemp(prefix="proxsdp_san_")
    try:
        exe = os.path.join(tmp, "driver")
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", os.path.join(ROOT, "include"),
               os.path.join(ROOT, "paper_1810_05231_amd", "csrc", "proxsdp.hip"),
               os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp"),
               "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
        b = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
        assert b.returncode == 0, b.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
        assert "all ok" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
