"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): the
driver tests/oracle_sanitize_driver.c runs pair searches and full steps with contact history
for every physics variant; any out-of-bounds access, leak or undefined behaviour aborts it."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "drv")
    flags = ["-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    cmd = [gcc, *flags, os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "dss_oracle.c"),
           "-o", exe, "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and ("asan" in build.stderr or "ubsan" in build.stderr):
        pytest.skip("gcc without the sanitizer runtimes")
    assert build.returncode == 0, build.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0"))
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert out.count("variant ") == 4, out
