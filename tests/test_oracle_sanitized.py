"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): `oracle_sanitize_main.c` includes the oracle's source and runs small
problems over every boundary kind, the shortest lines, the limiter near
vacuum, all reconstructions and fluxes, the 2D operator and the batched
driver; an out-of-bounds access, a leak or an undefined operation aborts it."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_sanitized")
    build = subprocess.run(
        [gcc, "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         os.path.join(HERE, "oracle_sanitize_main.c"), "-o", exe, "-lm"],
        capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("sanitizer runtime not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert run.stdout.strip().endswith("ok")
