"""The FP64 oracles built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): small and degenerate grids of every wall scheme, collision
operator and boundary variant step without an out-of-bounds access or
undefined behaviour, stay finite and, with link walls, keep their mass.
The drivers are tests/native/oracle_sanitize.c (2D) and oracle3_sanitize.c
(3D); gcc aborts the run at the first sanitizer report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]


def _sanitizers_available(tmp_path) -> bool:
    if shutil.which("gcc") is None:
        return False
    src = tmp_path / "probe.c"
    src.write_text("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", *FLAGS, str(src), "-o", str(tmp_path / "probe")],
                       capture_output=True, text=True)
    return r.returncode == 0


@pytest.mark.parametrize("driver", ["oracle_sanitize.c", "oracle3_sanitize.c"])
def test_oracle_under_sanitizers(tmp_path, driver):
    if not _sanitizers_available(tmp_path):
        pytest.skip("gcc with ASan/UBSan runtimes is not available")
    exe = tmp_path / driver.replace(".c", "")
    subprocess.run(["gcc", *FLAGS, os.path.join(HERE, "native", driver), "-lm", "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "all ok" in r.stdout
