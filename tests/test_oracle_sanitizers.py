"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

oracle/sanitize_driver.cpp runs every entry point of the oracle once on a
small seeded input (trees, the h solve, hydro with and without the
switches, velocity gradients, conduction, gravity at three opening angles,
the three list kinds, the three adjoints, a refit). Built with
-fsanitize=address,undefined and no recovery, any out-of-bounds access,
use-after-free, leak or undefined operation ends the run with a report. A
planted heap overflow in a separate two-line program checks that the
toolchain's sanitizer is active at all.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")
FLAGS = ["-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)


def test_sanitizer_catches_a_planted_overflow(tmp_path):
    src = tmp_path / "planted.cpp"
    src.write_text("#include <vector>\nint main() { std::vector<int> v(4); "
                   "return v.data()[4]; }\n")
    exe = tmp_path / "planted"
    subprocess.run(["g++", *FLAGS, str(src), "-o", str(exe)], check=True)
    r = run(str(exe))
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "g3ref_sanitized"
    subprocess.run(["g++", *FLAGS, f"-I{ORACLE}", os.path.join(ORACLE, "g3ref.cpp"),
                    os.path.join(ORACLE, "sanitize_driver.cpp"), "-o", str(exe)], check=True)
    r = run(str(exe))
    print(r.stdout)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "LeakSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    assert "sanitized oracle run: rc 0, 0 non-finite outputs" in r.stdout
