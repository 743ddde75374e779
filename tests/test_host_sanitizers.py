"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Three separate programs, so the oracle and the library share nothing even
here: the library's host setup (CSR validation, weights, alias table, record
packing, augmented system), the C oracle, and the serving-stream generator,
each driven over valid and invalid inputs by a small driver in tests/native/.
"""
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
NATIVE = ROOT / "tests" / "native"
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _have_sanitizers(tmp_path):
    if not shutil.which("gcc") or not shutil.which("g++"):
        return False
    probe = tmp_path / "probe.c"
    probe.write_text("int main(void){return 0;}\n")
    r = subprocess.run(["gcc", *SAN, str(probe), "-o", str(tmp_path / "probe")], capture_output=True)
    return r.returncode == 0


def _run(cmd_build, exe, expect):
    b = subprocess.run(cmd_build, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600,
                       env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "PATH": "/usr/bin:/bin"})
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert expect in r.stdout


def test_setup_under_sanitizers(tmp_path):
    if not _have_sanitizers(tmp_path):
        pytest.skip("gcc sanitizer runtime not available")
    exe = tmp_path / "san_setup"
    csrc = ROOT / "paper_1401_4780_amd" / "csrc"
    _run(["g++", "-std=c++17", *SAN, "-ffp-contract=off", "-pthread", f"-I{csrc}",
          str(NATIVE / "sanitize_setup.cpp"), str(csrc / "setup.cpp"), "-o", str(exe)],
         exe, "0 failed checks")


def test_setup_under_thread_sanitizer(tmp_path):
    """The threaded validation (row scans beside the in-order column pass)
    and record writing under ThreadSanitizer: no data race."""
    probe = tmp_path / "p.cpp"
    probe.write_text("int main(){return 0;}\n")
    if not shutil.which("g++") or subprocess.run(["g++", "-fsanitize=thread", str(probe), "-o",
                                                  str(tmp_path / "p")], capture_output=True).returncode:
        pytest.skip("ThreadSanitizer runtime not available")
    exe = tmp_path / "tsan_setup"
    csrc = ROOT / "paper_1401_4780_amd" / "csrc"
    b = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-ffp-contract=off", "-pthread",
                        f"-I{csrc}", str(NATIVE / "sanitize_setup.cpp"), str(csrc / "setup.cpp"), "-o", str(exe)],
                       capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600,
                       env={"TSAN_OPTIONS": "halt_on_error=1", "PATH": "/usr/bin:/bin"})
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "0 failed checks" in r.stdout


def test_oracle_under_sanitizers(tmp_path):
    if not _have_sanitizers(tmp_path):
        pytest.skip("gcc sanitizer runtime not available")
    exe = tmp_path / "san_oracle"
    _run(["gcc", "-std=c99", *SAN, "-ffp-contract=off", str(NATIVE / "sanitize_oracle.c"),
          str(ROOT / "oracle" / "rk_oracle.c"), "-o", str(exe), "-lm"], exe, "0 failed checks")


def test_serving_generator_under_sanitizers(tmp_path):
    if not _have_sanitizers(tmp_path):
        pytest.skip("gcc sanitizer runtime not available")
    exe = tmp_path / "san_sg"
    _run(["gcc", "-std=c99", *SAN, str(NATIVE / "sanitize_serving_gen.c"),
          str(ROOT / "synth" / "serving_gen.c"), "-o", str(exe), "-lm"], exe, "ok")
