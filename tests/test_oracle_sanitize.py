"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code, CPU only)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_clean_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_asan"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
                    os.path.join(ROOT, "oracle", "wc_oracle.cpp"),
                    os.path.join(ROOT, "oracle", "sanitize_driver.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "entries" in r.stdout
