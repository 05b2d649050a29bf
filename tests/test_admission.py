"""The request server's memory policy on the CPU (no GPU): tests/admission_sim.cpp drives the
host-only policy header of the server with a fake executor and a fake clock (count and
resident admission, the fragmentation sequence that used to fail a request, deferred release of
tables a merge reads, deterministic replays), built with gcc under the address and undefined
behaviour sanitizers."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_admission_policy_with_fake_executor(tmp_path):
    exe = tmp_path / "admission_sim"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined",
                    "-I", os.path.join(ROOT, "paper_2206_05269_amd", "csrc"),
                    os.path.join(ROOT, "tests", "admission_sim.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    for name in ("fragmentation", "resident_full", "resident_waiters", "merge_pins", "executor"):
        assert f"ok {name}" in r.stdout
