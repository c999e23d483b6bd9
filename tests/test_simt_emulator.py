"""The library's kernels compiled for the host and run on the CPU SIMT
emulator (tests/simt) under AddressSanitizer: every GPU thread a fiber,
block barriers and wave64 collectives emulated, several blocks in flight at
once.  Checks results against the oracle and catches out-of-bounds accesses
to device buffers and LDS arrays without a GPU."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "simt"))


@pytest.fixture(scope="module")
def emu_dir(tmp_path_factory):
    import build as simt_build  # tests/simt/build.py
    d = str(tmp_path_factory.mktemp("simt"))
    simt_build.build(d)
    return d


def run(exe, *args, workers=4, timeout=600):
    env = dict(os.environ, SIMT_WORKERS=str(workers), ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=timeout, env=env)
    return r


def test_emulated_kernels_match_oracle(emu_dir):
    # 1,024-thread passes run four look-back agent workgroups beside the tile
    # workgroups: emulate more blocks at once than that.
    r = run(os.path.join(emu_dir, "emu_driver"), "quick", workers=8)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "0 failure(s)" in r.stdout


def test_lookback_under_concurrency(emu_dir):
    exe = os.path.join(emu_dir, "lookback_stress")
    inc = ["-I" + os.path.join(HERE, "simt", "include"), "-I" + os.path.join(os.path.dirname(HERE), "include"),
           "-I" + os.path.join(os.path.dirname(HERE), "paper_1105_6040_amd", "csrc")]
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-w", "-U_FORTIFY_SOURCE", "-fsanitize=address,undefined",
                    *inc, os.path.join(HERE, "simt", "lookback_stress.cpp"), os.path.join(HERE, "simt", "simt.cpp"),
                    "-o", exe, "-lpthread"], check=True)
    r = run(exe, workers=8)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert r.stdout.count("ok   lookback") == 7
