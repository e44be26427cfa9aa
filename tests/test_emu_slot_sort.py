"""CPU: the round-based slot sort (the bucket sort of the wide split and of
handed-on level buckets) run on the host through a HIP emulation, one OS
thread per GPU thread of a 1024-thread work-group, under AddressSanitizer,
in both LDS layouts the library builds (30720 keys a round over 2^14 slots,
16000 keys a round over 2^13 slots).

Buckets of 1 to 130,000 keys (one round, two rounds, many rounds with
32-bit slot counters; full-range, dense, duplicate-heavy and two-valued
keys; bucket bounds known or found) must come out equal to std::sort, and a
call whose input is its output and needs more than one round must be
refused with the buffer untouched (a later round re-reads the input after
an earlier one wrote the output)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_slot_sort_rounds_on_host_emulation(tmp_path):
    exe = str(tmp_path / "slot_sort_emu")
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address", "-pthread", "-w", "-I", EMU,
           os.path.join(EMU, "slot_sort_emu.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "total wrong 0 " in r.stdout, r.stdout
