"""The call-slot bookkeeping of persistent launches (csrc/pn_slots.hpp) on the
host, with a fake runtime: a slot is reused only after the new call's
stream waits for the event recorded after the slot's last launch; captured
calls take dedicated slots and no events; an exhausted capture pool fails
without launching; host threads never run two launches on one slot at once.
Guards against the silent failures the paper describes for GPU runs
(Sec. III): a slot rewritten under a running launch would give wrong outputs
with no error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_slot_bookkeeping(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "slots_check"
    src = os.path.join(ROOT, "tests", "native", "slots_check.cpp")
    inc = os.path.join(ROOT, "paper_0908_3889_amd", "csrc")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-pthread", "-I", inc, src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
