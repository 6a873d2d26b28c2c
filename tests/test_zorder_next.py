"""The library's next-key-in-box step (the box pre-filter scan's skip over z-order
key runs outside the box) against brute force: a host build of csrc/zorder.h."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc (host build only)")
def test_znext_is_the_next_box_key(tmp_path):
    exe = str(tmp_path / "zcheck")
    subprocess.check_call(["hipcc", "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(HERE, "zorder_next_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("bad 0"), out.stdout
