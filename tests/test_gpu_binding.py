"""The binding in a fresh process: a context created before anything imports torch
(the library must bind to the HIP runtime torch loads, not a second one)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_context_first_in_a_fresh_process():
    code = ("import paper_2301_05518_amd as tl\n"
            "c = tl.Context(0)\n"
            "c.sync()\n"
            "c.close()\n"
            "print('context ok')\n")
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert res.returncode == 0, res.stderr[-2000:]
    assert "context ok" in res.stdout
