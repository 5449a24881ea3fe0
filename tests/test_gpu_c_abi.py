"""The library called from a C program (tests/c_abi/abi_check.c), on the GPU: counts
of hipMalloc'd buffers at an unaligned start and a ragged length against closed
forms (all-ones words: every position once per word, for k = 8, 16, 32, 64 and for
each kernel variant; all-zero words: nothing; constant ids: one category or the
outside counter), and an overlap refused before launch."""
import os
import subprocess

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_caller_on_gpu():
    exe = os.path.join(ROOT, "tests", "c_abi", "abi_check")
    if not os.path.exists(exe):
        pytest.fail("tests/c_abi/abi_check is not built (run __graft_entry__.build())")
    say("c abi: gpu checks")
    res = subprocess.run([exe, "gpu"], capture_output=True, text=True, timeout=120)
    say(res.stdout.strip())
    assert res.returncode == 0, res.stdout + res.stderr
