"""The C ABI driven from plain C (tests/native/abi_check.c, built by
__graft_entry__.build()): solves in both precisions and both cycle types,
read-backs, a ragged batch, a three-level AMR problem, a server with more
requests than slots and an invalid domain, all through include/emg.h."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "native", "abi_check")


def test_c_abi_driver():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.fail("tests/native/abi_check is not built (run __graft_entry__.build())")
    print("[gpu] C ABI driver", flush=True)
    res = subprocess.run([EXE], capture_output=True, text=True, timeout=240)
    print(res.stdout + res.stderr, flush=True)
    assert res.returncode == 0 and "abi_check: 0 failure(s)" in res.stdout
