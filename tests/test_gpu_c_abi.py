"""The C ABI from plain C on the GPU: the example program (built by
__graft_entry__.build() from paper_1905_01141_amd/examples/tb_roundtrip.c
against include/tdec.h and libtdec.so only) encodes a transport block on the
GPU, decodes its noiseless LLRs and must get the payload back with CRC24A
passing."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1905_01141_amd", "examples", "tb_roundtrip")


@pytest.mark.parametrize("tbs", [75376, 40, 6121])
def test_c_example_round_trip(tbs):
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is missing: run __graft_entry__.build() first")
    print(f"[c-abi] tb_roundtrip {tbs}", flush=True)
    sys.stdout.flush()
    r = subprocess.run([EXE, str(tbs)], capture_output=True, text=True, timeout=60)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "tb_ok=1" in r.stdout and "payload identical" in r.stdout
