"""The device probes on the GPU return plausible ceilings: the packed int16
VALU rate near the published 78.6 TOP/s (it cannot exceed the issue rate of
256 CUs x 4 SIMDs), HBM streaming well under the published 8 TB/s, and
launch overheads of microseconds."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_1905_01141_amd as T
    if not torch.cuda.is_available():
        pytest.fail("a GPU is required for the gpu-marked tests")
    return T


def test_valu_probe(T):
    v = T.probe_valu_int16(0, 20000)
    say(f"[probe] packed int16 VALU {v:.2f} TOP/s")
    assert 20.0 < v <= 78.64 * 1.02


def test_hbm_probe(T):
    r, c = T.probe_hbm(0, 1 << 30)
    say(f"[probe] HBM read {r:.0f} GB/s, copy {c:.0f} GB/s")
    assert 1000.0 < r < 8000.0 * 1.05 and 1000.0 < c < 8000.0 * 1.05


def test_launch_probe(T):
    a, g = T.probe_launch(0, 500)
    say(f"[probe] launch {a:.2f} us, graph node {g:.2f} us")
    assert 0.05 < a < 200.0 and 0.05 < g < 200.0
