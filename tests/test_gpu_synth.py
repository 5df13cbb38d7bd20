"""The GPU input generator reproduces the CPU twin bit for bit (same counter
hash, Irwin-Hall innovations and fma recursion), so any channel of a GPU-fed
run can be regenerated on the CPU for the oracle."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_helpers import say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_ou_gpu_equals_cpu(dtype):
    say(f"[synth] OU {np.dtype(dtype).name}")
    spec = synth.OUSpec.make(seed=11, stream=3, n=5000, comps=3, tau=10, tau_hi=1000,
                             dtype=dtype)
    ref, _ = spec.series(0, 37)
    g = synth.GpuOU(spec)
    out = torch.empty((37, spec.n), dtype=g.tdt, device="cuda")
    g.fill(out[:20], 20)
    g.fill(out[20:], 17)
    got = out.cpu().numpy()
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))


def test_positions_gpu_equals_cpu():
    say("[synth] positions")
    spec = synth.PositionSpec(seed=5, stream=7, n_atoms=3000, box=100.0)
    ref, _ = spec.series(0, 9)
    g = synth.GpuPositions(spec)
    out = torch.empty((9, 3, spec.n_atoms), dtype=torch.float32, device="cuda")
    g.fill(out, 9)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.view(np.uint32))


def test_cpu_twin_channel_subset():
    spec = synth.OUSpec.make(seed=1, stream=1, n=100, comps=3, tau=20, tau_hi=200)
    full, _ = spec.series(0, 50)
    sub, _ = spec.series(0, 50, channels=[99, 0, 50])
    assert np.array_equal(sub, full[:, [99, 0, 50]])
