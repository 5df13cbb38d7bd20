"""corr_finalize_noalloc (the readout that allocates no device memory) against
corr_finalize: the same results bit for bit, on two calls in a row on the
same GPU, the second with a smaller input, so that the fixed scratch array
keeps the first call's contents when the second runs.  The first context's
block-deferred group is large enough that its readout is reduced in several
passes over the scratch array."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_helpers import say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

KEYS = ("t", "c", "count", "gk_running")


def _same(a, b, label):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), f"{label}: {k} differs"
    assert a["gk_at_cut"] == b["gk_at_cut"], f"{label}: gk_at_cut differs"
    if "c_per_channel" in a or "c_per_channel" in b:
        assert np.array_equal(a["c_per_channel"], b["c_per_channel"]), f"{label}: slice differs"


def _fill_and_push(corr, gens, bufs, S, chunk):
    done = 0
    while done < S:
        n = min(chunk, S - done)
        for gen, buf in zip(gens, bufs):
            gen.fill(buf, n)
        for j in range(n):
            corr.push([buf[j] for buf in bufs])
        done += n
    torch.cuda.synchronize()


def _compare(corr, g, n_ch, label, **kw):
    ref = corr.finalize(g, **kw)
    got = corr.finalize(g, noalloc=True, **kw)
    _same(ref, got, label)
    say(f"  {label}: {len(ref['t'])} entries identical")
    return ref


def test_noalloc_readout_matches_finalize():
    from paper_2503_07526_amd import Correlator, GroupDesc
    from paper_2503_07526_amd.corr import CORR_E_UNSUPPORTED, CorrError

    # First call: 3e6 block-deferred FP32 channels with compensated sums (b=10):
    # after 600 pushes 57 (level, lag) entries, so the per-chunk sums (46864
    # rows x 57 doubles) exceed the 16 MiB array and are reduced in two passes;
    # beside it a direct-form FP64 group.
    n1, S1 = 3_000_000, 600
    say(f"[noalloc] first context: {n1} deferred channels + 9 FP64 channels, {S1} pushes")
    g1 = [GroupDesc(n1, 10, 16, 2, dtype="f32", accum="kahan"),
          GroupDesc(9, 12, 16, 2, dtype="f64", accum="f64")]
    specs = [synth.OUSpec.make(seed=11, stream=1, n=n1, comps=3, tau=20, tau_hi=200),
             synth.OUSpec.make(seed=11, stream=2, n=9, tau=50, dtype=np.float64)]
    chunk = 100
    bufs = [torch.empty((chunk, n1), dtype=torch.float32, device="cuda"),
            torch.empty((chunk, 9), dtype=torch.float64, device="cuda")]
    with Correlator(g1) as c1:
        _fill_and_push(c1, [synth.GpuOU(s) for s in specs], bufs, S1, chunk)
        say("  pushes done")
        _compare(c1, 0, n1, "deferred group, all channels", slice_=(n1 - 5, n1))
        _compare(c1, 0, n1, "deferred group, channel range",
                 ch=(123_457, 2_987_654), slice_=(0, 3))
        _compare(c1, 1, 9, "FP64 group", slice_=(0, 9), gk_kind=1, volume=2.0, kB=1.0,
                 temperature=1.5)
        # a slice beyond the fixed array is refused (host-side check, nothing launched)
        with pytest.raises(CorrError) as ei:
            c1.finalize(0, slice_=(0, 100_000), noalloc=True)
        assert ei.value.code == CORR_E_UNSUPPORTED
    del bufs
    torch.cuda.empty_cache()

    # Second call, smaller: a 5000-channel deferred group (one pass), a pair
    # group and a long one-level window, readouts between flush boundaries.
    n2, S2 = 5000, 777
    say(f"[noalloc] second context: {n2} deferred + 64 pair + 256 window channels, {S2} pushes")
    g2 = [GroupDesc(n2, 6, 16, 2, dtype="f32", accum="kahan"),
          GroupDesc(64, 5, 16, 2, dtype="f32", accum="f64", pair=True),
          GroupDesc(256, 1, 1024, 2, dtype="f32", accum="kahan")]
    specs2 = [synth.OUSpec.make(seed=12, stream=1, n=n2, tau=30),
              synth.OUSpec.make(seed=12, stream=2, n=128, tau=40),
              synth.OUSpec.make(seed=12, stream=3, n=256, tau=50)]
    chunk = 111
    bufs = [torch.empty((chunk, n2), dtype=torch.float32, device="cuda"),
            torch.empty((chunk, 128), dtype=torch.float32, device="cuda"),
            torch.empty((chunk, 256), dtype=torch.float32, device="cuda")]
    with Correlator(g2) as c2:
        _fill_and_push(c2, [synth.GpuOU(s) for s in specs2], bufs, S2, chunk)
        _compare(c2, 0, n2, "small deferred group", slice_=(17, 33))
        _compare(c2, 1, 64, "pair group", slice_=(0, 64))
        _compare(c2, 2, 256, "window group", slice_=(250, 256))
        # readouts do not change later results: push on and compare again
        _fill_and_push(c2, [synth.GpuOU(s) for s in specs2], bufs, 2 * chunk, chunk)
        _compare(c2, 0, n2, "small deferred group, later", ch=(1, n2 - 1))
