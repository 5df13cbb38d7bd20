"""GPU parity: the HIP correlator (through the C ABI) against the CPU FP64
oracle on the same seeded inputs.  Counts and lag times must match exactly;
C(t) within the tolerance of its precision class (tests/gpu_helpers.TOL),
measured as max |dC| / |C(0)| over the group mean and over sampled channels.
Sizes span several 512-channel tiles with a ragged tail."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_helpers import TOL, gate, oracle_run, ou_inputs, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def corrmod():
    import paper_2503_07526_amd as m
    m.lib()  # fails loudly if the HIP library is missing
    return m


def _push_all(corr, xs):
    dev = torch.device("cuda:0")
    ts = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in xs]
    for s in range(xs[0].shape[0]):
        corr.push([t[s] for t in ts])
    torch.cuda.synchronize()


KINDS = [("f32", "f64"), ("f32", "kahan"), ("f32", "f32"), ("f64", "f64"),
         ("cf32", "f64"), ("cf32", "kahan"), ("cf32", "f32"), ("cf64", "f64")]


@pytest.mark.parametrize("direct", [False, True])
@pytest.mark.parametrize("dtype,accum", KINDS)
def test_parity_each_kind(corrmod, dtype, accum, direct):
    """Every (sample, accumulator) kind; single-precision real kinds with p=16,
    m=2 run the block-deferred form unless direct=True."""
    n, S, b, p, m = 1300, 1200, 7, 16, 2
    say(f"[parity kind] dtype={dtype} accum={accum} direct={direct} n={n} S={S} b={b} p={p}")
    x = ou_inputs(7, 11, n, S, dtype)
    o = oracle_run(x, b, p, m)
    with corrmod.Correlator([corrmod.GroupDesc(n, b, p, m, dtype=dtype, accum=accum)],
                            direct=direct) as c:
        _push_all(c, [x])
        sl = (n - 5, n)
        res = c.finalize(0, slice_=sl)
        err = gate(res, o, TOL[(dtype, accum)], slice_=sl, label=f"{dtype}/{accum}")
        res0 = c.finalize(0, slice_=(0, 4))
        gate(res0, o, TOL[(dtype, accum)], slice_=(0, 4), label=f"{dtype}/{accum} head")
    say(f"  max |dC|/|C(0)| = {err:.2e}")


@pytest.mark.parametrize("n,S,b,p,m", [
    (1, 50, 4, 16, 2),        # one channel
    (513, 5, 4, 16, 2),       # fewer pushes than points
    (700, 0, 4, 16, 2),       # no push at all
    (700, 777, 5, 7, 3),      # m does not divide p
    (700, 400, 3, 4, 2),      # small p
    (700, 300, 6, 3, 2),      # p = 3, lag0 = 1
    (600, 700, 4, 9, 4),      # m = 4
    (1100, 600, 6, 32, 2),    # p = 32 (two lag chunks)
    (520, 1000, 1, 16, 2),    # single level
    (520, 1000, 2, 16, 2),    # two levels
    (1030, 2048, 12, 16, 2),  # pushes = 2^11: deepest level just reached
])
def test_parity_shapes(corrmod, n, S, b, p, m):
    say(f"[parity shape] n={n} S={S} b={b} p={p} m={m}")
    x = ou_inputs(3, 5, n, max(S, 1), "f64")[:S]
    o = oracle.OracleCorrelator(n, b, p, m)
    for row in x:
        o.push(row)
    with corrmod.Correlator([corrmod.GroupDesc(n, b, p, m, dtype="f64", accum="f64")]) as c:
        if S:
            _push_all(c, [x])
        res = c.finalize(0, slice_=(0, min(n, 3)))
        assert c.n_pushes() == S
        if S == 0:
            assert len(res["t"]) == 0
            return
        gate(res, o, 1e-12, slice_=(0, min(n, 3)), label="shape")


@pytest.mark.parametrize("tuning", [
    dict(tile_channels=256, chans_per_thread=1, lag_chunk=16, grid_blocks=0),
    dict(tile_channels=256, chans_per_thread=1, lag_chunk=8, grid_blocks=0),
    dict(tile_channels=512, chans_per_thread=2, lag_chunk=8, grid_blocks=0),
    dict(tile_channels=256, chans_per_thread=2, lag_chunk=4, grid_blocks=3),
    dict(tile_channels=1024, chans_per_thread=4, lag_chunk=4, grid_blocks=0),
    dict(tile_channels=256, chans_per_thread=4, lag_chunk=8, grid_blocks=5),
])
def test_tile_invariance_bitwise(corrmod, tuning):
    """Every launch shape gives bit-identical results (one thread owns each
    channel; the readout reduction order does not depend on the tiling)."""
    n, S = 2100, 600
    say(f"[tile invariance] {tuning}")
    xs = [ou_inputs(1, 2, n, S, "f32"), ou_inputs(1, 3, 300, S, "cf32")]
    groups = [corrmod.GroupDesc(n, 6, 16, 2, dtype="f32", accum="kahan"),
              corrmod.GroupDesc(300, 5, 32, 2, dtype="cf32", accum="f64")]
    ref = []
    with corrmod.Correlator(groups) as c:
        _push_all(c, xs)
        ref = [c.finalize(g, slice_=(0, 7)) for g in range(2)]
    with corrmod.Correlator(groups, tuning=tuning) as c:
        _push_all(c, xs)
        got = [c.finalize(g, slice_=(0, 7)) for g in range(2)]
    for r, g in zip(ref, got):
        assert np.array_equal(r["c"], g["c"])
        assert np.array_equal(r["c_per_channel"], g["c_per_channel"])


def test_snapshot_is_non_destructive(corrmod):
    n, S = 900, 500
    say("[snapshot] finalize mid-run then continue")
    x = ou_inputs(9, 9, n, S, "f32")
    with corrmod.Correlator([corrmod.GroupDesc(n, 6, 16, 2, accum="kahan")]) as a, \
            corrmod.Correlator([corrmod.GroupDesc(n, 6, 16, 2, accum="kahan")]) as b:
        _push_all(a, [x[:123]])
        mid = a.finalize(0)
        _push_all(a, [x[123:]])
        _push_all(b, [x])
        ra, rb = a.finalize(0), b.finalize(0)
        assert np.array_equal(ra["c"], rb["c"]) and np.array_equal(ra["count"], rb["count"])
        o = oracle_run(x[:123], 6, 16, 2)
        gate(mid, o, TOL[("f32", "kahan")], label="mid-run")


@pytest.mark.parametrize("rhok_valu", [False, True])
def test_rhok_magnitude_and_phase(corrmod, rhok_valu):
    """One push: C(0) of k = |n(k)|^2 / N.  Two pushes with every atom moved by
    d: C(lag 1) = exp(i k.d) |n(k)|^2 / N (later times conj(earlier)).  Both
    producers: matrix cores (default) and vector units."""
    kv = synth.kvectors(300)
    N, box = 5000, 100.0
    say(f"[rho(k)] N={N} nk={len(kv)} valu={rhok_valu}")
    ps = synth.PositionSpec(4, 4, N, box)
    r0 = ps.r0.copy()
    d = np.array([0.37, -1.25, 2.5], dtype=np.float32)
    r1 = (r0 + d[:, None]).astype(np.float32)
    g = corrmod.GroupDesc(len(kv), 3, 8, 2, dtype="cf32", accum="f64", source="rhok", kvec=kv,
                          n_atoms=N, box=box)
    with corrmod.Correlator([g], rhok_valu=rhok_valu) as c:
        _push_all(c, [r0[None]])
        res = c.finalize(0, slice_=(0, len(kv)))
        rho0 = oracle.rhok(r0, kv, box)
        expect = np.abs(rho0) ** 2 / N
        got = res["c_per_channel"][:, 0]
        assert np.max(np.abs(got - expect)) / np.max(expect) < 2e-6
        _push_all(c, [r1[None]])
        res = c.finalize(0, slice_=(0, len(kv)))
        rho1 = oracle.rhok(r1, kv, box)
        expect1 = rho1 * np.conj(rho0) / N
        got1 = res["c_per_channel"][:, 1]
        assert np.max(np.abs(got1 - expect1)) / np.max(np.abs(expect1)) < 2e-6


@pytest.mark.parametrize("case", ["wide_nz", "large_n", "nmax15", "duplicates", "ragged_atoms"])
def test_rhok_kset_shapes(corrmod, case):
    """A k-set with a component above 15 takes the vector-unit producer; wide
    n_z ranges, components up to the matrix-core limit of 15, repeated
    k-vectors and atom counts that are not a multiple of the atom tile: every
    listed k gets |n(k)|^2 / N at lag 0, and both producers agree."""
    rng = np.random.default_rng(11)
    N, box = 3001, 50.0
    if case == "wide_nz":
        kv = np.stack([rng.integers(-3, 4, 200), rng.integers(-3, 4, 200),
                       rng.integers(-20, 21, 200)], axis=1).astype(np.int32)
    elif case == "large_n":
        kv = np.stack([rng.integers(-16, 17, 150), rng.integers(-2, 3, 150),
                       rng.integers(-2, 3, 150)], axis=1).astype(np.int32)
        kv[0] = (16, 0, 0)
    elif case == "nmax15":
        kv = np.stack([rng.integers(-15, 16, 300), rng.integers(-15, 16, 300),
                       rng.integers(-15, 16, 300)], axis=1).astype(np.int32)
        kv[0] = (15, -15, 15)
    elif case == "duplicates":
        base = synth.kvectors(100)
        kv = np.concatenate([base, base[::7], base[:3]]).astype(np.int32)
    else:
        kv = synth.kvectors(257)
        N = 64 * 37 + 19
    kv = kv[np.any(kv != 0, axis=1)]  # k = 0 would only measure N
    say(f"[rho(k) k-set] {case} nk={len(kv)} N={N}")
    ps = synth.PositionSpec(9, 1, N, box)
    r0 = ps.r0.copy()
    expect = np.abs(oracle.rhok(r0, kv, box)) ** 2 / N
    got = {}
    for valu in (False, True):
        g = corrmod.GroupDesc(len(kv), 2, 4, 2, dtype="cf32", accum="f64", source="rhok",
                              kvec=kv, n_atoms=N, box=box)
        with corrmod.Correlator([g], rhok_valu=valu) as c:
            _push_all(c, [r0[None]])
            got[valu] = c.finalize(0, slice_=(0, len(kv)))["c_per_channel"][:, 0]
        err = np.max(np.abs(got[valu] - expect)) / np.max(expect)
        assert err < 2e-6, (case, valu, err)
    assert np.max(np.abs(got[False] - got[True])) / np.max(expect) < 2e-6


@pytest.mark.parametrize("rhok_valu", [False, True])
def test_batched_mixed_groups_and_modes(corrmod, rhok_valu):
    """Three uneven groups in one context (compensated FP32 velocities, the
    k-space density, FP64 global channels): parity with the oracle, and
    bit-identical state from the batched launch, the per-group launches, the
    HIP graph replay and both forked issue orders (producers forked; per-step
    updates forked beside the flush), with either k-density producer, and from
    captured runs of 100 pushes with the producers forked (corr_push_steps:
    two chains joined every 4 pushes, one capture replayed four
    times across the first fold block)."""
    S, nv, N, box = 400, 2500, 3000, 100.0
    kv = synth.kvectors(200)
    say(f"[batched] S={S} nv={nv} N={N} nk={len(kv)}")
    xv = ou_inputs(5, 1, nv, S, "f32")
    xg = ou_inputs(5, 2, 9, S, "f64", tau=50, tau_hi=None)
    pos = synth.PositionSpec(5, 3, N, box)
    xp, _ = pos.series(0, S)
    groups = [corrmod.GroupDesc(nv, 7, 16, 2, dtype="f32", accum="kahan"),
              corrmod.GroupDesc(len(kv), 6, 32, 2, dtype="cf32", accum="kahan", source="rhok",
                                kvec=kv, n_atoms=N, box=box),
              corrmod.GroupDesc(9, 9, 16, 2, dtype="f64", accum="f64")]
    ov = oracle_run(xv, 7, 16, 2)
    og = oracle_run(xg, 9, 16, 2)
    orh = oracle.OracleCorrelator(len(kv), 6, 32, 2, complex_=True)
    for s in range(S):
        orh.push(oracle.rhok(xp[s], kv, box))
    results = {}
    modes = ("batched", "per_group", "graph", "overlap", "overlap_graph", "overlap2",
             "overlap2_graph", "overlap_steps")
    for mode in modes:
        say(f"  mode {mode}")
        tuning = None
        if mode.startswith("overlap"):
            tuning = {"overlap_producers": 2 if mode.startswith("overlap2") else 1}
        with corrmod.Correlator(groups, graph=mode.endswith(("graph", "steps")),
                                per_group=(mode == "per_group"), rhok_valu=rhok_valu,
                                tuning=tuning) as c:
            dev = torch.device("cuda:0")
            tv = torch.from_numpy(xv).to(dev)
            tg = torch.from_numpy(xg).to(dev)
            tp = torch.from_numpy(xp).to(dev)
            if mode.endswith("steps"):
                ch = 100
                bufs = [torch.empty((ch,) + tuple(t.shape[1:]), dtype=t.dtype, device=dev)
                        for t in (tv, tp, tg)]
                for s0 in range(0, S, ch):
                    for b, t in zip(bufs, (tv, tp, tg)):
                        b.copy_(t[s0:s0 + ch])  # the same buffers every call: one capture
                    c.push_steps(bufs)
            elif mode.endswith("graph"):
                bv = torch.empty_like(tv[0]); bp = torch.empty_like(tp[0]); bg = torch.empty_like(tg[0])
                c.bind_input(0, bv); c.bind_input(1, bp); c.bind_input(2, bg)
                for s in range(S):
                    bv.copy_(tv[s]); bp.copy_(tp[s]); bg.copy_(tg[s])
                    c.push()
            else:
                for s in range(S):
                    c.push([tv[s], tp[s], tg[s]])
            results[mode] = [c.finalize(g, slice_=(0, 5)) for g in range(3)]
    for mode in modes[1:]:
        for g in range(3):
            assert np.array_equal(results[mode][g]["c"], results["batched"][g]["c"]), (mode, g)
            assert np.array_equal(results[mode][g]["c_per_channel"],
                                  results["batched"][g]["c_per_channel"]), (mode, g)
    r = results["batched"]
    e1 = gate(r[0], ov, TOL[("f32", "kahan")], slice_=(0, 5), label="velocity")
    e2 = gate(r[1], orh, TOL[("cf32", "kahan")], scale=1.0 / N, slice_=(0, 5), label="rho(k)")
    e3 = gate(r[2], og, TOL[("f64", "f64")], slice_=(0, 5), label="global")
    say(f"  errors: velocity {e1:.2e} rho(k) {e2:.2e} global {e3:.2e}")


def test_green_kubo_readout(corrmod):
    """gk_running / gk_at_cut follow the trapezoid integral of the oracle's C
    with the viscosity and conductivity prefactors (Section 2.3)."""
    S = 3000
    x = ou_inputs(2, 8, 9, S, "f64", tau=50, tau_hi=None)
    o = oracle_run(x, 10, 16, 2)
    V, kB, T = 1000.0, 1.380649e-23 * 1e23, 300.0
    with corrmod.Correlator([corrmod.GroupDesc(9, 10, 16, 2, dtype="f64", dt=0.001)]) as c:
        _push_all(c, [x])
        for kind, ch, fn in ((1, (3, 6), oracle.green_kubo_viscosity),
                             (2, (6, 9), oracle.green_kubo_conductivity)):
            res = c.finalize(0, ch=ch, gk_kind=kind, volume=V, kB=kB, temperature=T, t_cut=0.5)
            t, cm, _ = o.readout(*ch)
            run, at = fn(t * 0.001, cm, V, kB, T, t_cut=0.5)
            assert np.allclose(res["gk_running"], run, rtol=1e-12, atol=1e-12 * abs(run).max())
            assert abs(res["gk_at_cut"] - at) <= 1e-12 * abs(at)


@pytest.mark.parametrize("accum", ["kahan", "f64"])
def test_deferred_readout_at_many_push_counts(corrmod, accum):
    """Block-deferred groups: readouts before the first flush, exactly at flush
    boundaries and with pending pushes all match the oracle at that push count,
    and never change later results (bitwise against an uninterrupted run)."""
    n, b, p, m = 700, 12, 16, 2
    marks = [1, 2, 15, 16, 17, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257, 511, 512, 513, 700,
             767, 768, 769, 1024, 1500]
    S = marks[-1]
    say(f"[deferred readouts] accum={accum} n={n}")
    x = ou_inputs(4, 4, n, S, "f32")
    o = oracle.OracleCorrelator(n, b, p, m)
    dev = torch.device("cuda:0")
    tx = torch.from_numpy(x).to(dev)
    g = [corrmod.GroupDesc(n, b, p, m, dtype="f32", accum=accum)]
    with corrmod.Correlator(g) as c, corrmod.Correlator(g) as ref:
        done = 0
        for mk in marks:
            for s in range(done, mk):
                c.push([tx[s]])
                ref.push([tx[s]])
                o.push(x[s].astype(np.float64))
            done = mk
            res = c.finalize(0, slice_=(n - 3, n))
            gate(res, o, TOL[("f32", accum)], slice_=(n - 3, n), label=f"S={mk}")
        a, r = c.finalize(0, slice_=(0, n)), ref.finalize(0, slice_=(0, n))
        assert np.array_equal(a["c"], r["c"])
        assert np.array_equal(a["c_per_channel"], r["c_per_channel"])


@pytest.mark.parametrize("b", [1, 2, 3, 9])
def test_deferred_level_counts(corrmod, b):
    """The block-deferred fold streams levels 0 and 1 through each block and
    runs the cascade from level 2: groups with one, two and three levels (no
    level 1, no cascade, a one-level cascade) and a deep one, across several
    blocks, read out at a block boundary and with pushes pending."""
    n = 300
    say(f"[deferred levels] b={b}")
    x = ou_inputs(6, 9, n, 1300, "f32")
    o = oracle.OracleCorrelator(n, b, 16, 2)
    dev = torch.device("cuda:0")
    tx = torch.from_numpy(x).to(dev)
    with corrmod.Correlator([corrmod.GroupDesc(n, b, 16, 2, dtype="f32", accum="kahan")]) as c:
        done = 0
        for mk in (768, 1300):
            for s in range(done, mk):
                c.push([tx[s]])
                o.push(x[s].astype(np.float64))
            done = mk
            res = c.finalize(0, slice_=(0, 3))
            gate(res, o, TOL[("f32", "kahan")], slice_=(0, 3), label=f"b={b} S={mk}")


def test_deferred_equals_direct_within_rounding(corrmod):
    """The block-deferred form regroups the same sums as the per-step form."""
    n, S = 2000, 3000
    say("[deferred vs direct]")
    x = ou_inputs(8, 8, n, S, "f32")
    g = [corrmod.GroupDesc(n, 12, 16, 2, dtype="f32", accum="f64")]
    with corrmod.Correlator(g) as d, corrmod.Correlator(g, direct=True) as e:
        _push_all(d, [x])
        _push_all(e, [x])
        rd, re_ = d.finalize(0, slice_=(0, 50)), e.finalize(0, slice_=(0, 50))
        assert np.array_equal(rd["count"], re_["count"])
        assert np.max(np.abs(rd["c"] - re_["c"])) <= 1e-12 * abs(re_["c"][0])
        assert np.max(np.abs(rd["c_per_channel"] - re_["c_per_channel"])) <= 1e-9


def test_autotune_picks_and_caches(corrmod, tmp_path):
    """The autotuner returns a valid launch shape, writes it to the cache, reads
    it back without timing, and a context created with it matches the oracle."""
    import time as _t
    cache = str(tmp_path / "tune.jsonl")
    groups = [corrmod.GroupDesc(5000, 6, 16, 2, dtype="f32", accum="kahan"),
              corrmod.GroupDesc(9, 8, 16, 2, dtype="f64", accum="f64")]
    say("[autotune]")
    t0 = _t.perf_counter()
    tn = corrmod.autotune(groups, cache_path=cache, max_trial_channels=1 << 14)
    first = _t.perf_counter() - t0
    assert tn["tile_channels"] % (64 * tn["chans_per_thread"]) == 0
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"key":"arch=gfx950' in lines[0]
    t0 = _t.perf_counter()
    tn2 = corrmod.autotune(groups, cache_path=cache, max_trial_channels=1 << 14)
    assert tn2 == tn and _t.perf_counter() - t0 < first
    x = ou_inputs(6, 6, 5000, 300, "f32")
    o = oracle_run(x, 6, 16, 2)
    with corrmod.Correlator(groups[:1], tuning=tn) as c:
        assert c.tuning() == tn
        _push_all(c, [x])
        gate(c.finalize(0, slice_=(0, 3)), o, TOL[("f32", "kahan")], slice_=(0, 3),
             label="autotuned")


def test_kernel_time_pools(corrmod):
    """CORR_FLAG_TIMING: one push-event pair, one flush-fold pair and one
    producer pair per push in a context with a block-deferred group and a
    k-density group; positive summed times; reset clears the counters; with a
    timing stride only one push in `stride` is timed, and state is unchanged."""
    S, nv, N, box = 70, 4096, 2000, 50.0
    kv = synth.kvectors(64)
    xv = ou_inputs(8, 1, nv, S, "f32")
    xp, _ = synth.PositionSpec(8, 2, N, box).series(0, S)
    groups = [corrmod.GroupDesc(nv, 6, 16, 2, dtype="f32", accum="kahan"),
              corrmod.GroupDesc(len(kv), 4, 16, 2, dtype="cf32", accum="f64", source="rhok",
                                kvec=kv, n_atoms=N, box=box)]
    with corrmod.Correlator(groups, timing=True) as c:
        _push_all(c, [xv, xp])
        for which in (0, 1, 2, 3, 4):
            ms, n = c.kernel_time(which)
            assert n == S and ms > 0.0, (which, n, ms)
        # the device stamps of the fold and of the producer span their events'
        # intervals at most
        assert c.kernel_time(3)[0] <= c.kernel_time(1)[0] * 1.05 + 0.01
        assert c.kernel_time(4)[0] <= c.kernel_time(2)[0] * 1.05 + 0.01
        ms, n = c.kernel_time(2, reset=True)
        assert c.kernel_time(2) == (0.0, 0)
        for which in (3, 4):
            c.kernel_time(which, reset=True)
            assert c.kernel_time(which) == (0.0, 0)
        with pytest.raises(corrmod.CorrError):
            c.kernel_time(5)
    # one push in 8 timed (pushes 0, 8, ..., 64 of 70): same state as every push timed
    with corrmod.Correlator(groups, timing=True) as c, corrmod.Correlator(groups) as ref:
        c.set_timing_stride(8)
        with pytest.raises(corrmod.CorrError):
            c.set_timing_stride(0)
        _push_all(c, [xv, xp])
        _push_all(ref, [xv, xp])
        for which in (0, 1, 2):
            ms, n = c.kernel_time(which)
            assert n == 9 and ms > 0.0, (which, n, ms)
        # the device stamps follow the stride too (the device push counter)
        assert c.kernel_time(3)[1] == 9 and c.kernel_time(4)[1] == 9
        assert np.array_equal(c.finalize(0, slice_=(0, 3))["c_per_channel"],
                              ref.finalize(0, slice_=(0, 3))["c_per_channel"])
        with pytest.raises(corrmod.CorrError):
            ref.set_timing_stride(4)  # no CORR_FLAG_TIMING
    # captured graphs: stamps on pushes 0, 8, ..., 64 whatever the chunks, same state
    # (also with the producers forked, where a captured run joins the two
    # streams every few pushes and each stream ends its pushes with its own
    # counter; the runs of 13, 32 and 25 pushes end between joins)
    for tuning in (None, {"overlap_producers": 1}):
        with corrmod.Correlator(groups, timing=True, graph=True, tuning=tuning) as c, \
                corrmod.Correlator(groups) as ref:
            c.set_timing_stride(8)
            xv_d = torch.as_tensor(xv, device="cuda")
            xp_d = torch.as_tensor(xp, device="cuda")
            for a, b in ((0, 13), (13, 45), (45, S)):
                c.push_steps([xv_d[a:b], xp_d[a:b]])
            _push_all(ref, [xv, xp])
            assert c.kernel_time(3)[1] == 9 and c.kernel_time(4)[1] == 9, tuning
            for g in range(2):
                assert np.array_equal(c.finalize(g, slice_=(0, 3))["c_per_channel"],
                                      ref.finalize(g, slice_=(0, 3))["c_per_channel"]), tuning


def _currents_inputs(seed, N, box, S):
    """[S][6][N] float32: positions (seeded lattice-free uniform + OU drift)
    then velocities (unit-variance OU series, tau 20)."""
    pos, _ = synth.PositionSpec(seed, 1, N, box).series(0, S)
    vel = ou_inputs(seed, 7, 3 * N, S, "f32").reshape(S, 3, N)
    return np.ascontiguousarray(np.concatenate([pos, vel], axis=1))


@pytest.mark.parametrize("source,valu", [("rhok", False), ("rhok", True), ("currents", False)])
def test_producers_with_double_samples(corrmod, source, valu):
    """Producer groups with complex-double samples (the producers' double
    output path) and FP64 accumulators: C(0) and C(1) of two pushes against
    the oracle's direct double sums; the producer's own precision (about 22
    significant bits per product on the matrix cores) sets the bound."""
    N, box = 4000, 40.0
    kv = synth.kvectors(96)
    say(f"[double samples] {source} valu={valu}")
    x = _currents_inputs(46, N, box, 2)
    nch = len(kv) * (3 if source == "currents" else 1)
    g = corrmod.GroupDesc(nch, 3, 8, 2, dtype="cf64", accum="f64", source=source, kvec=kv,
                          n_atoms=N, box=box)
    inp = x if source == "currents" else np.ascontiguousarray(x[:, :3])
    with corrmod.Correlator([g], rhok_valu=valu) as c:
        _push_all(c, [inp])
        res = c.finalize(0, slice_=(0, nch))
    if source == "currents":
        v = [oracle.currents(x[s, :3], x[s, 3:], kv, box).reshape(-1) for s in range(2)]
    else:
        v = [oracle.rhok(x[s, :3], kv, box) for s in range(2)]
    c0 = (np.abs(v[0]) ** 2 + np.abs(v[1]) ** 2) / 2 / N
    c1 = v[1] * np.conj(v[0]) / N
    e0 = np.max(np.abs(res["c_per_channel"][:, 0] - c0)) / np.max(c0)
    e1 = np.max(np.abs(res["c_per_channel"][:, 1] - c1)) / np.max(c0)
    say(f"  C(0) {e0:.2e}  C(1) {e1:.2e}")
    assert e0 < 2e-6 and e1 < 2e-6


@pytest.mark.parametrize("N", [1, 7, 130])
@pytest.mark.parametrize("source,valu", [("rhok", False), ("rhok", True), ("currents", False)])
def test_producers_with_few_atoms(corrmod, source, valu, N):
    """Fewer atoms than one atom tile (1, 7) or one tile and a ragged rest
    (130): a single atom block whose tiles are mostly past the last atom.  With
    one atom |n(k)|^2 / N = 1 for every k (a closed form); otherwise C(0) of
    one push against the oracle's direct double sums."""
    box = 30.0
    kv = np.concatenate([synth.kvectors(96), [[15, -15, 15], [0, 0, -7]]]).astype(np.int32)
    say(f"[few atoms] {source} valu={valu} N={N} nk={len(kv)}")
    x = _currents_inputs(41 + N, N, box, 1)
    nch = len(kv) * (3 if source == "currents" else 1)
    if source == "currents":
        expect = np.abs(oracle.currents(x[0, :3], x[0, 3:], kv, box).reshape(-1)) ** 2 / N
        inp = x
    else:
        expect = np.abs(oracle.rhok(x[0, :3], kv, box)) ** 2 / N
        if N == 1:
            assert np.max(np.abs(expect - 1.0)) < 1e-12
        inp = np.ascontiguousarray(x[:, :3])
    g = corrmod.GroupDesc(nch, 2, 4, 2, dtype="cf32", accum="f64", source=source, kvec=kv,
                          n_atoms=N, box=box)
    with corrmod.Correlator([g], rhok_valu=valu) as c:
        _push_all(c, [inp])
        got = c.finalize(0, slice_=(0, nch))["c_per_channel"][:, 0]
    err = np.max(np.abs(got - expect)) / np.max(expect)
    say(f"  C(0) error {err:.2e}")
    assert err < 2e-6


def test_currents_lag0_against_oracle(corrmod):
    """One push: C(0) of channel 3q+c = |J_c(k_q)|^2 / N with J from the
    oracle's direct double sums, for a k-set spanning |n| up to 15 and
    repeated vectors; a second push checks the phase of C(lag 1)."""
    N, box = 3001, 50.0
    kv = synth.kvectors(120)
    kv = np.concatenate([kv, [[15, -15, 15], [0, 0, -7]], kv[:3]]).astype(np.int32)
    say(f"[currents] N={N} nk={len(kv)}")
    x = _currents_inputs(21, N, box, 2)
    g = corrmod.GroupDesc(3 * len(kv), 3, 8, 2, dtype="cf32", accum="f64", source="currents",
                          kvec=kv, n_atoms=N, box=box)
    with corrmod.Correlator([g]) as c:
        _push_all(c, [x[:1]])
        res = c.finalize(0, slice_=(0, 3 * len(kv)))
        j0 = oracle.currents(x[0, :3], x[0, 3:], kv, box).reshape(-1)
        expect = np.abs(j0) ** 2 / N
        got = res["c_per_channel"][:, 0]
        err = np.max(np.abs(got - expect)) / np.max(expect)
        say(f"  lag-0 error {err:.2e}")
        assert err < 2e-6
        _push_all(c, [x[1:2]])
        res = c.finalize(0, slice_=(0, 3 * len(kv)))
        j1 = oracle.currents(x[1, :3], x[1, 3:], kv, box).reshape(-1)
        expect1 = j1 * np.conj(j0) / N
        got1 = res["c_per_channel"][:, 1]
        assert np.max(np.abs(got1 - expect1)) / np.max(np.abs(expect1)) < 2e-6


@pytest.mark.parametrize("scale", [(1e-3, 1e-3, 1e-3), (1e5, 1e5, 1e5), (1e-3, 1.0, 1e4)])
def test_currents_in_any_velocity_units(corrmod, scale):
    """Velocities far from unit size (e.g. Angstrom/fs, or large units) and
    components of very different size: the producer scales each component by
    a power of two per atom block before the fp16 split, so C(0) and C(1) of
    two pushes keep the precision of unit velocities (against the oracle's
    direct double sums of the same float inputs)."""
    N, box = 2500, 40.0
    kv = synth.kvectors(64)
    say(f"[currents units] velocity scale per component {scale}")
    x = _currents_inputs(31, N, box, 2)
    x[:, 3:] *= np.array(scale, dtype=np.float32)[None, :, None]
    g = corrmod.GroupDesc(3 * len(kv), 3, 8, 2, dtype="cf32", accum="f64", source="currents",
                          kvec=kv, n_atoms=N, box=box)
    with corrmod.Correlator([g]) as c:
        _push_all(c, [x])
        res = c.finalize(0, slice_=(0, 3 * len(kv)))
    v = [oracle.currents(x[s, :3], x[s, 3:], kv, box).reshape(-1) for s in range(2)]
    c0 = (np.abs(v[0]) ** 2 + np.abs(v[1]) ** 2) / 2 / N
    c1 = v[1] * np.conj(v[0]) / N
    assert np.all(np.isfinite(res["c_per_channel"]))
    e0 = np.max(np.abs(res["c_per_channel"][:, 0] - c0)) / np.max(c0)
    e1 = np.max(np.abs(res["c_per_channel"][:, 1] - c1)) / np.max(c0)
    say(f"  C(0) {e0:.2e}  C(1) {e1:.2e}")
    assert e0 < 2e-6 and e1 < 2e-6


@pytest.mark.parametrize("accum", ["kahan", "f64"])
def test_currents_correlator_parity(corrmod, accum):
    """S pushes of moving atoms: the currents group against the oracle
    correlator fed the oracle's currents; times and counts exact, C within the
    tolerance of the accumulator."""
    S, N, box = 200, 1500, 40.0
    kv = synth.kvectors(48)
    x = _currents_inputs(22, N, box, S)
    say(f"[currents parity] S={S} N={N} nk={len(kv)} accum={accum}")
    o = oracle.OracleCorrelator(3 * len(kv), 5, 16, 2, complex_=True)
    for s in range(S):
        o.push(oracle.currents(x[s, :3], x[s, 3:], kv, box).reshape(-1))
    g = corrmod.GroupDesc(3 * len(kv), 5, 16, 2, dtype="cf32", accum=accum, source="currents",
                          kvec=kv, n_atoms=N, box=box)
    with corrmod.Correlator([g]) as c:
        _push_all(c, [x])
        res = c.finalize(0, slice_=(0, 6))
    e = gate(res, o, TOL[("cf32", accum)], scale=1.0 / N, slice_=(0, 6), label="currents")
    say(f"  error {e:.2e}")


def test_currents_with_other_groups_all_launch_modes(corrmod):
    """A currents group next to a k-density group and a velocity group: the
    batched launch, the per-group launches and the graph replay give
    bit-identical state."""
    S, N, box, nv = 130, 1200, 30.0, 3000
    kv = synth.kvectors(40)
    x = _currents_inputs(23, N, box, S)
    xv = ou_inputs(23, 3, nv, S, "f32")
    pos = np.ascontiguousarray(x[:, :3])
    groups = [corrmod.GroupDesc(3 * len(kv), 4, 16, 2, dtype="cf32", accum="kahan",
                                source="currents", kvec=kv, n_atoms=N, box=box),
              corrmod.GroupDesc(len(kv), 4, 16, 2, dtype="cf32", accum="kahan", source="rhok",
                                kvec=kv, n_atoms=N, box=box),
              corrmod.GroupDesc(nv, 6, 16, 2, dtype="f32", accum="kahan")]
    out = {}
    dev = torch.device("cuda:0")
    for mode in ("batched", "per_group", "graph"):
        with corrmod.Correlator(groups, graph=(mode == "graph"),
                                per_group=(mode == "per_group")) as c:
            tx, tp, tv = (torch.from_numpy(a).to(dev) for a in (x, pos, xv))
            if mode == "graph":
                bx, bp, bv = torch.empty_like(tx[0]), torch.empty_like(tp[0]), torch.empty_like(tv[0])
                c.bind_input(0, bx); c.bind_input(1, bp); c.bind_input(2, bv)
                for s in range(S):
                    bx.copy_(tx[s]); bp.copy_(tp[s]); bv.copy_(tv[s])
                    c.push()
            else:
                for s in range(S):
                    c.push([tx[s], tp[s], tv[s]])
            torch.cuda.synchronize()
            out[mode] = [c.finalize(g, slice_=(0, 6)) for g in range(3)]
    for mode in ("per_group", "graph"):
        for g in range(3):
            assert np.array_equal(out[mode][g]["c_per_channel"], out["batched"][g]["c_per_channel"])
    # the longitudinal current with all velocities = khat would be n(k); here
    # check the density group against the oracle instead
    orh = oracle.OracleCorrelator(len(kv), 4, 16, 2, complex_=True)
    for s in range(S):
        orh.push(oracle.rhok(pos[s], kv, box))
    gate(out["batched"][1], orh, TOL[("cf32", "kahan")], scale=1.0 / N, slice_=(0, 6),
         label="rho(k) beside currents")


@pytest.mark.parametrize("dtype,accum,direct", [("cf32", "kahan", False), ("cf32", "kahan", True),
                                                ("f32", "f64", False), ("f64", "f64", False)])
def test_large_window(corrmod, dtype, accum, direct):
    """One block of p = 10240 points (the paper's long single-window
    correlations, p = 10240 with u = 10): parity with the oracle after the
    ring has wrapped, in the block-deferred window form (single-precision
    samples) and the per-step window kernel (direct, or double samples); lag
    times carry u = 10."""
    n, S, p = 16, 10500, 10240
    say(f"[large window] n={n} S={S} p={p} {dtype}/{accum} direct={direct}")
    x = ou_inputs(31, 2, n, S, dtype, tau=200.0, tau_hi=None)
    o = oracle_run(x, 1, p, 2)
    with corrmod.Correlator([corrmod.GroupDesc(n, 1, p, 2, dtype=dtype, accum=accum,
                                               update_every=10, dt=0.001)], direct=direct) as c:
        _push_all(c, [x])
        res = c.finalize(0, slice_=(0, 4))
    t, _, _ = o.readout()
    np.testing.assert_allclose(res["t"], t * 10 * 0.001, rtol=1e-15)
    res["t"] = t  # the oracle reports steps
    e = gate(res, o, TOL[(dtype, accum)], slice_=(0, 4), label="large window")
    say(f"  error {e:.2e}")


def test_limits_of_the_descriptor(corrmod):
    """The largest window (p = 16384, block-deferred window form, past the
    ring's wrap) and the most levels (b = 40) against the oracle; one point
    more of either is refused as unsupported."""
    n, S, p = 8, 16600, 16384
    say(f"[limits] window p={p} S={S}")
    x = ou_inputs(32, 2, n, S, "f32", tau=300.0, tau_hi=None)
    o = oracle_run(x, 1, p, 2)
    with corrmod.Correlator([corrmod.GroupDesc(n, 1, p, 2, dtype="f32", accum="kahan")]) as c:
        _push_all(c, [x])
        res = c.finalize(0, slice_=(0, 3))
    e = gate(res, o, TOL[("f32", "kahan")], slice_=(0, 3), label="p = 16384")
    say(f"  window error {e:.2e}")
    n, S, b = 300, 3000, 40
    say(f"[limits] levels b={b} S={S}")
    x = ou_inputs(33, 2, n, S, "f64", tau=50.0, tau_hi=None)
    o = oracle_run(x, b, 16, 2)
    with corrmod.Correlator([corrmod.GroupDesc(n, b, 16, 2, dtype="f64", accum="f64")]) as c:
        _push_all(c, [x])
        res = c.finalize(0, slice_=(0, 3))
    e = gate(res, o, TOL[("f64", "f64")], slice_=(0, 3), label="b = 40")
    say(f"  levels error {e:.2e}")
    for kw in (dict(points=16385, levels=1), dict(points=16, levels=41)):
        with pytest.raises(corrmod.CorrError) as ei:
            corrmod.Correlator([corrmod.GroupDesc(8, kw["levels"], kw["points"], 2)])
        assert ei.value.code == -5


WINDOW_KINDS = [("cf32", "kahan"), ("cf32", "f64"), ("cf32", "f32"),
                ("f32", "kahan"), ("f32", "f64"), ("f32", "f32")]


@pytest.mark.parametrize("dtype,accum", WINDOW_KINDS)
def test_window_deferred_readouts(corrmod, dtype, accum):
    """One-level windows of p >= 512 points with single-precision samples run
    block-deferred: each push stages its sample and folds one of 64 lag blocks
    of the last complete block of 64 pushes.  Readouts before the first fold,
    at block boundaries, with up to 126 pending pushes, before and after the
    window fills all match the oracle at that push count, and never change
    later results (bitwise against an uninterrupted run).  p = 600 is not a
    multiple of 64 (lag blocks of 10 lags, the last four empty); 300 channels
    leave a ragged tile."""
    n, p = 300, 600
    marks = [1, 2, 63, 64, 65, 127, 128, 129, 190, 599, 600, 601, 700, 777, 1400]
    S = marks[-1]
    say(f"[window deferred readouts] {dtype}/{accum} n={n} p={p}")
    x = ou_inputs(41, 3, n, S, dtype, tau=50.0, tau_hi=None)
    cplx = np.iscomplexobj(x)
    o = oracle.OracleCorrelator(n, 1, p, 2, complex_=cplx)
    dev = torch.device("cuda:0")
    tx = torch.from_numpy(x).to(dev)
    g = [corrmod.GroupDesc(n, 1, p, 2, dtype=dtype, accum=accum)]
    with corrmod.Correlator(g) as c, corrmod.Correlator(g) as ref:
        done = 0
        for mk in marks:
            for s in range(done, mk):
                c.push([tx[s]])
                ref.push([tx[s]])
                o.push(x[s].astype(np.complex128 if cplx else np.float64))
            done = mk
            res = c.finalize(0, slice_=(n - 3, n))
            gate(res, o, TOL[(dtype, accum)], slice_=(n - 3, n), label=f"S={mk}")
        a, r = c.finalize(0, slice_=(0, n)), ref.finalize(0, slice_=(0, n))
        assert np.array_equal(a["c"], r["c"])
        assert np.array_equal(a["c_per_channel"], r["c_per_channel"])


def test_window_folds_sharing_launches(corrmod):
    """Four block-deferred windows in one context: two of one kind and
    length (their folds share a launch, the second's channel blocks after the
    first's), one of another length and one of another kind (launched alone).
    The shared launches give the same state bit for bit as one launch per
    window (the per-group form), and every window matches the oracle."""
    S = 700
    specs = [(300, 512, "f32", "kahan"), (700, 512, "f32", "kahan"), (200, 576, "f32", "kahan"),
             (100, 512, "cf32", "kahan")]
    say(f"[windows sharing launches] {[sp[:2] for sp in specs]}")
    xs = [ou_inputs(47, 20 + i, n, S, dt, tau=50.0, tau_hi=None) for i, (n, p, dt, acc) in enumerate(specs)]
    groups = [corrmod.GroupDesc(n, 1, p, 2, dtype=dt, accum=acc) for (n, p, dt, acc) in specs]
    dev = torch.device("cuda:0")
    out = {}
    for per_group in (False, True):
        with corrmod.Correlator(groups, per_group=per_group) as c:
            _push_all(c, xs)
            out[per_group] = [c.finalize(i, slice_=(0, sp[0])) for i, sp in enumerate(specs)]
    for i in range(len(specs)):
        assert np.array_equal(out[True][i]["c_per_channel"], out[False][i]["c_per_channel"]), i
        assert np.array_equal(out[True][i]["c"], out[False][i]["c"]), i
    for i, (n, p, dt, acc) in enumerate(specs):
        cplx = np.iscomplexobj(xs[i])
        o = oracle.OracleCorrelator(n, 1, p, 2, complex_=cplx)
        for s in range(S):
            o.push(xs[i][s].astype(np.complex128 if cplx else np.float64))
        res = dict(out[False][i], c_per_channel=out[False][i]["c_per_channel"][n - 3:n])
        gate(res, o, TOL[(dt, acc)], slice_=(n - 3, n), label=f"window {i}")


@pytest.mark.parametrize("dtype", ["f32", "cf32"])
def test_window_deferred_equals_direct(corrmod, dtype):
    """The block-deferred window regroups the sums of the per-step window
    kernel: with FP64 sums of exact single-precision products the two agree to
    rounding, per channel and for the group mean."""
    n, S, p = 1000, 1500, 1024
    say(f"[window deferred vs direct] {dtype}")
    x = ou_inputs(42, 5, n, S, dtype, tau=80.0, tau_hi=None)
    g = [corrmod.GroupDesc(n, 1, p, 2, dtype=dtype, accum="f64")]
    with corrmod.Correlator(g) as d, corrmod.Correlator(g, direct=True) as e:
        _push_all(d, [x])
        _push_all(e, [x])
        rd, re_ = d.finalize(0, slice_=(0, 40)), e.finalize(0, slice_=(0, 40))
    assert np.array_equal(rd["count"], re_["count"])
    assert np.max(np.abs(rd["c"] - re_["c"])) <= 1e-12 * abs(re_["c"][0])
    scale = np.abs(re_["c_per_channel"][:, :1])
    assert np.max(np.abs(rd["c_per_channel"] - re_["c_per_channel"]) / scale) <= 1e-12


def test_window_deferred_fed_by_producer_all_launch_modes(corrmod):
    """A long window fed by the k-density producer (staged after the
    producer), next to a block-deferred group and a per-step group: batched,
    per-group, graph and overlapped-producer launches give bit-identical window
    results, which match the oracle."""
    S, N, box, p = 700, 1000, 30.0, 512
    kv = synth.kvectors(48)
    xv = ou_inputs(44, 1, 1500, S, "f32")
    xg = ou_inputs(44, 2, 9, S, "f64")
    pos, _ = synth.PositionSpec(44, 3, N, box).series(0, S)
    groups = [corrmod.GroupDesc(1500, 5, 16, 2, dtype="f32", accum="kahan"),
              corrmod.GroupDesc(9, 6, 16, 2, dtype="f64", accum="f64"),
              corrmod.GroupDesc(len(kv), 1, p, 2, dtype="cf32", accum="kahan", source="rhok",
                                kvec=kv, n_atoms=N, box=box)]
    dev = torch.device("cuda:0")
    out = {}
    for mode in ("batched", "per_group", "graph", "overlap", "overlap2"):
        say(f"[window fed by producer] mode={mode}")
        tuning = {"overlap": {"overlap_producers": 1},
                  "overlap2": {"overlap_producers": 2}}.get(mode)
        with corrmod.Correlator(groups, graph=(mode == "graph"), per_group=(mode == "per_group"),
                                tuning=tuning) as c:
            ta, tb, tc = (torch.from_numpy(a).to(dev) for a in (xv, xg, pos))
            if mode == "graph":
                ba, bb, bc = torch.empty_like(ta[0]), torch.empty_like(tb[0]), torch.empty_like(tc[0])
                c.bind_input(0, ba); c.bind_input(1, bb); c.bind_input(2, bc)
                for s in range(S):
                    ba.copy_(ta[s]); bb.copy_(tb[s]); bc.copy_(tc[s])
                    c.push()
            else:
                for s in range(S):
                    c.push([ta[s], tb[s], tc[s]])
            torch.cuda.synchronize()
            out[mode] = c.finalize(2, slice_=(0, 4))
    for mode in ("per_group", "graph", "overlap", "overlap2"):
        assert np.array_equal(out[mode]["c_per_channel"], out["batched"]["c_per_channel"]), mode
        assert np.array_equal(out[mode]["c"], out["batched"]["c"]), mode
    o = oracle.OracleCorrelator(len(kv), 1, p, 2, complex_=True)
    for s in range(S):
        o.push(oracle.rhok(pos[s], kv, box))
    gate(out["batched"], o, TOL[("cf32", "kahan")], scale=1.0 / N, slice_=(0, 4),
         label="window fed by rho(k)")


def test_two_producer_groups_all_launch_modes(corrmod):
    """Producer groups only (currents and n(k) of the same atoms, long windows
    and a multi-level group): one stream, the forked order (which keeps
    producer-only contexts on one stream), per-group launches and a graph give
    bit-identical results, which match the oracle."""
    S, N, box = 600, 1200, 30.0
    kv = synth.kvectors(40)
    x = _currents_inputs(45, N, box, S)  # [S][6][N]: positions, velocities
    pos = np.ascontiguousarray(x[:, :3])
    groups = [corrmod.GroupDesc(3 * len(kv), 1, 512, 2, dtype="cf32", accum="kahan",
                                source="currents", kvec=kv, n_atoms=N, box=box),
              corrmod.GroupDesc(len(kv), 1, 512, 2, dtype="cf32", accum="kahan", source="rhok",
                                kvec=kv, n_atoms=N, box=box),
              corrmod.GroupDesc(len(kv), 5, 16, 2, dtype="cf32", accum="f64", source="rhok",
                                kvec=kv, n_atoms=N, box=box)]
    base = dict(tile_channels=256, chans_per_thread=1, lag_chunk=8, grid_blocks=0)
    dev = torch.device("cuda:0")
    out = {}
    for mode in ("serial", "forked", "per_group", "forked_graph"):
        say(f"[two producers] mode={mode}")
        ov = 1 if mode.startswith("forked") else 0
        with corrmod.Correlator(groups, graph=(mode == "forked_graph"),
                                per_group=(mode == "per_group"),
                                tuning=dict(base, overlap_producers=ov)) as c:
            ta, tb = torch.from_numpy(x).to(dev), torch.from_numpy(pos).to(dev)
            if mode == "forked_graph":
                ba, bb, bc = torch.empty_like(ta[0]), torch.empty_like(tb[0]), torch.empty_like(tb[0])
                c.bind_input(0, ba); c.bind_input(1, bb); c.bind_input(2, bc)
                for s in range(S):
                    ba.copy_(ta[s]); bb.copy_(tb[s]); bc.copy_(tb[s])
                    c.push()
            else:
                for s in range(S):
                    c.push([ta[s], tb[s], tb[s]])
            torch.cuda.synchronize()
            out[mode] = [c.finalize(g, slice_=(0, 4)) for g in range(3)]
    for mode in ("forked", "per_group", "forked_graph"):
        for g in range(3):
            assert np.array_equal(out[mode][g]["c_per_channel"], out["serial"][g]["c_per_channel"]), (mode, g)
            assert np.array_equal(out[mode][g]["c"], out["serial"][g]["c"]), (mode, g)
    oc = oracle.OracleCorrelator(3 * len(kv), 1, 512, 2, complex_=True)
    orw = oracle.OracleCorrelator(len(kv), 1, 512, 2, complex_=True)
    orl = oracle.OracleCorrelator(len(kv), 5, 16, 2, complex_=True)
    for s in range(S):
        oc.push(oracle.currents(x[s, :3], x[s, 3:], kv, box).reshape(-1))
        r = oracle.rhok(x[s, :3], kv, box)
        orw.push(r)
        orl.push(r)
    gate(out["serial"][0], oc, TOL[("cf32", "kahan")], scale=1.0 / N, slice_=(0, 4), label="currents")
    gate(out["serial"][1], orw, TOL[("cf32", "kahan")], scale=1.0 / N, slice_=(0, 4), label="n(k) window")
    gate(out["serial"][2], orl, TOL[("cf32", "f64")], scale=1.0 / N, slice_=(0, 4), label="n(k)")


def _pair_inputs(seed, n, S, dtype):
    """x: OU series; y: 0.6 x + an independent OU series (cross-correlated)."""
    x = ou_inputs(seed, 11, n, S, dtype)
    z = ou_inputs(seed, 12, n, S, dtype)
    y = (0.6 * x + z).astype(x.dtype)
    return x, y


@pytest.mark.parametrize("dtype,accum,b,p,m", [
    ("f32", "kahan", 6, 16, 2), ("f32", "f64", 5, 16, 2), ("f64", "f64", 4, 9, 3),
    ("cf32", "kahan", 5, 16, 2), ("cf64", "f64", 4, 8, 2), ("f32", "kahan", 1, 1024, 2)])
def test_pair_parity(corrmod, dtype, accum, b, p, m):
    """Pair groups, C(L) = <x(s) conj(y(s - L))>, against the oracle's pair
    form: times and counts exact, values within the accumulator's tolerance.
    The last case is a one-level window of 1024 points (window kernel)."""
    n, S = 700, 1500
    say(f"[pair] {dtype}/{accum} b={b} p={p} m={m}")
    x, y = _pair_inputs(41, n, S, dtype)
    o = oracle.OracleCorrelator(n, b, p, m, complex_=np.iscomplexobj(x))
    for s in range(S):
        o.push_pair(x[s], y[s])
    xy = np.ascontiguousarray(np.stack([x, y], axis=1))  # [S][2][n]
    with corrmod.Correlator([corrmod.GroupDesc(n, b, p, m, dtype=dtype, accum=accum,
                                               pair=True)]) as c:
        _push_all(c, [xy])
        res = c.finalize(0, slice_=(0, 5))
    e = gate(res, o, TOL[(dtype, accum)], slice_=(0, 5), label="pair")
    say(f"  error {e:.2e}")


def test_pair_with_itself_equals_direct_autocorrelation(corrmod):
    """pair(x, x) and the per-step autocorrelation of x: identical arithmetic,
    bit-identical state."""
    n, S = 900, 700
    x = ou_inputs(42, 1, n, S, "cf32")
    xx = np.ascontiguousarray(np.stack([x, x], axis=1))
    with corrmod.Correlator([corrmod.GroupDesc(n, 5, 16, 2, dtype="cf32", accum="kahan",
                                               pair=True),
                             corrmod.GroupDesc(n, 5, 16, 2, dtype="cf32", accum="kahan")],
                            direct=True) as c:
        _push_all(c, [xx, x])
        a, b = c.finalize(0, slice_=(0, n)), c.finalize(1, slice_=(0, n))
    assert np.array_equal(a["c_per_channel"], b["c_per_channel"])
    assert np.array_equal(a["count"], b["count"])


def test_pair_group_in_all_launch_modes(corrmod):
    """A pair group next to a block-deferred group and a k-density group:
    batched, per-group and graph launches give bit-identical pair results,
    and they match the oracle."""
    n, S, N, box = 500, 300, 1000, 30.0
    kv = synth.kvectors(32)
    x, y = _pair_inputs(43, n, S, "f32")
    xy = np.ascontiguousarray(np.stack([x, y], axis=1))
    xv = ou_inputs(43, 3, 2000, S, "f32")
    pos, _ = synth.PositionSpec(43, 1, N, box).series(0, S)
    groups = [corrmod.GroupDesc(n, 5, 16, 2, dtype="f32", accum="kahan", pair=True),
              corrmod.GroupDesc(2000, 5, 16, 2, dtype="f32", accum="kahan"),
              corrmod.GroupDesc(len(kv), 4, 16, 2, dtype="cf32", accum="f64", source="rhok",
                                kvec=kv, n_atoms=N, box=box)]
    out = {}
    dev = torch.device("cuda:0")
    for mode in ("batched", "per_group", "graph"):
        with corrmod.Correlator(groups, graph=(mode == "graph"),
                                per_group=(mode == "per_group")) as c:
            ta, tb, tc = (torch.from_numpy(a).to(dev) for a in (xy, xv, pos))
            if mode == "graph":
                ba, bb, bc = torch.empty_like(ta[0]), torch.empty_like(tb[0]), torch.empty_like(tc[0])
                c.bind_input(0, ba); c.bind_input(1, bb); c.bind_input(2, bc)
                for s in range(S):
                    ba.copy_(ta[s]); bb.copy_(tb[s]); bc.copy_(tc[s])
                    c.push()
            else:
                for s in range(S):
                    c.push([ta[s], tb[s], tc[s]])
            torch.cuda.synchronize()
            out[mode] = c.finalize(0, slice_=(0, 5))
    for mode in ("per_group", "graph"):
        assert np.array_equal(out[mode]["c_per_channel"], out["batched"]["c_per_channel"])
    o = oracle.OracleCorrelator(n, 5, 16, 2)
    for s in range(S):
        o.push_pair(x[s], y[s])
    gate(out["batched"], o, TOL[("f32", "kahan")], slice_=(0, 5), label="pair in mix")


def test_push_steps_equals_single_pushes(corrmod):
    """corr_push_steps replays a stored history: the same state, bit for bit,
    as one push per step -- for block-deferred, per-step, pair, k-density and
    long-window groups in one context, across flush boundaries (three whole
    256-push blocks inside one replay), with a readout between two replays --
    and both against the oracle fed the same series."""
    S, nv, N, box = 900, 3000, 800, 25.0
    kv = synth.kvectors(24)
    xv = ou_inputs(51, 1, nv, S, "f32")
    xg = ou_inputs(51, 2, 9, S, "f64")
    x, y = _pair_inputs(51, 300, S, "f32")
    xy = np.ascontiguousarray(np.stack([x, y], axis=1))
    pos, _ = synth.PositionSpec(51, 3, N, box).series(0, S)
    xw = ou_inputs(51, 4, 200, S, "cf32")
    groups = [corrmod.GroupDesc(nv, 6, 16, 2, dtype="f32", accum="kahan"),
              corrmod.GroupDesc(9, 8, 16, 2, dtype="f64", accum="f64"),
              corrmod.GroupDesc(300, 5, 16, 2, dtype="f32", accum="kahan", pair=True),
              corrmod.GroupDesc(len(kv), 4, 16, 2, dtype="cf32", accum="kahan", source="rhok",
                                kvec=kv, n_atoms=N, box=box),
              corrmod.GroupDesc(200, 1, 640, 2, dtype="cf32", accum="kahan")]
    dev = torch.device("cuda:0")
    hs = [torch.from_numpy(a).to(dev) for a in (xv, xg, xy, pos, xw)]
    with corrmod.Correlator(groups) as a, corrmod.Correlator(groups) as b:
        for s in range(S):
            a.push([h[s] for h in hs])
        b.push_steps([h[:77] for h in hs])
        mid = [b.finalize(g, slice_=(0, 3)) for g in range(5)]
        b.push_steps([h[77:] for h in hs])
        torch.cuda.synchronize()
        assert a.n_pushes() == b.n_pushes() == S
        res = []
        for g in range(5):
            ra, rb = a.finalize(g, slice_=(0, 3)), b.finalize(g, slice_=(0, 3))
            assert np.array_equal(ra["c"], rb["c"]), g
            assert np.array_equal(ra["c_per_channel"], rb["c_per_channel"]), g
            res.append(rb)
        assert len(mid[0]["t"]) > 0
        short = torch.zeros((2, 10), dtype=torch.float32, device=dev)  # rows below 3N floats
        with pytest.raises(corrmod.CorrError):
            b.push_steps([hs[0][:2], hs[1][:2], hs[2][:2], short, hs[4][:2]])
        assert b.n_pushes() == S  # rejected before anything was issued
    # the replayed state against the oracle
    gate(res[0], oracle_run(xv, 6, 16, 2), TOL[("f32", "kahan")], slice_=(0, 3), label="deferred")
    gate(res[1], oracle_run(xg, 8, 16, 2), TOL[("f64", "f64")], slice_=(0, 3), label="FP64")
    o = oracle.OracleCorrelator(300, 5, 16, 2)
    for s in range(S):
        o.push_pair(x[s], y[s])
    gate(res[2], o, TOL[("f32", "kahan")], slice_=(0, 3), label="pair")
    o = oracle.OracleCorrelator(len(kv), 4, 16, 2, complex_=True)
    for s in range(S):
        o.push(oracle.rhok(pos[s], kv, box))
    gate(res[3], o, TOL[("cf32", "kahan")], scale=1.0 / N, slice_=(0, 3), label="n(k)")
    gate(res[4], oracle_run(xw, 1, 640, 2), TOL[("cf32", "kahan")], slice_=(0, 3), label="window")


@pytest.mark.parametrize("fold_block", [128, 256])
def test_fold_block_lengths_against_oracle(corrmod, fold_block):
    """The block-deferred form with 128- and 256-push blocks (tuning
    fold_block): compensated and FP64 sums against the oracle at readouts on
    both sides of block boundaries, and a replay that folds whole blocks from
    the history bit for bit equal to single pushes."""
    S, n = 3 * fold_block + 37, 2500
    x = ou_inputs(61, 1, n, S, "f32")
    dev = torch.device("cuda:0")
    hx = torch.from_numpy(x).to(dev)
    say(f"[fold block {fold_block}] n={n} S={S}")
    tn = dict(tile_channels=256, chans_per_thread=1, lag_chunk=8, grid_blocks=0,
              fold_block=fold_block)
    groups = [corrmod.GroupDesc(n, 7, 16, 2, dtype="f32", accum="kahan"),
              corrmod.GroupDesc(n, 7, 16, 2, dtype="f32", accum="f64")]
    o = oracle.OracleCorrelator(n, 7, 16, 2)
    with corrmod.Correlator(groups, tuning=tn) as a, corrmod.Correlator(groups, tuning=tn) as b:
        assert a.group_form(0) == (1, fold_block)
        done = 0
        for stop in (fold_block - 1, fold_block, fold_block + 1, 2 * fold_block + 5, S):
            for s in range(done, stop):
                a.push([hx[s], hx[s]])
            o.push_series(x[done:stop])
            done = stop
            for g, accum in ((0, "kahan"), (1, "f64")):
                gate(a.finalize(g, slice_=(0, 3)), o, TOL[("f32", accum)], slice_=(0, 3),
                     label=f"T={fold_block} {accum} at {stop}")
        b.push_steps([hx[:29], hx[:29]])
        b.push_steps([hx[29:], hx[29:]])  # crosses whole blocks: folded from the history
        torch.cuda.synchronize()
        for g in (0, 1):
            ra, rb = a.finalize(g, slice_=(n - 3, n)), b.finalize(g, slice_=(n - 3, n))
            assert np.array_equal(ra["c"], rb["c"]) and np.array_equal(ra["c_per_channel"],
                                                                        rb["c_per_channel"])


def test_fold_threads_bitwise(corrmod):
    """Threads per block of the scheduled fold (64, 128, 256) change only the
    launch shape: identical results bit for bit."""
    S, n = 600, 3000
    x = ou_inputs(62, 1, n, S, "f32")
    out = {}
    for nt in (64, 128, 256):
        tn = dict(tile_channels=512, chans_per_thread=2, lag_chunk=8, grid_blocks=0,
                  fold_threads=nt)
        with corrmod.Correlator([corrmod.GroupDesc(n, 6, 16, 2, dtype="f32", accum="kahan")],
                                tuning=tn) as c:
            assert c.tuning()["fold_threads"] == nt
            _push_all(c, [x])
            out[nt] = c.finalize(0, slice_=(0, n))["c_per_channel"]
    assert np.array_equal(out[64], out[128]) and np.array_equal(out[256], out[128])


def test_chained_runs_of_any_length(corrmod):
    """Captured corr_push_steps runs with the producers forked beside a
    block-deferred group (the two streams joined every few pushes, each
    ending its pushes with its own counter): runs of 1, 3, 4, 5, 8, 255 and 257
    pushes, across the first fold blocks, give the state of single pushes bit
    for bit, with a readout of every group after every run, and the oracle's
    result at the end."""
    lengths = [1, 3, 4, 5, 8, 255, 257]
    S, nv, N, box = sum(lengths), 2048, 1500, 40.0
    kv = synth.kvectors(40)
    xv = ou_inputs(71, 1, nv, S, "f32")
    xg = ou_inputs(71, 2, 9, S, "f64")
    pos, _ = synth.PositionSpec(71, 3, N, box).series(0, S)
    say(f"[chained runs] S={S} lengths={lengths}")
    groups = [corrmod.GroupDesc(nv, 6, 16, 2, dtype="f32", accum="kahan"),
              corrmod.GroupDesc(len(kv), 5, 16, 2, dtype="cf32", accum="kahan", source="rhok",
                                kvec=kv, n_atoms=N, box=box),
              corrmod.GroupDesc(9, 8, 16, 2, dtype="f64", accum="f64")]
    dev = torch.device("cuda:0")
    hs = [torch.from_numpy(a).to(dev) for a in (xv, pos, xg)]
    tune = {"overlap_producers": 1}
    with corrmod.Correlator(groups, tuning=tune) as a, \
            corrmod.Correlator(groups, graph=True, tuning=tune) as b:
        s0 = 0
        for n in lengths:
            for s in range(s0, s0 + n):
                a.push([h[s] for h in hs])
            b.push_steps([h[s0:s0 + n] for h in hs])
            s0 += n
            torch.cuda.synchronize()
            assert a.n_pushes() == b.n_pushes() == s0
            for g in range(3):
                ra, rb = a.finalize(g, slice_=(0, 3)), b.finalize(g, slice_=(0, 3))
                assert np.array_equal(ra["t"], rb["t"]) and np.array_equal(ra["count"], rb["count"])
                assert np.array_equal(ra["c_per_channel"], rb["c_per_channel"]), (n, g)
        gate(b.finalize(0, slice_=(0, 3)), oracle_run(xv, 6, 16, 2), TOL[("f32", "kahan")],
             slice_=(0, 3), label="velocity")
        gate(b.finalize(2, slice_=(0, 3)), oracle_run(xg, 8, 16, 2), TOL[("f64", "f64")],
             slice_=(0, 3), label="global")


def test_graph_replay_equals_single_pushes(corrmod):
    """Graph mode: corr_push_steps captures its pushes once and replays the
    graph for later calls with the same histories -- the same state bit for
    bit as single pushes, for block-deferred, FP64, n(k) and window groups,
    with readouts between replays."""
    S, nv, N, box, chunk = 4 * 150, 3000, 600, 20.0, 150
    kv = synth.kvectors(16)
    xv = ou_inputs(63, 1, nv, S, "f32")
    xg = ou_inputs(63, 2, 9, S, "f64")
    pos, _ = synth.PositionSpec(63, 3, N, box).series(0, S)
    xw = ou_inputs(63, 4, 100, S, "f32")
    groups = [corrmod.GroupDesc(nv, 6, 16, 2, dtype="f32", accum="kahan"),
              corrmod.GroupDesc(9, 8, 16, 2, dtype="f64", accum="f64"),
              corrmod.GroupDesc(len(kv), 4, 16, 2, dtype="cf32", accum="kahan", source="rhok",
                                kvec=kv, n_atoms=N, box=box),
              corrmod.GroupDesc(100, 1, 600, 2, dtype="f32", accum="f64")]
    dev = torch.device("cuda:0")
    hs = [torch.from_numpy(a).to(dev) for a in (xv, xg, pos, xw)]
    bufs = [torch.empty((chunk,) + tuple(h.shape[1:]), dtype=h.dtype, device=dev) for h in hs]
    with corrmod.Correlator(groups) as a, corrmod.Correlator(groups, graph=True) as b:
        for s0 in range(0, S, chunk):
            for buf, h in zip(bufs, hs):
                buf.copy_(h[s0:s0 + chunk])  # the same buffers every call: one capture
            for s in range(s0, s0 + chunk):
                a.push([h[s] for h in hs])
            b.push_steps(bufs)
            torch.cuda.synchronize()
            for g in range(4):
                ra, rb = a.finalize(g, slice_=(0, 3)), b.finalize(g, slice_=(0, 3))
                assert np.array_equal(ra["c_per_channel"], rb["c_per_channel"]), (s0, g)
        assert a.n_pushes() == b.n_pushes() == S
    gate(rb, oracle_run(xw, 1, 600, 2), TOL[("f32", "f64")], slice_=(0, 3), label="window")


def test_state_that_fits_only_with_the_shorter_block(corrmod):
    """A block-deferred group too large for 256-push blocks in the device's
    free memory (3648 B per channel) but not for 128-push blocks (2624 B): the
    library takes T = 128 by itself; sampled channels against the oracle."""
    free, total = torch.cuda.mem_get_info()
    n = int(0.80 * free / 2624) // 1024 * 1024
    assert n * 3648 > free  # the longer block could not fit
    S, chunk = 300, 20
    say(f"[fit] free {free / 1e9:.1f} GB: {n} channels, b=12, compensated")
    spec = synth.OUSpec.make(seed=64, stream=1, n=n, comps=3, tau=20, tau_hi=200)
    gen = synth.GpuOU(spec)
    buf = torch.empty((chunk, n), dtype=torch.float32, device="cuda")
    with corrmod.Correlator([corrmod.GroupDesc(n, 12, 16, 2, dtype="f32", accum="kahan")]) as c:
        assert c.group_form(0) == (1, 128)
        say(f"  state {c.state_bytes(0) / 1e9:.1f} GB")
        for _ in range(0, S, chunk):
            gen.fill(buf, chunk)
            c.push_steps([buf])
        torch.cuda.synchronize()
        ranges = [(0, 2), (n // 2, n // 2 + 2), (n - 2, n)]
        res = [c.finalize(0, slice_=r) for r in ranges]
    del buf
    torch.cuda.empty_cache()
    chans = np.concatenate([np.arange(lo, hi) for lo, hi in ranges])
    xs, _ = spec.series(0, S, channels=chans)
    o = oracle.OracleCorrelator(len(chans), 12, 16, 2)
    o.push_series(xs)
    i = 0
    for r, (lo, hi) in zip(res, ranges):
        for j in range(hi - lo):
            t, cc, cnt = o.readout(i, i + 1)
            assert np.array_equal(r["t"], t) and np.array_equal(r["count"], cnt)
            err = np.max(np.abs(r["c_per_channel"][j] - cc)) / abs(cc[0])
            assert err <= TOL[("f32", "kahan")], (lo + j, err)
            i += 1
