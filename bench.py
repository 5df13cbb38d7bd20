#!/usr/bin/env python3
"""Throughput benchmark of the on-the-fly multiple-tau correlator on one MI355X.

One "step" is one push: every channel of every group receives one sample and
is updated (Algorithm 1 of the paper's Appendix D with block index 1), plus
the k-space density producer for k-density groups.  Inputs are synthetic
(seeded Ornstein-Uhlenbeck series and atom positions, see synth/) generated on
the GPU into HBM in chunks *before* each timed chunk, so every timed push
reads inputs already resident in HBM.  The timed region is the sum of the
chunks' push intervals, each bracketed by torch.cuda.synchronize().

Workloads (--config):
  plain    3x10^6 FP32 channels, FP64 sums, 12 levels x 16 points, m=2, one
           group, one kernel launch per push (the plain per-group form)
  batched  3x10^7 FP32 channels with compensated FP32 sums (10 levels x 16),
           n(k) of 2048 k-vectors from 10^6 atoms (complex FP32, compensated,
           16 levels x 32), 9 FP64 global channels (20 levels x 16); one
           batched push kernel per step (default)
  large    6x10^7 FP32 channels with compensated FP32 sums + 9 FP64 channels,
           12 levels x 16 points
  rhok     the k-density group of `batched` alone (2048 k-vectors, 10^6 atoms):
           the producer kernel's own roofline line
  currents longitudinal and transverse currents of the same 2048 k-vectors and
           10^6 atoms (6144 complex channels), the current producer's line
  kgap     the long single-window form: currents and n(k) of the same k-vectors
           and atoms, one block of 10240 points updated every 10 MD steps
           (8192 complex channels, block-deferred window); the producers
           dominate, and the window update is reported beside them
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
MFMA_F16_PEAK_TFS = 2500.0  # MI355X dense fp16 matrix peak
VALU_F32_PEAK_TFS = 157.3   # MI355X fp32 vector peak
RHOK_FLOP_PER_ATOM_K = 14  # factorised phases: 2 complex multiplies + 1 complex add
# currents: the phase as for n(k) plus, per velocity component, a real x complex
# multiply-add (4 flop)
CURRENTS_FLOP_PER_ATOM_K = RHOK_FLOP_PER_ATOM_K + 3 * 4
PRODUCER_KINDS = ("rhok", "currents", "momentum")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--config", default="batched",
                    choices=["plain", "batched", "large", "rhok", "currents", "kgap", "massflux",
                             "precision"])
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the launch-shape autotuner (library defaults)")
    ap.add_argument("--precision-steps", type=int, default=1_000_000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy 8 times (reference for "
                         "the rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--chunk", type=int, default=None,
                    help="pushes per generated input chunk (default 128; with --replay 256, one "
                         "fold block)")
    ap.add_argument("--replay", action="store_true",
                    help="push each generated chunk with one corr_push_steps call (a stored "
                         "history replayed) instead of one corr_push per step")
    ap.add_argument("--mode", default=None, choices=["batched", "per_group"],
                    help="launch form (default: per_group for plain, batched otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare-plain", action="store_true",
                    help="skip the bounded leg that times the plain FP64 per-group form on the "
                         "largest sample-fed group (run by default)")
    ap.add_argument("--eager", action="store_true",
                    help="time every workload eagerly (one corr_push per step); by default "
                         "block-deferred workloads are timed as captured HIP graphs per chunk of "
                         "pushes")
    ap.add_argument("--no-mode-leg", action="store_true",
                    help="skip the leg that times the other issue form (eager beside a graph "
                         "headline, graphs beside an eager one)")
    ap.add_argument("--plain-steps", type=int, default=64,
                    help="timed pushes of the plain-form leg (after %d fill pushes)" % 256)
    ap.add_argument("--tuning", default=None, help="JSON dict of corr_tuning fields")
    ap.add_argument("--timing-stride", type=int, default=7,
                    help="record the HIP timing events on one push in this many (each event pair "
                         "costs a few microseconds of the push it brackets); odd, so that the "
                         "timed pushes cycle through every level schedule (m^k | s) and flush group")
    ap.add_argument("--direct", action="store_true",
                    help="per-step update of every channel (no block-deferred form)")
    ap.add_argument("--rhok-valu", action="store_true",
                    help="k-density producer on the vector units instead of the matrix cores")
    ap.add_argument("--overlap", type=int, choices=[0, 1, 2], default=None,
                    help="issue order instead of the autotuner's choice: 0 one stream, 1 producers "
                         "forked, 2 per-step updates forked beside the flush")
    return ap.parse_args()


# ------------------------------------------------------------------ workloads
def workload(name):
    import synth
    if name == "plain":
        return dict(
            name=("plain: 3e6 FP32 channels (1e6 atoms), FP64 sums, b=12 p=16 m=2, per-step update, "
                  "per-group launch"),
            steps=10_000, direct=True,
            groups=[dict(kind="ou", n=3_000_000, levels=12, points=16, m=2, dtype="f32",
                         accum="f64", comps=3, tau=(20, 200), sigma=1.0, seed=1, stream=1)])
    if name == "batched":
        return dict(
            name=("batched: 3e7 FP32 channels compensated b=10 p=16 + rho(k) 2048 k from 1e6 atoms "
                  "cFP32 compensated b=16 p=32 + 9 FP64 channels b=20 p=16, m=2, one batched launch"),
            steps=10_000,
            groups=[dict(kind="ou", n=30_000_000, levels=10, points=16, m=2, dtype="f32",
                         accum="kahan", comps=3, tau=(20, 200), sigma=1.0, seed=3, stream=1),
                    dict(kind="rhok", n=2048, levels=16, points=32, m=2, dtype="cf32",
                         accum="kahan", n_atoms=1_000_000, box=100.0, seed=3, stream=3,
                         kvec=synth.kvectors(2048)),
                    dict(kind="ou", n=9, levels=20, points=16, m=2, dtype="f64", accum="f64",
                         comps=1, tau=(100, 100), sigma=1.0, seed=3, stream=2)])
    if name == "large":
        return dict(
            name=("large: 6e7 FP32 channels (2e7 atoms, tau 10..1000) compensated b=12 p=16 + "
                  "9 FP64 channels b=12, m=2, one batched launch"),
            steps=50_000,
            groups=[dict(kind="ou", n=60_000_000, levels=12, points=16, m=2, dtype="f32",
                         accum="kahan", comps=3, tau=(10, 1000), sigma=1.0, seed=4, stream=1),
                    dict(kind="ou", n=9, levels=12, points=16, m=2, dtype="f64", accum="f64",
                         comps=1, tau=(100, 100), sigma=1.0, seed=4, stream=2)])
    if name == "rhok":
        return dict(
            name="rhok: n(k) of 2048 k-vectors (|n| <= 12 half-space) from 1e6 atoms in a box of 100, "
                 "cFP32 compensated b=16 p=32 m=2",
            steps=10_000,
            groups=[dict(kind="rhok", n=2048, levels=16, points=32, m=2, dtype="cf32",
                         accum="kahan", n_atoms=1_000_000, box=100.0, seed=3, stream=3,
                         kvec=synth.kvectors(2048))])
    if name == "currents":
        return dict(
            name="currents: j_L and j_T of 2048 k-vectors (|n| <= 12 half-space) from 1e6 atoms in "
                 "a box of 100 with OU velocities (tau 20..200), 6144 cFP32 channels compensated "
                 "b=16 p=32 m=2",
            steps=10_000,
            groups=[dict(kind="currents", n=3 * 2048, levels=16, points=32, m=2, dtype="cf32",
                         accum="kahan", n_atoms=1_000_000, box=100.0, seed=5, stream=3,
                         vtau=(20, 200), kvec=synth.kvectors(2048))])
    if name == "kgap":
        kv = synth.kvectors(2048)
        return dict(
            name="kgap: j_L, j_T and n(k) of 2048 k-vectors from 1e6 atoms, one window of p=10240 "
                 "points (b=1), u=10, 8192 cFP32 channels compensated",
            steps=1024, warmup=10240, dominant="producer",  # timed once the window is full
            groups=[dict(kind="currents", n=3 * 2048, levels=1, points=10240, m=2, dtype="cf32",
                         accum="kahan", n_atoms=1_000_000, box=100.0, seed=6, stream=3,
                         vtau=(20, 200), kvec=kv, update_every=10),
                    dict(kind="rhok", n=2048, levels=1, points=10240, m=2, dtype="cf32",
                         accum="kahan", n_atoms=1_000_000, box=100.0, seed=6, stream=3, kvec=kv,
                         update_every=10, shares_positions=True)])
    if name == "massflux":
        return dict(
            name=("massflux: partial momentum densities of 2 species (masses 6.941 and 18.998, "
                  "half the atoms each) from 2e7 atoms with OU velocities in a box of 600, "
                  "correlated with a 3-component heat-flux series (<q(s) j(s-L)>, 6 FP32 pair "
                  "channels) + the heat-flux autocorrelation (3 FP32 channels), compensated, "
                  "b=12 p=16 m=2"),
            steps=4096, dominant="momentum",
            groups=[dict(kind="ou", n=3, levels=12, points=16, m=2, dtype="f32", accum="kahan",
                         comps=3, tau=(50, 50), sigma=1.0, seed=7, stream=2),
                    dict(kind="momentum", n=6, levels=12, points=16, m=2, dtype="f32",
                         accum="kahan", n_atoms=20_000_000, box=600.0, masses=(6.941, 18.998),
                         seed=7, stream=5, vtau=(20, 200), pair_with=0)])
    raise ValueError(name)


def momentum_species(g):
    """Seeded species ids of a momentum workload (uniform over the species)."""
    rng = np.random.default_rng([g["seed"], g["stream"]])
    return rng.integers(0, len(g["masses"]), g["n_atoms"]).astype(np.int32)


class MomentumInput:
    """Velocities [3][N] (OU series, generated on the GPU) then, for a pair
    group, the x samples: the heat-flux components of another group's input,
    repeated for every species."""

    def __init__(self, g, xbuf):
        import synth
        self.n = g["n_atoms"]
        self.ns = len(g["masses"])
        self.xbuf = xbuf
        self.vel = synth.GpuOU(synth.OUSpec.make(g["seed"], g["stream"], 3 * self.n, comps=3,
                                                 tau=g["vtau"][0], tau_hi=g["vtau"][1],
                                                 sigma=1.0))

    def fill(self, buf, n_steps):
        self.vel.fill(buf[:, :3 * self.n], n_steps)
        if self.xbuf is not None:
            q = self.xbuf[:n_steps]
            for s in range(self.ns):
                buf[:n_steps, 3 * self.n + 3 * s:3 * self.n + 3 * s + 3].copy_(q)


class CurrentsInput:
    """Positions then velocities, [steps][6][N] float32, generated on the GPU."""

    def __init__(self, g):
        import synth
        self.n = g["n_atoms"]
        self.pos = synth.GpuPositions(synth.PositionSpec(g["seed"], g["stream"], self.n, g["box"],
                                                         0.1, 50.0))
        self.vel = synth.GpuOU(synth.OUSpec.make(g["seed"], g["stream"] + 1, 3 * self.n, comps=3,
                                                 tau=g["vtau"][0], tau_hi=g["vtau"][1],
                                                 sigma=1.0))

    def fill(self, buf, n_steps):
        flat = buf.view(buf.shape[0], 6 * self.n)
        self.pos.fill(flat[:, :3 * self.n], n_steps)
        self.vel.fill(flat[:, 3 * self.n:], n_steps)


# rocprofv3 counter records of the flush kernel (profiles/flush_traffic_<config>.md)
# are valid only for the kernel source they were taken on: the fold kernel's
# file and, of the shared header, the definitions it uses.
TRAFFIC_SOURCE = "paper_2503_07526_amd/csrc/corr_deferred.hip"
TRAFFIC_HEADER = "paper_2503_07526_amd/csrc/corr_internal.h"
TRAFFIC_HEADER_PARTS = ("enum Kind", "struct GroupArgs", "struct DeferredArgs", "kDeferT",
                        "kFlushGroups", "acc_planes", "kind_complex", "kind_sample_bytes",
                        "kind_acc_bytes", "struct FoldStamps", "kStampSlots", "stamp_")


def _strip_comments(src):
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    return re.sub(r"//[^\n]*", " ", src)


def flush_source_hash():
    """Hash of the fold kernel's source and of the header definitions it uses,
    with comments and whitespace removed (a comment edit, or a change to other
    kernels' argument structs, does not change this kernel)."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, TRAFFIC_SOURCE)) as f:
        h.update(" ".join(_strip_comments(f.read()).split()).encode())
    with open(os.path.join(ROOT, TRAFFIC_HEADER)) as f:
        header = _strip_comments(f.read())
    # top-level declarations: split at lines that start a new definition
    decls, cur = [], []
    for line in header.splitlines():
        if line and not line[0].isspace() and line[0] not in "{}" and cur:
            decls.append("\n".join(cur))
            cur = []
        cur.append(line)
    decls.append("\n".join(cur))
    for part in TRAFFIC_HEADER_PARTS:
        for d in decls:
            first = d.strip().split("\n", 1)[0]
            if part in first:
                h.update(" ".join(d.split()).encode())
    return h.hexdigest()[:16]


def traffic_record(config):
    """HBM bytes per flush launch from the committed counter summary of this
    workload (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or
    None when there is none or it was taken on another kernel source."""
    path = os.path.join(ROOT, "profiles", f"flush_traffic_{config}.md")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("record:"):
                rec = dict(kv.split("=", 1) for kv in line.split()[1:])
    if rec is None or rec.get("source_sha256") != flush_source_hash():
        return None
    return rec


SB = {"f32": 4, "f64": 8, "cf32": 8, "cf64": 16}
AB = {("f32", "f64"): 8, ("f32", "kahan"): 8, ("f32", "f32"): 4, ("f64", "f64"): 8,
      ("cf32", "f64"): 16, ("cf32", "kahan"): 16, ("cf32", "f32"): 8, ("cf64", "f64"): 16}


DEFER_T = 256   # pushes per block of the block-deferred form (the library's default T)
WINDOW_T = 64   # pushes per block of the block-deferred window


def deferred(g, direct=False):
    """Groups the library runs in the block-deferred form (as it reports them
    once the context exists: corr_group_form)."""
    if "form" in g:
        return g["form"] == 1
    return (not direct and g["kind"] == "ou" and g["dtype"] == "f32" and g["points"] == 16
            and g["m"] == 2)


def block_of(g):
    return g.get("T", DEFER_T)


def fold_bytes(g, s, level0_new):
    """Algorithmic HBM bytes per channel of folding the block of T pushes that
    ends at push s (s a multiple of T): level 0 moves level0_new bytes for the
    T new values and reads+writes its 16 accumulators; every level k that
    receives n_k > 0 new values reads its 15 older ring values, writes
    min(n_k, 16) slots and reads+writes its 8 accumulators."""
    sb, ab = SB[g["dtype"]], AB[(g["dtype"], g["accum"])]
    p, b, T = g["points"], g["levels"], block_of(g)
    B = level0_new + 2 * p * ab
    for k in range(1, b):
        nk = s // 2 ** k - (s - T) // 2 ** k
        if nk <= 0:
            break
        B += (p - 1) * sb + min(nk, p) * sb + 2 * (p - p // 2) * ab
    return B


def flush_bytes(g, s):
    """Algorithmic HBM bytes of the flush at push s (s a multiple of T) for one
    block-deferred group: level 0 reads the T new and 15 older values from the
    ring (the staging wrote them there), then the levels as in fold_bytes."""
    sb, p, T = SB[g["dtype"]], g["points"], block_of(g)
    return fold_bytes(g, s, (p - 1 + T) * sb) * g["n"]


def history_fold_bytes(g, s):
    """The same block folded straight from a stored history (corr_push_steps):
    level 0 reads the T new values from the history and the 15 older ones from
    the ring, and writes the block's last 15 values to the ring."""
    sb, p, T = SB[g["dtype"]], g["points"], block_of(g)
    return fold_bytes(g, s, (T + 2 * (p - 1)) * sb) * g["n"]


def group_channels(g, tw, j):
    """Channels of tile group j (T groups of contiguous tiles) of a block-deferred group."""
    n_tiles = -(-g["n"] // tw)
    tpg = -(-n_tiles // block_of(g))
    t0, t1 = j * tpg, min((j + 1) * tpg, n_tiles)
    if t0 >= t1:
        return 0
    return max(0, min(t1 * tw, g["n"]) - t0 * tw)


def staggered_flush_bytes(g, s, tw):
    """Bytes of the flush issued with push s: tile group s mod T folds block
    s // T (pushes (T (q-1), T q])."""
    T = block_of(g)
    j, q = s % T, s // T
    if q < 1:
        return 0
    per_channel = flush_bytes(dict(g, n=1), q * T)
    return per_channel * group_channels(g, tw, j)


def window_deferred(g, direct=False):
    """One-level groups of >= 512 points with single-precision samples: the
    library's fold kernel of each push writes the sample into the ring and folds
    one of 64 lag blocks."""
    return (not direct and g["levels"] == 1 and g["points"] >= 512
            and g["dtype"] in ("f32", "cf32"))


def window_push_cost(g):
    """Algorithmic bytes and flop of one push of a block-deferred window, per
    group: the sample is read and written to its ring slot; the fold of lag
    block j (lpb = p / 64 lags) reads the 64 new and 63 + lpb older ring values
    and reads+writes lpb accumulators, and does 64 x lpb products (complex: 4
    fma = 8 flop each; real: 2 flop)."""
    sb, ab = SB[g["dtype"]], AB[(g["dtype"], g["accum"])]
    lpb = -(-g["points"] // WINDOW_T)
    per_ch = 2 * sb + (2 * WINDOW_T - 1 + lpb) * sb + 2 * lpb * ab
    flop = g["points"] * (8 if g["dtype"] == "cf32" else 2)
    return per_ch * g["n"], flop * g["n"]


def producer_flop(g):
    """Algorithmic flop of one producer launch (matrix-core forms; the
    momentum densities are an HBM-bound reduction and count no flop here)."""
    if g["kind"] == "momentum":
        return 0
    if g["kind"] == "currents":
        return CURRENTS_FLOP_PER_ATOM_K * (g["n"] // 3) * g["n_atoms"]
    return RHOK_FLOP_PER_ATOM_K * g["n"] * g["n_atoms"]


def push_bytes(g, s, direct=False):
    """Bytes of the push kernel at push s: staging (read sample, write ring slot)
    for block-deferred groups, the full per-step update otherwise."""
    if deferred(g, direct):
        return 2 * SB[g["dtype"]] * g["n"]
    return step_bytes(g, s)


def step_bytes(g, s):
    """Algorithmic HBM bytes of push s (1-based) for one group: per channel,
    level 0 reads the sample, the min(s,p)-1 lagged ring values and writes the
    new slot, and reads+writes min(s,p) accumulators; level k (when m^k | s)
    reads m-1 values of level k-1 for the block mean, writes its slot, reads
    its active lags and reads+writes their accumulators (a compensated
    accumulator counts value and compensation)."""
    sb, ab = SB[g["dtype"]], AB[(g["dtype"], g["accum"])]
    p, m, b = g["points"], g["m"], g["levels"]
    lag0 = p // m
    nl = min(s, p)
    B = sb + (nl - 1) * sb + sb + 2 * nl * ab
    sk = s
    for _k in range(1, b):
        if sk % m:
            break
        sk //= m
        nlk = max(0, min(sk, p) - lag0)
        B += (m - 1) * sb + sb + nlk * sb + 2 * nlk * ab
    return B * g["n"]


# -------------------------------------------------------------------- CPU leg
def cpu_baseline(wl):
    """The FP64 oracle on a bounded sample of the workload's largest group."""
    import oracle
    import synth
    if wl.get("dominant") == "momentum":
        return cpu_baseline_momentum(wl)
    if all(g["kind"] in PRODUCER_KINDS for g in wl["groups"]):
        return cpu_baseline_rhok(wl["groups"][0])
    g = max(wl["groups"], key=lambda x: x["n"])
    n_ch, S = 12000, 6000
    real = np.float32 if g["dtype"] == "f32" else np.float64
    spec = synth.OUSpec.make(g["seed"], g["stream"], n_ch, comps=g.get("comps", 1),
                             tau=g["tau"][0], tau_hi=g["tau"][1], dtype=real)
    x, _ = spec.series(0, S)
    o = oracle.OracleCorrelator(n_ch, g["levels"], g["points"], g["m"])
    x64 = x.astype(np.float64)
    t0 = time.perf_counter()
    for row in x64:
        o.push(row)
    dt = time.perf_counter() - t0
    out = {"value": n_ch * S / dt, "unit": "channel-samples/s", "cores": 1, "kind": "oracle",
           "sample": (f"{n_ch} channels x {S} pushes of the {g['dtype']} group "
                      f"(b={g['levels']}, p={g['points']}, m={g['m']}), single thread, "
                      f"{dt:.1f} s")}
    # the same sample on every host core at once: one oracle per thread (its C
    # calls release the interpreter lock), each pushing the same series; a GPU
    # box gives one GPU a share of 16 host cores, whatever the affinity mask says
    import threading
    n_thr = min(16, len(os.sched_getaffinity(0)))
    if n_thr > 1:
        S2 = S // 2

        def work():
            oo = oracle.OracleCorrelator(n_ch, g["levels"], g["points"], g["m"])
            for row in x64[:S2]:
                oo.push(row)

        ths = [threading.Thread(target=work) for _ in range(n_thr)]
        t0 = time.perf_counter()
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        dt2 = time.perf_counter() - t0
        # the reported baseline is the oracle on every core; the single-thread
        # figure stays beside it
        single = dict(out)
        del single["kind"]
        out = {"value": n_thr * n_ch * S2 / dt2, "unit": "channel-samples/s", "cores": n_thr,
               "kind": "oracle",
               "sample": (f"{n_thr} threads, each an oracle of {n_ch} channels of the "
                          f"{g['dtype']} group (b={g['levels']}, p={g['points']}, m={g['m']}) "
                          f"pushed {S2} times, {dt2:.1f} s"),
               "single_thread": single}
    return out


def cpu_baseline_rhok(g):
    """The oracle's direct n(k) (or current) sums (one double cos and sin per
    atom and k) on a bounded sample of atoms, scaled linearly to the workload's
    atom count; the correlator update of the k-channels is negligible beside
    it."""
    import oracle
    import synth
    n_sample, reps = 50_000, 3
    spec = synth.PositionSpec(g["seed"], g["stream"], n_sample, g["box"], 0.1, 50.0)
    pos, _ = spec.series(0, reps)
    vel = np.random.default_rng(0).standard_normal((reps, 3, n_sample)).astype(np.float32)
    t0 = time.perf_counter()
    for r in range(reps):
        if g["kind"] == "currents":
            oracle.currents(pos[r], vel[r], g["kvec"], g["box"])
        else:
            oracle.rhok(pos[r], g["kvec"], g["box"])
    dt = (time.perf_counter() - t0) / reps
    per_push = dt * g["n_atoms"] / n_sample
    return {"value": g["n"] / per_push, "unit": "channel-samples/s", "cores": 1, "kind": "oracle",
            "sample": (f"{g['kind']} of {len(g['kvec'])} k-vectors over {n_sample} of "
                       f"{g['n_atoms']} atoms, "
                       f"{reps} pushes, {dt:.2f} s each, scaled to the full atom count; "
                       f"single thread")}


def cpu_baseline_momentum(wl):
    """The oracle's partial momentum densities (plain double sums) over all
    atoms of the workload for a few pushes; the correlator updates of the few
    channels are negligible beside it."""
    import oracle
    g = next(x for x in wl["groups"] if x["kind"] == "momentum")
    n_sample, reps = g["n_atoms"], 3
    rng = np.random.default_rng(0)
    vel = rng.standard_normal((3, n_sample)).astype(np.float32)
    sp = momentum_species(dict(g, n_atoms=n_sample))
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.partial_momentum(vel, sp, g["masses"], g["box"] ** 3)
    dt = (time.perf_counter() - t0) / reps
    per_push = dt * g["n_atoms"] / n_sample
    n_total = sum(x["n"] for x in wl["groups"])
    return {"value": n_total / per_push, "unit": "channel-samples/s", "cores": 1, "kind": "oracle",
            "sample": (f"partial momentum densities of {len(g['masses'])} species over all "
                       f"{n_sample} atoms, {reps} pushes, {dt:.2f} s each; single thread")}


# -------------------------------------------------------------------- GPU leg
def make_inputs(wl, chunk, dev):
    """Group descriptors, device input generators and chunk buffers ([chunk]
    rows of one push's input each) of a workload."""
    import torch

    import synth
    from paper_2503_07526_amd import GroupDesc
    descs, gens, bufs = [], [], []
    for g in wl["groups"]:
        if g.get("shares_positions"):
            # positions are the first [3][N] floats of the previous group's input
            descs.append(GroupDesc(g["n"], g["levels"], g["points"], g["m"], dtype=g["dtype"],
                                   accum=g["accum"], source="rhok", kvec=g["kvec"],
                                   n_atoms=g["n_atoms"], box=g["box"],
                                   update_every=g.get("update_every", 1)))
            gens.append(None)
            bufs.append(bufs[-1])
        elif g["kind"] == "momentum":
            pair = g.get("pair_with") is not None
            descs.append(GroupDesc(g["n"], g["levels"], g["points"], g["m"], dtype=g["dtype"],
                                   accum=g["accum"], source="momentum", n_atoms=g["n_atoms"],
                                   box=g["box"], species=momentum_species(g),
                                   masses=np.array(g["masses"]), pair=pair))
            gens.append(MomentumInput(g, bufs[g["pair_with"]] if pair else None))
            bufs.append(torch.empty((chunk, 3 * g["n_atoms"] + (g["n"] if pair else 0)),
                                    dtype=torch.float32, device=dev))
        elif g["kind"] == "currents":
            descs.append(GroupDesc(g["n"], g["levels"], g["points"], g["m"], dtype=g["dtype"],
                                   accum=g["accum"], source="currents", kvec=g["kvec"],
                                   n_atoms=g["n_atoms"], box=g["box"],
                                   update_every=g.get("update_every", 1)))
            gens.append(CurrentsInput(g))
            bufs.append(torch.empty((chunk, 6, g["n_atoms"]), dtype=torch.float32, device=dev))
        elif g["kind"] == "rhok":
            descs.append(GroupDesc(g["n"], g["levels"], g["points"], g["m"], dtype=g["dtype"],
                                   accum=g["accum"], source="rhok", kvec=g["kvec"],
                                   n_atoms=g["n_atoms"], box=g["box"],
                                   update_every=g.get("update_every", 1)))
            spec = synth.PositionSpec(g["seed"], g["stream"], g["n_atoms"], g["box"], 0.1, 50.0)
            gens.append(synth.GpuPositions(spec))
            bufs.append(torch.empty((chunk, 3, g["n_atoms"]), dtype=torch.float32, device=dev))
        else:
            real = np.float32 if g["dtype"] == "f32" else np.float64
            descs.append(GroupDesc(g["n"], g["levels"], g["points"], g["m"], dtype=g["dtype"],
                                   accum=g["accum"]))
            spec = synth.OUSpec.make(g["seed"], g["stream"], g["n"], comps=g["comps"],
                                     tau=g["tau"][0], tau_hi=g["tau"][1], sigma=g["sigma"],
                                     dtype=real)
            gens.append(synth.GpuOU(spec))
            tdt = torch.float32 if real == np.float32 else torch.float64
            bufs.append(torch.empty((chunk, g["n"]), dtype=tdt, device=dev))
    return descs, gens, bufs


def run(args):
    import torch

    import synth
    from paper_2503_07526_amd import Correlator, GroupDesc, autotune

    wl = workload(args.config)
    K = args.steps if args.steps is not None else wl["steps"]
    W = args.warmup if args.warmup is not None else wl.get("warmup", 256)
    mode = args.mode or ("per_group" if args.config == "plain" else "batched")
    args.direct = args.direct or wl.get("direct", False)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)

    if args.replay:
        chunk = args.chunk or DEFER_T
    else:
        chunk = max(1, min(args.chunk or 128, K))
    descs, gens, bufs = make_inputs(wl, chunk, dev)
    tuning = json.loads(args.tuning) if args.tuning else None
    tune_s = 0.0
    if tuning is None and not args.no_autotune:
        t0 = time.perf_counter()
        tuning = autotune(descs, per_group=(mode == "per_group"), direct=args.direct,
                          rhok_valu=args.rhok_valu)
        tune_s = time.perf_counter() - t0
    if args.overlap is not None:
        tuning = dict(tuning or {}, overlap_producers=args.overlap)
    # Block-deferred workloads are timed as captured HIP graphs (one graph per
    # chunk of pushes, corr_push_steps on a CORR_FLAG_GRAPH context), the eager
    # form beside them (1.5 to 6% slower on every such line once the timing
    # stamps sample one push in timing_stride); the others eagerly, one
    # corr_push per step.
    use_graph = (not args.eager and not args.replay and not args.direct and mode != "per_group"
                 and any(deferred(g) for g in wl["groups"]))
    corr = Correlator(descs, per_group=(mode == "per_group"), tuning=tuning, timing=True,
                      direct=args.direct, rhok_valu=args.rhok_valu, graph=use_graph)
    state_gb = sum(corr.state_bytes(i) for i in range(len(descs))) / 1e9
    # events and device stamps on one push in timing_stride (a stored-history
    # replay stamps every block fold: there are few of them)
    corr.set_timing_stride(1 if args.replay else args.timing_stride)
    # the update form and fold block the library chose for each group
    wl = dict(wl, groups=[dict(g) for g in wl["groups"]])
    for i, g in enumerate(wl["groups"]):
        g["form"], blk = corr.group_form(i)
        if g["form"] == 1:
            g["T"] = blk
    if args.replay:
        return run_replay(args, wl, corr, descs, gens, bufs, K, W, mode, state_gb, tune_s)

    def push_chunk(n):
        for gen, buf in zip(gens, bufs):
            if gen is not None:
                gen.fill(buf, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if use_graph:
            corr.push_steps([buf[:n] for buf in bufs])
        else:
            for j in range(n):
                corr.push([buf[j] for buf in bufs])
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # Fill, then the declared warm-up.  A block-deferred group folds its first
    # block at push T (256), so at least one whole block is pushed before the
    # warm-up: the timed pushes then carry their scheduled folds whatever
    # --warmup says (steady state).  In graph mode the fill also captures the
    # graph of every chunk length the timed pushes use.
    direct = args.direct
    fill = max([block_of(g) for g in wl["groups"] if deferred(g, direct)], default=0)
    lead = [min(chunk, fill - d) for d in range(0, fill, chunk)]
    if use_graph:
        lead += [n for n in {chunk, K % chunk} if n and n not in lead]
    fill = sum(lead)
    for n in lead:
        push_chunk(n)
    done = 0
    while done < W:
        n = min(chunk, W - done)
        push_chunk(n)
        done += n
    for which in (0, 1, 2, 3, 4):
        corr.kernel_time(which, reset=True)
    s_first = fill + W + 1
    wall = 0.0
    done = 0
    while done < K:
        n = min(chunk, K - done)
        wall += push_chunk(n)
        done += n
    steps = range(s_first, s_first + K)
    n_total = sum(g["n"] for g in wl["groups"])
    value = n_total * K / wall
    tw = corr.tuning()["tile_channels"]
    has_rhok = any(g["kind"] in PRODUCER_KINDS for g in wl["groups"])
    # the groups whose update the push events bracket (a forked producer
    # branch runs beside them)
    timed = [g for g in wl["groups"]
             if not (has_rhok and len(wl["groups"]) > 1 and g["kind"] in PRODUCER_KINDS)]
    # device stamps of one push in timing_stride: the folds (3) and the producers (4)
    fs_ms, fs_n = corr.kernel_time(which=3)
    ps_ms, ps_n = corr.kernel_time(which=4)
    fl_bytes_all = sum(staggered_flush_bytes(g, s, tw) for g in timed if deferred(g, direct)
                       for s in steps)
    # HIP events (eager pushes only), like the stamps on one push in timing_stride
    kern_ms, kern_n = corr.kernel_time(0)
    fl_ms, fl_n = corr.kernel_time(which=1)
    rk_ms, rk_n = corr.kernel_time(which=2)
    sampled = [s for s in steps if (s - 1) % args.timing_stride == 0]
    if not use_graph:
        assert kern_n == len(sampled), (kern_n, len(sampled))
    stage_bytes = sum(push_bytes(g, s, direct) for g in timed for s in sampled)
    fl_bytes = sum(staggered_flush_bytes(g, s, tw) for g in timed if deferred(g, direct)
                   for s in sampled)
    rhok_only = (all(g["kind"] in PRODUCER_KINDS for g in wl["groups"])
                 and wl.get("dominant") not in ("push", "producer"))
    producer_dominant = wl.get("dominant") == "producer"
    push_dominant = wl.get("dominant") == "push"
    momentum_dominant = wl.get("dominant") == "momentum"
    flop_per = None
    if momentum_dominant:
        # the momentum density producers: per atom three velocity components
        # and a one-byte species id; device stamps of the sampled pushes' producers
        per_launch_bytes = sum(g["n_atoms"] * (3 * SB[g["dtype"]] + 1) for g in wl["groups"]
                               if g["kind"] == "momentum")
        per_launch_ms = ps_ms / ps_n
        achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
        kname = ("momentum density producer (HBM-bound reduction over the atoms), device stamps "
                 "of one push in %d" % args.timing_stride)
    elif producer_dominant:
        # the producers of every k-space group, per push
        flop_per = sum(producer_flop(g) for g in wl["groups"] if g["kind"] in PRODUCER_KINDS)
        per_launch_ms = ps_ms / ps_n
        achieved = flop_per / (per_launch_ms * 1e-3) / 1e12
        kname = ("k-space producers (matrix cores), device stamps spanning the producer launches "
                 "of one push in %d" % args.timing_stride)
        per_launch_bytes = None
    elif push_dominant:
        # the per-step correlator update of every group (direct form): the
        # push events minus the producer launches they contain
        push_ms = (kern_ms - rk_ms) / kern_n
        push_bytes_step = sum(step_bytes(g, s) for g in wl["groups"] for s in sampled) / kern_n
        achieved = push_bytes_step / (push_ms * 1e-3) / 1e9
        kname = ("push kernel (per-step update of every channel's window), HIP events per push "
                 "less the producer launches")
        per_launch_ms, per_launch_bytes = push_ms, push_bytes_step
    elif rhok_only:
        g0 = wl["groups"][0]
        if g0["kind"] == "currents":
            flop_per = CURRENTS_FLOP_PER_ATOM_K * (g0["n"] // 3) * g0["n_atoms"]
            kname = ("current producer (matrix cores), device stamps of one launch in %d"
                     % args.timing_stride)
        else:
            flop_per = RHOK_FLOP_PER_ATOM_K * g0["n"] * g0["n_atoms"]
            kname = ("k-density producer (%s), device stamps of one launch in %d"
                     % ("vector units" if args.rhok_valu else "matrix cores", args.timing_stride))
        achieved = flop_per / (ps_ms / ps_n * 1e-3) / 1e12
        per_launch_ms, per_launch_bytes = ps_ms / ps_n, None
    elif fs_n:
        # dominant kernel: the flush of the block-deferred groups, stamped on the
        # sampled pushes
        assert fs_n == len(sampled), (fs_n, len(sampled))
        if fl_bytes_all <= 0:
            raise RuntimeError("the timed pushes carried no fold work (pushes %d..%d): the "
                               "block-deferred line would not measure its dominant kernel"
                               % (s_first, s_first + K - 1))
        achieved = fl_bytes / (fs_ms * 1e-3) / 1e9
        T0 = max(block_of(g) for g in timed if deferred(g, direct))
        kname = ("flush kernel (block-deferred fold of %d pushes for 1/%d of the channels per "
                 "push), device stamps of one launch in %d" % (T0, T0, args.timing_stride))
        per_launch_ms, per_launch_bytes = fs_ms / fs_n, fl_bytes / fs_n
    else:
        achieved = (stage_bytes + fl_bytes) / (kern_ms * 1e-3) / 1e9
        kname = ("push kernel (correlator update of %d of %d groups), HIP events per launch"
                 % (len(timed), len(wl["groups"])))
        per_launch_ms, per_launch_bytes = kern_ms / kern_n, (stage_bytes + fl_bytes) / kern_n
    out = {
        "metric": "channel-samples/sec into correlators",
        "value": value,
        "unit": "channel-samples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "fill_pushes": fill,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+kahan" if any(g["accum"] == "kahan" for g in wl["groups"]) else "f32+f64",
        "data": "synthetic (seeded OU series and atom positions generated in HBM before each "
                "timed chunk)",
        "config": {"workload": wl["name"], "channels": n_total, "launch": mode,
                   "update_form": "direct" if args.direct else "block-deferred where supported",
                   "rhok_producer": ("vector units (fp32 phases, fp32 tile sums added in fp64)"
                                     if args.rhok_valu else
                                     "matrix cores (fp16 hi/lo operand split: about 22 "
                                     "significant bits per product; fp32 tile sums added in "
                                     "fp64)"),
                   "push_calls": ("one captured HIP graph per chunk of %d pushes (corr_push_steps "
                                  "with CORR_FLAG_GRAPH)" % chunk if use_graph
                                  else "one corr_push per step"),
                   "fold_block": {str(i): g["T"] for i, g in enumerate(wl["groups"]) if "T" in g},
                   "producer_stream": {0: "the context's stream, before the other updates",
                                       1: ("a side stream with the per-step updates, forked and "
                                           "joined every 4 pushes of a captured chunk (each "
                                           "stream ends its pushes with its own counter)"
                                           if use_graph and any(deferred(g, args.direct)
                                                                for g in wl["groups"]) else
                                           "forked at the start of the push (with the per-step "
                                           "updates when block-deferred groups flush beside "
                                           "them)"),
                                       2: "the context's stream; the per-step updates forked "
                                          "beside the flush"}[corr.tuning()["overlap_producers"]],
                   "tuning": corr.tuning(), "state_GB": round(state_gb, 2)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kname,
                     "kernel_ms_per_launch": per_launch_ms,
                     "alg_bytes_per_launch": per_launch_bytes},
    }
    r = out["roofline"]
    if kern_n:
        r.update({"update_kernels_GBs": (stage_bytes + fl_bytes) / (kern_ms * 1e-3) / 1e9,
                  "update_ms_per_step": kern_ms / kern_n,
                  "alg_bytes_per_step": (stage_bytes + fl_bytes) / kern_n,
                  "timed_pushes": kern_n, "timing_stride": args.timing_stride})
    if fs_n:
        # context for the byte model of the per-step form (Algorithm 1 push by
        # push): its algorithmic bytes for the same pushes of the same groups,
        # over this form's wall time per push (an equivalent, not traffic)
        eq = sum(step_bytes(g, s) for g in wl["groups"] if g["kind"] not in PRODUCER_KINDS
                 for s in steps) / K
        eq_gbs = eq / (wall / K) / 1e9
        out["per_step_form_model"] = {
            "note": "the per-step form's algorithmic bytes for the same pushes of the sample-fed "
                    "groups, divided by this form's wall time per push (a model figure, not HBM "
                    "traffic)",
            "bytes_per_push": eq, "GBs": eq_gbs, "x_peak": eq_gbs / HBM_PEAK_GBS}
    if fs_n and fl_n:
        r["kernel_ms_per_launch_events"] = fl_ms / fl_n
        r["events_note"] = ("HIP events on the timed pushes (one in %d); they separate the "
                            "push's kernels" % args.timing_stride)
    if ps_n:
        r["producer_ms_per_push"] = ps_ms / ps_n
        if not (rhok_only or producer_dominant or momentum_dominant):
            # the producers beside the dominant kernel (forked, they may be the
            # longer branch of the step)
            pf = sum(producer_flop(g) for g in wl["groups"] if g["kind"] in PRODUCER_KINDS)
            pms = ps_ms / ps_n
            out["producers"] = {
                "ms_per_push": pms, "alg_flop_per_push": pf,
                "TFLOPs": pf / (pms * 1e-3) / 1e12,
                "frac_of_fp16_matrix_peak": pf / (pms * 1e-3) / 1e12 / MFMA_F16_PEAK_TFS,
                "timing": "device stamps from the first producer block's start to the end of "
                          "its final reduction, every push",
                "stream": "forked beside the other updates"
                          if corr.tuning()["overlap_producers"] == 1 else "the context's stream"}
    wins = [g for g in wl["groups"] if window_deferred(g, direct)]
    if wins and len(wins) == len(wl["groups"]) and kern_n:
        # the correlator update of the block-deferred windows: the push events
        # less the producer launches they contain
        wb = sum(window_push_cost(g)[0] for g in wins)
        wf = sum(window_push_cost(g)[1] for g in wins)
        wms = (kern_ms - rk_ms) / kern_n
        out["window_update"] = {
            "kernels": "one lag-block fold per group and push (which also stages the sample)",
            "ms_per_push": wms, "alg_bytes_per_push": wb, "alg_flop_per_push": wf,
            "GBs": wb / (wms * 1e-3) / 1e9, "hbm_frac": wb / (wms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "TFLOPs": wf / (wms * 1e-3) / 1e12,
            "alu_frac": wf / (wms * 1e-3) / 1e12 / VALU_F32_PEAK_TFS}
    if rhok_only or producer_dominant:
        bound, peak = ("alu", VALU_F32_PEAK_TFS) if args.rhok_valu else ("mfma", MFMA_F16_PEAK_TFS)
        r.update({"bound": bound, "unit": "TFLOP/s", "peak": peak, "frac": achieved / peak,
                  "alg_flop_per_launch": flop_per})
        for key in ("alg_bytes_per_launch", "update_kernels_GBs", "alg_bytes_per_step"):
            r.pop(key, None)
    elif fs_n:
        rec = traffic_record(args.config)
        if rec is not None:
            tb = float(rec["read_bytes_per_launch"]) + float(rec["write_bytes_per_launch"])
            r["traffic"] = tb
            r["traffic_detail"] = {
                "hbm_bytes_per_launch": tb,
                "alg_bytes_per_launch_same_pushes": float(rec["alg_bytes_per_launch"]),
                "ratio": tb / float(rec["alg_bytes_per_launch"]),
                "pushes": rec["pushes"], "source": f"profiles/flush_traffic_{args.config}.md"}
    out["config"]["autotune_s"] = round(tune_s, 2)
    if max(wl["groups"], key=lambda x: x["n"])["kind"] == "ou":
        out["error_vs_fp64"] = spot_check(corr, wl, fill + W + K)
    tuned = corr.tuning()
    corr.close()
    if fs_n and tuned["overlap_producers"] != 0:
        # the same flush kernel with nothing beside it: a short second context
        # with every push on one stream, timed by the same device stamps
        t0n = dict(tuned, overlap_producers=0)
        c0 = Correlator(descs, per_group=(mode == "per_group"), tuning=t0n, timing=True,
                        direct=args.direct, rhok_valu=args.rhok_valu)
        n_alone = 256
        T0 = max(block_of(g) for g in timed if deferred(g, direct))
        for lead_n in (T0, n_alone):  # one block to fill the rings, then the timed pushes
            if lead_n == n_alone:
                c0.kernel_time(3, reset=True)
            done = 0
            while done < lead_n:
                n = min(chunk, lead_n - done)
                for gen, buf in zip(gens, bufs):
                    if gen is not None:
                        gen.fill(buf, n)
                for j in range(n):
                    c0.push([buf[j] for buf in bufs])
                done += n
        torch.cuda.synchronize()
        a_ms, a_n = c0.kernel_time(3)
        c0.close()
        a_bytes = sum(staggered_flush_bytes(g, s, tw) for g in timed if deferred(g, direct)
                      for s in range(T0 + 1, T0 + n_alone + 1))
        if a_n:
            a_gbs = a_bytes / (a_ms * 1e-3) / 1e9
            r["alone"] = {
                "note": "the same flush kernel with every push on one stream (nothing beside "
                        "it), %d pushes after one block, device stamps" % n_alone,
                "kernel_ms_per_launch": a_ms / a_n, "achieved": a_gbs,
                "frac": a_gbs / HBM_PEAK_GBS}
    if use_graph and not args.no_mode_leg:
        out["eager"] = mode_leg(args, wl, descs, gens, bufs, tuned, mode, chunk, False, value)
    elif fs_n and not args.no_mode_leg and mode != "per_group":
        out["graph"] = mode_leg(args, wl, descs, gens, bufs, tuned, mode, chunk, True, value)
    big = max(wl["groups"], key=lambda x: x["n"])
    if not args.no_compare_plain and big["kind"] == "ou" and big["dtype"] == "f32":
        out["plain_form"] = compare_plain(wl, args.plain_steps, chunk, args.timing_stride)
        out["plain_form"]["speedup_of_this_form"] = value / out["plain_form"]["value"]
    return out, wl


def mode_leg(args, wl, descs, gens, bufs, tuned, mode, chunk, graph, headline_value):
    """The same workload in the other issue form, timed like the headline
    beside it: graph=True replays every chunk of pushes as one captured HIP
    graph (corr_push_steps with CORR_FLAG_GRAPH), graph=False issues one
    corr_push per step (eager)."""
    import torch

    from paper_2503_07526_amd import Correlator
    n_total = sum(g["n"] for g in wl["groups"])
    corr = Correlator(descs, per_group=(mode == "per_group"), tuning=tuned, graph=graph,
                      direct=args.direct, rhok_valu=args.rhok_valu)
    T0 = max([block_of(g) for g in wl["groups"] if deferred(g, args.direct)], default=0)

    def chunk_run(n):
        for gen, buf in zip(gens, bufs):
            if gen is not None:
                gen.fill(buf, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if graph:
            corr.push_steps([buf[:n] for buf in bufs])
        else:
            for j in range(n):
                corr.push([buf[j] for buf in bufs])
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    lead = [min(chunk, T0 - d) for d in range(0, T0, chunk)] + [chunk]
    for n in lead:  # one fold block, then a chunk (which captures the timed graph)
        chunk_run(n)
    steps = max(256, chunk) // chunk * chunk
    wall = sum(chunk_run(chunk) for _ in range(steps // chunk))
    corr.close()
    v = n_total * steps / wall
    return {"note": ("the same pushes as one captured HIP graph per chunk of %d (corr_push_steps "
                     "with CORR_FLAG_GRAPH)" % chunk) if graph else
                    "the same pushes issued eagerly, one corr_push per step",
            "fill_pushes": sum(lead), "steps": steps, "ms_per_step": wall / steps * 1e3,
            "value": v, "ratio_to_headline": v / headline_value}


def run_replay(args, wl, corr, descs, gens, bufs, K, W, mode, state_gb, tune_s):
    """Replay of stored histories (corr_push_steps without a graph): every
    chunk of pushes is handed over at once, block-aligned, so the
    block-deferred groups fold each whole block straight from the history; the
    other groups are pushed row by row.  The dominant kernel is that history
    fold, timed by its own device stamps."""
    import torch
    chunk = bufs[0].shape[0]
    Ts = [block_of(g) for g in wl["groups"] if deferred(g, args.direct)]
    T = max(Ts, default=DEFER_T)
    if chunk % T:
        raise SystemExit(f"--replay needs --chunk a multiple of the fold block ({T})")
    W = -(-W // T) * T          # block-aligned warm-up
    K = max(chunk, -(-K // chunk) * chunk)
    n_total = sum(g["n"] for g in wl["groups"])

    def chunk_run(n):
        for gen, buf in zip(gens, bufs):
            if gen is not None:
                gen.fill(buf, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        corr.push_steps([buf[:n] for buf in bufs])
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    done = 0
    while done < W:
        n = min(chunk, W - done)
        chunk_run(n)
        done += n
    corr.kernel_time(3, reset=True)
    wall = sum(chunk_run(chunk) for _ in range(K // chunk))
    fs_ms, fs_n = corr.kernel_time(3)
    blocks = [s for s in range(W + T, W + K + 1, T)]
    fold_b = sum(history_fold_bytes(g, s) for g in wl["groups"] if deferred(g, args.direct)
                 for s in blocks)
    achieved = fold_b / (fs_ms * 1e-3) / 1e9 if fs_n else 0.0
    value = n_total * K / wall
    out = {
        "metric": "channel-samples/sec into correlators (replay of stored histories)",
        "value": value, "unit": "channel-samples/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+kahan" if any(g["accum"] == "kahan" for g in wl["groups"]) else "f32+f64",
        "data": "synthetic (seeded OU series and atom positions generated in HBM before each "
                "timed chunk)",
        "config": {"workload": wl["name"], "channels": n_total, "launch": mode,
                   "push_calls": "one corr_push_steps per chunk of %d stored pushes" % chunk,
                   "fold_block": T, "tuning": corr.tuning(), "state_GB": round(state_gb, 2),
                   "autotune_s": round(tune_s, 2)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "history fold (a whole block of %d pushes of every channel read "
                               "straight from the stored history), device stamps" % T,
                     "kernel_ms_per_launch": fs_ms / fs_n if fs_n else None,
                     "alg_bytes_per_launch": fold_b / max(fs_n, 1),
                     "alg_bytes_per_channel_step": fold_b / max(len(blocks), 1) / T /
                     sum(g["n"] for g in wl["groups"] if deferred(g, args.direct)),
                     "launches": fs_n},
    }
    if max(wl["groups"], key=lambda x: x["n"])["kind"] == "ou":
        out["error_vs_fp64"] = spot_check(corr, wl, W + K)
    corr.close()
    return out, wl


def spot_check(corr, wl, S):
    """Readout of a few channels of the largest group after the timed run,
    against the FP64 oracle fed with the same series regenerated on the CPU:
    max |C_gpu - C_oracle| / |C_oracle(0)| per channel, counts exact."""
    import oracle
    import synth
    gi = max(range(len(wl["groups"])), key=lambda i: wl["groups"][i]["n"])
    g = wl["groups"][gi]
    real = np.float32 if g["dtype"] == "f32" else np.float64
    spec = synth.OUSpec.make(g["seed"], g["stream"], g["n"], comps=g["comps"], tau=g["tau"][0],
                             tau_hi=g["tau"][1], sigma=g["sigma"], dtype=real)
    worst, chans, counts_ok = 0.0, [], True
    for lo in (0, g["n"] // 2, g["n"] - 2):
        res = corr.finalize(gi, slice_=(lo, lo + 2))
        x, _ = spec.series(0, S, channels=np.arange(lo, lo + 2))
        o = oracle.OracleCorrelator(2, g["levels"], g["points"], g["m"])
        for row in x:
            o.push(row.astype(np.float64))
        for i in range(2):
            t, c, n = o.readout(i, i + 1)
            counts_ok &= bool(np.array_equal(res["count"], n) and np.array_equal(res["t"], t))
            worst = max(worst, float(np.max(np.abs(res["c_per_channel"][i] - c)) / abs(c[0])))
            chans.append(lo + i)
    return {"max_abs_dC_over_C0": worst, "counts_and_lags_exact": counts_ok, "channels": chans,
            "pushes": S, "accumulator": g["accum"]}


def ou_expected(a, var, t_steps, p, m):
    """E[C] of a stationary AR(1) series (autocorrelation a^l) block-averaged
    over M = m^k samples at the multiple-tau lag grid (level k, lag L)."""
    out = []
    for t in t_steps:
        k = 0
        while t >= p * m ** k:
            k += 1
        M = m ** k
        L = int(round(t)) // M
        if k == 0:
            out.append(var * a ** L)
        else:
            g = (1 - a ** M) / (1 - a)
            out.append(var * a ** (M * L - (M - 1)) * g * g / (M * M))
    return np.array(out)


def precision(args):
    """Compensated FP32 vs FP64 (vs plain FP32) sums on the precision workload:
    10^5 velocity channels (tau=100) + 9 FP64 global channels (tau=100), 20
    levels x 16 points, m=2, sigma 1 and 10^3, against the FP64 oracle on
    sampled channels and against the closed-form OU expectation / sigma^2 tau
    Green-Kubo integral for the group mean."""
    import torch

    import oracle
    import synth
    from paper_2503_07526_amd import Correlator, GroupDesc
    S = args.precision_steps
    nv, b, p, m, tau = 100_000, 20, 16, 2, 100.0
    chunk = 512
    sample = np.r_[0:16, nv - 16:nv]
    runs = []
    for sigma in (1.0, 1000.0):
        vspec = synth.OUSpec.make(2, 1, nv, comps=3, tau=tau, sigma=sigma)
        gspec = synth.OUSpec.make(2, 2, 9, tau=tau, sigma=sigma, dtype=np.float64)
        # oracle on the sampled velocity channels and all global channels
        xs, _ = vspec.series(0, S, channels=sample)
        xg, _ = gspec.series(0, S)
        ov = oracle.OracleCorrelator(len(sample), b, p, m)
        og = oracle.OracleCorrelator(9, b, p, m)
        for i, (r1, r2) in enumerate(zip(xs, xg)):
            ov.push(r1.astype(np.float64))
            og.push(r2)
            if (i + 1) % 100_000 == 0:
                print(f"precision sigma={sigma:g}: oracle {i + 1}/{S} pushes", file=sys.stderr,
                      flush=True)
        var = float(synth.stationary_variance(vspec.a[0], vspec.b[0]))
        a64 = float(vspec.a[0])
        for accum in ("kahan", "f64", "f32"):
            t0 = time.perf_counter()
            gv, gg = synth.GpuOU(vspec), synth.GpuOU(gspec)
            bv = torch.empty((chunk, nv), dtype=torch.float32, device="cuda")
            bg = torch.empty((chunk, 9), dtype=torch.float64, device="cuda")
            corr = Correlator([GroupDesc(nv, b, p, m, dtype="f32", accum=accum),
                               GroupDesc(9, b, p, m, dtype="f64", accum="f64")])
            done = 0
            while done < S:
                n = min(chunk, S - done)
                gv.fill(bv, n)
                gg.fill(bg, n)
                for j in range(n):
                    corr.push([bv[j], bg[j]])
                done += n
                if done % 102_400 == 0:
                    print(f"precision sigma={sigma:g} {accum}: {done}/{S} pushes", file=sys.stderr,
                          flush=True)
            torch.cuda.synchronize()
            res_s = [corr.finalize(0, slice_=(0, 16)), corr.finalize(0, slice_=(nv - 16, nv))]
            per = np.vstack([r["c_per_channel"] for r in res_s])
            err_v = 0.0
            for i in range(len(sample)):
                t, c, n_ = ov.readout(i, i + 1)
                err_v = max(err_v, float(np.max(np.abs(per[i] - c)) / abs(c[0])))
            rg = corr.finalize(1, slice_=(0, 9))
            err_g = 0.0
            for i in range(9):
                t, c, n_ = og.readout(i, i + 1)
                err_g = max(err_g, float(np.max(np.abs(rg["c_per_channel"][i] - c)) / abs(c[0])))
            full = corr.finalize(0)
            t_s = full["t"]
            expect = ou_expected(a64, var, t_s, p, m)
            gk_grid = oracle.trapezoid(t_s, expect)[1]
            tau_eff = -1.0 / np.log(a64)
            corr.close()
            del bv, bg
            torch.cuda.empty_cache()
            runs.append({"sigma": sigma, "accumulator": accum,
                         "velocity_max_abs_dC_over_C0_vs_fp64_oracle": err_v,
                         "global_fp64_max_abs_dC_over_C0_vs_fp64_oracle": err_g,
                         "group_gk": full["gk_at_cut"],
                         "gk_grid_expected": gk_grid,
                         "gk_closed_form_sigma2_tau": var * tau_eff,
                         "c0_group_mean": float(full["c"][0]), "c0_expected": var,
                         "seconds": round(time.perf_counter() - t0, 1)})
            print(json.dumps(runs[-1]), file=sys.stderr, flush=True)
    worst = max(r["velocity_max_abs_dC_over_C0_vs_fp64_oracle"] for r in runs
                if r["accumulator"] == "kahan")
    return {"metric": "max |C_gpu - C_fp64oracle| / |C(0)|, compensated FP32 sums",
            "value": worst, "unit": "relative", "higher_is_better": False,
            "steps": S, "n_gpus": 1, "data": "synthetic OU series",
            "config": {"workload": "precision: 1e5 FP32 channels + 9 FP64 channels, tau=100, "
                                   "b=20 p=16 m=2, sigma 1 and 1e3",
                       "sampled_velocity_channels": len(sample)},
            "runs": runs}


def compare_plain(wl, K, chunk, stride):
    """The largest sample-fed group alone in the plain form (FP64 sums, per-step
    update, per-group launch): one whole 256-push block to fill the level-0
    window and the first levels, then K timed pushes."""
    import torch

    import synth
    from paper_2503_07526_amd import Correlator, GroupDesc
    g = max(wl["groups"], key=lambda x: x["n"])
    spec = synth.OUSpec.make(g["seed"], g["stream"], g["n"], comps=g["comps"], tau=g["tau"][0],
                             tau_hi=g["tau"][1], sigma=g["sigma"])
    gen = synth.GpuOU(spec)
    buf = torch.empty((chunk, g["n"]), dtype=torch.float32, device="cuda")
    corr = Correlator([GroupDesc(g["n"], g["levels"], g["points"], g["m"], dtype="f32",
                                 accum="f64")], per_group=True, timing=True, direct=True)
    corr.set_timing_stride(stride)
    W = DEFER_T
    wall, done, reset = 0.0, 0, False
    while done < W + K:
        if done >= W and not reset:
            corr.kernel_time(0, reset=True)  # time the chunks that count as timed
            w_first, reset = done + 1, True
        n = min(chunk, W + K - done)
        gen.fill(buf, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(n):
            corr.push([buf[j]])
        torch.cuda.synchronize()
        if done >= W:
            wall += time.perf_counter() - t0
        done += n
    kern_ms, kern_n = corr.kernel_time(0)
    corr.close()
    # bytes of the timed pushes the events cover (push s is timed when s - 1 % stride == 0)
    timed_s = [s for s in range(w_first, W + K + 1) if (s - 1) % stride == 0]
    alg = sum(step_bytes(g, s) for s in timed_s) / max(len(timed_s), 1)
    return {"value": g["n"] * K / wall, "unit": "channel-samples/s",
            "ms_per_step": wall / K * 1e3,
            "push_kernel_ms": kern_ms / kern_n if kern_n else None,
            "push_kernel_GBs": alg / (kern_ms / kern_n * 1e-3) / 1e9 if kern_n else None,
            "channels": g["n"], "steps": K, "fill_pushes": W,
            "form": "the largest group alone: FP32 samples, FP64 sums, per-step update of every "
                    "channel, one launch per group and push"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU sharding "
                                   "is a design note only (--gpus 1)", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(8):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_copy": src.numel() * 4,
                          "bytes_written_per_copy": dst.numel() * 4, "copies": 8}), flush=True)
        return
    if args.config == "precision":
        print(json.dumps(precision(args)), flush=True)
        return
    out, wl = run(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
