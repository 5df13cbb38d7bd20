"""Partial momentum densities of the mass-flux correction (Section "Viscosity
and thermal conductivity"; reading R22) on the GPU against the oracle: the
densities at lag 0, their correlations, and the pair form <q(s) j(s - L)>
with a caller series, in every launch mode."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import TOL, gate, ou_inputs, say

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def corrmod():
    import paper_2503_07526_amd as m
    m.lib()  # fails loudly if the HIP library is missing
    return m


def _system(seed, N, n_species, S, dtype):
    """Species ids, masses and [S][3][N] velocities (unit-variance OU series)."""
    rng = np.random.default_rng(seed)
    sp = rng.integers(0, n_species, N).astype(np.int32)
    masses = rng.uniform(1.0, 40.0, n_species)
    vel = ou_inputs(seed, 5, 3 * N, S, dtype).reshape(S, 3, N)
    return sp, masses, np.ascontiguousarray(vel)


def _push_all(corr, xs):
    dev = torch.device("cuda:0")
    ts = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in xs]
    for s in range(xs[0].shape[0]):
        corr.push([t[s] for t in ts])
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype,accum", [("f32", "kahan"), ("f32", "f64"), ("f64", "f64")])
@pytest.mark.parametrize("n_species,N", [(1, 1), (3, 5003), (8, 70001), (2, 4), (5, 400_000)])
def test_momentum_lag0_against_oracle(corrmod, dtype, accum, n_species, N):
    """One push: C(0) of channel 3s + a is j_{s,a}^2 (no 1/N), j from the
    oracle's plain double sums; atom counts of one atom, ragged counts (one
    atom per load), multiples of 4 (four atoms per load) and several blocks
    of the reduction."""
    box = 17.0
    say(f"[momentum lag 0] {dtype}/{accum} species={n_species} N={N}")
    sp, masses, vel = _system(31, N, n_species, 1, dtype)
    g = corrmod.GroupDesc(3 * n_species, 3, 8, 2, dtype=dtype, accum=accum, source="momentum",
                          n_atoms=N, box=box, species=sp, masses=masses)
    with corrmod.Correlator([g]) as c:
        _push_all(c, [vel])
        res = c.finalize(0, slice_=(0, 3 * n_species))
    j = oracle.partial_momentum(vel[0], sp, masses, box ** 3)
    got = res["c_per_channel"][:, 0]
    expect = j ** 2
    err = np.max(np.abs(got - expect)) / np.max(expect)
    say(f"  error {err:.2e}")
    assert err < (1e-12 if dtype == "f64" else 1e-6)


@pytest.mark.parametrize("dtype,accum", [("f32", "kahan"), ("f64", "f64")])
def test_momentum_correlator_parity(corrmod, dtype, accum):
    """Correlations of the densities of 2 species over 600 pushes against the
    oracle correlator fed with the oracle's densities."""
    N, S, box, b, p, m = 3000, 600, 12.0, 5, 16, 2
    say(f"[momentum parity] {dtype}/{accum}")
    sp, masses, vel = _system(32, N, 2, S, dtype)
    o = oracle.OracleCorrelator(6, b, p, m)
    for s in range(S):
        o.push(oracle.partial_momentum(vel[s], sp, masses, box ** 3))
    g = corrmod.GroupDesc(6, b, p, m, dtype=dtype, accum=accum, source="momentum", n_atoms=N,
                          box=box, species=sp, masses=masses)
    with corrmod.Correlator([g]) as c:
        _push_all(c, [vel])
        res = c.finalize(0, slice_=(0, 6))
    e = gate(res, o, TOL[(dtype, accum)], slice_=(0, 6), label="momentum")
    say(f"  error {e:.2e}")


@pytest.mark.parametrize("dtype,accum", [("f32", "kahan"), ("f64", "f64")])
def test_momentum_pair_with_heat_flux_all_launch_modes(corrmod, dtype, accum):
    """Pair group: x = a heat-flux series q (component a for channel 3s + a),
    y = the densities, C(L) = <q(s) j(s - L)>, beside a block-deferred group:
    one stream, forked producers, forked updates and a graph give
    bit-identical results, which match the oracle's pair form."""
    N, S, box, ns = 2500, 400, 9.0, 2
    sp, masses, vel = _system(33, N, ns, S, dtype)
    q = ou_inputs(33, 9, 3, S, dtype)                 # [S][3]
    x = np.ascontiguousarray(np.tile(q, (1, ns)))     # [S][3 ns]
    inp = np.ascontiguousarray(np.concatenate([vel.reshape(S, -1), x], axis=1))
    xv = ou_inputs(33, 4, 3000, S, "f32")
    groups = [corrmod.GroupDesc(3 * ns, 5, 16, 2, dtype=dtype, accum=accum, source="momentum",
                                n_atoms=N, box=box, species=sp, masses=masses, pair=True),
              corrmod.GroupDesc(3000, 5, 16, 2, dtype="f32", accum="kahan")]
    base = dict(tile_channels=256, chans_per_thread=1, lag_chunk=8, grid_blocks=0)
    out = {}
    dev = torch.device("cuda:0")
    for mode in ("serial", "fork", "fork_updates", "graph"):
        say(f"[momentum pair] {dtype} {mode}")
        ov = {"serial": 0, "fork": 1, "fork_updates": 2, "graph": 1}[mode]
        with corrmod.Correlator(groups, graph=(mode == "graph"),
                                tuning=dict(base, overlap_producers=ov)) as c:
            ta, tb = torch.from_numpy(inp).to(dev), torch.from_numpy(xv).to(dev)
            if mode == "graph":
                ba, bb = torch.empty_like(ta[0]), torch.empty_like(tb[0])
                c.bind_input(0, ba)
                c.bind_input(1, bb)
                for s in range(S):
                    ba.copy_(ta[s])
                    bb.copy_(tb[s])
                    c.push()
            else:
                for s in range(S):
                    c.push([ta[s], tb[s]])
            torch.cuda.synchronize()
            out[mode] = c.finalize(0, slice_=(0, 3 * ns))
    for mode in ("fork", "fork_updates", "graph"):
        assert np.array_equal(out[mode]["c_per_channel"], out["serial"]["c_per_channel"]), mode
    o = oracle.OracleCorrelator(3 * ns, 5, 16, 2)
    for s in range(S):
        o.push_pair(x[s].astype(np.float64), oracle.partial_momentum(vel[s], sp, masses, box ** 3))
    e = gate(out["serial"], o, TOL[(dtype, accum)], slice_=(0, 3 * ns), label="momentum pair")
    say(f"  error {e:.2e}")


def test_momentum_full_size_against_oracle(corrmod):
    """The mass-flux workload's size (2 species, 2e7 atoms, the bench's
    launch configuration with the pair form beside a sample-fed group): the
    densities of three pushes against the oracle's, through C(0) and C(1) of
    the autocorrelation and the pair group's C(0) = <q j>."""
    N, box, S = 20_000_000, 600.0, 3
    rng = np.random.default_rng(71)
    sp = rng.integers(0, 2, N).astype(np.int32)
    masses = np.array([6.941, 18.998])
    vel = rng.standard_normal((S, 3, N)).astype(np.float32)
    q = rng.standard_normal((S, 3)).astype(np.float32)
    x = np.ascontiguousarray(np.tile(q, (1, 2)))
    say(f"[momentum full size] N={N}")
    inp = np.ascontiguousarray(np.concatenate([vel.reshape(S, -1), x], axis=1))
    groups = [corrmod.GroupDesc(6, 4, 16, 2, dtype="f32", accum="kahan", source="momentum",
                                n_atoms=N, box=box, species=sp, masses=masses),
              corrmod.GroupDesc(6, 4, 16, 2, dtype="f32", accum="kahan", source="momentum",
                                n_atoms=N, box=box, species=sp, masses=masses, pair=True),
              corrmod.GroupDesc(3000, 4, 16, 2, dtype="f32", accum="kahan")]
    xv = ou_inputs(71, 1, 3000, S, "f32")
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(inp).to(dev)
    tv = ti[:, :3 * N]
    tx = torch.from_numpy(xv).to(dev)
    with corrmod.Correlator(groups, tuning=dict(tile_channels=256, chans_per_thread=1,
                                                lag_chunk=16, grid_blocks=0,
                                                overlap_producers=1)) as c:
        for s in range(S):
            c.push([tv[s], ti[s], tx[s]])
        torch.cuda.synchronize()
        auto = c.finalize(0, slice_=(0, 6))
        pair = c.finalize(1, slice_=(0, 6))
    j = np.stack([oracle.partial_momentum(vel[s], sp, masses, box ** 3) for s in range(S)])
    c0 = np.mean(j * j, axis=0)
    c1 = np.mean(j[1:] * j[:-1], axis=0)
    cq = np.mean(x * j, axis=0)
    e0 = np.max(np.abs(auto["c_per_channel"][:, 0] - c0)) / np.max(np.abs(c0))
    e1 = np.max(np.abs(auto["c_per_channel"][:, 1] - c1)) / np.max(np.abs(c0))
    eq = np.max(np.abs(pair["c_per_channel"][:, 0] - cq)) / np.max(np.abs(cq))
    say(f"  C(0) {e0:.2e}  C(1) {e1:.2e}  <q j> {eq:.2e}")
    assert e0 < 1e-6 and e1 < 1e-6 and eq < 1e-6
