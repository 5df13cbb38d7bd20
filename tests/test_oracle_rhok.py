"""Pins of the oracle's k-space density n(k) = sum_j exp(i k.r_j), k = 2 pi n/L
(Section "Currents", Eq. k-density)."""
import numpy as np


def test_all_atoms_at_one_point(oracle_mod, synth_mod):
    """All N atoms at r: n(k) = N exp(i k.r)."""
    kv = synth_mod.kvectors(64)
    N, box = 50, 100.0
    r = np.array([12.5, 50.0, 75.0], dtype=np.float32)
    pos = np.repeat(r[:, None], N, axis=1)
    got = oracle_mod.rhok(pos, kv, box)
    ph = 2 * np.pi * (kv @ r.astype(np.float64)) / box
    assert np.allclose(got, N * np.exp(1j * ph), rtol=0, atol=1e-11 * N)


def test_cubic_grid_selection_rule(oracle_mod, synth_mod):
    """G^3 atoms on a simple cubic grid of spacing L/G: n(k) = G^3 when every
    component of n is a multiple of G, else 0."""
    G, box = 4, 100.0
    g = (np.arange(G) * (box / G)).astype(np.float32)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    kv = synth_mod.kvectors(600)
    got = oracle_mod.rhok(pos, kv, box)
    sel = np.all(kv % G == 0, axis=1)
    assert sel.any() and (~sel).any()
    assert np.allclose(got[sel], G**3, rtol=0, atol=1e-9)
    assert np.max(np.abs(got[~sel])) < 1e-9


def test_mirror_conjugates(oracle_mod, synth_mod):
    """Reflecting every position through the origin conjugates n(k)."""
    rng = np.random.default_rng(2)
    pos = (rng.random((3, 200)) * 100.0).astype(np.float32)
    kv = synth_mod.kvectors(100)
    a = oracle_mod.rhok(pos, kv, 100.0)
    b = oracle_mod.rhok(-pos, kv, 100.0)
    assert np.allclose(b, np.conj(a), rtol=0, atol=1e-10)


def test_kvector_set(synth_mod):
    """The 2048 k-vectors: distinct, half-space, 0 < |n|^2 <= 99 (<= 12^2), sorted."""
    kv = synth_mod.kvectors(2048)
    n2 = (kv.astype(np.int64) ** 2).sum(1)
    assert len({tuple(v) for v in kv}) == 2048
    assert n2.min() > 0 and n2.max() == 99
    assert np.all(np.diff(n2) >= 0)
    first = np.where(kv[:, 0] != 0, kv[:, 0], np.where(kv[:, 1] != 0, kv[:, 1], kv[:, 2]))
    assert np.all(first > 0)
