"""Host-side checks of the C ABI (no GPU compute): the library loads, exports
every entry point declared in include/corr.h, and rejects invalid descriptors
before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "corr.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(corr_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def corrmod():
    import paper_2503_07526_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("HIP library not built (run __graft_entry__.build())")
    return m


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("corr_create", "corr_push", "corr_finalize", "corr_destroy", "corr_input_buffer"):
        assert n in names


def test_library_exports_every_declared_symbol(corrmod):
    L = ctypes.CDLL(corrmod.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(corrmod.EXPORTS) == _declared()


def test_library_is_gfx950_only(corrmod):
    data = open(corrmod.LIB_PATH, "rb").read()
    assert b"gfx950" in data
    for other in (b"gfx942", b"gfx90a", b"gfx1100"):
        assert other not in data


def _create(corrmod, desc, tuning=None):
    L = corrmod.lib()
    arr = (corrmod.corr._GroupDesc * 1)(desc.to_c())
    h = ctypes.c_void_p()
    tn = corrmod.Tuning(**tuning) if tuning else None
    rc = L.corr_create(arr, 1, 0, None, 0, ctypes.byref(tn) if tn else None, ctypes.byref(h))
    return rc, L.corr_last_error(None).decode()


@pytest.mark.parametrize("kw,needle", [
    (dict(n_channels=0, levels=4, points=16), "n_channels"),
    (dict(n_channels=8, levels=0, points=16), "levels"),
    (dict(n_channels=8, levels=4, points=1), "points"),
    (dict(n_channels=8, levels=4, points=16, m=1), "m must be >= 2"),
    (dict(n_channels=8, levels=4, points=16, m=16), "m must be < p"),
    (dict(n_channels=8, levels=4, points=16, update_every=0), "update_every"),
    (dict(n_channels=8, levels=4, points=16, dtype="f64", accum="kahan"), "double samples"),
    (dict(n_channels=8, levels=4, points=16, dtype="cf32", source="rhok"), "k-density"),
])
def test_invalid_descriptors_rejected(corrmod, kw, needle):
    rc, msg = _create(corrmod, corrmod.GroupDesc(**kw))
    assert rc == -1, (rc, msg)
    assert needle in msg


def test_rhok_descriptor_needs_positions_and_box(corrmod):
    kv = np.array([[1, 0, 0]], dtype=np.int32)
    rc, msg = _create(corrmod, corrmod.GroupDesc(1, 4, 16, dtype="cf32", source="rhok", kvec=kv,
                                                 n_atoms=0, box=10.0))
    assert rc == -1 and "n_atoms" in msg
    rc, msg = _create(corrmod, corrmod.GroupDesc(1, 4, 16, dtype="cf32", source="rhok", kvec=kv,
                                                 n_atoms=10, box=0.0))
    assert rc == -1 and "box" in msg


@pytest.mark.parametrize("kv,n_channels,rc_want,needle", [
    ([[1, 0, 0], [0, 0, 0]], 6, -1, "zero k-vector"),
    ([[1, 0, 0], [16, 0, 0]], 6, -5, "+-15"),
    ([[1, 0, 0]], 4, -1, "3 x k-vectors"),
])
def test_currents_descriptor_checks(corrmod, kv, n_channels, rc_want, needle):
    rc, msg = _create(corrmod, corrmod.GroupDesc(n_channels, 4, 16, dtype="cf32",
                                                 source="currents",
                                                 kvec=np.array(kv, dtype=np.int32),
                                                 n_atoms=10, box=10.0))
    assert rc == rc_want and needle in msg, (rc, msg)


@pytest.mark.parametrize("tuning", [
    dict(tile_channels=100, chans_per_thread=1, lag_chunk=16, grid_blocks=0),
    dict(tile_channels=256, chans_per_thread=3, lag_chunk=8, grid_blocks=0),
    dict(tile_channels=4096, chans_per_thread=1, lag_chunk=16, grid_blocks=0),
    dict(tile_channels=512, chans_per_thread=1, lag_chunk=16, grid_blocks=0),
    dict(tile_channels=2048, chans_per_thread=4, lag_chunk=4, grid_blocks=0),
    dict(tile_channels=256, chans_per_thread=1, lag_chunk=8, grid_blocks=0, overlap_producers=3),
    dict(tile_channels=256, chans_per_thread=1, lag_chunk=8, grid_blocks=0, overlap_producers=-1),
])
def test_invalid_tuning_rejected(corrmod, tuning):
    rc, msg = _create(corrmod, corrmod.GroupDesc(64, 4, 16), tuning)
    assert rc == -1 and "tuning" in msg


def test_null_arguments(corrmod):
    L = corrmod.lib()
    assert L.corr_push(None, None) == -1
    assert L.corr_sync(None) == -1
    assert L.corr_destroy(None) == -1
    assert isinstance(L.corr_last_error(None), bytes)


def test_pair_descriptor_checks(corrmod):
    kv = np.array([[1, 0, 0]], dtype=np.int32)
    rc, msg = _create(corrmod, corrmod.GroupDesc(1, 4, 16, dtype="cf32", source="rhok", kvec=kv,
                                                 n_atoms=10, box=10.0, pair=True))
    assert rc == -1 and "pair" in msg


def _mom(n_channels=6, n_atoms=10, box=10.0, dtype="f32", species=None, masses=(1.0, 2.0),
         **kw):
    sp = (np.zeros(n_atoms, np.int32) if species is None else
          None if isinstance(species, str) else np.asarray(species, np.int32))
    return dict(n_channels=n_channels, levels=4, points=16, dtype=dtype, source="momentum",
                n_atoms=n_atoms, box=box, species=sp,
                masses=None if masses is None else np.asarray(masses, np.float64), **kw)


@pytest.mark.parametrize("kw,needle", [
    (_mom(dtype="cf32"), "real dtype"),
    (_mom(n_channels=5), "3 x n_species"),
    (_mom(n_channels=27, masses=[1.0] * 9), "n_species"),
    (_mom(species="none"), "species or masses"),
    (_mom(masses=None), "n_species"),
    (_mom(n_atoms=0, species=np.zeros(1, np.int32)), "n_atoms"),
    (_mom(box=0.0), "box"),
    (_mom(species=[0] * 9 + [2]), "out of range"),
    (_mom(species=[0] * 9 + [-1]), "out of range"),
    (_mom(masses=[1.0, float("nan")]), "finite"),
])
def test_momentum_descriptor_checks(corrmod, kw, needle):
    """Partial momentum density groups: a real dtype, 3 channels per species,
    1..8 species with ids in range, finite masses, atoms and a box."""
    rc, msg = _create(corrmod, corrmod.GroupDesc(**kw))
    assert rc == -1 and needle in msg, (rc, msg)


def test_missing_library_fails_loudly(corrmod, monkeypatch, tmp_path):
    """No fallback: without the built HIP library every entry point raises."""
    import paper_2503_07526_amd.corr as c
    monkeypatch.setattr(c, "_lib", None)
    monkeypatch.setattr(c, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        c.lib()
    with pytest.raises(ImportError):
        c.Correlator([c.GroupDesc(8, 4, 16)])
