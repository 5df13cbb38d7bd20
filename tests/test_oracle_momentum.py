"""Pins of the oracle's partial momentum densities (the mass-flux correction of
Section "Viscosity and thermal conductivity"; reading R22 of
oracle/corr_oracle.c) against facts the definition fixes, independent of the
function's own loop: a hand-worked example, the total momentum computed from
per-atom masses in one dot product, momentum conservation of a binary
system, invariance under atom order, relabelled species, linearity and the
1/V scaling."""
import numpy as np
import pytest

import oracle


def test_hand_worked_example():
    # atoms: (1, 0, 0) species 0, (0, 2, 0) species 1, (3, 0, -1) species 0;
    # masses 2 and 5, V = 10: j_0 = 2 (4, 0, -1) / 10, j_1 = 5 (0, 2, 0) / 10
    v = np.array([[1.0, 0.0, 3.0], [0.0, 2.0, 0.0], [0.0, 0.0, -1.0]])
    j = oracle.partial_momentum(v, [0, 1, 0], [2.0, 5.0], 10.0)
    np.testing.assert_array_equal(j, [0.8, 0.0, -0.2, 0.0, 1.0, 0.0])


def _system(seed, n, n_species):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3, n))
    sp = rng.integers(0, n_species, n).astype(np.int32)
    masses = rng.uniform(1.0, 40.0, n_species)
    return v, sp, masses


def test_species_sum_is_the_total_momentum_density():
    v, sp, masses = _system(1, 5000, 3)
    j = oracle.partial_momentum(v, sp, masses, 123.0).reshape(3, 3)
    total = (v @ masses[sp]) / 123.0  # per-atom masses, one dot product per component
    np.testing.assert_allclose(j.sum(axis=0), total, rtol=1e-12, atol=1e-12)


def test_binary_system_at_rest_has_opposite_densities():
    v, sp, masses = _system(2, 4000, 2)
    m = masses[sp]
    v -= (v @ m / m.sum())[:, None]  # remove the centre-of-mass velocity
    j = oracle.partial_momentum(v, sp, masses, 50.0).reshape(2, 3)
    scale = np.abs(j).max()
    np.testing.assert_allclose(j[0], -j[1], atol=1e-12 * scale * 4000)


def test_atom_order_and_species_labels():
    v, sp, masses = _system(3, 3000, 4)
    j = oracle.partial_momentum(v, sp, masses, 7.0).reshape(4, 3)
    perm = np.random.default_rng(4).permutation(3000)
    jp = oracle.partial_momentum(v[:, perm], sp[perm], masses, 7.0).reshape(4, 3)
    np.testing.assert_allclose(jp, j, rtol=1e-12, atol=1e-12)
    relabel = np.array([2, 0, 3, 1])  # species s becomes relabel[s]
    m2 = np.empty(4)
    m2[relabel] = masses
    jr = oracle.partial_momentum(v, relabel[sp], m2, 7.0).reshape(4, 3)
    np.testing.assert_allclose(jr[relabel], j, rtol=1e-12, atol=1e-12)


def test_linearity_and_volume_scaling():
    v1, sp, masses = _system(5, 2000, 2)
    v2 = np.random.default_rng(6).standard_normal(v1.shape)
    a = oracle.partial_momentum(v1, sp, masses, 3.0)
    b = oracle.partial_momentum(v2, sp, masses, 3.0)
    ab = oracle.partial_momentum(2.0 * v1 - v2, sp, masses, 3.0)
    np.testing.assert_allclose(ab, 2.0 * a - b, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(oracle.partial_momentum(v1, sp, masses, 6.0), a / 2.0,
                               rtol=1e-14)


def test_single_species_is_mass_times_velocity_sum():
    v, _, _ = _system(7, 1000, 1)
    j = oracle.partial_momentum(v, np.zeros(1000, np.int32), [4.0], 2.0)
    np.testing.assert_allclose(j, 2.0 * v.sum(axis=1), rtol=1e-12)


def test_empty_species_gives_zero_and_bad_ids_are_rejected():
    v, _, _ = _system(8, 10, 1)
    j = oracle.partial_momentum(v, np.zeros(10, np.int32), [1.0, 2.0], 1.0)
    np.testing.assert_array_equal(j[3:], 0.0)
    with pytest.raises(ValueError):
        oracle.partial_momentum(v, np.full(10, 2, np.int32), [1.0, 2.0], 1.0)
