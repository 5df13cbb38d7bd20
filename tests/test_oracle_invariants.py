"""Exact invariants and hand-worked golden examples that pin the oracle."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_golden(name):
    rows = np.loadtxt(os.path.join(GOLDEN, name), comments="#")
    return rows[:, 0], rows[:, 1].astype(np.int64), rows[:, 2] + 1j * rows[:, 3]


def test_golden_real(oracle_mod):
    t_g, n_g, c_g = _load_golden("handworked_real_b3_p4_m2.txt")
    o = oracle_mod.OracleCorrelator(1, 3, 4, 2)
    o.push_series(np.arange(1, 9, dtype=np.float64)[:, None])
    t, c, n = o.readout()
    assert np.array_equal(t, t_g)
    assert np.array_equal(n, n_g)
    assert np.allclose(c, c_g.real, rtol=1e-15, atol=0)


def test_golden_complex(oracle_mod):
    t_g, n_g, c_g = _load_golden("handworked_complex_b1_p4.txt")
    o = oracle_mod.OracleCorrelator(1, 1, 4, 2, complex_=True)
    o.push_series(np.array([1, 1j, -1, -1j])[:, None])
    t, c, n = o.readout()
    assert np.array_equal(t, t_g) and np.array_equal(n, n_g)
    assert np.array_equal(c, c_g)


@pytest.mark.parametrize("b,p,m,S", [(6, 16, 2, 1000), (4, 8, 2, 333), (3, 9, 3, 500)])
def test_constant_series(oracle_mod, b, p, m, S):
    """A constant c gives C = c^2 at every level and lag (block means of a
    constant are the constant).  c = 0.75 keeps every sum exact."""
    c0 = 0.75
    o = oracle_mod.OracleCorrelator(2, b, p, m)
    o.push_series(np.full((S, 2), c0))
    t, c, n = o.readout()
    assert np.all(c == c0 * c0)


def test_alternating_series(oracle_mod):
    """x_s = (-1)^s: level 0 gives (-1)^L exactly; with m = 2 every block mean is
    0, so all coarser levels give exactly 0."""
    S, b, p = 1000, 6, 16
    x = np.array([(-1.0) ** s for s in range(S)])[:, None]
    o = oracle_mod.OracleCorrelator(1, b, p, 2)
    o.push_series(x)
    t, c, n = o.readout()
    lvl0 = t < p
    assert np.array_equal(c[lvl0], np.array([(-1.0) ** L for L in range(p)]))
    assert np.all(c[~lvl0] == 0.0)


def test_impulse(oracle_mod):
    """A single unit impulse: level 0 has C(0) = 1/S and C(L>0) = 0."""
    S, p = 100, 8
    x = np.zeros((S, 1))
    x[37, 0] = 1.0
    o = oracle_mod.OracleCorrelator(1, 1, p, 2)
    o.push_series(x)
    t, c, n = o.readout()
    assert c[0] == 1.0 / S
    assert np.all(c[1:] == 0.0)


def test_scaling_by_power_of_two(oracle_mod):
    """Scaling the input by 2^j scales every C by 4^j exactly."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((500, 2))
    o1 = oracle_mod.OracleCorrelator(2, 5, 16, 2)
    o2 = oracle_mod.OracleCorrelator(2, 5, 16, 2)
    o1.push_series(x)
    o2.push_series(x * 8.0)
    _, c1, _ = o1.readout()
    _, c2, _ = o2.readout()
    assert np.array_equal(c2, c1 * 64.0)


def test_c0_is_mean_of_squares(oracle_mod):
    rng = np.random.default_rng(11)
    x = rng.standard_normal((777, 4))
    o = oracle_mod.OracleCorrelator(4, 4, 16, 2)
    o.push_series(x)
    for ch in range(4):
        t, c, n = o.readout(ch, ch + 1)
        assert t[0] == 0 and n[0] == 777
        assert abs(c[0] - np.mean(x[:, ch] ** 2)) <= 1e-14 * c[0]


def test_complex_symmetry(oracle_mod):
    """Conjugating the input conjugates every C; a real series gives a real C."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((300, 2)) + 1j * rng.standard_normal((300, 2))
    o1 = oracle_mod.OracleCorrelator(2, 4, 8, 2, complex_=True)
    o2 = oracle_mod.OracleCorrelator(2, 4, 8, 2, complex_=True)
    o1.push_series(x)
    o2.push_series(np.conj(x))
    _, c1, _ = o1.readout()
    _, c2, _ = o2.readout()
    assert np.allclose(c2, np.conj(c1), rtol=0, atol=1e-15)


def test_trapezoid_closed_forms(oracle_mod):
    """Trapezoid rule (reading R14) is exact for piecewise-linear data; a cut-off
    inside an interval interpolates C linearly."""
    t = np.array([0.0, 1.0, 3.0, 7.0])
    c = np.array([2.0, 1.0, 1.0, -1.0])
    run, at = oracle_mod.trapezoid(t, c)
    assert np.array_equal(run, [0.0, 1.5, 3.5, 3.5])
    assert at == 3.5
    _, at_mid = oracle_mod.trapezoid(t, c, t_cut=5.0)   # C(5) = 0
    assert at_mid == 3.5 + 0.5 * 2.0 * (1.0 + 0.0)
    _, at0 = oracle_mod.trapezoid(t, c, t_cut=0.0)
    assert at0 == 0.0
    # integral of exp(-t) on a fine grid -> 1 within the trapezoid error h^2/12
    tt = np.linspace(0, 40, 40001)
    _, at = oracle_mod.trapezoid(tt, np.exp(-tt))
    assert abs(at - (1 - np.exp(-40))) < 1e-3 ** 2 / 12 * 1.01


def test_green_kubo_prefactors(oracle_mod):
    """Eq. (viscosity) and Eq. (thermal conductivity) prefactors on a constant C."""
    t = np.array([0.0, 2.0])
    c = np.array([3.0, 3.0])
    _, eta = oracle_mod.green_kubo_viscosity(t, c, volume=10.0, kB=2.0, temperature=5.0)
    assert eta == 10.0 / (2.0 * 5.0) * 6.0
    _, kap = oracle_mod.green_kubo_conductivity(t, c, volume=10.0, kB=2.0, temperature=5.0)
    assert np.isclose(kap, 10.0 / (3 * 2.0 * 25.0) * 3 * 6.0, rtol=1e-15)


def test_conductivity_from_the_component_sum(oracle_mod):
    """Reading R16 pinned independently of the oracle's prefactor: the heat
    flux autocorrelation in Eq. (thermal conductivity) is the dot product
    <q(t).q(0)> = sum over x, y, z of the component autocorrelations.  Here it
    is formed directly from a 3-component series with numpy dot products (one
    level, so every lag is Eq. (1) exactly), and from three one-channel oracle
    readouts summed; its trapezoid integral (numpy) times V/(3 kB T^2) must
    equal green_kubo_conductivity on the mean of the three channels."""
    rng = np.random.default_rng(2503)
    S, p = 600, 48
    q = np.zeros((S, 3))
    for s in range(1, S):  # correlated components of unequal variance
        q[s] = 0.9 * q[s - 1] + rng.standard_normal(3) * np.array([1.0, 2.0, 0.5])
    o = oracle_mod.OracleCorrelator(3, 1, p, 2)
    o.push_series(q)
    t, c_mean, n = o.readout()
    lags = np.arange(len(t))
    dot = np.array([np.einsum("ij,ij->", q[L:], q[:S - L]) / (S - L) for L in lags])
    comp = np.zeros(len(t))
    for a in range(3):
        oa = oracle_mod.OracleCorrelator(1, 1, p, 2)
        oa.push_series(q[:, a:a + 1])
        comp += oa.readout()[1]
    assert np.allclose(comp, dot, rtol=1e-12, atol=0)
    V, kB, T = 27.0, 1.380649e-23, 300.0
    integ = getattr(np, "trapezoid", None) or np.trapz
    kappa_direct = V / (3 * kB * T * T) * float(integ(dot, t))
    _, kappa = oracle_mod.green_kubo_conductivity(t, c_mean, volume=V, kB=kB, temperature=T)
    assert np.isclose(kappa, kappa_direct, rtol=1e-12, atol=0), (kappa, kappa_direct)
    # and with several levels: three one-channel readouts summed = 3 x the mean
    o3 = oracle_mod.OracleCorrelator(3, 4, 16, 2)
    o3.push_series(q)
    t3, c3, _ = o3.readout()
    s3 = np.zeros(len(t3))
    for a in range(3):
        oa = oracle_mod.OracleCorrelator(1, 4, 16, 2)
        oa.push_series(q[:, a:a + 1])
        s3 += oa.readout()[1]
    assert np.allclose(s3, 3 * c3, rtol=1e-13, atol=1e-13 * abs(s3[0]))
