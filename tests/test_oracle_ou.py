"""Statistical pins of the oracle on Ornstein-Uhlenbeck inputs.

For a stationary discrete OU series x' = a x + b xi (unit-variance iid xi) the
autocorrelation is var * a^L with var = b^2 / (1 - a^2); block means of
M = m^k samples have the closed-form covariance in tests/bruteforce.py.  The
Green-Kubo integral of var * exp(-t/tau) is var * tau (Section 2.3, Eqs. for
viscosity and thermal conductivity).  Every emitted point of the oracle run on
3000 channels x 10^4 steps (the tiny plain workload: 8 levels, 16 points,
m = 2, tau = 50) must lie within 5 standard errors (estimated from 30
independent channel batches) of its expectation.
"""
import numpy as np
import pytest

from tests.bruteforce import ou_level_expectation

N_CH, S, B, P, M, TAU = 3000, 10_000, 8, 16, 2, 50.0


@pytest.fixture(scope="module")
def ou_run(oracle_mod, synth_mod):
    spec = synth_mod.OUSpec.make(seed=0, stream=1, n=N_CH, tau=TAU, sigma=1.0, dtype=np.float64)
    x, _ = spec.series(0, S)
    o = oracle_mod.OracleCorrelator(N_CH, B, P, M)
    o.push_series(x)
    per_ch = []
    for ch in range(N_CH):
        t, c, n = o.readout(ch, ch + 1)
        per_ch.append(c)
    per_ch = np.array(per_ch)  # [ch][n_out]
    a = float(spec.a[0])
    var = float(synth_mod.stationary_variance(spec.a[0], spec.b[0]))
    return t, n, per_ch, a, var


def _levels_lags(t):
    out = []
    for tt in t:
        k = 0
        while tt >= P * M**k and k < B - 1:
            k += 1
        out.append((k, int(tt) // M**k))
    return out


def test_ou_levels_match_closed_form(ou_run):
    t, n, per_ch, a, var = ou_run
    batches = per_ch.reshape(30, -1, per_ch.shape[1]).mean(axis=1)
    mean = per_ch.mean(axis=0)
    se = batches.std(axis=0, ddof=1) / np.sqrt(batches.shape[0])
    expect = np.array([ou_level_expectation(a, var, k, M, L) for (k, L) in _levels_lags(t)])
    z = (mean - expect) / se
    assert np.max(np.abs(z)) < 5.0, np.max(np.abs(z))
    # C(0) is the variance
    assert abs(mean[0] - var) < 5 * se[0]


def test_ou_green_kubo(oracle_mod, ou_run):
    t, n, per_ch, a, var = ou_run
    gk_ch = np.array([oracle_mod.trapezoid(t, c)[1] for c in per_ch])
    batches = gk_ch.reshape(30, -1).mean(axis=1)
    se = batches.std(ddof=1) / np.sqrt(len(batches))
    expect_grid = np.array([ou_level_expectation(a, var, k, M, L) for (k, L) in _levels_lags(t)])
    gk_grid = oracle_mod.trapezoid(t, expect_grid)[1]
    assert abs(gk_ch.mean() - gk_grid) < 5 * se
    # the grid-expected integral is within 1% of var * tau_eff, tau_eff = -1/ln(a)
    tau_eff = -1.0 / np.log(a)
    tail = var * tau_eff * np.exp(-t[-1] / tau_eff)   # integral beyond the last lag
    assert abs(gk_grid + tail - var * tau_eff) / (var * tau_eff) < 1e-2
