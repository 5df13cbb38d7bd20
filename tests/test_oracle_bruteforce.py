"""Pin the oracle's Algorithm 1/2 against the brute-force closed definition.

The multiple-tau estimate at level k and lag L equals Eq. (1) (Section 2.2)
applied to the level-k block-averaged series.  A dropped term, a wrong lag
index, a wrong averaging count or a swapped conjugate in the oracle changes
at least one of these values or counts.
"""
import numpy as np
import pytest

from tests.bruteforce import multitau_bruteforce

CASES = [
    # (S, b, p, m)
    (1000, 4, 8, 2),
    (777, 5, 7, 3),   # m does not divide p (floor(p/m) = 2, coinciding lag times)
    (50, 6, 16, 2),
    (3, 3, 4, 2),
    (2000, 3, 9, 4),
    (1, 2, 4, 2),
    (64, 4, 4, 2),
    (300, 8, 16, 2),
    (513, 3, 32, 2),
    (1024, 10, 16, 2),
    (2600, 1, 1000, 2),  # one long window that wraps (the large-p form)
    (1500, 2, 1200, 2),
]


@pytest.mark.parametrize("S,b,p,m", CASES)
@pytest.mark.parametrize("complex_", [False, True])
def test_oracle_matches_bruteforce(oracle_mod, S, b, p, m, complex_):
    rng = np.random.default_rng(1000 * S + 10 * p + m + complex_)
    n_ch = 3
    x = rng.standard_normal((S, n_ch))
    if complex_:
        x = x + 1j * rng.standard_normal((S, n_ch))
    o = oracle_mod.OracleCorrelator(n_ch, b, p, m, complex_=complex_)
    o.push_series(x)
    t_bf, c_bf, n_bf = multitau_bruteforce(x, b, p, m)
    for ch in range(n_ch):
        t, c, n = o.readout(ch, ch + 1)
        assert np.array_equal(t, t_bf), (t, t_bf)
        assert np.array_equal(n, n_bf)
        ref = c_bf[:, ch]
        scale = np.abs(ref).max()
        assert np.max(np.abs(c - ref)) <= 1e-12 * scale
    # group mean over channels
    t, c, n = o.readout()
    ref = c_bf.mean(axis=1)
    assert np.max(np.abs(c - ref)) <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("S,b,p,m", CASES)
def test_counts_closed_form(oracle_mod, S, b, p, m):
    """count_k(L) = max(0, floor(S/m^k) - L) for every (level, lag) of the range."""
    o = oracle_mod.OracleCorrelator(1, b, p, m)
    o.push_series(np.ones((S, 1)))
    _, cnt = o.raw(0)
    for k in range(b):
        Sk = S // m**k
        lag0 = 0 if k == 0 else p // m
        for L in range(p):
            expect = max(0, Sk - L) if L >= lag0 else 0
            assert cnt[k, L] == expect, (k, L, cnt[k, L], expect)


def test_level0_equals_eq1_exactly_ordered(oracle_mod):
    """Level 0 is Eq. (1) itself: integer-valued samples make every sum exact,
    so the values must agree bit for bit."""
    rng = np.random.default_rng(7)
    x = rng.integers(-50, 50, size=(400, 2)).astype(np.float64)
    o = oracle_mod.OracleCorrelator(2, 1, 16, 2)
    o.push_series(x)
    for ch in range(2):
        t, c, n = o.readout(ch, ch + 1)
        for L in range(16):
            s = np.sum(x[L:, ch] * x[: 400 - L, ch])
            assert t[L] == L and n[L] == 400 - L
            assert c[L] == s / (400 - L)


def test_max_lag_and_point_count(oracle_mod):
    """Maximum lag (p-1) m^(b-1) (Section 2.2, reading l = b-1) and the number of
    emitted points p + (b-1)(p - floor(p/m)) once every level is full."""
    for (b, p, m) in [(8, 16, 2), (4, 8, 2), (3, 9, 3), (5, 6, 2)]:
        S = (p + 1) * m ** (b - 1)
        o = oracle_mod.OracleCorrelator(1, b, p, m)
        o.push_series(np.ones((S, 1)))
        t, c, n = o.readout()
        assert t.max() == (p - 1) * m ** (b - 1)
        assert len(t) == p + (b - 1) * (p - p // m)
        if p % m == 0:
            assert np.all(np.diff(t) > 0)


@pytest.mark.parametrize("S,b,p,m", CASES)
@pytest.mark.parametrize("complex_", [False, True])
def test_oracle_pair_matches_bruteforce(oracle_mod, S, b, p, m, complex_):
    """Pair form: C(L) = <x(s) conj(y(s - L))> with both series block-averaged."""
    from tests.bruteforce import multitau_bruteforce_pair
    rng = np.random.default_rng(7000 * S + 10 * p + m + complex_)
    n_ch = 3
    x = rng.standard_normal((S, n_ch))
    y = 0.5 * x + rng.standard_normal((S, n_ch))
    if complex_:
        x = x + 1j * rng.standard_normal((S, n_ch))
        y = y + 1j * rng.standard_normal((S, n_ch))
    o = oracle_mod.OracleCorrelator(n_ch, b, p, m, complex_=complex_)
    for s in range(S):
        o.push_pair(x[s], y[s])
    t_bf, c_bf, n_bf = multitau_bruteforce_pair(x, y, b, p, m)
    for ch in range(n_ch):
        t, c, n = o.readout(ch, ch + 1)
        assert np.array_equal(t, t_bf) and np.array_equal(n, n_bf)
        ref = c_bf[:, ch]
        assert np.max(np.abs(c - ref)) <= 1e-12 * np.abs(ref).max()


def test_oracle_pair_with_itself_is_the_autocorrelation(oracle_mod):
    """pair(x, x) equals the autocorrelation of x bit for bit (same operations
    in the same order), and the roles of x and y are not interchangeable."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((700, 4)) + 1j * rng.standard_normal((700, 4))
    y = rng.standard_normal((700, 4)) + 1j * rng.standard_normal((700, 4))
    a = oracle_mod.OracleCorrelator(4, 5, 16, 2, complex_=True)
    q = oracle_mod.OracleCorrelator(4, 5, 16, 2, complex_=True)
    xy = oracle_mod.OracleCorrelator(4, 5, 16, 2, complex_=True)
    yx = oracle_mod.OracleCorrelator(4, 5, 16, 2, complex_=True)
    for s in range(700):
        a.push(x[s])
        q.push_pair(x[s], x[s])
        xy.push_pair(x[s], y[s])
        yx.push_pair(y[s], x[s])
    ta, ca, na = a.readout()
    tq, cq, nq = q.readout()
    assert np.array_equal(ta, tq) and np.array_equal(na, nq) and np.array_equal(ca, cq)
    # C_xy(0) = conj(C_yx(0)); at L > 0 the two differ (x later vs y later)
    _, cxy, _ = xy.readout()
    _, cyx, _ = yx.readout()
    assert abs(cxy[0] - np.conj(cyx[0])) < 1e-12 * abs(cxy[0])
    assert np.max(np.abs(cxy[1:] - np.conj(cyx[1:]))) > 1e-3
    with pytest.raises(RuntimeError):
        q.push(x[0])  # a pair record takes pairs only
