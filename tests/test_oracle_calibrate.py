"""Pins of the calibration oracle (Section 5.1, Fig. 1, Tables 1 and 2)
against facts that do not come from the oracle itself: the coefficients the
paper prints, hand-worked selections and percentages, the first-order
optimality conditions of the least-squares problem, a brute-force scan of
its objective, and a textbook straight-line fit."""
import os

import numpy as np
import pytest

from oracle import calibrate as cal

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gscale_law_tables.txt")


def paper_laws():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, k1, k2, k3, a, b, s = line.split()
        rows.append((name, (float(k1), float(k2), float(k3)), np.arange(float(a), float(b) + 1e-9, float(s))))
    return rows


@pytest.mark.parametrize("name,k,x", paper_laws(), ids=[r[0] for r in paper_laws()])
def test_fit_recovers_printed_coefficients(name, k, x):
    # points on the paper's product form (gScale - k3)(nConn + k2) = k1
    y = k[2] + k[0] / (x + k[1])
    got = cal.fit(x, y)
    np.testing.assert_allclose(got, k, rtol=1e-7, atol=1e-12)
    assert cal.mape(got, x, y) < 1e-6


def test_law_limits_table1():
    # Table 1 at nConn = 0: 1318 / 109.9 - 0.28 = 11.712720...; far out it tends to k3
    k = (1.318e3, 1.099e2, -2.800e-1)
    assert cal.law(k, [0.0])[0] == pytest.approx(11.7127206551, rel=1e-10)
    assert cal.law(k, [1e12])[0] == pytest.approx(-0.28, abs=1e-8)
    assert cal.law(k, [1000.0])[0] == pytest.approx(0.9074943688, rel=1e-9)


def test_mape_hand_example():
    # k1 = 0 makes the law the constant k3 = 2; against 1, 2, 4 the errors
    # are 100%, 0% and 50%, so the mean is 50%
    assert cal.mape((0.0, 1.0, 2.0), [1.0, 2.0, 3.0], [1.0, 2.0, 4.0]) == pytest.approx(50.0)


def noisy(seed, k=(1.318e3, 1.099e2, -2.800e-1), rel=0.03):
    rng = np.random.default_rng(seed)
    x = np.arange(100.0, 1001.0, 50.0)
    return x, (k[2] + k[0] / (x + k[1])) * (1.0 + rel * rng.standard_normal(x.size))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fit_is_stationary(seed):
    # gradient of the sum of squares, differentiated by hand, vanishes at the fit
    x, y = noisy(seed)
    k1, k2, k3 = cal.fit(x, y)
    r = k1 / (k2 + x) + k3 - y
    grad = np.array([np.sum(r / (k2 + x)), -np.sum(r * k1 / (k2 + x) ** 2), np.sum(r)])
    scale = np.array([np.sum(np.abs(r / (k2 + x))), np.sum(np.abs(r * k1 / (k2 + x) ** 2)), np.sum(np.abs(r))])
    assert np.all(np.abs(grad) <= 1e-6 * scale)


@pytest.mark.parametrize("seed", [1, 4])
def test_fit_beats_a_brute_force_scan(seed):
    x, y = noisy(seed)
    k = cal.fit(x, y)
    best = cal.sse(k, x, y)
    k2s = k[1] + np.linspace(-60.0, 60.0, 61)
    k2s = k2s[k2s > -x.min() + 1.0]
    for k1 in k[0] * np.linspace(0.8, 1.2, 41):
        for k3 in k[2] + np.linspace(-0.2, 0.2, 41):
            r = k1 / (k2s[:, None] + x[None, :]) + k3 - y[None, :]
            assert np.min(np.sum(r * r, axis=1)) >= best * (1.0 - 1e-12)


def test_conditional_line_fit_matches_polyfit():
    # at the fitted k2 the law is a straight line in u = 1/(k2 + nConn), so
    # k1 and k3 are that line's least-squares slope and intercept
    x, y = noisy(5)
    k = cal.fit(x, y)
    slope, icpt = np.polyfit(1.0 / (k[1] + x), y, 1)
    np.testing.assert_allclose([slope, icpt], [k[0], k[2]], rtol=1e-6, atol=1e-9)


def test_fit_needs_three_distinct_nconn():
    with pytest.raises(ValueError):
        cal.fit([100.0, 100.0, 200.0, 200.0], [1.0, 1.1, 0.5, 0.6])


def test_selection_hand_table():
    # runs: nConn, gScale, avgSpike, NaNs; reference run 4 (avgSpike 10)
    table = [
        (100, 0.5, 3.0, 0),    # 0
        (100, 1.0, 9.0, 0),    # 1  |d| = 1
        (100, 2.0, 11.0, 0),   # 2  |d| = 1, larger gScale: loses the tie to run 1
        (200, 0.5, 10.5, 0),   # 3
        (200, 1.0, 10.0, 0),   # 4  reference, |d| = 0
        (200, 2.0, 10.0, 3),   # 5  NaNs: excluded although |d| = 0
        (300, 0.25, 10.0, 2),  # 6  NaNs
        (300, 0.5, np.nan, 0), # 7  non-finite count: excluded
        (150, 0.25, 4.0, 0),   # 8  only run of its nConn
        (150, 0.5, 16.0, 0),   # 9  |d| = 6 = |4 - 10|, larger gScale: loses to run 8
    ]
    n, g, a, z = (list(c) for c in zip(*table))
    groups, picked = cal.select(n, g, a, z, 4)
    assert list(groups) == [100.0, 150.0, 200.0, 300.0]
    assert list(picked) == [1, 8, 4, -1]


def test_selection_tie_on_equal_gscale_takes_earlier_run():
    groups, picked = cal.select([5, 5, 5], [1.0, 1.0, 1.0], [2.0, 3.0, 3.0], [0, 0, 0], 0)
    assert list(picked) == [0]
    groups, picked = cal.select([5, 5, 7, 7], [1.0, 1.0, 2.0, 2.0], [2.0, 3.0, 1.0, 3.0], [0, 0, 0, 0], 0)
    assert list(picked) == [0, 2]


def test_selection_rejects_nan_reference():
    with pytest.raises(ValueError):
        cal.select([1, 2], [1.0, 1.0], [1.0, 2.0], [1, 0], 0)
