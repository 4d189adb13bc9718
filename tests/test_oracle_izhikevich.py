"""Pins of the Izhikevich neuron oracle (the model of Section 5.1's first
network, reference [9]) against closed forms of the model: its fixed points,
the input at which they vanish (saddle-node), the exact reset, and the
monotone frequency-current relation."""
import math

import numpy as np
import pytest

from oracle import izhikevich as iz


def fixed_points(b, i_in):
    # u = b v and 0.04 v^2 + (5 - b) v + 140 + I = 0
    disc = (5.0 - b) ** 2 - 0.16 * (140.0 + i_in)
    if disc < 0:
        return None
    r = math.sqrt(disc)
    return (-(5.0 - b) - r) / 0.08, (-(5.0 - b) + r) / 0.08


def one(a=0.02, b=0.2, c=-65.0, d=8.0):
    return [np.array([x], np.float64) for x in (a, b, c, d)]


def test_regular_spiking_rest_is_minus_70():
    lo, hi = fixed_points(0.2, 0.0)
    assert lo == pytest.approx(-70.0) and hi == pytest.approx(-50.0)
    a, b, c, d = one()
    v, u, n = iz.run(np.array([-70.0]), np.array([-14.0]), 0.0, a, b, c, d, 0.1, 5000)
    assert n[0] == 0
    assert v[0] == pytest.approx(-70.0, abs=1e-12) and u[0] == pytest.approx(-14.0, abs=1e-12)


def test_relaxes_to_the_stable_fixed_point_below_rheobase():
    # below I = (5 - b)^2 / 0.16 - 140 (= 4 for b = 0.2) the lower fixed point
    # exists; a step of I from rest small enough that v keeps a fixed point
    # while u lags (0.04 v^2 + 5 v + 154 + I = 0 solvable: I <= 2.25) relaxes
    # onto it without a spike
    a, b, c, d = one()
    for i_in in (0.0, 1.0, 2.0):
        v, u, n = iz.run(np.array([-70.0]), np.array([-14.0]), i_in, a, b, c, d, 0.1, 40000)
        lo, _ = fixed_points(0.2, i_in)
        assert n[0] == 0
        assert v[0] == pytest.approx(lo, abs=1e-6) and u[0] == pytest.approx(0.2 * lo, abs=1e-6)


def test_spikes_above_rheobase():
    assert fixed_points(0.2, 4.0 + 1e-9) is None
    a, b, c, d = one()
    v0, u0 = iz.initial_state(b)
    _, _, n = iz.run(v0, u0, 4.5, a, b, c, d, 0.1, 40000)
    assert n[0] > 0


def test_reset_is_exact():
    a, b, c, d = one(c=-55.0, d=4.0)
    v, u, s = iz.step(np.array([29.0]), np.array([-10.0]), 100.0, a, b, c, d, 0.1)
    assert s[0] and v[0] == -55.0
    # u took its Euler step from the pre-reset state, then gained d
    assert u[0] == -10.0 + 0.1 * 0.02 * (0.2 * 29.0 + 10.0) + 4.0
    v, u, s = iz.step(np.array([-60.0]), np.array([-12.0]), 0.0, a, b, c, d, 0.1)
    assert not s[0] and v[0] == -60.0 + 0.1 * (0.04 * 3600.0 - 300.0 + 140.0 + 12.0)


def test_frequency_current_relation_is_monotone():
    a, b, c, d = one()
    counts = []
    for i_in in (5.0, 7.0, 10.0, 15.0, 20.0):
        v0, u0 = iz.initial_state(b)
        counts.append(int(iz.run(v0, u0, i_in, a, b, c, d, 0.1, 10000)[2][0]))
    assert counts[0] > 0 and all(x < y for x, y in zip(counts, counts[1:]))


def test_parameters_of_the_4_to_1_population():
    rng = np.random.default_rng(3)
    re, ri = rng.random(800), rng.random(200)
    a, b, c, d = iz.params(800, 200, re, ri)
    assert np.all(a[:800] == 0.02) and np.all(b[:800] == 0.2)
    assert np.all((c[:800] >= -65.0) & (c[:800] < -50.0)) and np.all((d[:800] > 2.0) & (d[:800] <= 8.0))
    assert np.all((a[800:] >= 0.02) & (a[800:] < 0.1)) and np.all((b[800:] > 0.2) & (b[800:] <= 0.25))
    assert np.all(c[800:] == -65.0) and np.all(d[800:] == 2.0)
    # r = 0 gives the regular-spiking and the fast-spiking-like corner cases
    a, b, c, d = iz.params(1, 1, [0.0], [1.0 - 2 ** -53])
    assert (a[0], b[0], c[0], d[0]) == (0.02, 0.2, -65.0, 8.0)
    assert a[1] == pytest.approx(0.1) and b[1] == pytest.approx(0.2)
    v, u = iz.initial_state(b)
    assert np.all(v == -65.0) and np.allclose(u, b * -65.0)
