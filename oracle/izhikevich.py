"""FP64 oracle of the Izhikevich neuron and of the 4:1 excitatory/inhibitory
population of Section 5.1's first scalability network.

TEST INFRASTRUCTURE ONLY: the test suite may use it; the product library
never does.  The paper names the model (its reference [9]) but prints none of
its equations or parameters; they are taken from that reference, Izhikevich,
"Simple model of spiking neurons", IEEE Trans. Neural Networks 14 (2003):

    dv/dt = 0.04 v^2 + 5 v + 140 - u + I      (v in mV, t in ms)
    du/dt = a (b v - u)
    if v >= 30 mV:  v <- c,  u <- u + d

with, per neuron and a uniform draw r in [0, 1),
    excitatory: a = 0.02, b = 0.2, c = -65 + 15 r^2, d = 8 - 6 r^2
    inhibitory: a = 0.02 + 0.08 r, b = 0.25 - 0.05 r, c = -65, d = 2
and the initial state v = -65, u = b v.

Reading: the state is advanced by forward Euler with step h on v and u
together (both right-hand sides from the state at the start of the step),
and the threshold is tested after each step; a step that ends at or above
30 mV is a spike and resets the neuron.
"""
from __future__ import annotations

import numpy as np

V_PEAK = 30.0


def params(n_exc, n_inh, r_exc, r_inh):
    """(a, b, c, d) arrays for n_exc excitatory then n_inh inhibitory neurons
    from their uniform draws."""
    re = np.asarray(r_exc, np.float64)
    ri = np.asarray(r_inh, np.float64)
    assert re.size == n_exc and ri.size == n_inh
    a = np.concatenate([np.full(n_exc, 0.02), 0.02 + 0.08 * ri])
    b = np.concatenate([np.full(n_exc, 0.2), 0.25 - 0.05 * ri])
    c = np.concatenate([-65.0 + 15.0 * re * re, np.full(n_inh, -65.0)])
    d = np.concatenate([8.0 - 6.0 * re * re, np.full(n_inh, 2.0)])
    return a, b, c, d


def initial_state(b):
    v = np.full(np.asarray(b).size, -65.0)
    return v, np.asarray(b, np.float64) * v


def step(v, u, i_in, a, b, c, d, h):
    """One forward-Euler step of length h (ms) for every neuron; returns the
    new (v, u) and the boolean spike mask."""
    dv = 0.04 * v * v + 5.0 * v + 140.0 - u + i_in
    du = a * (b * v - u)
    v_new = v + h * dv
    u_new = u + h * du
    spiked = v_new >= V_PEAK
    v_new = np.where(spiked, c, v_new)
    u_new = np.where(spiked, u_new + d, u_new)
    return v_new, u_new, spiked


def run(v, u, i_in, a, b, c, d, h, n_steps):
    """n_steps steps under a constant input current; returns the final
    state and each neuron's spike count."""
    counts = np.zeros(np.asarray(v).size, np.int64)
    for _ in range(n_steps):
        v, u, s = step(v, u, i_in, a, b, c, d, h)
        counts += s
    return v, u, counts
