"""Hand-derived values that tie the oracle's Traub-Miles kinetics to the
published model, and a checker that reports which of them a build of the
oracle violates.

Every literal below is worked out from the model's constants alone, at
voltages where a rate's exponent is exactly +1 or -1, so that the slope
divisors (not only the offsets) are fixed; the ionic current is evaluated at
gate values where m^3 h and n^4 differ from every neighbouring power; the
resting point (the stable root of the steady-state membrane current) comes
from an independent computation of the same published kinetics.
"""
import math

E = math.e

# rate name -> (V in mV, exact value in 1/ms)
RATE_POINTS = {
    "orc_alpha_m": [(-56.0, 1.28 / (E - 1.0))],          # x = (-52 - V)/4 = 1: 1.28 * 1/(e - 1)
    "orc_beta_m": [(-20.0, 1.4 / (E - 1.0)),              # x = (V + 25)/5 = 1
                   (-30.0, 1.4 * (-1.0) / (math.exp(-1.0) - 1.0))],
    "orc_alpha_h": [(-66.0, 0.128 * E),                   # (-48 - V)/18 = 1
                    (-30.0, 0.128 / E)],                  # (-48 - V)/18 = -1
    "orc_beta_h": [(-20.0, 4.0 / (1.0 + 1.0 / E)),        # (-25 - V)/5 = -1
                   (-30.0, 4.0 / (E + 1.0))],             # (-25 - V)/5 = +1
    "orc_alpha_n": [(-55.0, 0.16 / (E - 1.0)),            # (-50 - V)/5 = 1
                    (-45.0, 0.16 * (-1.0) / (math.exp(-1.0) - 1.0))],
    "orc_beta_n": [(-95.0, 0.5 * E),                      # (-55 - V)/40 = 1
                   (-15.0, 0.5 / E)],                     # (-55 - V)/40 = -1
}

# (V, m, h, n) -> I_ion in nA with g_Na 7.15, E_Na 50, g_K 1.43, E_K -95,
# g_L 0.02672, E_L -63.563:  g_Na m^3 h (V - E_Na) + g_K n^4 (V - E_K) + g_L (V - E_L)
ION_POINTS = [
    ((0.0, 0.5, 1.0, 0.5), 7.15 * 0.125 * 1.0 * (0.0 - 50.0) + 1.43 * 0.0625 * 95.0 + 0.02672 * 63.563),
    ((0.0, 1.0, 0.5, 1.0), 7.15 * 1.0 * 0.5 * (0.0 - 50.0) + 1.43 * 1.0 * 95.0 + 0.02672 * 63.563),
    ((-80.0, 0.3, 0.7, 0.6), 7.15 * 0.027 * 0.7 * (-130.0) + 1.43 * 0.1296 * 15.0 + 0.02672 * (-16.437)),
]

# Resting point of the unstimulated neuron (mV and gate values), with the
# tolerance each is held to.
REST = {"V": (-63.3020692, 5e-8), "m": (0.02079827, 1e-8), "h": (0.99375047, 1e-8), "n": (0.04943329, 1e-8)}


def violations(L, hh):
    """Names of the pins that library L (the oracle's ctypes handle, any
    build of its source) violates; hh is a double[7] array of the published
    parameters."""
    import ctypes as C

    import numpy as np
    bad = []
    for name, pts in RATE_POINTS.items():
        f = getattr(L, name)
        f.restype = C.c_double
        f.argtypes = [C.c_double]
        for v, want in pts:
            got = f(v)
            if not abs(got - want) <= 1e-14 * abs(want):
                bad.append(f"{name}({v}) = {got!r}, not {want!r}")
    L.orc_i_ion.restype = C.c_double
    L.orc_i_ion.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double]
    for (v, m, h, n), want in ION_POINTS:
        got = L.orc_i_ion(hh.ctypes.data, v, m, h, n)
        if not abs(got - want) <= 1e-12 * abs(want):
            bad.append(f"I_ion{(v, m, h, n)} = {got!r}, not {want!r}")
    L.orc_rest.restype = C.c_int
    L.orc_rest.argtypes = [C.c_void_p] * 5
    o = [np.zeros(1) for _ in range(4)]
    if L.orc_rest(hh.ctypes.data, *[x.ctypes.data for x in o]) != 0:
        bad.append("no resting point in [-80, -60] mV")
    else:
        for (k, (want, tol)), x in zip(REST.items(), o):
            if not abs(x[0] - want) <= tol:
                bad.append(f"rest {k} = {x[0]!r}, not {want!r} +- {tol}")
    return bad
