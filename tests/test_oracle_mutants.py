"""The kinetics pins must catch plausible misreadings of the Traub-Miles
model: each case below compiles the oracle with one planted mistake (a wrong
slope divisor, gate exponent, sign or constant) on the CPU and checks that at
least one hand-derived pin of tests/tm_pins.py fails for it."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import tm_pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "snn_oracle.c")

MUTANTS = {
    "n^3 for n^4": ("p[HH_GK] * n * n * n * n", "p[HH_GK] * n * n * n"),
    "m^2 for m^3": ("p[HH_GNA] * m * m * m * h", "p[HH_GNA] * m * m * h"),
    "h^2 for h": ("p[HH_GNA] * m * m * m * h", "p[HH_GNA] * m * m * m * h * h"),
    "beta_n /80": ("exp((-55.0 - V) / 40.0)", "exp((-55.0 - V) / 80.0)"),
    "beta_n /20": ("exp((-55.0 - V) / 40.0)", "exp((-55.0 - V) / 20.0)"),
    "alpha_h /20": ("exp((-48.0 - V) / 18.0)", "exp((-48.0 - V) / 20.0)"),
    "beta_h /4": ("exp((-25.0 - V) / 5.0)", "exp((-25.0 - V) / 4.0)"),
    "alpha_m /5": ("orc_phi((-52.0 - V) / 4.0)", "orc_phi((-52.0 - V) / 5.0)"),
    "beta_m /4": ("orc_phi((V + 25.0) / 5.0)", "orc_phi((V + 25.0) / 4.0)"),
    "alpha_n /4": ("orc_phi((-50.0 - V) / 5.0)", "orc_phi((-50.0 - V) / 4.0)"),
    "beta_n offset -50": ("exp((-55.0 - V) / 40.0)", "exp((-50.0 - V) / 40.0)"),
    "E_K sign in I_ion": ("(V - p[HH_EK])", "(V + p[HH_EK])"),
    "leak E_L -63.56": ("p[HH_EL] = -63.563", "p[HH_EL] = -63.56"),
    "g_L 0.0267": ("p[HH_GL] = 0.02672", "p[HH_GL] = 0.0267"),
}


def _build(tmp_path, name, old, new):
    with open(SRC) as fh:
        text = fh.read()
    assert text.count(old) == 1, f"mutation site of {name!r} not unique"
    src = tmp_path / "mut.c"
    src.write_text(text.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                           "-I", os.path.join(ROOT, "oracle"), "-o", str(so), str(src), "-lm"])
    return ctypes.CDLL(str(so))


def test_pins_hold_for_the_oracle_source(tmp_path):
    L = _build(tmp_path, "none", "double orc_phi(double x)", "double orc_phi(double x)")
    hh = np.zeros(7)
    L.orc_default_hh.argtypes = [ctypes.c_void_p]
    L.orc_default_hh(hh.ctypes.data)
    assert tm_pins.violations(L, hh) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    L = _build(tmp_path, name, old, new)
    hh = np.zeros(7)
    L.orc_default_hh.argtypes = [ctypes.c_void_p]
    L.orc_default_hh(hh.ctypes.data)
    assert tm_pins.violations(L, hh), f"no pin fails for the mutant {name!r}"
