"""ctypes wrapper of the FP64 reference simulator in ``snn_oracle.c``.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may use it; the product library never does.
It takes one instance of a network spec (see the package's ``netgen``) and
simulates it in double precision with plain loops.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "snn_oracle.c"), os.path.join(HERE, "snn_adjoint.c")]
DEPS = SRC + [os.path.join(HERE, "snn_oracle.h")]
LIB = os.path.join(HERE, "liboracle.so")

POISSON, HH, IZH = 0, 1, 2
V, M, H, N = 0, 1, 2, 3


def build(force=True):
    """Compile the oracle with gcc (portable flags, no fast-math)."""
    srcs = [s for s in SRC if os.path.exists(s)]
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(s) for s in DEPS):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-fopenmp",
                           "-o", tmp, *srcs, "-lm"])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB)
        d, i32, i64, u64, vp = C.c_double, C.c_int32, C.c_int64, C.c_uint64, C.c_void_p
        sig = {
            "orc_phi": (d, [d]), "orc_alpha_m": (d, [d]), "orc_beta_m": (d, [d]),
            "orc_alpha_h": (d, [d]), "orc_beta_h": (d, [d]), "orc_alpha_n": (d, [d]),
            "orc_beta_n": (d, [d]),
            "orc_default_hh": (None, [vp]),
            "orc_i_ion": (d, [vp, d, d, d, d]),
            "orc_i_ss": (d, [vp, d]),
            "orc_substep": (None, [vp, d, d, vp, vp, vp, vp]),
            "orc_rest": (C.c_int, [vp, vp, vp, vp, vp]),
            "orc_philox4x32_10": (None, [vp, vp, vp]),
            "orc_poisson_threshold": (u64, [d, d]),
            "orc_poisson_fires": (C.c_int, [u64, i64, i32, i32, u64]),
            "orc_create": (vp, [d, C.c_int, d, u64]),
            "orc_add_pop": (C.c_int, [vp, C.c_int, C.c_int, d, d, vp]),
            "orc_add_proj": (C.c_int, [vp, C.c_int, C.c_int, i64, vp, vp, vp, d, d, C.c_int, d, d, d, d]),
            "orc_init": (C.c_int, [vp]),
            "orc_step": (C.c_int, [vp, i64]),
            "orc_step_trace": (C.c_int, [vp, i64, C.c_int, vp]),
            "orc_get_var": (C.c_int, [vp, C.c_int, C.c_int, vp]),
            "orc_set_var": (C.c_int, [vp, C.c_int, C.c_int, vp]),
            "orc_get_G": (C.c_int, [vp, C.c_int, vp]),
            "orc_set_G": (C.c_int, [vp, C.c_int, vp]),
            "orc_get_weights": (C.c_int, [vp, C.c_int, vp]),
            "orc_get_traces": (C.c_int, [vp, C.c_int, vp, vp]),
            "orc_get_counts": (C.c_int, [vp, C.c_int, vp]),
            "orc_get_vsum": (C.c_int, [vp, C.c_int, vp]),
            "orc_get_last_spikes": (C.c_int, [vp, C.c_int, vp]),
            "orc_set_last_spikes": (C.c_int, [vp, C.c_int, vp]),
            "orc_nan_count": (i64, [vp]),
            "orc_set_threads": (None, [vp, C.c_int]),
            "orc_set_izh_params": (C.c_int, [vp, C.c_int, vp]),
            "orc_izh_substep": (None, [d, d, d, d, vp, vp]),
            "orc_time": (i64, [vp]),
            "orc_set_g_scale": (None, [vp, d]),
            "orc_log_events": (None, [vp, C.c_int]),
            "orc_event_count": (i64, [vp]),
            "orc_take_events": (i64, [vp, vp, vp, vp, i64]),
            "orc_set_replay": (C.c_int, [vp, C.c_int, C.c_int, vp, vp, i64]),
            "orc_destroy": (None, [vp]),
            "orc_dphi": (d, [d]),
            "orc_substep_vjp": (None, [vp, d, vp, vp, vp, vp]),
            "orc_adjoint": (C.c_int, [vp, i64, C.c_int, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            if not hasattr(L, name):
                continue
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def default_hh():
    out = np.zeros(7)
    lib().orc_default_hh(_p(out))
    return out


def rest(hh=None):
    hh = default_hh() if hh is None else np.asarray(hh, np.float64)
    o = [np.zeros(1) for _ in range(4)]
    rc = lib().orc_rest(_p(hh), *[_p(x) for x in o])
    if rc != 0:
        raise ValueError("no resting point in [-80, -60] mV")
    return tuple(float(x[0]) for x in o)


def substep_vjp(hh, hs, x, lam_out):
    """(lam_in[4], lam_I) of one Euler substep at state x = (V, m, h, n)."""
    hh = np.ascontiguousarray(hh, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    lo = np.ascontiguousarray(lam_out, np.float64)
    li = np.zeros(4)
    lI = np.zeros(1)
    lib().orc_substep_vjp(_p(hh), float(hs), _p(x), _p(lo), _p(li), _p(lI))
    return li, float(lI[0])


def substep(hh, hs, i_in, x):
    hh = np.ascontiguousarray(hh, np.float64)
    v = [np.array([float(a)]) for a in x]
    lib().orc_substep(_p(hh), float(hs), float(i_in), *[_p(a) for a in v])
    return np.array([a[0] for a in v])


def raster_arrays(events, n_pops, T):
    """(offsets, ids) of an event log for orc_set_replay: ids ascending per
    (step, population)."""
    t, p, i = events
    key = t.astype(np.int64) * n_pops + p
    order = np.lexsort((i, key))
    off = np.zeros(T * n_pops + 1, np.int64)
    np.cumsum(np.bincount(key, minlength=T * n_pops)[:T * n_pops], out=off[1:])
    return off, i[order].astype(np.int32)


def philox(ctr, key):
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def step_many(nets, n, threads=1):
    """Advance independent instances by n steps each, on up to `threads`
    host threads at once (ctypes drops the interpreter lock during each call,
    so the instances really run in parallel).  Every instance does exactly
    the arithmetic of a serial run."""
    if threads <= 1 or len(nets) <= 1:
        for net in nets:
            net.step(n)
        return
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=int(threads)) as ex:
        list(ex.map(lambda net: net.step(n), nets))


class OracleNet:
    """One network instance in FP64.  ``inst`` is an entry of spec["instances"]."""

    def __init__(self, inst, dt=0.1, substeps=3, hh_params=None, log_events=False):
        L = lib()
        self.inst = inst
        self.dt = dt
        self.h = L.orc_create(dt, substeps, float(inst["g_scale"]), int(inst["seed"]))
        if not self.h:
            raise ValueError("bad dt/substeps")
        self.pops = inst["pops"]
        self._keep = []
        for k, p in enumerate(self.pops):
            kind = {"poisson": POISSON, "hh": HH, "izh": IZH}[p["kind"]]
            hh = None
            if hh_params is not None and hh_params.get(k) is not None:
                hh = np.asarray(hh_params[k], np.float64)
                self._keep.append(hh)
            r = L.orc_add_pop(self.h, kind, int(p["n"]), float(p.get("rate_hz", 0.0)),
                              float(p.get("i_ext", 0.0)), _p(hh) if hh is not None else None)
            if r < 0:
                raise ValueError("bad population")
            if kind == IZH:
                abcd = np.ascontiguousarray(p["abcd"], np.float32)
                assert abcd.shape == (4, int(p["n"]))
                self._keep.append(abcd)
                if L.orc_set_izh_params(self.h, k, _p(abcd)) != 0:
                    raise ValueError("bad Izhikevich parameters")
        for q in inst["projs"]:
            rp = np.ascontiguousarray(q["row_ptr"], np.int32)
            ci = np.ascontiguousarray(q["col_idx"], np.int32)
            g = np.ascontiguousarray(q["g"], np.float32)
            st = q.get("stdp")
            r = L.orc_add_proj(self.h, int(q["pre"]), int(q["post"]), int(ci.size), _p(rp), _p(ci), _p(g),
                               float(q["e_rev"]), float(q["tau"]), 1 if st else 0,
                               float(st["a_plus"]) if st else 0.0, float(st["a_minus"]) if st else 0.0,
                               float(st["tau"]) if st else 1.0, float(st["g_max"]) if st else 0.0)
            if r < 0:
                raise ValueError("bad projection")
        if L.orc_init(self.h) != 0:
            raise ValueError("init failed")
        if log_events:
            L.orc_log_events(self.h, 1)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def step(self, n=1):
        lib().orc_step(self.h, int(n))

    def trace(self, n, pop):
        out = np.zeros((int(n), int(self.pops[pop]["n"])), np.float64)
        if lib().orc_step_trace(self.h, int(n), int(pop), _p(out)) != 0:
            raise ValueError("trace of a non-HH population")
        return out

    def get(self, pop, var):
        out = np.zeros(int(self.pops[pop]["n"]), np.float64)
        if lib().orc_get_var(self.h, int(pop), int(var), _p(out)) != 0:
            raise ValueError("bad pop/var")
        return out

    def set(self, pop, var, vals):
        a = np.ascontiguousarray(vals, np.float64)
        assert a.size == self.pops[pop]["n"]
        if lib().orc_set_var(self.h, int(pop), int(var), _p(a)) != 0:
            raise ValueError("bad pop/var")

    def G(self, proj):
        q = self.inst["projs"][proj]
        out = np.zeros(int(self.pops[q["post"]]["n"]), np.float64)
        lib().orc_get_G(self.h, int(proj), _p(out))
        return out

    def set_G(self, proj, vals):
        a = np.ascontiguousarray(vals, np.float64)
        lib().orc_set_G(self.h, int(proj), _p(a))

    def weights(self, proj):
        out = np.zeros(int(np.asarray(self.inst["projs"][proj]["col_idx"]).size), np.float64)
        lib().orc_get_weights(self.h, int(proj), _p(out))
        return out

    def traces(self, proj):
        q = self.inst["projs"][proj]
        x = np.zeros(int(self.pops[q["pre"]]["n"]))
        y = np.zeros(int(self.pops[q["post"]]["n"]))
        if lib().orc_get_traces(self.h, int(proj), _p(x), _p(y)) != 0:
            raise ValueError("not plastic")
        return x, y

    def counts(self, pop):
        out = np.zeros(int(self.pops[pop]["n"]), np.int32)
        lib().orc_get_counts(self.h, int(pop), _p(out))
        return out

    def vsum(self, pop):
        out = np.zeros(int(self.pops[pop]["n"]), np.float64)
        lib().orc_get_vsum(self.h, int(pop), _p(out))
        return out

    def last_spikes(self, pop):
        out = np.zeros(int(self.pops[pop]["n"]), np.uint8)
        lib().orc_get_last_spikes(self.h, int(pop), _p(out))
        return out

    def set_last_spikes(self, pop, flags):
        a = np.ascontiguousarray(flags, np.uint8)
        lib().orc_set_last_spikes(self.h, int(pop), _p(a))

    def set_threads(self, n):
        """Run the HH neuron loop of every step on n OpenMP threads (1: serial)."""
        lib().orc_set_threads(self.h, int(n))

    @property
    def nan_count(self):
        return int(lib().orc_nan_count(self.h))

    @property
    def t(self):
        return int(lib().orc_time(self.h))

    def events(self):
        """(t, pop, id) arrays of every spike since the last call (log_events=True)."""
        n = int(lib().orc_event_count(self.h))
        t, p, i = (np.zeros(n, np.int32) for _ in range(3))
        lib().orc_take_events(self.h, _p(t), _p(p), _p(i), n)
        return t, p, i

    def adjoint(self, T, loss_pop, dLdVbar):
        """Run T steps from the initial state and the reverse pass: returns
        (vbar, [dL/dg per projection], dL/dg_scale)."""
        n = int(self.pops[loss_pop]["n"])
        dv = np.ascontiguousarray(dLdVbar, np.float64)
        assert dv.size == n
        grads = [np.zeros(max(1, int(np.asarray(q["col_idx"]).size))) for q in self.inst["projs"]]
        ptrs = (C.c_void_p * max(1, len(grads)))(*[g.ctypes.data for g in grads])
        dls = np.zeros(1)
        vbar = np.zeros(n)
        rc = lib().orc_adjoint(self.h, int(T), int(loss_pop), _p(dv), C.cast(ptrs, C.c_void_p), _p(dls), _p(vbar))
        if rc != 0:
            raise ValueError("adjoint: bad arguments or plastic network")
        grads = [g[:int(np.asarray(q["col_idx"]).size)] for g, q in zip(grads, self.inst["projs"])]
        return vbar, grads, float(dls[0])

    def set_replay(self, pop, off, ids, T):
        """Population pop takes its spikes from a raster; off has T*n_pops+1 entries."""
        self._rp = (np.ascontiguousarray(off, np.int64), np.ascontiguousarray(ids, np.int32))
        if lib().orc_set_replay(self.h, int(pop), 1, _p(self._rp[0]), _p(self._rp[1]), int(T)) != 0:
            raise ValueError("bad pop")
