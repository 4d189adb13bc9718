"""Pins of the FP64 oracle adjoint (gradient with the spike raster fixed).

Checked against central finite differences of the oracle's own forward map
(a different computation than the transposed Jacobians), the structural
zero for projections that cannot reach the loss population, and the exact
identity dL/ds = (1/s) sum_k g_k dL/dg_k.
"""
import copy

import numpy as np
import pytest

from paper_1412_0595_amd import netgen


def test_dphi_matches_difference_quotient_and_series(orc):
    L = orc.lib()
    for x in [-3.0, -0.7, -2e-3, 2e-3, 0.4, 5.0]:
        h = 1e-6 * max(1.0, abs(x))
        fd = (L.orc_phi(x + h) - L.orc_phi(x - h)) / (2 * h)
        assert abs(L.orc_dphi(x) - fd) < 1e-8
    # the series branch and the closed form agree where they meet
    for x in [0.999e-3, -0.999e-3]:
        em1 = np.expm1(x * 1.002)
        closed = (em1 * (1 - x * 1.002) - x * 1.002) / em1 ** 2
        assert abs(L.orc_dphi(x * 1.002) - closed) < 1e-9
    assert L.orc_dphi(0.0) == -0.5


@pytest.mark.parametrize("x", [(-63.3, 0.02, 0.99, 0.05), (-52.0, 0.3, 0.5, 0.4), (-25.0, 0.9, 0.2, 0.6),
                               (-50.0, 0.1, 0.8, 0.3), (20.0, 0.98, 0.1, 0.7), (-90.0, 0.001, 0.99, 0.01)])
def test_substep_vjp_matches_central_differences(orc, x):
    """Per-substep vector-Jacobian product against central differences of the
    substep map, for every input and the injected current (FP64, relative
    1e-7)."""
    hh = orc.default_hh()
    hs = 0.1 / 3
    rng = np.random.default_rng(int(abs(x[0]) * 10))
    lam = rng.normal(size=4)
    i_in = 0.3
    li, lI = orc.substep_vjp(hh, hs, np.array(x), lam)
    f = lambda xx, ii: float(lam @ orc.substep(hh, hs, ii, xx))
    x = np.array(x, np.float64)
    for k in range(4):
        e = 1e-6 * (abs(x[k]) if k == 0 else 1.0) + 1e-9
        xp, xm = x.copy(), x.copy()
        xp[k] += e
        xm[k] -= e
        fd = (f(xp, i_in) - f(xm, i_in)) / (2 * e)
        assert abs(li[k] - fd) <= 1e-7 * max(1.0, abs(fd)), (k, li[k], fd)
    e = 1e-6
    fd = (f(x, i_in + e) - f(x, i_in - e)) / (2 * e)
    assert abs(lI - fd) <= 1e-7 * max(1.0, abs(fd))


def _setup(scale=0.1, T=300, seed=0):
    spec = netgen.make_config(5, n_instances=1, scale=scale)
    inst = spec["instances"][0]
    y = spec["target"][0]
    return inst, y, T


def _raster(orc, inst, T):
    net = orc.OracleNet(inst, log_events=True)
    net.step(T)
    return orc.raster_arrays(net.events(), len(inst["pops"]), T)


def _loss(orc, inst, y, T, off, ids, replay=True):
    net = orc.OracleNet(inst, log_events=not replay)
    if replay:
        for p in (1, 2):
            net.set_replay(p, off, ids, T)
    net.step(T)
    vbar = net.vsum(2) / T
    L = float(np.sum((vbar - y) ** 2) / y.size)
    return L, (net.events() if not replay else None)


def _adjoint(orc, inst, y, T, off, ids):
    net = orc.OracleNet(inst)
    for p in (1, 2):
        net.set_replay(p, off, ids, T)
    # dL/dVbar = 2 (Vbar - y) / C needs Vbar first: one forward, then the adjoint run
    fwd = orc.OracleNet(inst)
    for p in (1, 2):
        fwd.set_replay(p, off, ids, T)
    fwd.step(T)
    vbar = fwd.vsum(2) / T
    dv = 2 * (vbar - y) / y.size
    vb2, grads, dls = net.adjoint(T, 2, dv)
    assert np.array_equal(vb2, vbar)
    return grads, dls


def _richardson(f, eps):
    """Central difference extrapolated from steps 2 eps and eps: the O(eps^2)
    truncation term cancels (the spike upstroke makes it large: 1.5e-6
    relative at eps = 1e-6 on this network, 5e-9 after extrapolation)."""
    d1 = (f(2 * eps) - f(-2 * eps)) / (4 * eps)
    d2 = (f(eps) - f(-eps)) / (2 * eps)
    return (4 * d2 - d1) / 3


def test_full_run_gradient_matches_central_differences(orc):
    """dL/dg_scale and 20 random B->C and C->C weights against Richardson-
    extrapolated central differences (eps = 1e-6 * s, 1e-4 * g) with the
    raster replayed (held fixed); relative 1e-6."""
    inst, y, T = _setup()
    off, ids = _raster(orc, inst, T)
    grads, dls = _adjoint(orc, inst, y, T, off, ids)
    s = inst["g_scale"]
    fd = _richardson(lambda e: _loss(orc, dict(inst, g_scale=s + e), y, T, off, ids)[0], 1e-6 * s)
    assert abs(dls - fd) <= 1e-6 * abs(fd), (dls, fd)
    rng = np.random.default_rng(1)
    for q in (1, 2):
        g = inst["projs"][q]["g"]
        big = np.nonzero(np.abs(grads[q]) > 1e-3 * np.abs(grads[q]).max())[0]
        for k in rng.choice(big, size=10, replace=False):
            def loss_at(e, q=q, k=k):
                # the weights are fp32 inputs: perturb in double through a copy
                I2 = copy.deepcopy(inst)
                I2["projs"][q]["g"] = g.astype(np.float64)
                I2["projs"][q]["g"][k] += e
                return _loss_f64(orc, I2, y, T, off, ids)
            # a single weight moves L by little: a larger step keeps rounding
            # noise of L (~1e-14) well below the derivative
            fdk = _richardson(loss_at, 1e-4 * float(g[k]))
            assert abs(grads[q][k] - fdk) <= 1e-6 * max(abs(fdk), 1e-3 * np.abs(grads[q]).max()), (q, k)


def _loss_f64(orc, inst, y, T, off, ids):
    """Loss with fp64 weights: the oracle widens fp32 inputs, so feed it a
    float64 array through a float32-exact split (g = hi + lo) of two
    parallel projections."""
    I2 = copy.deepcopy(inst)
    extra = []
    for q in I2["projs"]:
        g64 = np.asarray(q["g"], np.float64)
        hi = g64.astype(np.float32)
        lo = (g64 - hi.astype(np.float64)).astype(np.float32)
        q["g"] = hi
        if np.any(lo != 0):
            extra.append(dict(q, g=lo))
    I2["projs"] = I2["projs"] + extra
    return _loss(orc, I2, y, T, off, ids)[0]


def test_input_projection_gradient_is_exactly_zero(orc):
    """With the raster fixed, A->B weights cannot reach the output layer:
    their gradient is exactly 0 and perturbing them leaves L bitwise equal."""
    inst, y, T = _setup()
    off, ids = _raster(orc, inst, T)
    grads, _ = _adjoint(orc, inst, y, T, off, ids)
    assert np.all(grads[0] == 0.0)
    I2 = copy.deepcopy(inst)
    I2["projs"][0]["g"] = (I2["projs"][0]["g"] * np.float32(1.01)).astype(np.float32)
    assert _loss(orc, I2, y, T, off, ids)[0] == _loss(orc, inst, y, T, off, ids)[0]


def test_gscale_identity(orc):
    """g_scale multiplies every delivered weight, so dL/ds = (1/s) sum g dL/dg."""
    inst, y, T = _setup()
    inst = dict(inst, g_scale=1.7)
    off, ids = _raster(orc, inst, T)
    grads, dls = _adjoint(orc, inst, y, T, off, ids)
    tot = sum(float(np.dot(inst["projs"][q]["g"].astype(np.float64), grads[q])) for q in range(3))
    assert abs(dls - tot / 1.7) <= 1e-12 * abs(dls)


def test_free_running_fd_with_unchanged_raster(orc):
    """Without replay, a small perturbation of g_scale that leaves every spike
    in place gives the same derivative."""
    inst, y, T = _setup(T=200)
    off, ids = _raster(orc, inst, T)
    grads, dls = _adjoint(orc, inst, y, T, off, ids)
    s = inst["g_scale"]
    eps = 1e-7 * s
    for _ in range(4):
        (Lp, ep), (Lm, em) = (_loss(orc, dict(inst, g_scale=s + e), y, T, off, ids, replay=False) for e in (eps, -eps))
        same = all(np.array_equal(a, b) for a, b in zip(ep, em))
        if same:
            break
        eps /= 2
    assert same
    fd = (Lp - Lm) / (2 * eps)
    assert abs(dls - fd) <= 1e-5 * abs(fd)
