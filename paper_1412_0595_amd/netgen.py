"""Seeded synthetic spiking networks shaped like the paper's layered models.

This module only draws inputs: population sizes, Bernoulli CSR connectivity
(Compressed Row Storage, Section 3: values along the pre-synaptic index, the
post-synaptic index of each value, and the start of every pre-synaptic row),
uniform weights, per-instance conductance scales, Poisson seeds and loss
targets.  It holds none of the simulation arithmetic, so both the FP64 oracle
and the HIP library consume exactly the same arrays.

The layered shape follows the insect-olfaction model of Section 5.1 (input
projection neurons -> Kenyon cells -> detection neurons, called A -> B -> C
here), with Poisson input sources (the model's non-deterministic inputs,
Section 4 "Discussion").  The batched configuration is the conductance-scaling
sweep of Section 2 ("a series of simulations in the likely range of the
scaling factors") drawn as many uneven instances.

A network spec is a plain dict::

    {"dt": 0.1, "substeps": 3,
     "instances": [{"g_scale": s, "seed": k,
                    "pops":  [{"name", "kind": "poisson"|"hh"|"izh", "n", "rate_hz", "i_ext",
                               "abcd" (izh only: float32[4, n] rows a, b, c, d)}],
                    "projs": [{"pre", "post", "row_ptr" int32[n_pre+1],
                               "col_idx" int32[nnz], "g" float32[nnz],
                               "e_rev", "tau", "stdp": None | {...}}]}]}

Units: mV, ms, uS, nA, Hz.
"""
from __future__ import annotations

import math

import numpy as np

# Conductance scales of the layered model (uS).  The paper fixes none of them;
# they are chosen by its own criterion (a moderate spiking level with no NaNs).
G0_AB = 0.1      # A->B: g = U[0,1) * G0_AB / (n_A * p_AB)
G1_BC = 0.05     # B->C: g = U[0,1) * G1_BC / (n_B * p_BC)
G_INH_CC = 0.0005  # C->C at n_C = 100: g = U[0,1) * G_INH_CC * 100 / n_C

E_EXC, TAU_AB, TAU_BC = 0.0, 1.0, 5.0
E_INH, TAU_CC = -92.0, 2.5

# STDP of the plastic B->C projection (amplitudes in units of g_max)
STDP_A_PLUS, STDP_A_MINUS, STDP_TAU = 0.01, 0.012, 20.0


def bernoulli_csr(rng, n_pre, n_post, p, *, no_self=False, chunk_elems=1 << 24):
    """Bernoulli(p) connectivity for every (pre, post) pair, as CSR with
    ascending column indices in each row.  ``no_self`` drops i == j."""
    if n_pre == 0 or n_post == 0:
        return np.zeros(n_pre + 1, np.int32), np.zeros(0, np.int32)
    counts = np.zeros(n_pre, np.int64)
    cols = []
    rows_per = max(1, chunk_elems // max(1, n_post))
    for r0 in range(0, n_pre, rows_per):
        r1 = min(n_pre, r0 + rows_per)
        if p >= 1.0:
            m = np.ones((r1 - r0, n_post), bool)
        else:
            m = rng.random((r1 - r0, n_post), dtype=np.float32) < np.float32(p)
        if no_self:
            idx = np.arange(r0, r1)
            ok = idx < n_post
            m[np.nonzero(ok)[0], idx[ok]] = False
        counts[r0:r1] = m.sum(axis=1)
        cols.append(np.nonzero(m)[1].astype(np.int32))
    row_ptr = np.zeros(n_pre + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("projection too large for int32 CSR")
    return row_ptr.astype(np.int32), (np.concatenate(cols) if cols else np.zeros(0, np.int32))


def uniform_weights(rng, nnz, scale):
    """g = U[0,1) * scale, stored as fp32 (uS)."""
    return (rng.random(nnz) * scale).astype(np.float32)


def layered_instance(rng, n_a, n_b, n_c, *, rate_hz=20.0, p_ab=0.5, p_bc=1.0,
                     g_scale=1.0, seed=0, stdp_bc=False, i_ext=0.0, ab_norm=None):
    """One A(Poisson) -> B(HH) -> C(HH) network with C->C all-to-all inhibition.
    A->B weights are U[0,1) * G0_AB / ab_norm, ab_norm = n_A * p_AB (the
    expected in-degree) unless given."""
    pops = [dict(name="A", kind="poisson", n=int(n_a), rate_hz=float(rate_hz), i_ext=0.0),
            dict(name="B", kind="hh", n=int(n_b), rate_hz=0.0, i_ext=float(i_ext)),
            dict(name="C", kind="hh", n=int(n_c), rate_hz=0.0, i_ext=float(i_ext))]
    rp, ci = bernoulli_csr(rng, n_a, n_b, p_ab)
    ab = dict(pre=0, post=1, row_ptr=rp, col_idx=ci,
              g=uniform_weights(rng, ci.size, G0_AB / (n_a * p_ab if ab_norm is None else ab_norm)),
              e_rev=E_EXC, tau=TAU_AB, stdp=None)
    rp, ci = bernoulli_csr(rng, n_b, n_c, p_bc)
    g1 = G1_BC / (n_b * p_bc)
    bc = dict(pre=1, post=2, row_ptr=rp, col_idx=ci, g=uniform_weights(rng, ci.size, g1),
              e_rev=E_EXC, tau=TAU_BC, stdp=None)
    if stdp_bc:
        bc["stdp"] = dict(a_plus=STDP_A_PLUS, a_minus=STDP_A_MINUS, tau=STDP_TAU, g_max=g1)
    rp, ci = bernoulli_csr(rng, n_c, n_c, 1.0, no_self=True)
    cc = dict(pre=2, post=2, row_ptr=rp, col_idx=ci,
              g=uniform_weights(rng, ci.size, G_INH_CC * 100.0 / n_c),
              e_rev=E_INH, tau=TAU_CC, stdp=None)
    return dict(g_scale=float(g_scale), seed=int(seed), pops=pops, projs=[ab, bc, cc])


def instance_seed(key, i):
    """Poisson key of instance i: every instance draws its own stream."""
    return (int(key) << 20) | int(i)


def _loguniform_int(rng, lo, hi, size):
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size))).astype(np.int64)


def make_config(k, *, n_instances=None, scale=1.0):
    """Workloads 1..5 (dt = 0.1 ms, 3 Euler substeps).  Seeds: base = 1000*k,
    +1 connectivity, +2 Poisson key, +3 instance sizes and g_scale, +4 target.

    1: A=100 @20 Hz, B=1000, C=100; A->B p=0.5, B->C and C->C all-to-all.
    2: A=1000 @20 Hz, B=20000, C=1000; p_AB=0.2, p_BC=0.5.
    3: A=2000 @30 Hz, B=100000, C=1000; p_AB=0.2, p_BC=0.5 with pair STDP.
    4: 256 instances, A~LU[200,1000], B~LU[2000,20000], C~LU[100,1000],
       g_scale~LU[0.1,10], p=0.2/0.5.
    5: 64 x (A=500, B=5000, C=200), p=0.2/0.5, plus a seeded target
       y~U[-64,-58] mV per output neuron (returned under "target").

    ``n_instances`` trims workloads 4 and 5; ``scale`` shrinks every
    population (rounded, >= 2) for reduced-size tests.
    """
    base = 1000 * k
    rng_c = np.random.default_rng(base + 1)
    seed_key = base + 2
    sz = lambda n: max(2, int(round(n * scale)))
    spec = dict(dt=0.1, substeps=3, instances=[])
    if k == 1:
        spec["instances"].append(layered_instance(rng_c, sz(100), sz(1000), sz(100), rate_hz=20.0,
                                                  p_ab=0.5, p_bc=1.0, seed=seed_key))
        spec["steps"] = 10000
    elif k == 2:
        spec["instances"].append(layered_instance(rng_c, sz(1000), sz(20000), sz(1000), rate_hz=20.0,
                                                  p_ab=0.2, p_bc=0.5, seed=seed_key))
        spec["steps"] = 10000
    elif k == 3:
        spec["instances"].append(layered_instance(rng_c, sz(2000), sz(100000), sz(1000), rate_hz=30.0,
                                                  p_ab=0.2, p_bc=0.5, seed=seed_key, stdp_bc=True))
        spec["steps"] = 5000
    elif k == 4:
        n = 256 if n_instances is None else int(n_instances)
        rng_s = np.random.default_rng(base + 3)
        a = _loguniform_int(rng_s, 200, 1000, 256)[:n]
        b = _loguniform_int(rng_s, 2000, 20000, 256)[:n]
        c = _loguniform_int(rng_s, 100, 1000, 256)[:n]
        gs = np.exp(rng_s.uniform(math.log(0.1), math.log(10.0), 256))[:n]
        for i in range(n):
            spec["instances"].append(layered_instance(rng_c, sz(a[i]), sz(b[i]), sz(c[i]), rate_hz=20.0,
                                                      p_ab=0.2, p_bc=0.5, g_scale=float(gs[i]),
                                                      seed=instance_seed(seed_key, i)))
        spec["steps"] = 5000
    elif k == 5:
        n = 64 if n_instances is None else int(n_instances)
        for i in range(n):
            spec["instances"].append(layered_instance(rng_c, sz(500), sz(5000), sz(200), rate_hz=20.0,
                                                      p_ab=0.2, p_bc=0.5, seed=instance_seed(seed_key, i)))
        rng_t = np.random.default_rng(base + 4)
        spec["target"] = [rng_t.uniform(-64.0, -58.0, inst["pops"][2]["n"]) for inst in spec["instances"]]
        spec["steps"] = 2000
        spec["ckpt_every"] = 100
    else:
        raise ValueError(f"unknown workload {k}")
    return spec


def calibration_config(n_conn_values, g_scales, *, n_b=1000, n_c=100, p_ab=0.2, ref_n_conn=100.0,
                       rate_hz=20.0, steps=5000, key=6000):
    """A conductance-scaling sweep laid out for the calibration of Section 5.1
    (Fig. 1): one instance per (nConn, gScale) pair, nConn being the expected
    number of A inputs per B neuron (n_A = nConn / p_AB).  A->B weights are
    normalised by the fixed ref_n_conn, so the drive of B grows with nConn
    and gScale has to shrink to hold B's spiking level.  All gScale values of
    one nConn share its connectivity and Poisson stream.  Returns the spec
    with per-instance "n_conn" and the index of every instance under
    "grid" as (nConn index, gScale index)."""
    spec = dict(dt=0.1, substeps=3, instances=[], steps=int(steps), n_conn=[], grid=[])
    for i, x in enumerate(n_conn_values):
        n_a = int(round(float(x) / p_ab))
        base = layered_instance(np.random.default_rng(key + 1 + i), n_a, n_b, n_c, rate_hz=rate_hz,
                                p_ab=p_ab, p_bc=0.5, seed=instance_seed(key + 2, i), ab_norm=ref_n_conn)
        for j, g in enumerate(g_scales):
            inst = dict(base, g_scale=float(g))
            spec["instances"].append(inst)
            spec["n_conn"].append(float(x))
            spec["grid"].append((i, j))
    return spec


# Lateral horn interneurons (LHI) of the insect-olfaction model: excited by
# the projection neurons (PN), they inhibit the Kenyon cells (KC) feed-forward.
G_PN_LHI = 0.1     # PN->LHI: g = U[0,1) * G_PN_LHI / ref_nConn_LHI
G_LHI_KC = 0.02    # LHI->KC: g = U[0,1) * G_LHI_KC / n_LHI
TAU_LHI_KC = 5.0


def mushroom_body_instance(n_pn, n_lhi, *, n_kc=1000, n_dn=100, p_pn_kc=0.2, p_pn_lhi=0.5, rate_hz=20.0,
                           ref_n_pn=100, scale_kc=1.0, scale_lhi=1.0, seed=0, conn_seed=0):
    """The LHI variant of the layered model (Section 5.1's PN, LHI, KC, DN):
    PN(Poisson) -> KC and PN -> LHI excitatory, LHI -> KC all-to-all
    inhibitory, KC -> DN excitatory, DN -> DN all-to-all inhibitory.  PN->KC
    and PN->LHI weights are normalised by the in-degree at ref_n_pn PNs and
    multiplied by scale_kc and scale_lhi, the two swept conductance scales."""
    rng = np.random.default_rng(conn_seed)
    pops = [dict(name="PN", kind="poisson", n=int(n_pn), rate_hz=float(rate_hz), i_ext=0.0),
            dict(name="LHI", kind="hh", n=int(n_lhi), rate_hz=0.0, i_ext=0.0),
            dict(name="KC", kind="hh", n=int(n_kc), rate_hz=0.0, i_ext=0.0),
            dict(name="DN", kind="hh", n=int(n_dn), rate_hz=0.0, i_ext=0.0)]
    projs = []
    rp, ci = bernoulli_csr(rng, n_pn, n_kc, p_pn_kc)
    projs.append(dict(pre=0, post=2, row_ptr=rp, col_idx=ci, e_rev=E_EXC, tau=TAU_AB, stdp=None,
                      g=(uniform_weights(rng, ci.size, G0_AB / (ref_n_pn * p_pn_kc)) * np.float32(scale_kc))))
    rp, ci = bernoulli_csr(rng, n_pn, n_lhi, p_pn_lhi)
    projs.append(dict(pre=0, post=1, row_ptr=rp, col_idx=ci, e_rev=E_EXC, tau=TAU_AB, stdp=None,
                      g=(uniform_weights(rng, ci.size, G_PN_LHI / (ref_n_pn * p_pn_lhi)) * np.float32(scale_lhi))))
    rp, ci = bernoulli_csr(rng, n_lhi, n_kc, 1.0)
    projs.append(dict(pre=1, post=2, row_ptr=rp, col_idx=ci, e_rev=E_INH, tau=TAU_LHI_KC, stdp=None,
                      g=uniform_weights(rng, ci.size, G_LHI_KC / n_lhi)))
    rp, ci = bernoulli_csr(rng, n_kc, n_dn, 0.5)
    projs.append(dict(pre=2, post=3, row_ptr=rp, col_idx=ci, e_rev=E_EXC, tau=TAU_BC, stdp=None,
                      g=uniform_weights(rng, ci.size, G1_BC / (n_kc * 0.5))))
    rp, ci = bernoulli_csr(rng, n_dn, n_dn, 1.0, no_self=True)
    projs.append(dict(pre=3, post=3, row_ptr=rp, col_idx=ci, e_rev=E_INH, tau=TAU_CC, stdp=None,
                      g=uniform_weights(rng, ci.size, G_INH_CC * 100.0 / n_dn)))
    return dict(g_scale=1.0, seed=int(seed), pops=pops, projs=projs)


def mushroom_body_calibration_config(n_pn_values, scales, *, swept="kc", n_lhi=20, n_kc=1000, n_dn=100,
                                     p_pn_kc=0.2, p_pn_lhi=0.5, ref_n_pn=100, steps=5000, key=7000):
    """Calibration sweep of the LHI variant for one of its two swept scales:
    swept="kc" scales PN->KC (criterion: KC spiking, nConn = p_PN_KC * n_PN),
    swept="lhi" scales PN->LHI (criterion: LHI spiking, nConn = p_PN_LHI *
    n_PN); the other scale stays 1.  Runs of one PN count share connectivity
    and Poisson stream.  The spec carries per-run "n_conn", the criterion
    population under "pop" and the swept projection under "proj"."""
    if swept not in ("kc", "lhi"):
        raise ValueError("swept must be 'kc' or 'lhi'")
    spec = dict(dt=0.1, substeps=3, instances=[], steps=int(steps), n_conn=[], grid=[],
                pop=2 if swept == "kc" else 1, proj=0 if swept == "kc" else 1)
    p = p_pn_kc if swept == "kc" else p_pn_lhi
    for i, n_pn in enumerate(n_pn_values):
        for j, s in enumerate(scales):
            kw = dict(scale_kc=float(s)) if swept == "kc" else dict(scale_lhi=float(s))
            inst = mushroom_body_instance(int(n_pn), n_lhi, n_kc=n_kc, n_dn=n_dn, p_pn_kc=p_pn_kc,
                                          p_pn_lhi=p_pn_lhi, ref_n_pn=ref_n_pn, seed=instance_seed(key + 2, i),
                                          conn_seed=key + 1 + i, **kw)
            inst["g_scale_swept"] = float(s)
            spec["instances"].append(inst)
            spec["n_conn"].append(float(p * n_pn))
            spec["grid"].append((i, j))
    return spec


# The 4:1 excitatory/inhibitory Izhikevich network of Section 5.1 (the
# paper's first scalability network; its neuron model is reference [9]).
# The paper gives the size (1000 neurons, E:I = 4:1) and the swept number of
# connections per neuron (nConn = 100 .. 1000), nothing else; the rest is
# this module's reading: per-neuron a, b, c, d drawn as in Izhikevich (2003)
# (excitatory: a 0.02, b 0.2, c -65 + 15 r^2, d 8 - 6 r^2; inhibitory:
# a 0.02 + 0.08 r, b 0.25 - 0.05 r, c -65, d 2; r ~ U[0,1) per neuron),
# rounded to fp32; the random thalamic input of that reference replaced by
# Poisson sources with conductance synapses (as the other workloads' inputs);
# recurrent connections Bernoulli(nConn / n) per (pre, post) pair without
# self-connections, conductance synapses onto v with reversal 0 mV
# (excitatory) or -80 mV (inhibitory), 5 ms decay.
IZH_G_IN = 0.01      # input -> E/I: g = U[0,1) * IZH_G_IN (uS)
IZH_G_E = 0.005      # E -> E/I:     g = U[0,1) * IZH_G_E * gScale
IZH_G_I = 0.0025     # I -> E/I:     g = U[0,1) * IZH_G_I * gScale
IZH_E_INH = -80.0
IZH_TAU = 5.0


def izhikevich_params(rng, n_exc, n_inh):
    """float32[4, n_exc + n_inh] rows a, b, c, d (excitatory neurons first)."""
    re, ri = rng.random(n_exc), rng.random(n_inh)
    a = np.concatenate([np.full(n_exc, 0.02), 0.02 + 0.08 * ri])
    b = np.concatenate([np.full(n_exc, 0.2), 0.25 - 0.05 * ri])
    c = np.concatenate([-65.0 + 15.0 * re * re, np.full(n_inh, -65.0)])
    d = np.concatenate([8.0 - 6.0 * re * re, np.full(n_inh, 2.0)])
    return np.stack([a, b, c, d]).astype(np.float32)


def izhikevich_instance(n_conn, *, n_exc=800, n_inh=200, n_in=1000, p_in=0.1, rate_hz=20.0, g_scale=1.0,
                        seed=0, conn_seed=0):
    """One 4:1 E/I Izhikevich network: populations IN (Poisson), E, I; the
    recurrent projections E->E, E->I, I->E, I->I with p = nConn / (n_exc +
    n_inh) and weights scaled by g_scale (built into the fp32 weights: the
    instance g_scale stays 1, so the input projections are not scaled)."""
    rng = np.random.default_rng(conn_seed)
    n = n_exc + n_inh
    abcd = izhikevich_params(rng, n_exc, n_inh)
    pops = [dict(name="IN", kind="poisson", n=int(n_in), rate_hz=float(rate_hz), i_ext=0.0),
            dict(name="E", kind="izh", n=int(n_exc), rate_hz=0.0, i_ext=0.0, abcd=abcd[:, :n_exc].copy()),
            dict(name="I", kind="izh", n=int(n_inh), rate_hz=0.0, i_ext=0.0, abcd=abcd[:, n_exc:].copy())]
    p = min(1.0, float(n_conn) / n)
    projs = []

    def add(pre, post, n_pre, n_post, pp, scale, e_rev, no_self=False):
        rp, ci = bernoulli_csr(rng, n_pre, n_post, pp, no_self=no_self)
        g = uniform_weights(rng, ci.size, scale)
        projs.append(dict(pre=pre, post=post, row_ptr=rp, col_idx=ci, g=g, e_rev=e_rev, tau=IZH_TAU, stdp=None))

    add(0, 1, n_in, n_exc, p_in, IZH_G_IN, E_EXC)
    add(0, 2, n_in, n_inh, p_in, IZH_G_IN, E_EXC)
    add(1, 1, n_exc, n_exc, p, IZH_G_E * g_scale, E_EXC, no_self=True)
    add(1, 2, n_exc, n_inh, p, IZH_G_E * g_scale, E_EXC)
    add(2, 1, n_inh, n_exc, p, IZH_G_I * g_scale, IZH_E_INH)
    add(2, 2, n_inh, n_inh, p, IZH_G_I * g_scale, IZH_E_INH, no_self=True)
    return dict(g_scale=1.0, seed=int(seed), pops=pops, projs=projs, g_scale_swept=float(g_scale))


def izhikevich_calibration_config(n_conn_values, g_scales, *, n_exc=800, n_inh=200, steps=5000, key=8000):
    """Calibration sweep of the 4:1 Izhikevich network (Section 5.1, Fig. 1
    and Table 1): one run per (nConn, gScale) pair; the runs of one nConn
    share the network's neurons, connectivity pattern and Poisson stream, and
    differ in the recurrent weights' scale only.  The criterion population is
    E (avgSpike of the excitatory neurons)."""
    spec = dict(dt=0.1, substeps=3, instances=[], steps=int(steps), n_conn=[], grid=[], pop=1)
    for i, x in enumerate(n_conn_values):
        for j, g in enumerate(g_scales):
            inst = izhikevich_instance(float(x), n_exc=n_exc, n_inh=n_inh, g_scale=float(g),
                                       seed=instance_seed(key + 2, i), conn_seed=key + 1 + i)
            spec["instances"].append(inst)
            spec["n_conn"].append(float(x))
            spec["grid"].append((i, j))
    return spec


def random_tiny(seed, *, n_pops=3, max_n=64, p=0.3, n_poisson=1, rate_hz=200.0, stdp=False,
                integer_g=False, g_scale=1.0):
    """Small random network for brute-force checks: arbitrary sizes, empty rows,
    all-to-all rows, self-projections.  ``integer_g`` draws g in {0,..,7} so
    that every sum is exact in any order."""
    rng = np.random.default_rng(seed)
    pops = []
    for i in range(n_pops):
        kind = "poisson" if i < n_poisson else "hh"
        pops.append(dict(name=f"P{i}", kind=kind, n=int(rng.integers(1, max_n + 1)),
                         rate_hz=rate_hz if kind == "poisson" else 0.0, i_ext=0.0))
    projs = []
    for post in range(n_poisson, n_pops):
        for pre in range(n_pops):
            if rng.random() < 0.6 or pre == post - 1:
                pp = p if rng.random() < 0.7 else 1.0
                rp, ci = bernoulli_csr(rng, pops[pre]["n"], pops[post]["n"], pp)
                if integer_g:
                    g = rng.integers(0, 8, ci.size).astype(np.float32)
                else:
                    g = uniform_weights(rng, ci.size, 0.02)
                e_rev = 0.0 if rng.random() < 0.7 else -92.0
                projs.append(dict(pre=pre, post=post, row_ptr=rp, col_idx=ci, g=g, e_rev=e_rev,
                                  tau=float(rng.choice([1.0, 2.5, 5.0])), stdp=None))
    if stdp:
        for pr in projs:
            if pops[pr["pre"]]["kind"] == "hh":
                pr["stdp"] = dict(a_plus=STDP_A_PLUS, a_minus=STDP_A_MINUS, tau=STDP_TAU,
                                  g_max=float(pr["g"].max() if pr["g"].size else 0.02) * 1.5 + 1e-6)
                break
    return dict(dt=0.1, substeps=3, instances=[dict(g_scale=float(g_scale), seed=int(seed) + 77,
                                                    pops=pops, projs=projs)])


def forced_spikes(rng, n, frac):
    """Seeded synthetic spike set: a sorted random subset of round(frac*n) ids."""
    k = int(round(frac * n))
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)
