"""The conductance-scale calibration of Section 5.1 (Fig. 1) driven through
the library: the sweep over (nConn, gScale) runs as one batched network on
the GPU, its per-run table (nConn, gScale, avgSpike, NaN count) is read back,
and snn_gscale_select and snn_gscale_fit pick one gScale per nConn and fit
gScale = k1 / (k2 + nConn) + k3."""
from __future__ import annotations

import numpy as np

from . import snn


def swept_scale(inst):
    """The run's swept conductance scale: the instance g_scale, or the scale
    built into the swept projection's weights (the LHI variant's two scales)."""
    return float(inst.get("g_scale_swept", inst["g_scale"]))


def reference_run(spec, ref_n_conn, ref_g_scale):
    """Index of the run at the reference (nConn, gScale) of Fig. 1."""
    hits = [k for k, inst in enumerate(spec["instances"])
            if spec["n_conn"][k] == float(ref_n_conn) and swept_scale(inst) == float(ref_g_scale)]
    if len(hits) != 1:
        raise ValueError(f"the sweep has {len(hits)} runs at nConn {ref_n_conn}, gScale {ref_g_scale}")
    return hits[0]


def sweep_table(net, spec, pop=None):
    """Per-run table of a stepped sweep: nConn, gScale, avgSpike (mean spike
    count per neuron of population pop since create; default: the sweep's
    criterion population, B of the layered model) and NaN count."""
    n = len(spec["instances"])
    pop = spec.get("pop", 1) if pop is None else pop
    n_conn = np.asarray(spec["n_conn"], np.float64)
    g_scale = np.array([swept_scale(inst) for inst in spec["instances"]], np.float64)
    avg = np.array([net.spikes(k, pop).mean() for k in range(n)], np.float64)
    return n_conn, g_scale, avg, net.nan_counts()


def calibrate(net, spec, ref_run, pop=None):
    """Fig. 1 on a stepped sweep: returns the table, the distinct nConn, the
    picked run per nConn (-1: none NaN-free), the fitted (k1, k2, k3) and the
    fit's MAPE in percent."""
    n_conn, g_scale, avg, nans = sweep_table(net, spec, pop)
    groups, picked = snn.gscale_select(n_conn, g_scale, avg, nans, ref_run)
    ok = picked >= 0
    k, mape = snn.gscale_fit(groups[ok], g_scale[picked[ok]])
    return dict(n_conn=n_conn, g_scale=g_scale, avg_spike=avg, n_nans=nans, groups=groups, picked=picked,
                k=k, mape=mape)
