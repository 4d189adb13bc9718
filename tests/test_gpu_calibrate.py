"""The calibration of Section 5.1 (Fig. 1) end to end: a (nConn, gScale)
sweep stepped as one batched network on the GPU, its per-run table against
the FP64 oracle's, and the library's selection and law fit against the
calibration oracle's on the same table."""
import numpy as np
import pytest

from oracle import calibrate as ocal
from oracle import oracle as O
from paper_1412_0595_amd import netgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def snn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_0595_amd import snn as S
    S.load()
    return S


def say(*a):
    print(*a, flush=True)


def check_sweep(snn, spec, ref_n_conn, T):
    """Step the sweep on the GPU, compare its table with the oracle's and the
    library's selection and fit with the calibration oracle's."""
    from paper_1412_0595_amd import calibrate as cal
    pop = spec.get("pop", 1)
    ref = cal.reference_run(spec, ref_n_conn, 1.0)
    net = snn.Network(spec)
    net.step(T)
    res = cal.calibrate(net, spec, ref)
    # the per-run table against the oracle run by run
    o_avg, o_nan, differing, total = [], [], 0, 0
    for k, inst in enumerate(spec["instances"]):
        orc = O.OracleNet(inst)
        orc.step(T)
        c = orc.counts(pop)
        g = net.spikes(k, pop)
        if orc.nan_count == 0 and res["n_nans"][k] == 0:
            differing += int(np.sum(c != g))
            total += c.size
        o_avg.append(c.mean())
        o_nan.append(orc.nan_count)
    net.close()
    nan_runs = np.asarray(o_nan) > 0
    say(f"  criterion neurons with a different spike count: {differing} of {total} (NaN-free runs); "
        f"runs with NaNs {int(nan_runs.sum())}; NaN counts differing from the oracle's in "
        f"{int(np.sum(np.asarray(o_nan) != res['n_nans']))} runs")
    assert differing == 0
    np.testing.assert_array_equal(res["n_nans"], np.asarray(o_nan))
    # selection and fit: bit-exact picks and 1e-6 coefficients on the same table
    groups, picked = ocal.select(res["n_conn"], res["g_scale"], res["avg_spike"], res["n_nans"], ref)
    np.testing.assert_array_equal(res["groups"], groups)
    np.testing.assert_array_equal(res["picked"], picked)
    ok = picked >= 0
    k = ocal.fit(groups[ok], res["g_scale"][picked[ok]])
    say(f"  picked gScale {res['g_scale'][picked].round(3).tolist()}; k {res['k'].tolist()} MAPE {res['mape']:.2f}%")
    np.testing.assert_allclose(res["k"], k, rtol=1e-6, atol=1e-9 * np.abs(k).max())
    assert res["mape"] == pytest.approx(ocal.mape(k, groups[ok], res["g_scale"][picked[ok]]), rel=1e-6)
    # where the oracle's own table agrees, so does its selection
    o_avg = np.where(nan_runs, res["avg_spike"], np.asarray(o_avg))
    if np.array_equal(o_avg, res["avg_spike"]):
        np.testing.assert_array_equal(ocal.select(res["n_conn"], res["g_scale"], o_avg, o_nan, ref)[1], picked)
    assert not np.any(nan_runs[picked[ok]])
    # the calibrated gScale falls as nConn grows (more inputs, each as strong)
    assert np.all(np.diff(res["g_scale"][picked]) <= 0)
    return res, nan_runs


def test_calibration_sweep_matches_oracle(snn):
    T = 1000
    # gScale 3000 drives every run to NaNs while its B spike level stays
    # near the reference's: Fig. 1's NaN filter has to keep those runs out
    gs = list(10.0 ** np.linspace(-1.0, 1.0, 17)) + [3000.0]
    spec = netgen.calibration_config([20, 30, 40, 60, 80], gs, n_b=200, n_c=20, ref_n_conn=20.0, steps=T)
    say(f"case: calibration sweep of {len(spec['instances'])} runs, {T} steps, batched on the GPU")
    res, nan_runs = check_sweep(snn, spec, 20.0, T)
    assert np.all(nan_runs[res["g_scale"] == 3000.0])
    ref = int(np.flatnonzero((res["n_conn"] == 20.0) & (res["g_scale"] == 1.0))[0])
    unfiltered = ocal.select(res["n_conn"], res["g_scale"], res["avg_spike"], np.zeros_like(res["n_nans"]), ref)[1]
    say(f"  nConn groups whose pick a selection without the NaN filter would change: "
        f"{int(np.sum(unfiltered != res['picked']))}")


@pytest.mark.parametrize("swept", ["kc", "lhi"])
def test_lhi_variant_calibration_matches_oracle(snn, swept):
    """The LHI variant (PN -> LHI -| KC feed-forward inhibition): the PN->KC
    and the PN->LHI scale each swept with the other held at 1."""
    T = 1000
    spec = netgen.mushroom_body_calibration_config([40, 60, 80, 120, 160], 10.0 ** np.linspace(-1.0, 1.0, 17),
                                                   swept=swept, n_lhi=20, n_kc=100, n_dn=10, ref_n_pn=40, steps=T)
    say(f"case: LHI variant, PN->{swept.upper()} scale swept, {len(spec['instances'])} runs, {T} steps")
    check_sweep(snn, spec, spec["n_conn"][0], T)
