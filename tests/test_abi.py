"""The C-ABI library loads, exports every declared symbol, and rejects invalid
network descriptions on the host before touching the GPU."""
import copy
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1412_0595_amd import netgen, snn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "snn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(snn_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = snn.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(snn.EXPORTS) == names


def test_default_parameters():
    assert list(snn.default_hh()) == [7.15, 50.0, 1.43, -95.0, 0.02672, -63.563, 0.143]


def _tiny():
    return netgen.random_tiny(3, n_pops=3, max_n=20)


def _bad(mutate):
    spec = copy.deepcopy(_tiny())
    mutate(spec["instances"][0])
    rc, msg = snn.create_status(spec)
    return rc, msg


def _first_nonempty(inst):
    for q in inst["projs"]:
        if q["col_idx"].size > 2:
            return q
    raise AssertionError


@pytest.mark.parametrize("name,mutate,needle", [
    ("row_ptr0", lambda I: _first_nonempty(I)["row_ptr"].__setitem__(0, 1), "row_ptr[0]"),
    ("nnz", lambda I: _first_nonempty(I).__setitem__("row_ptr", _first_nonempty(I)["row_ptr"] + 0) or
     _first_nonempty(I)["row_ptr"].__setitem__(-1, _first_nonempty(I)["row_ptr"][-1] - 1), "nnz"),
    ("col_range", lambda I: _first_nonempty(I)["col_idx"].__setitem__(0, 10 ** 6), "out of range"),
    ("col_neg", lambda I: _first_nonempty(I)["col_idx"].__setitem__(0, -1), "out of range"),
    ("g_nan", lambda I: _first_nonempty(I)["g"].__setitem__(0, np.nan), "g["),
    ("g_neg", lambda I: _first_nonempty(I)["g"].__setitem__(0, -1.0), "g["),
    ("pop_index", lambda I: I["projs"][0].__setitem__("post", 99), "population index"),
    ("post_poisson", lambda I: I["projs"][0].__setitem__("post", 0), "Traub-Miles"),
    ("tau", lambda I: I["projs"][0].__setitem__("tau", 0.0), "tau"),
    ("gscale", lambda I: I.__setitem__("g_scale", float("inf")), "g_scale"),
    ("rate", lambda I: I["pops"][0].__setitem__("rate_hz", -1.0), "rate"),
    ("n_neg", lambda I: I["pops"][1].__setitem__("n", -5), "n < 0"),
])
def test_invalid_description_rejected(name, mutate, needle):
    rc, msg = _bad(mutate)
    assert rc == snn.SNN_EINVAL, (rc, msg)
    assert needle in msg, msg


def test_unsorted_row_rejected():
    spec = copy.deepcopy(_tiny())
    q = _first_nonempty(spec["instances"][0])
    rp = q["row_ptr"]
    for i in range(rp.size - 1):
        if rp[i + 1] - rp[i] >= 2:
            a = q["col_idx"][rp[i]]
            q["col_idx"][rp[i]] = q["col_idx"][rp[i] + 1]
            q["col_idx"][rp[i] + 1] = a
            break
    rc, msg = snn.create_status(spec)
    assert rc == snn.SNN_EINVAL and "not strictly ascending" in msg


def test_duplicate_synapse_rejected():
    """A row may not list the same post neuron twice: the tiled propagation
    relies on distinct columns within a row."""
    spec = copy.deepcopy(_tiny())
    q = _first_nonempty(spec["instances"][0])
    rp = q["row_ptr"]
    for i in range(rp.size - 1):
        if rp[i + 1] - rp[i] >= 2:
            q["col_idx"][rp[i] + 1] = q["col_idx"][rp[i]]
            break
    rc, msg = snn.create_status(spec)
    assert rc == snn.SNN_EINVAL and "not strictly ascending" in msg


def test_decreasing_row_ptr_rejected():
    spec = copy.deepcopy(_tiny())
    q = _first_nonempty(spec["instances"][0])
    rp = q["row_ptr"].astype(np.int32).copy()
    i = int(np.argmax(np.diff(rp) > 0))
    rp[i + 1] = rp[i] - 1 if rp[i] > 0 else rp[i + 1]
    if rp[i + 1] >= rp[i]:
        rp[i + 1], rp[i] = 0, 1
    q["row_ptr"] = rp
    rc, msg = snn.create_status(spec)
    assert rc == snn.SNN_EINVAL


def test_bad_config_rejected():
    spec = copy.deepcopy(_tiny())
    spec["dt"] = 0.0
    assert snn.create_status(spec)[0] == snn.SNN_EINVAL
    spec = copy.deepcopy(_tiny())
    spec["substeps"] = 0
    assert snn.create_status(spec)[0] == snn.SNN_EINVAL


def test_too_many_incoming_projections_rejected():
    spec = copy.deepcopy(_tiny())
    inst = spec["instances"][0]
    q = inst["projs"][0]
    inst["projs"] = [copy.deepcopy(q) for _ in range(5)]
    rc, msg = snn.create_status(spec)
    assert rc == snn.SNN_EINVAL and "incoming" in msg


def test_conductance_range_rejected():
    spec = copy.deepcopy(_tiny())
    spec["instances"][0]["g_scale"] = 3e38
    rc, msg = snn.create_status(spec)
    assert rc == snn.SNN_ERANGE, msg


def test_single_weight_range_rejected():
    """One synapse with g_scale * g of 2^11 uS or more is rejected even when
    the reachable conductance is in range (the kernels round every increment
    with a method exact below 2^51 units of 2^-40 uS)."""
    spec = copy.deepcopy(_tiny())
    q = _first_nonempty(spec["instances"][0])
    q["g"] = np.asarray(q["g"], np.float32).copy()
    q["g"][0] = 3000.0
    rc, msg = snn.create_status(spec)
    assert rc == snn.SNN_ERANGE and "largest weight" in msg, msg


def _izh_spec(n_conn=50):
    inst = netgen.izhikevich_instance(n_conn, n_exc=80, n_inh=20, n_in=50, seed=1, conn_seed=2)
    return dict(dt=0.1, substeps=3, instances=[inst])


def test_izhikevich_description_validated():
    """An Izhikevich population passes the host checks; a non-finite a, b, c
    or d, missing parameters or a wrong kind are rejected before any device
    call."""
    rc, msg = snn.create_status(_izh_spec())
    assert rc in (snn.SNN_OK, snn.SNN_EDEVICE), msg
    for k in range(4):
        spec = _izh_spec()
        bad = spec["instances"][0]["pops"][1]["abcd"].copy()
        bad[k, 7] = np.inf
        spec["instances"][0]["pops"][1]["abcd"] = bad
        rc, msg = snn.create_status(spec)
        assert rc == snn.SNN_EINVAL and "Izhikevich parameter" in msg, msg
    L = snn.load()
    cfg, keep = snn.build_config(_izh_spec())
    inst = snn.InstDesc.from_address(cfg.inst)
    pops = (snn.PopDesc * inst.n_pops).from_address(inst.pops)
    pops[2].izh_abcd = None
    h = ctypes.c_void_p()
    rc = L.snn_create(ctypes.byref(cfg), ctypes.byref(h))
    assert rc == snn.SNN_EINVAL and "izh_abcd is NULL" in snn.last_error()
    pops[2].izh_abcd = pops[1].izh_abcd
    pops[2].kind = 7
    rc = L.snn_create(ctypes.byref(cfg), ctypes.byref(h))
    assert rc == snn.SNN_EINVAL and "bad kind" in snn.last_error()


def test_valid_description_passes_validation():
    """A valid network passes every host check; without a GPU the first
    device call then fails cleanly with SNN_EDEVICE (on a GPU it succeeds)."""
    rc, msg = snn.create_status(_tiny())
    assert rc in (snn.SNN_OK, snn.SNN_EDEVICE), msg


def test_null_arguments():
    L = snn.load()
    assert L.snn_create(None, None) == snn.SNN_EINVAL
    assert L.snn_step(None, 1) == snn.SNN_EINVAL
    assert L.snn_time(None) == -1
    ms = (ctypes.c_double * 3)()
    cnt = (ctypes.c_int64 * 3)()
    assert L.snn_profile_steps(None, 10, ms, cnt) == snn.SNN_EINVAL
    L.snn_destroy(None)


def test_header_compiles_as_c_and_host_routines_run(tmp_path):
    """include/snn.h is a plain C11 header; a C program linked against
    libsnn.so calls the host calibration routines (no GPU involved)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    lib_dir = os.path.dirname(snn.LIB_PATH)
    exe = str(tmp_path / "abi_calibrate")
    subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "c", "abi_calibrate.c"), "-o", exe,
                           "-L", lib_dir, "-lsnn", f"-Wl,-rpath,{lib_dir}", "-lm"])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    fit, sel = out.stdout.strip().splitlines()
    k1, k2, k3, mape = (float(v) for v in fit.split())
    assert k1 == pytest.approx(1318.0, rel=1e-7) and k2 == pytest.approx(109.9, rel=1e-7)
    assert k3 == pytest.approx(-0.28, rel=1e-7) and mape < 1e-6
    # nConn 10 -> run 0 (the reference); nConn 20 -> run 1 (|5.5 - 5| = |4 - 5| / 2; run 3 has NaNs)
    assert sel.split() == ["2", "10", "0", "20", "1"]


def test_neuron_count_limit_rejected():
    """The neuron update addresses its 8-byte per-neuron arrays by 32-bit byte
    offsets, so more than 2^29 neurons (each population padded to 64) are
    refused before any device call."""
    pops = [dict(name="A", kind="poisson", n=1 << 29, rate_hz=1.0, i_ext=0.0),
            dict(name="B", kind="hh", n=1, rate_hz=0.0, i_ext=0.0)]
    spec = dict(dt=0.1, substeps=3, instances=[dict(g_scale=1.0, seed=1, pops=pops, projs=[])])
    rc, msg = snn.create_status(spec)
    assert rc == snn.SNN_ERANGE and "neurons" in msg, msg
