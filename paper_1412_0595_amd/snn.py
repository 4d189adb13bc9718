"""Python binding of libsnn.so (include/snn.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels; PyTorch only
supplies device memory (its caching allocator, through the library's
alloc/free hooks) and the stream the work is enqueued on.  If the library
has not been built, importing works but creating a network raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnn.so")

SNN_OK, SNN_EINVAL, SNN_ENOMEM, SNN_EDEVICE, SNN_ESTATE, SNN_ERANGE = 0, -1, -2, -3, -4, -5
POISSON, TRAUB_MILES, IZHIKEVICH = 0, 1, 2
V, M, H, N = 0, 1, 2, 3
U = 1   # recovery variable of an Izhikevich population
NOALLOC_SCRATCH_BYTES = 64 << 20   # SNN_NOALLOC_SCRATCH_BYTES of include/snn.h

# Every symbol include/snn.h declares.
EXPORTS = [
    "snn_default_hh", "snn_create", "snn_destroy", "snn_step", "snn_sync", "snn_time",
    "snn_get_spikes", "snn_get_raster", "snn_get_state", "snn_set_state", "snn_get_state_f64",
    "snn_set_state_f64", "snn_get_conductance", "snn_set_conductance", "snn_get_last_spikes",
    "snn_set_last_spikes", "snn_get_vbar", "snn_get_nan_counts", "snn_set_gscale", "snn_get_weights",
    "snn_memory_bytes", "snn_get_launch", "snn_set_launch", "snn_time_steps", "snn_time_kernel", "snn_profile_steps",
    "snn_last_error", "snn_reset", "snn_weight_count", "snn_weight_offset", "snn_get_weights_device",
    "snn_set_weights_device", "snn_forward_record", "snn_backward", "snn_gscale_select", "snn_gscale_fit",
    "snn_backward_noalloc",
]


class PopDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("rate_hz", C.c_double), ("i_ext_nA", C.c_double),
                ("hh", C.c_double * 7), ("record_vbar", C.c_int32), ("izh_abcd", C.c_void_p)]


class ProjDesc(C.Structure):
    _fields_ = [("pre_pop", C.c_int32), ("post_pop", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("g", C.c_void_p),
                ("e_rev_mV", C.c_float), ("tau_ms", C.c_float), ("stdp", C.c_int32),
                ("a_plus", C.c_float), ("a_minus", C.c_float), ("tau_stdp_ms", C.c_float), ("g_max", C.c_float)]


class InstDesc(C.Structure):
    _fields_ = [("n_pops", C.c_int32), ("n_projs", C.c_int32), ("pops", C.c_void_p), ("projs", C.c_void_p),
                ("g_scale", C.c_float), ("seed", C.c_uint64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Config(C.Structure):
    _fields_ = [("dt_ms", C.c_double), ("substeps", C.c_int32), ("n_instances", C.c_int32),
                ("inst", C.c_void_p), ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", C.c_void_p), ("raster_steps", C.c_int32), ("autotune", C.c_int32),
                ("tune_cache", C.c_char_p)]


class Launch(C.Structure):
    _fields_ = [("neuron_block", C.c_int32), ("prop_blocks", C.c_int32), ("prop_block", C.c_int32),
                ("chunk", C.c_int32), ("mode", C.c_int32)]


class SNNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"snn error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libsnn.so; raise if it was not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime; loading it first makes libsnn.so bind
    # to that same runtime (one HSA runtime per process) instead of pulling
    # in a second copy from /opt/rocm
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "snn_default_hh": (None, [vp]),
        "snn_create": (C.c_int, [vp, vp]),
        "snn_destroy": (None, [vp]),
        "snn_step": (C.c_int, [vp, i64]),
        "snn_sync": (C.c_int, [vp]),
        "snn_time": (i64, [vp]),
        "snn_get_spikes": (C.c_int, [vp, i32, i32, vp]),
        "snn_get_raster": (C.c_int, [vp, i32, i32, i64, i64, vp, vp, i64]),
        "snn_get_state": (C.c_int, [vp, i32, i32, i32, vp]),
        "snn_set_state": (C.c_int, [vp, i32, i32, i32, vp]),
        "snn_get_state_f64": (C.c_int, [vp, i32, i32, i32, vp]),
        "snn_set_state_f64": (C.c_int, [vp, i32, i32, i32, vp]),
        "snn_get_conductance": (C.c_int, [vp, i32, i32, vp]),
        "snn_set_conductance": (C.c_int, [vp, i32, i32, vp]),
        "snn_get_last_spikes": (C.c_int, [vp, i32, i32, vp]),
        "snn_set_last_spikes": (C.c_int, [vp, i32, i32, vp]),
        "snn_get_vbar": (C.c_int, [vp, i32, i32, vp]),
        "snn_get_nan_counts": (C.c_int, [vp, vp]),
        "snn_set_gscale": (C.c_int, [vp, vp]),
        "snn_get_weights": (C.c_int, [vp, i32, i32, vp]),
        "snn_memory_bytes": (C.c_int, [vp, vp]),
        "snn_get_launch": (C.c_int, [vp, vp]),
        "snn_set_launch": (C.c_int, [vp, vp]),
        "snn_time_steps": (C.c_int, [vp, i64, vp]),
        "snn_time_kernel": (C.c_int, [vp, i32, i64, vp]),
        "snn_profile_steps": (C.c_int, [vp, i64, vp, vp]),
        "snn_last_error": (C.c_char_p, []),
        "snn_reset": (C.c_int, [vp]),
        "snn_weight_count": (i64, [vp]),
        "snn_weight_offset": (C.c_int, [vp, i32, i32, vp]),
        "snn_get_weights_device": (C.c_int, [vp, vp]),
        "snn_set_weights_device": (C.c_int, [vp, vp]),
        "snn_forward_record": (C.c_int, [vp, i32, i64, i32, vp]),
        "snn_backward": (C.c_int, [vp, vp, vp, vp, vp]),
        "snn_backward_noalloc": (C.c_int, [vp, vp, vp, vp]),
        "snn_gscale_select": (C.c_int, [i64, vp, vp, vp, vp, i64, vp, vp, vp]),
        "snn_gscale_fit": (C.c_int, [i64, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def last_error():
    return load().snn_last_error().decode()


def _check(rc):
    if rc != SNN_OK:
        raise SNNError(rc, last_error())


def default_hh():
    out = np.zeros(7)
    load().snn_default_hh(out.ctypes.data)
    return out


def _p(a):
    return C.c_void_p(a.ctypes.data)


def build_config(spec, *, record_vbar=(), raster_steps=0, autotune=False, tune_cache=None, hh_params=None):
    """Marshal a network spec (see netgen) into snn_config; returns (cfg, keepalive)."""
    keep = []
    hh_default = default_hh() if _lib is not None or os.path.exists(LIB_PATH) else None
    insts = (InstDesc * len(spec["instances"]))()
    for b, inst in enumerate(spec["instances"]):
        pops = (PopDesc * len(inst["pops"]))()
        for k, p in enumerate(inst["pops"]):
            pops[k].kind = {"poisson": POISSON, "hh": TRAUB_MILES, "izh": IZHIKEVICH}[p["kind"]]
            if p["kind"] == "izh":
                abcd = np.ascontiguousarray(p["abcd"], np.float32)
                if abcd.shape != (4, int(p["n"])):
                    raise ValueError("abcd must be float32[4, n]")
                keep.append(abcd)
                pops[k].izh_abcd = abcd.ctypes.data
            pops[k].n = int(p["n"])
            pops[k].rate_hz = float(p.get("rate_hz", 0.0))
            pops[k].i_ext_nA = float(p.get("i_ext", 0.0))
            hp = None
            if hh_params is not None:
                hp = hh_params.get(k)
            vals = hp if hp is not None else hh_default
            for i in range(7):
                pops[k].hh[i] = float(vals[i])
            pops[k].record_vbar = 1 if (p.get("name") in record_vbar or k in record_vbar) else 0
        projs = (ProjDesc * max(1, len(inst["projs"])))()
        for k, q in enumerate(inst["projs"]):
            rp = np.ascontiguousarray(q["row_ptr"], np.int32)
            ci = np.ascontiguousarray(q["col_idx"], np.int32)
            g = np.ascontiguousarray(q["g"], np.float32)
            keep += [rp, ci, g]
            projs[k].pre_pop, projs[k].post_pop = int(q["pre"]), int(q["post"])
            projs[k].nnz = int(ci.size)
            projs[k].row_ptr, projs[k].col_idx, projs[k].g = rp.ctypes.data, ci.ctypes.data, g.ctypes.data
            projs[k].e_rev_mV, projs[k].tau_ms = float(q["e_rev"]), float(q["tau"])
            st = q.get("stdp")
            if st:
                projs[k].stdp = 1
                projs[k].a_plus, projs[k].a_minus = float(st["a_plus"]), float(st["a_minus"])
                projs[k].tau_stdp_ms, projs[k].g_max = float(st["tau"]), float(st["g_max"])
        keep += [pops, projs]
        insts[b].n_pops, insts[b].n_projs = len(inst["pops"]), len(inst["projs"])
        insts[b].pops, insts[b].projs = C.addressof(pops), C.addressof(projs)
        insts[b].g_scale = float(inst["g_scale"])
        insts[b].seed = int(inst["seed"])
    keep.append(insts)
    cfg = Config()
    cfg.dt_ms = float(spec.get("dt", 0.1))
    cfg.substeps = int(spec.get("substeps", 3))
    cfg.n_instances = len(spec["instances"])
    cfg.inst = C.addressof(insts)
    cfg.raster_steps = int(raster_steps)
    cfg.autotune = 1 if autotune else 0
    if tune_cache:
        tc = str(tune_cache).encode()
        keep.append(tc)
        cfg.tune_cache = tc
    return cfg, keep


class Network:
    """A batch of network instances on one GPU, driven through libsnn.so."""

    def __init__(self, spec, *, device=0, stream=None, record_vbar=(), raster_steps=0, autotune=False,
                 tune_cache=None, torch_alloc=True, hh_params=None):
        L = load()
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the spiking-network library runs only on the GPU")
        self._torch = torch
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.spec = spec
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        cfg, self._keep = build_config(spec, record_vbar=record_vbar, raster_steps=raster_steps, autotune=autotune,
                                       tune_cache=tune_cache, hh_params=hh_params)
        cfg.stream = self.stream.cuda_stream
        if torch_alloc:
            dev, strm = self.device.index, self.stream

            def _alloc(nbytes, ctx):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, strm)
                except Exception:
                    return None

            def _free(ptr, ctx):
                torch.cuda.caching_allocator_delete(ptr)

            self._alloc_cb, self._free_cb = ALLOC_FN(_alloc), FREE_FN(_free)
            cfg.alloc, cfg.free = self._alloc_cb, self._free_cb
        self.h = C.c_void_p()
        _check(L.snn_create(C.byref(cfg), C.byref(self.h)))
        self.n_instances = len(spec["instances"])
        # bumped by every call that changes what a backward pass would read
        # (the recording, the weights, g_scale): an autograd tape remembers it
        self.tape_generation = 0

    # ---------------------------------------------------------------- life
    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().snn_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -------------------------------------------------------------- stepping
    def step(self, n=1):
        _check(load().snn_step(self.h, int(n)))

    def sync(self):
        _check(load().snn_sync(self.h))

    @property
    def t(self):
        return int(load().snn_time(self.h))

    def time_steps(self, n):
        out = C.c_double()
        _check(load().snn_time_steps(self.h, int(n), C.byref(out)))
        return out.value

    def time_kernel(self, which, launches):
        """Mean ms per launch of one kernel (0 propagate, 1 potentiate,
        2 neuron) over back-to-back launches on a snapshot of the state."""
        out = C.c_double()
        _check(load().snn_time_kernel(self.h, int(which), int(launches), C.byref(out)))
        return out.value

    def profile_steps(self, n):
        """Advance n steps with direct, event-stamped launches; returns
        {kernel: (total ms, launches)} for propagate, potentiate, neuron."""
        ms = (C.c_double * 3)()
        cnt = (C.c_int64 * 3)()
        _check(load().snn_profile_steps(self.h, int(n), ms, cnt))
        return {k: (ms[i], int(cnt[i])) for i, k in enumerate(("propagate", "potentiate", "neuron"))}

    def reset(self):
        _check(load().snn_reset(self.h))

    # ------------------------------------------------------ weights / adjoint
    @property
    def weight_count(self):
        return int(load().snn_weight_count(self.h))

    def weight_offset(self, inst, proj):
        out = C.c_int64()
        _check(load().snn_weight_offset(self.h, int(inst), int(proj), C.byref(out)))
        return out.value

    def get_weights_device(self, out):
        """Copy the weight pool into a float32 CUDA tensor."""
        assert out.dtype == self._torch.float32 and out.is_cuda and out.numel() == self.weight_count
        _check(load().snn_get_weights_device(self.h, C.c_void_p(out.data_ptr())))

    def set_weights_device(self, src):
        src = src.contiguous()
        assert src.dtype == self._torch.float32 and src.is_cuda and src.numel() == self.weight_count
        self.tape_generation += 1
        _check(load().snn_set_weights_device(self.h, C.c_void_p(src.data_ptr())))

    def loss_size(self, pop):
        return sum(int(inst["pops"][pop]["n"]) for inst in self.spec["instances"])

    def forward_record(self, pop, n_steps, ckpt_every, vbar=None):
        """Reset, run n_steps recording raster and checkpoints; returns Vbar of
        population pop (float64 CUDA tensor, instance-major)."""
        t = self._torch
        if vbar is None:
            vbar = t.empty(self.loss_size(pop), dtype=t.float64, device=self.device)
        self.tape_generation += 1
        _check(load().snn_forward_record(self.h, int(pop), int(n_steps), int(ckpt_every), C.c_void_p(vbar.data_ptr())))
        return vbar

    def backward(self, dvbar, check=False):
        """Returns (dL/dg float32 [weight_count], dL/dg_scale float64 [n_inst],
        recompute mismatches or None)."""
        t = self._torch
        dvbar = dvbar.contiguous().to(t.float64)
        dg = t.empty(self.weight_count, dtype=t.float32, device=self.device)
        ds = t.empty(self.n_instances, dtype=t.float64, device=self.device)
        mm = C.c_int64(-1)
        _check(load().snn_backward(self.h, C.c_void_p(dvbar.data_ptr()), C.c_void_p(dg.data_ptr()),
                                   C.c_void_p(ds.data_ptr()), C.byref(mm) if check else None))
        return dg, ds, (mm.value if check else None)

    def backward_noalloc(self, dvbar, dg, ds):
        """snn_backward_noalloc into caller-owned tensors dg (float32
        [weight_count]) and ds (float64 [n_inst]); the library allocates
        nothing for it."""
        t = self._torch
        assert dvbar.dtype == t.float64 and dvbar.is_contiguous()
        assert dg.dtype == t.float32 and dg.is_contiguous() and dg.numel() == self.weight_count
        assert ds.dtype == t.float64 and ds.is_contiguous() and ds.numel() == self.n_instances
        _check(load().snn_backward_noalloc(self.h, C.c_void_p(dvbar.data_ptr()), C.c_void_p(dg.data_ptr()),
                                           C.c_void_p(ds.data_ptr())))

    # ----------------------------------------------------------------- state
    def _n(self, inst, pop):
        return int(self.spec["instances"][inst]["pops"][pop]["n"])

    def _npost(self, inst, proj):
        q = self.spec["instances"][inst]["projs"][proj]
        return int(self.spec["instances"][inst]["pops"][q["post"]]["n"])

    def spikes(self, inst, pop):
        out = np.zeros(self._n(inst, pop), np.int32)
        _check(load().snn_get_spikes(self.h, inst, pop, _p(out)))
        return out

    def raster(self, inst, pop, t0, t1):
        """List of ascending id arrays, one per step in [t0, t1)."""
        off = np.zeros(t1 - t0 + 1, np.int64)
        cap = max(16, self._n(inst, pop) * (t1 - t0) // 8)
        while True:
            ids = np.zeros(cap, np.int32)
            rc = load().snn_get_raster(self.h, inst, pop, int(t0), int(t1), _p(off), _p(ids), int(cap))
            if rc == SNN_ERANGE and off[-1] > cap:
                cap = int(off[-1])
                continue
            _check(rc)
            return [ids[off[k]:off[k + 1]].copy() for k in range(t1 - t0)]

    def state(self, inst, pop, var, f64=True):
        n = self._n(inst, pop)
        if f64:
            out = np.zeros(n, np.float64)
            _check(load().snn_get_state_f64(self.h, inst, pop, var, _p(out)))
        else:
            out = np.zeros(n, np.float32)
            _check(load().snn_get_state(self.h, inst, pop, var, _p(out)))
        return out

    def set_state(self, inst, pop, var, vals):
        a = np.ascontiguousarray(vals, np.float64)
        assert a.size == self._n(inst, pop)
        _check(load().snn_set_state_f64(self.h, inst, pop, var, _p(a)))

    def conductance(self, inst, proj):
        out = np.zeros(self._npost(inst, proj), np.float64)
        _check(load().snn_get_conductance(self.h, inst, proj, _p(out)))
        return out

    def set_conductance(self, inst, proj, vals):
        a = np.ascontiguousarray(vals, np.float64)
        _check(load().snn_set_conductance(self.h, inst, proj, _p(a)))

    def last_spikes(self, inst, pop):
        out = np.zeros(self._n(inst, pop), np.uint8)
        _check(load().snn_get_last_spikes(self.h, inst, pop, _p(out)))
        return out

    def set_last_spikes(self, inst, pop, flags):
        a = np.ascontiguousarray(flags, np.uint8)
        _check(load().snn_set_last_spikes(self.h, inst, pop, _p(a)))

    def vbar_sum(self, inst, pop):
        out = np.zeros(self._n(inst, pop), np.float64)
        _check(load().snn_get_vbar(self.h, inst, pop, _p(out)))
        return out

    def nan_counts(self):
        out = np.zeros(self.n_instances, np.int32)
        _check(load().snn_get_nan_counts(self.h, _p(out)))
        return out

    def set_gscale(self, per_instance):
        a = np.ascontiguousarray(per_instance, np.float32)
        assert a.size == self.n_instances
        self.tape_generation += 1
        _check(load().snn_set_gscale(self.h, _p(a)))

    def weights(self, inst, proj):
        n = int(np.asarray(self.spec["instances"][inst]["projs"][proj]["col_idx"]).size)
        out = np.zeros(n, np.float32)
        _check(load().snn_get_weights(self.h, inst, proj, _p(out)))
        return out

    def memory_bytes(self):
        n = sum(len(i["projs"]) for i in self.spec["instances"])
        out = np.zeros(max(n, 1), np.int64)
        _check(load().snn_memory_bytes(self.h, _p(out)))
        return out[:n]

    @property
    def launch(self):
        L = Launch()
        _check(load().snn_get_launch(self.h, C.byref(L)))
        return dict(neuron_block=L.neuron_block, prop_blocks=L.prop_blocks, prop_block=L.prop_block, chunk=L.chunk,
                    mode=L.mode)

    def set_launch(self, **kw):
        cur = self.launch
        cur.update(kw)
        L = Launch(**cur)
        _check(load().snn_set_launch(self.h, C.byref(L)))


def create_status(spec, **kw):
    """snn_create on a spec without keeping the net: (status, message).  On a
    machine without a GPU, validation errors still come back as SNN_EINVAL."""
    L = load()
    cfg, keep = build_config(spec, **kw)
    h = C.c_void_p()
    rc = L.snn_create(C.byref(cfg), C.byref(h))
    msg = last_error()
    if rc == SNN_OK:
        L.snn_destroy(h)
    return rc, msg


def gscale_select(n_conn, g_scale, avg_spike, n_nans, ref_run):
    """Fig. 1's selection over a sweep's per-run table (snn_gscale_select):
    returns (distinct nConn ascending, picked run index per nConn or -1)."""
    x = np.ascontiguousarray(n_conn, np.float64)
    n = x.size
    g = np.ascontiguousarray(g_scale, np.float64)
    a = np.ascontiguousarray(avg_spike, np.float64)
    z = np.ascontiguousarray(n_nans, np.int32)
    assert g.size == n and a.size == n and z.size == n
    groups = np.zeros(max(n, 1), np.float64)
    picked = np.zeros(max(n, 1), np.int64)
    ng = C.c_int64(0)
    _check(load().snn_gscale_select(n, _p(x), _p(g), _p(a), _p(z), int(ref_run), C.byref(ng),
                                    _p(groups), _p(picked)))
    return groups[:ng.value].copy(), picked[:ng.value].copy()


def gscale_fit(n_conn, g_scale):
    """Least-squares k1, k2, k3 of gScale = k1 / (k2 + nConn) + k3 and the
    fit's MAPE in percent (snn_gscale_fit)."""
    x = np.ascontiguousarray(n_conn, np.float64)
    y = np.ascontiguousarray(g_scale, np.float64)
    assert x.size == y.size
    k = np.zeros(3, np.float64)
    mape = C.c_double(0.0)
    _check(load().snn_gscale_fit(x.size, _p(x), _p(y), _p(k), C.byref(mape)))
    return k, mape.value
