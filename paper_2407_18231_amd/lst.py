"""Python binding of liblst (ctypes; argument marshalling only).

Every computation happens in the HIP library; this module converts numpy
arrays (or torch tensors on the GPU, via LST_DEVICE_PTRS) to the C structs of
``include/lst.h`` and copies results back.  If ``liblst.so`` has not been
built, importing the library raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblst.so")

LST_OK = 0
LST_PENDING = 1
STATUS = {0: "OK", 1: "PENDING", -1: "INVALID_ARG", -2: "DEVICE", -3: "NO_GEOMETRY",
          -4: "BAD_GEOMETRY", -5: "BAD_MODULE", -6: "NONFINITE", -7: "OOM",
          -8: "TOO_LARGE", -9: "QUEUE_FULL", -10: "UNKNOWN_TICKET", -11: "HIT_OUTSIDE"}
LST_FLAG_BEND = 1
LST_FLAG_STAGE_TIMES = 2
LST_FLAG_TC_CLEAN = 4
LST_FLAG_SEEDS_TRIPLETS = 8
LST_FLAG_SKIP_LAYER = 16
STAGES = ("ingest", "md", "ls", "t3", "t5", "seed_lookup", "pt", "tc")
LST_DEVICE_PTRS = 1
TC_PT5, TC_PT3, TC_T5, TC_PLS = 0, 1, 2, 3
NOALLOC_MAX_HITS, NOALLOC_MAX_PLS = 131072, 8192


class LstError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class lst_params(C.Structure):
    _fields_ = [("device", C.c_int32), ("B", C.c_double), ("pt_min", C.c_double),
                ("L", C.c_double), ("sig_rphi", C.c_double), ("sig_c", C.c_double),
                ("n_sigma", C.c_double), ("flags", C.c_uint32), ("max_batch", C.c_uint32),
                ("n_slots", C.c_uint32), ("queue_depth", C.c_uint32),
                ("mem_budget", C.c_uint64), ("n_phi_bins", C.c_uint32), ("n_kappa_bins", C.c_uint32),
                ("ls_group", C.c_uint32), ("ls_waves", C.c_uint32), ("stream", C.c_void_p)]


MODULE_DTYPE = np.dtype([("kind", "<u4"), ("layer", "<u4"), ("side", "<i4"), ("pad", "<u4"),
                         ("s_lo", "<f8"), ("s_hi", "<f8"), ("c_min", "<f8"), ("c_max", "<f8"),
                         ("phi_min", "<f8"), ("phi_max", "<f8")])


class lst_event_in(C.Structure):
    _fields_ = [("n_hits", C.c_uint32), ("n_pls", C.c_uint32),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("module", C.c_void_p), ("sensor", C.c_void_p),
                ("pls_par", C.c_void_p), ("pls_cov", C.c_void_p),
                ("flags", C.c_uint32), ("pad", C.c_uint32), ("pls_nhits", C.c_void_p)]


class lst_event_out(C.Structure):
    _fields_ = [("n_md", C.c_uint32), ("n_ls", C.c_uint32), ("n_t3", C.c_uint32),
                ("n_t5", C.c_uint32), ("n_pt3", C.c_uint32), ("n_pt5", C.c_uint32),
                ("n_tc", C.c_uint32), ("status", C.c_uint32),
                ("md", C.POINTER(C.c_uint32)), ("ls", C.POINTER(C.c_uint32)),
                ("t3", C.POINTER(C.c_uint32)), ("t5", C.POINTER(C.c_uint32)),
                ("pt3", C.POINTER(C.c_uint32)), ("pt5", C.POINTER(C.c_uint32)),
                ("tc", C.POINTER(C.c_uint32)), ("t3_kappa", C.POINTER(C.c_float)),
                ("latency_us", C.c_double), ("ticket", C.c_uint64),
                ("n_flag_regrow", C.c_uint32), ("n_stage", C.c_uint32),
                ("stage_ns", C.c_uint64 * len(STAGES)), ("batch_events", C.c_uint32),
                ("n_tcc", C.c_uint32), ("footprint", C.c_uint64), ("tcc", C.POINTER(C.c_uint32)),
                ("n_seeds", C.c_uint32), ("seeds", C.POINTER(C.c_uint32))]


_LISTS = ("md", "ls", "t3", "t5", "pt3", "pt5", "tc")


class lst_event_dev_out(C.Structure):
    _fields_ = ([(k, C.c_void_p) for k in _LISTS] + [("t3_kappa", C.c_void_p)]
                + [("cap_" + k, C.c_uint32) for k in _LISTS] + [("n_" + k, C.c_uint32) for k in _LISTS])


_P = C.POINTER
_lib = None


def load(path: str = LIB_PATH):
    """Load liblst.so; raises when it is missing (build it with
    ``python -m paper_2407_18231_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run python -m paper_2407_18231_amd.build")
    _share_hip_runtime_with_torch()
    L = C.CDLL(path)
    sig = {
        "lst_default_params": (None, [_P(lst_params)]),
        "lst_create": (C.c_int32, [_P(lst_params), _P(C.c_void_p)]),
        "lst_load_geometry": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint32]),
        "lst_get_connection_map": (C.c_int32, [C.c_void_p, _P(_P(C.c_uint32)), _P(_P(C.c_uint32)), _P(C.c_uint32)]),
        "lst_build_connection_map": (C.c_int32, [_P(lst_params), C.c_void_p, C.c_uint32,
                                                 _P(_P(C.c_uint32)), _P(_P(C.c_uint32)), _P(C.c_uint32)]),
        "lst_free_map": (None, [_P(C.c_uint32), _P(C.c_uint32)]),
        "lst_set_geometry_cache": (C.c_int32, [C.c_void_p, C.c_char_p]),
        "lst_geometry_from_cache": (C.c_int32, [C.c_void_p]),
        "lst_run_event": (C.c_int32, [C.c_void_p, _P(lst_event_in), _P(_P(lst_event_out))]),
        "lst_run_batch": (C.c_int32, [C.c_void_p, _P(lst_event_in), C.c_uint32, _P(_P(lst_event_out))]),
        "lst_submit": (C.c_int32, [C.c_void_p, _P(lst_event_in), _P(C.c_uint64)]),
        "lst_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_int64, _P(_P(lst_event_out))]),
        "lst_batch_upload": (C.c_int32, [C.c_void_p, _P(lst_event_in), C.c_uint32]),
        "lst_batch_execute": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_int32, C.c_int32, _P(C.c_double)]),
        "lst_kernel_times": (C.c_int32, [C.c_void_p, _P(C.c_char_p), _P(C.c_double), _P(C.c_uint32), _P(C.c_uint32)]),
        "lst_batch_download": (C.c_int32, [C.c_void_p, _P(_P(lst_event_out))]),
        "lst_batch_counts": (C.c_int32, [C.c_void_p, _P(C.c_uint64)]),
        "lst_time_only": (C.c_int32, [C.c_void_p, C.c_char_p]),
        "lst_run_event_noalloc": (C.c_int32, [C.c_void_p, _P(lst_event_in), _P(lst_event_dev_out), C.c_void_p]),
        "lst_free_output": (None, [_P(lst_event_out)]),
        "lst_destroy": (None, [C.c_void_p]),
        "lst_status_str": (C.c_char_p, [C.c_int32]),
        "lst_last_error": (C.c_char_p, [C.c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _share_hip_runtime_with_torch():
    """A process must hold a single HIP runtime.  PyTorch ships its own copy;
    when PyTorch is installed, load that copy first so that liblst binds to it
    (by soname) and torch tensors can be passed as device pointers."""
    import importlib.util
    try:
        spec = importlib.util.find_spec("torch")
    except Exception:
        spec = None
    if spec is None or not spec.origin:
        return
    hip = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
    if os.path.exists(hip):
        C.CDLL(hip, mode=C.RTLD_GLOBAL)


def default_params(**kw) -> lst_params:
    p = lst_params()
    load().lst_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "bend":
            p.flags = (p.flags & ~LST_FLAG_BEND) | (LST_FLAG_BEND if v else 0)
        elif k == "stage_times":
            p.flags = (p.flags & ~LST_FLAG_STAGE_TIMES) | (LST_FLAG_STAGE_TIMES if v else 0)
        elif k == "tc_clean":
            p.flags = (p.flags & ~LST_FLAG_TC_CLEAN) | (LST_FLAG_TC_CLEAN if v else 0)
        elif k == "seeds_triplets":
            p.flags = (p.flags & ~LST_FLAG_SEEDS_TRIPLETS) | (LST_FLAG_SEEDS_TRIPLETS if v else 0)
        elif k == "skip_layer":
            p.flags = (p.flags & ~LST_FLAG_SKIP_LAYER) | (LST_FLAG_SKIP_LAYER if v else 0)
        elif k == "stream":
            # a torch.cuda.Stream, or a raw hipStream_t handle
            p.stream = C.c_void_p(int(getattr(v, "cuda_stream", v)) if v is not None else None)
        else:
            setattr(p, k, v)
    return p


def module_table(geom) -> np.ndarray:
    """Geometry object (or dict of arrays) -> lst_module_desc array."""
    t = geom.table() if hasattr(geom, "table") else geom
    n = len(t["kind"])
    m = np.zeros(n, dtype=MODULE_DTYPE)
    for k in ("kind", "layer", "side", "s_lo", "s_hi", "c_min", "c_max", "phi_min", "phi_max"):
        m[k] = t[k]
    return m


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


class EventIn:
    """Keeps the arrays of one event alive while a C struct points at them."""

    def __init__(self, ev: dict):
        self.keep = []
        if _is_torch(ev.get("x")):
            self.c = lst_event_in()
            self.c.n_hits = int(ev["x"].numel())
            par, cov = ev.get("pls_par"), ev.get("pls_cov")
            self.c.n_pls = int(par.shape[0]) if par is not None else 0
            for f in ("x", "y", "z", "module", "sensor"):
                t = ev[f].contiguous()
                self.keep.append(t)
                setattr(self.c, f, C.c_void_p(t.data_ptr()))
            if self.c.n_pls:
                for f, name in (("pls_par", par), ("pls_cov", cov)):
                    t = name.contiguous()
                    self.keep.append(t)
                    setattr(self.c, f, C.c_void_p(t.data_ptr()))
                if ev.get("pls_nhits") is not None:
                    t = ev["pls_nhits"].contiguous()
                    self.keep.append(t)
                    self.c.pls_nhits = C.c_void_p(t.data_ptr())
            self.c.flags = LST_DEVICE_PTRS
            return
        x = np.ascontiguousarray(ev["x"], np.float32)
        y = np.ascontiguousarray(ev["y"], np.float32)
        z = np.ascontiguousarray(ev["z"], np.float32)
        mod = np.ascontiguousarray(ev["module"], np.uint32)
        sen = np.ascontiguousarray(ev["sensor"], np.uint8)
        par = np.ascontiguousarray(ev.get("pls_par", np.zeros((0, 5))), np.float32).reshape(-1)
        cov = np.ascontiguousarray(ev.get("pls_cov", np.zeros((0, 15))), np.float32).reshape(-1)
        self.keep = [x, y, z, mod, sen, par, cov]
        self.c = lst_event_in(x.size, par.size // 5, _ptr(x), _ptr(y), _ptr(z), _ptr(mod),
                              _ptr(sen), _ptr(par), _ptr(cov), 0, 0)
        if ev.get("pls_nhits") is not None:
            nh = np.ascontiguousarray(ev["pls_nhits"], np.uint8)
            self.keep.append(nh)
            self.c.pls_nhits = _ptr(nh)


def _is_torch(a):
    return a is not None and type(a).__module__.startswith("torch")


def _out_to_dict(o: lst_event_out) -> dict:
    def pairs(ptr, n):
        if n == 0:
            return np.zeros((0, 2), np.uint32)
        return np.ctypeslib.as_array(ptr, shape=(n, 2)).copy()
    d = dict(md=pairs(o.md, o.n_md), ls=pairs(o.ls, o.n_ls), t3=pairs(o.t3, o.n_t3),
             t5=pairs(o.t5, o.n_t5), pt3=pairs(o.pt3, o.n_pt3), pt5=pairs(o.pt5, o.n_pt5),
             tc=pairs(o.tc, o.n_tc))
    d["t3_kappa"] = (np.ctypeslib.as_array(o.t3_kappa, shape=(o.n_t3,)).copy()
                     if o.n_t3 else np.zeros(0, np.float32))
    d["latency_us"] = o.latency_us
    d["ticket"] = o.ticket
    d["n_flag_regrow"] = o.n_flag_regrow
    d["batch_events"] = o.batch_events
    d["tcc"] = pairs(o.tcc, o.n_tcc) if o.tcc else None
    d["seeds"] = (np.ctypeslib.as_array(o.seeds, shape=(o.n_seeds,)).copy()
                  if o.n_seeds else np.zeros(0, np.uint32))
    d["footprint"] = o.footprint
    d["stage_ns"] = {name: int(o.stage_ns[i]) for i, name in enumerate(STAGES)}
    return d


class Context:
    """One engine context on one device (lst_create ... lst_destroy)."""

    def __init__(self, params: lst_params | None = None, **kw):
        L = load()
        self.L = L
        if params is None and not any(k in kw for k in ("n_phi_bins", "n_kappa_bins", "ls_group", "ls_waves")):
            # the autotuner's cached choice for this GPU and batch size, if any
            from . import tune
            kw = {**(tune.cached_choice(kw.get("max_batch", 64)) or {}), **kw}
        p = params or default_params(**kw)
        h = C.c_void_p()
        self._check(L.lst_create(C.byref(p), C.byref(h)), ctx=False)
        self.h = h
        self.params = p

    # -- helpers ----------------------------------------------------------
    def _check(self, st, ctx=True):
        if st < 0:
            msg = self.L.lst_last_error(self.h).decode() if ctx and getattr(self, "h", None) else ""
            raise LstError(st, msg)
        return st

    def close(self):
        if getattr(self, "h", None):
            self.L.lst_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- geometry ------------------------------------------------------------
    def load_geometry(self, geom):
        m = module_table(geom)
        self._check(self.L.lst_load_geometry(self.h, _ptr(m), len(m)))
        self.n_mod = len(m)

    def set_geometry_cache(self, directory):
        """Directory of the geometry cache (None: none); see lst_set_geometry_cache."""
        self._check(self.L.lst_set_geometry_cache(self.h, directory.encode() if directory else None))

    @property
    def geometry_from_cache(self) -> bool:
        return bool(self.L.lst_geometry_from_cache(self.h))

    def connection_map(self):
        """(begin[n_mod+1], dst[n_edges]) of the loaded geometry."""
        b = _P(C.c_uint32)(); d = _P(C.c_uint32)(); n = C.c_uint32()
        self._check(self.L.lst_get_connection_map(self.h, C.byref(b), C.byref(d), C.byref(n)))
        begin = np.ctypeslib.as_array(b, shape=(self.n_mod + 1,)).copy()
        dst = np.ctypeslib.as_array(d, shape=(n.value,)).copy() if n.value else np.zeros(0, np.uint32)
        return begin, dst

    # -- runs ----------------------------------------------------------------
    def run_event(self, ev: dict) -> dict:
        e = EventIn(ev)
        o = _P(lst_event_out)()
        self._check(self.L.lst_run_event(self.h, C.byref(e.c), C.byref(o)))
        try:
            return _out_to_dict(o.contents)
        finally:
            self.L.lst_free_output(o)

    def run_event_in(self, e: EventIn, fetch: bool = True):
        """lst_run_event of an event already marshalled (EventIn); fetch=False
        drops the lists (timing of the library call alone)."""
        o = _P(lst_event_out)()
        self._check(self.L.lst_run_event(self.h, C.byref(e.c), C.byref(o)))
        try:
            return _out_to_dict(o.contents) if fetch else None
        finally:
            self.L.lst_free_output(o)

    def run_batch(self, evs: list) -> list:
        return self.run_batch_in([EventIn(ev) for ev in evs])

    def run_batch_in(self, es: list, fetch: bool = True):
        """lst_run_batch of events already marshalled (EventIn); fetch=False
        drops the lists (timing of the library call alone)."""
        arr = (lst_event_in * len(es))(*[e.c for e in es])
        outs = (_P(lst_event_out) * len(es))()
        self._check(self.L.lst_run_batch(self.h, arr, len(es), outs))
        res = []
        for o in outs:
            if fetch:
                res.append(_out_to_dict(o.contents))
            self.L.lst_free_output(o)
        return res if fetch else None

    def submit(self, ev: dict) -> int:
        e = EventIn(ev)
        t = C.c_uint64()
        self._check(self.L.lst_submit(self.h, C.byref(e.c), C.byref(t)))
        return t.value

    def submit_in(self, e: EventIn) -> int:
        """lst_submit of an event already marshalled (EventIn)."""
        t = C.c_uint64()
        self._check(self.L.lst_submit(self.h, C.byref(e.c), C.byref(t)))
        return t.value

    def poll(self, ticket: int, timeout_us: int = -1, fetch: bool = True):
        """Returns the output dict, or None while pending.  fetch=False returns
        only the diagnostics (latency, ticket, batch size, footprint) and
        drops the lists."""
        o = _P(lst_event_out)()
        st = self.L.lst_poll(self.h, ticket, timeout_us, C.byref(o))
        if st == LST_PENDING:
            return None
        try:
            self._check(st)
            if fetch:
                return _out_to_dict(o.contents)
            c = o.contents
            return dict(latency_us=c.latency_us, ticket=c.ticket, batch_events=c.batch_events,
                        footprint=c.footprint)
        finally:
            if o:
                self.L.lst_free_output(o)

    def run_event_noalloc(self, ev: dict, bufs: dict, t3_kappa=None, stream=None) -> dict:
        """lst_run_event_noalloc: ev holds torch tensors on the device; bufs
        maps each list name (md, ls, t3, t5, pt3, pt5, tc) to a caller-owned
        (capacity, 2) 32-bit integer device tensor.  Returns the counts; the
        pairs are in the first count rows of each buffer."""
        e = EventIn(ev)
        o = lst_event_dev_out()
        for k in _LISTS:
            t = bufs[k]
            setattr(o, k, C.c_void_p(t.data_ptr()) if t.numel() else None)
            setattr(o, "cap_" + k, int(t.shape[0]))
        o.t3_kappa = C.c_void_p(t3_kappa.data_ptr()) if t3_kappa is not None else None
        sp = C.c_void_p(int(getattr(stream, "cuda_stream", stream))) if stream is not None else None
        st = self.L.lst_run_event_noalloc(self.h, C.byref(e.c), C.byref(o), sp)
        counts = {k: int(getattr(o, "n_" + k)) for k in _LISTS}
        if st < 0:
            err = LstError(st, self.L.lst_last_error(self.h).decode())
            err.counts = counts
            raise err
        return counts

    # -- device-resident path ----------------------------------------------
    def batch_upload(self, evs: list):
        es = [EventIn(ev) for ev in evs]
        arr = (lst_event_in * len(es))(*[e.c for e in es])
        self._check(self.L.lst_batch_upload(self.h, arr, len(es)))

    def batch_execute(self, repeats: int = 1, graph: bool = True, timing: bool = False) -> float:
        ms = C.c_double()
        self._check(self.L.lst_batch_execute(self.h, repeats, 1 if graph else 0, 1 if timing else 0,
                                             C.byref(ms)))
        return ms.value

    def kernel_times(self) -> dict:
        cap = 64
        names = (C.c_char_p * cap)(); tot = (C.c_double * cap)(); cnt = (C.c_uint32 * cap)()
        n = C.c_uint32(cap)
        self._check(self.L.lst_kernel_times(self.h, names, tot, cnt, C.byref(n)))
        return {names[i].decode(): (tot[i], cnt[i]) for i in range(n.value)}

    def batch_download(self, n_events: int) -> list:
        outs = (_P(lst_event_out) * n_events)()
        self._check(self.L.lst_batch_download(self.h, outs))
        res = []
        for o in outs:
            res.append(_out_to_dict(o.contents))
            self.L.lst_free_output(o)
        return res

    def time_only(self, name: str | None):
        """Restrict batch_execute(timing=True) to the launches of this name
        (None: every launch)."""
        self._check(self.L.lst_time_only(self.h, name.encode() if name else None))

    def batch_counts(self) -> dict:
        v = (C.c_uint64 * 15)()
        self._check(self.L.lst_batch_counts(self.h, v))
        keys = ["md", "ls", "t3", "t5", "pt3", "pt5", "tc", "cand_md", "cand_ls", "cand_t3",
                "cand_t5", "cand_pt3", "cand_pt5", "eval_pt3", "eval_pt5"]
        return {k: int(x) for k, x in zip(keys, v)}


def build_connection_map(geom, params: lst_params | None = None):
    """Host-only connection map: (begin[n_mod+1], dst[n_edges])."""
    L = load()
    m = module_table(geom)
    p = params or default_params()
    b = _P(C.c_uint32)(); d = _P(C.c_uint32)(); n = C.c_uint32()
    st = L.lst_build_connection_map(C.byref(p), _ptr(m), len(m), C.byref(b), C.byref(d), C.byref(n))
    if st < 0:
        raise LstError(st, "connection map")
    try:
        begin = np.ctypeslib.as_array(b, shape=(len(m) + 1,)).copy()
        dst = np.ctypeslib.as_array(d, shape=(n.value,)).copy() if n.value else np.zeros(0, np.uint32)
    finally:
        L.lst_free_map(b, d)
    return begin, dst


def result_keys(res: dict) -> dict:
    """Expanded canonical keys of a library result (same convention as the
    oracle's keys): tuples of input hit indices, prefixed by the seed index
    for pT3/pT5 and by the type for track candidates."""
    md = [(int(a), int(b)) for a, b in res["md"]]
    ls_md = [(int(a), int(b)) for a, b in res["ls"]]
    ls = [md[a] + md[b] for a, b in ls_md]
    t3_md = [(ls_md[l1][0], ls_md[l1][1], ls_md[l2][1]) for l1, l2 in res["t3"]]
    t3 = [md[a] + md[b] + md[c] for a, b, c in t3_md]
    t5 = [t3[u] + md[t3_md[w][1]] + md[t3_md[w][2]] for u, w in res["t5"]]
    pt3 = [(int(p),) + t3[u] for p, u in res["pt3"]]
    pt5 = [(int(p),) + t5[v] for p, v in res["pt5"]]
    src = {0: pt5, 1: pt3, 2: t5}
    tc = [(int(t),) + (src[int(t)][i] if int(t) in src else (int(i),)) for t, i in res["tc"]]
    out = dict(md=md, ls=ls, t3=t3, t5=t5, pt3=pt3, pt5=pt5, tc=tc)
    if res.get("tcc") is not None:
        out["tcc"] = [(int(t),) + (src[int(t)][i] if int(t) in src else (int(i),)) for t, i in res["tcc"]]
    return out
