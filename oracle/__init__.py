"""CPU oracle of the Line Segment Tracking object chain (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the product library never does.  The arithmetic lives
in ``lst_oracle.c`` (plain C, built with gcc, no FMA contraction); this
module builds it, marshals numpy arrays through ctypes and turns the object
lists into canonical keys (tuples of input hit indices) for comparisons.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lst_oracle.c")
# LST_ORACLE_LIB: a build of the same source to load instead (the sanitizer
# tests load one built with the address and undefined-behaviour sanitizers)
_LIB = os.environ.get("LST_ORACLE_LIB") or os.path.join(_HERE, "liblst_oracle.so")

ST_ACC = 1
ST_FLAG = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary32/binary64 IEEE arithmetic, no
    contraction into FMA, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(C.Structure):
    _fields_ = [("n_mod", C.c_uint32),
                ("kind", C.POINTER(C.c_uint32)), ("layer", C.POINTER(C.c_uint32)),
                ("side", C.POINTER(C.c_int32)),
                ("s_lo", C.POINTER(C.c_double)), ("s_hi", C.POINTER(C.c_double)),
                ("c_min", C.POINTER(C.c_double)), ("c_max", C.POINTER(C.c_double)),
                ("phi_min", C.POINTER(C.c_double)), ("phi_max", C.POINTER(C.c_double))]


class _Params(C.Structure):
    _fields_ = [("B", C.c_double), ("pt_min", C.c_double), ("L", C.c_double),
                ("sig_rphi", C.c_double), ("sig_c", C.c_double),
                ("n_sigma", C.c_double), ("flag_margin", C.c_double),
                ("flags", C.c_uint32)]


class _Event(C.Structure):
    _fields_ = [("n_hits", C.c_uint32),
                ("x", C.POINTER(C.c_float)), ("y", C.POINTER(C.c_float)),
                ("z", C.POINTER(C.c_float)), ("module", C.POINTER(C.c_uint32)),
                ("sensor", C.POINTER(C.c_uint8)), ("n_pls", C.c_uint32),
                ("pls_par", C.POINTER(C.c_float)), ("pls_cov", C.POINTER(C.c_float))]


_OBJ = ["md", "ls", "t3", "t5", "pt3", "pt5", "tc"]


class _Result(C.Structure):
    _fields_ = [
        ("n_md", C.c_uint32), ("md", C.POINTER(C.c_uint32)), ("md_st", C.POINTER(C.c_uint8)),
        ("n_ls", C.c_uint32), ("ls", C.POINTER(C.c_uint32)), ("ls_st", C.POINTER(C.c_uint8)),
        ("n_t3", C.c_uint32), ("t3", C.POINTER(C.c_uint32)), ("t3_st", C.POINTER(C.c_uint8)),
        ("t3_k", C.POINTER(C.c_float)), ("t3_sk", C.POINTER(C.c_float)),
        ("n_t5", C.c_uint32), ("t5", C.POINTER(C.c_uint32)), ("t5_st", C.POINTER(C.c_uint8)),
        ("n_pt3", C.c_uint32), ("pt3", C.POINTER(C.c_uint32)), ("pt3_st", C.POINTER(C.c_uint8)),
        ("n_pt5", C.c_uint32), ("pt5", C.POINTER(C.c_uint32)), ("pt5_st", C.POINTER(C.c_uint8)),
        ("n_tc", C.c_uint32), ("tc", C.POINTER(C.c_uint32)), ("tc_st", C.POINTER(C.c_uint8)),
        ("md_cand", C.c_uint32), ("ls_cand", C.c_uint32), ("t3_cand", C.c_uint32),
        ("t5_cand", C.c_uint32), ("pt3_cand", C.c_uint32), ("pt5_cand", C.c_uint32),
        ("t5_k", C.POINTER(C.c_float)), ("t5_sk", C.POINTER(C.c_float)),
        ("tc_keep", C.POINTER(C.c_uint8))]


@dataclass
class Params:
    B: float = 3.8
    pt_min: float = 0.8
    L: float = 15.0
    sig_rphi: float = 30e-4
    sig_c: float = 0.1
    n_sigma: float = 3.0
    flag_margin: float = 1e-5
    bend: bool = True
    skip: bool = False   # segments may also bridge one surface

    def c(self) -> _Params:
        return _Params(self.B, self.pt_min, self.L, self.sig_rphi, self.sig_c,
                       self.n_sigma, self.flag_margin,
                       (1 if self.bend else 0) | (2 if self.skip else 0))


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        L.or_run.argtypes = [C.POINTER(_Geom), C.POINTER(_Params), C.POINTER(_Event), C.POINTER(_Result)]
        L.or_run.restype = C.c_int
        L.or_free.argtypes = [C.POINTER(_Result)]
        L.or_module_const.argtypes = [C.POINTER(_Geom), C.POINTER(_Params), C.c_uint32, C.POINTER(C.c_float)]
        L.or_pair_const.argtypes = [C.POINTER(_Geom), C.POINTER(_Params), C.c_uint32, C.c_uint32, C.POINTER(C.c_float)]
        L.or_kappa3.argtypes = [C.POINTER(_Geom), C.POINTER(_Params), C.POINTER(C.c_float)]
        L.or_kappa3.restype = C.c_float
        L.or_derived.argtypes = [C.POINTER(_Geom), C.POINTER(_Params), C.POINTER(C.c_float)]
        L.or_kappa3_res.argtypes = [C.POINTER(_Geom), C.POINTER(_Params), C.POINTER(C.c_float),
                                    C.POINTER(C.c_int), C.c_float, C.POINTER(C.c_float)]
        L.or_pls_anchor.argtypes = [C.POINTER(_Params), C.POINTER(C.c_float), C.POINTER(C.c_float),
                                    C.c_float, C.c_float, C.c_float, C.c_int, C.POINTER(C.c_double)]
        L.or_pls_anchor.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class _GeomHolder:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, geom):
        t = geom.table() if hasattr(geom, "table") else geom
        self.arrs = dict(
            kind=np.ascontiguousarray(t["kind"], dtype=np.uint32),
            layer=np.ascontiguousarray(t["layer"], dtype=np.uint32),
            side=np.ascontiguousarray(t["side"], dtype=np.int32),
            **{k: np.ascontiguousarray(t[k], dtype=np.float64)
               for k in ("s_lo", "s_hi", "c_min", "c_max", "phi_min", "phi_max")})
        a = self.arrs
        self.c = _Geom(len(a["kind"]), _ptr(a["kind"], C.c_uint32), _ptr(a["layer"], C.c_uint32),
                       _ptr(a["side"], C.c_int32),
                       *[_ptr(a[k], C.c_double) for k in ("s_lo", "s_hi", "c_min", "c_max",
                                                            "phi_min", "phi_max")])


def module_const(geom, m: int, params: Params | None = None) -> np.ndarray:
    g = _GeomHolder(geom); p = (params or Params()).c()
    out = np.zeros(4, np.float32)
    lib().or_module_const(C.byref(g.c), C.byref(p), m, _ptr(out, C.c_float))
    return out


def pair_const(geom, A: int, B: int, params: Params | None = None) -> np.ndarray:
    g = _GeomHolder(geom); p = (params or Params()).c()
    out = np.zeros(12, np.float32)
    lib().or_pair_const(C.byref(g.c), C.byref(p), A, B, _ptr(out, C.c_float))
    return out


def kappa3(geom, xy, params: Params | None = None) -> float:
    g = _GeomHolder(geom); p = (params or Params()).c()
    a = np.ascontiguousarray(xy, dtype=np.float32)
    return float(lib().or_kappa3(C.byref(g.c), C.byref(p), _ptr(a, C.c_float)))


def kappa3_res(geom, xy, disk=(0, 0, 0), r_c: float = 0.0, params: Params | None = None):
    """(curvature, resolution) of three anchors (xy: 6 floats); disk[i] = 1
    for an anchor on a disk, r_c the radius of the third anchor."""
    g = _GeomHolder(geom); p = (params or Params()).c()
    a = np.ascontiguousarray(xy, dtype=np.float32)
    dk = (C.c_int * 3)(*[int(v) for v in disk])
    out = np.zeros(2, np.float32)
    lib().or_kappa3_res(C.byref(g.c), C.byref(p), _ptr(a, C.c_float), dk, float(r_c), _ptr(out, C.c_float))
    return float(out[0]), float(out[1])


def pls_anchor(par, cov, x, y, z, disk=False, params: Params | None = None):
    """One pixel-seed anchor test: (code, azimuth difference, its window,
    coarse deviation, its window); code 0 = evaluated, 1 = helix does not
    reach the radius, 2 = no disk prediction."""
    p = (params or Params()).c()
    pa = np.ascontiguousarray(par, dtype=np.float32)
    cv = np.ascontiguousarray(cov, dtype=np.float32)
    out = np.zeros(4, np.float64)
    code = lib().or_pls_anchor(C.byref(p), _ptr(pa, C.c_float), _ptr(cv, C.c_float),
                               float(x), float(y), float(z), int(bool(disk)), _ptr(out, C.c_double))
    return (int(code),) + tuple(float(v) for v in out)


def derived(geom, params: Params | None = None) -> np.ndarray:
    g = _GeomHolder(geom); p = (params or Params()).c()
    out = np.zeros(8, np.float32)
    lib().or_derived(C.byref(g.c), C.byref(p), _ptr(out, C.c_float))
    return out


def run(geom, ev: dict, params: Params | None = None) -> dict:
    """Run the whole chain on one event; returns numpy copies of every object
    list (index pairs + status bytes) and the candidate counts."""
    g = _GeomHolder(geom)
    p = (params or Params()).c()
    x = np.ascontiguousarray(ev["x"], np.float32)
    y = np.ascontiguousarray(ev["y"], np.float32)
    z = np.ascontiguousarray(ev["z"], np.float32)
    mod = np.ascontiguousarray(ev["module"], np.uint32)
    sen = np.ascontiguousarray(ev["sensor"], np.uint8)
    par = np.ascontiguousarray(ev.get("pls_par", np.zeros((0, 5))), np.float32).reshape(-1)
    cov = np.ascontiguousarray(ev.get("pls_cov", np.zeros((0, 15))), np.float32).reshape(-1)
    n_pls = par.size // 5
    e = _Event(x.size, _ptr(x, C.c_float), _ptr(y, C.c_float), _ptr(z, C.c_float),
               _ptr(mod, C.c_uint32), _ptr(sen, C.c_uint8), n_pls,
               _ptr(par, C.c_float), _ptr(cov, C.c_float))
    r = _Result()
    rc = lib().or_run(C.byref(g.c), C.byref(p), C.byref(e), C.byref(r))
    if rc != 0:
        raise ValueError(f"oracle rejected the event (code {rc})")
    out = {}
    try:
        for name in _OBJ:
            n = getattr(r, "n_" + name)
            if n:
                out[name] = np.ctypeslib.as_array(getattr(r, name), shape=(n, 2)).copy()
                out[name + "_st"] = np.ctypeslib.as_array(getattr(r, name + "_st"), shape=(n,)).copy()
            else:
                out[name] = np.zeros((0, 2), np.uint32)
                out[name + "_st"] = np.zeros(0, np.uint8)
        n = r.n_t3
        out["t3_k"] = np.ctypeslib.as_array(r.t3_k, shape=(n,)).copy() if n else np.zeros(0, np.float32)
        out["t3_sk"] = np.ctypeslib.as_array(r.t3_sk, shape=(n,)).copy() if n else np.zeros(0, np.float32)
        n = r.n_t5
        out["t5_k"] = np.ctypeslib.as_array(r.t5_k, shape=(n,)).copy() if n else np.zeros(0, np.float32)
        out["t5_sk"] = np.ctypeslib.as_array(r.t5_sk, shape=(n,)).copy() if n else np.zeros(0, np.float32)
        n = r.n_tc
        out["tc_keep"] = (np.ctypeslib.as_array(r.tc_keep, shape=(n,)).copy().astype(bool) if n
                          else np.zeros(0, bool))
        out["cand"] = {k: getattr(r, k + "_cand") for k in ("md", "ls", "t3", "t5", "pt3", "pt5")}
    finally:
        lib().or_free(C.byref(r))
    return out


# ---------------------------------------------------------- seed export ---

def export_seeds(res: dict, pls_nhits=None, triplets: bool = False):
    """Seeds handed to a downstream seeded track finder (Sec. 2, Table 1: the
    recovery iteration seeded by LST pLS quads, or by quads and triplets).
    Reading: the seeds that are track candidates by themselves -- the pLS
    entries of the candidate list, seeds linked to no T3 or T5 -- with at
    least four pixel hits (quads), and with three as well (triplets) when
    triplets is set; pls_nhits None: every seed a quad.  Returns the seed
    indices in increasing order and, per entry, whether its candidate is
    flagged (near a cut boundary)."""
    tc = np.asarray(res["tc"]).reshape(-1, 2).astype(np.int64)
    st = np.asarray(res.get("tc_st", np.zeros(len(tc), np.uint8)))
    own = tc[:, 0] == 3
    seeds, flag = tc[own, 1], st[own] == ST_FLAG
    nh = np.full(seeds.size, 4) if pls_nhits is None else np.asarray(pls_nhits, np.int64)[seeds]
    keep = (nh >= 4) | (triplets & (nh == 3))
    order = np.argsort(seeds[keep], kind="stable")
    return seeds[keep][order], flag[keep][order]


# ----------------------------------------------------------------- keys ---

def object_keys(md, ls, t3, t5, pt3, pt5, tc):
    """Expanded keys: each object as the tuple of input hit indices of its
    mini-doublets (lower, upper per MD), prefixed by the seed index for
    pT3/pT5 and by the type for track candidates (0 pT5, 1 pT3, 2 T5,
    3 pixel seed).  Inputs are the (n, 2) index arrays of each stage."""
    md_k = [(int(a), int(b)) for a, b in md]
    ls_k = [md_k[a] + md_k[b] for a, b in ls]
    ls_md = [(int(a), int(b)) for a, b in ls]
    t3_md = [(ls_md[l1][0], ls_md[l1][1], ls_md[l2][1]) for l1, l2 in t3]
    t3_k = [md_k[a] + md_k[b] + md_k[c] for a, b, c in t3_md]
    t5_k = [t3_k[u] + md_k[t3_md[w][1]] + md_k[t3_md[w][2]] for u, w in t5]
    pt3_k = [(int(p),) + t3_k[u] for p, u in pt3]
    pt5_k = [(int(p),) + t5_k[v] for p, v in pt5]
    src = {0: pt5_k, 1: pt3_k, 2: t5_k}
    tc_k = [(int(t),) + (src[int(t)][i] if int(t) in src else (int(i),)) for t, i in tc]
    return dict(md=md_k, ls=ls_k, t3=t3_k, t5=t5_k, pt3=pt3_k, pt5=pt5_k, tc=tc_k)


def keyed(res: dict) -> dict:
    """{stage: {key: status}} from an oracle result."""
    ks = object_keys(res["md"], res["ls"], res["t3"], res["t5"], res["pt3"], res["pt5"], res["tc"])
    out = {}
    for name in _OBJ:
        st = res[name + "_st"]
        d = {}
        for k, s in zip(ks[name], st):
            d[k] = d.get(k, 0) | int(s)
        out[name] = d
    return out


def flag_breakdown(res: dict) -> dict:
    """Per stage: (objects kept, flagged, flagged by the object's own cut
    margin).  An object is flagged by its own margin when it is flagged and
    none of its constituents (MDs of a segment, segments of a T3, T3s of a
    T5, the T3 / T5 of a pT3 / pT5) is; the rest inherit the flag."""
    fl = {k: (res[k + "_st"] & ST_FLAG) > 0 for k in _OBJ}
    inherited = {
        "md": np.zeros(len(fl["md"]), bool),
        "ls": fl["md"][res["ls"][:, 0]] | fl["md"][res["ls"][:, 1]] if len(res["ls"]) else np.zeros(0, bool),
        "t3": fl["ls"][res["t3"][:, 0]] | fl["ls"][res["t3"][:, 1]] if len(res["t3"]) else np.zeros(0, bool),
        "t5": fl["t3"][res["t5"][:, 0]] | fl["t3"][res["t5"][:, 1]] if len(res["t5"]) else np.zeros(0, bool),
        "pt3": fl["t3"][res["pt3"][:, 1]] if len(res["pt3"]) else np.zeros(0, bool),
        "pt5": fl["t5"][res["pt5"][:, 1]] if len(res["pt5"]) else np.zeros(0, bool),
    }
    out = {}
    for k in _OBJ:
        f = fl[k]
        own = f & ~inherited[k] if k in inherited else np.zeros(len(f), bool)
        out[k] = (len(f), int(f.sum()), int(own.sum()))
    return out


def compare(oracle_keyed: dict, got: dict) -> dict:
    """Parity rule: outside flagged (borderline) objects the two sets must be
    identical.  ``got`` maps stage -> iterable of keys.  Returns per-stage
    dict(missing, extra, flagged, total)."""
    rep = {}
    for name, od in oracle_keyed.items():
        g = set(got.get(name, ()))
        certain = {k for k, s in od.items() if s == ST_ACC}
        flagged = {k for k, s in od.items() if s & ST_FLAG}
        missing = certain - g
        extra = {k for k in g if k not in od or (od[k] & (ST_ACC | ST_FLAG)) == 0}
        rep[name] = dict(missing=len(missing), extra=len(extra), flagged=len(flagged),
                         total=len(certain) + len(flagged), got=len(g),
                         missing_keys=sorted(missing)[:5], extra_keys=sorted(extra)[:5])
    return rep
