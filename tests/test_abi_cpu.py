"""CPU-side checks of the C-ABI library: it loads, exports every function
include/lst.h declares, and its host-only connection map is conservative
(every segment the brute-force oracle builds lies on a map edge)."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2407_18231_amd import lst, synth as s
from truth import _surface_ids, _is_next, _is_linked

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lst.LIB_PATH):
        from paper_2407_18231_amd import build
        build.build()
    return lst.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lst.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lst_\w+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for code in lst.STATUS:
        assert lib.lst_status_str(code)


def test_default_params(lib):
    p = lst.default_params()
    assert p.B == 3.8 and p.pt_min == 0.8 and p.L == 15.0 and p.n_sigma == 3.0
    assert p.flags == lst.LST_FLAG_BEND and p.max_batch == 64 and p.n_slots == 2


def test_bad_geometry_rejected(lib):
    g = s.make_geometry("tiny")
    m = lst.module_table(g)
    m["s_hi"][5] = m["s_lo"][5] - 1.0
    with pytest.raises(lst.LstError) as e:
        lst.build_connection_map(m)
    assert e.value.name == "BAD_GEOMETRY"
    m = lst.module_table(g)
    m["s_lo"][100] += 0.5           # one module of layer 1 off its surface
    with pytest.raises(lst.LstError):
        lst.build_connection_map(m)


@pytest.mark.parametrize("kind", ["tiny", "pu200"])
def test_connection_map_holds_every_oracle_segment(lib, kind):
    g, ev = s.standard_event(kind)
    begin, dst = lst.build_connection_map(g)
    assert begin.shape == (g.n_mod + 1,) and begin[-1] == dst.size
    # edges only to the next surface
    sid, nb, nd = _surface_ids(g)
    src = np.repeat(np.arange(g.n_mod), np.diff(begin))
    assert all(_is_next(nb, nd, int(sid[a]), int(sid[b])) for a, b in zip(src[::97], dst[::97]))
    edges = set(zip(src.tolist(), dst.tolist()))
    r = oracle.run(g, ev)
    md_mod = ev["module"][r["md"][:, 0]]
    pairs = {(int(md_mod[a]), int(md_mod[b])) for a, b in r["ls"]}
    assert len(pairs) > 100
    missing = pairs - edges
    assert not missing, list(missing)[:5]
    # and the map is selective: far fewer edges than next-surface module pairs
    n_pairs = sum(int((sid == t).sum()) for a in range(g.n_mod)
                  for t in set(range(nb + 2 * nd)) if _is_next(nb, nd, int(sid[a]), t)) if kind == "tiny" else None
    if n_pairs:
        assert dst.size < 0.5 * n_pairs


def test_skip_layer_map_holds_every_oracle_segment(lib):
    """With skip-layer links the map pairs modules on surfaces one or two
    steps apart, holds every edge of the plain map and every segment the
    oracle builds with the same links."""
    g, ev = s.standard_event("pu200")
    b0, d0 = lst.build_connection_map(g)
    b1, d1 = lst.build_connection_map(g, lst.default_params(skip_layer=True))
    sid, nb, nd = _surface_ids(g)
    src0 = np.repeat(np.arange(g.n_mod), np.diff(b0))
    src1 = np.repeat(np.arange(g.n_mod), np.diff(b1))
    e0 = set(zip(src0.tolist(), d0.tolist()))
    e1 = set(zip(src1.tolist(), d1.tolist()))
    assert e0 < e1
    surf = {(int(sid[a]), int(sid[b])) for a, b in e1}
    assert all(_is_linked(nb, nd, a, b, True) for a, b in surf)
    assert sum(1 for a, b in surf if not _is_next(nb, nd, a, b)) > 5
    r = oracle.run(g, ev, oracle.Params(skip=True))
    md_mod = ev["module"][r["md"][:, 0]]
    pairs = {(int(md_mod[a]), int(md_mod[b])) for a, b in r["ls"]}
    assert len(pairs - e0) > 100
    missing = pairs - e1
    assert not missing, list(missing)[:5]


def test_bucket_granularity_params(lib, tmp_path):
    """The seed-lookup bucket counts default to 0 (the library's 64 x 12) and
    out-of-range values are refused before any device is touched; the
    tuner's cache round-trips per architecture and workload."""
    p = lst.default_params()
    assert p.n_phi_bins == 0 and p.n_kappa_bins == 0
    for bad in (dict(n_phi_bins=3), dict(n_phi_bins=5000), dict(n_kappa_bins=1), dict(n_kappa_bins=200),
                dict(ls_group=5), dict(ls_waves=7)):
        with pytest.raises(lst.LstError) as e:
            lst.Context(**bad)
        assert e.value.name == "INVALID_ARG", bad
    from paper_2407_18231_amd import tune
    path = str(tmp_path / "cache.json")
    assert tune.load_choice("gfx950", "batch64-pu200", path) is None
    tune.store_choice("gfx950", "batch64-pu200", {"n_phi_bins": 64, "n_kappa_bins": 16}, path)
    tune.store_choice("gfx950", "batch8-pu100", {"n_phi_bins": 32, "n_kappa_bins": 12}, path)
    assert tune.load_choice("gfx950", "batch64-pu200", path) == {"n_phi_bins": 64, "n_kappa_bins": 16}
    assert tune.load_choice("gfx942", "batch64-pu200", path) is None
    per_arch = {"batch64-pu200": {"n_phi_bins": 64, "n_kappa_bins": 16, "ls_group": 4, "ls_waves": 8,
                                  "ms_per_batch": {}},
                "batch8-pu100": {"n_phi_bins": 32, "n_kappa_bins": 12}}
    assert tune.choice_for(per_arch, 64) == {"n_phi_bins": 64, "n_kappa_bins": 16, "ls_group": 4, "ls_waves": 8}
    assert tune.choice_for(per_arch, 8) == {"n_phi_bins": 32, "n_kappa_bins": 12}
    assert tune.choice_for(per_arch, 16) is None


def _c_layout(struct: str, fields: list) -> dict:
    """sizeof and offsetof of a struct of include/lst.h, as gcc lays it out."""
    import subprocess
    import tempfile
    body = "\n".join(f'printf("{f} %zu\\n", offsetof({struct}, {f}));' for f in fields)
    src = ('#include <stddef.h>\n#include <stdio.h>\n#include "lst.h"\n'
           f'int main(void) {{ printf("sizeof %zu\\n", sizeof({struct})); {body} return 0; }}\n')
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "t.c"), os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    return {k: int(v) for k, v in zip(out[::2], out[1::2])}


@pytest.mark.parametrize("cls,struct", [(lst.lst_params, "lst_params"), (lst.lst_event_in, "lst_event_in"),
                                        (lst.lst_event_out, "lst_event_out"),
                                        (lst.lst_event_dev_out, "lst_event_dev_out")])
def test_struct_layout_matches_header(lib, cls, struct):
    """The binding's ctypes structs have the header's size and field offsets
    (stage_ns and n_flag_regrow of the output, the caller stream of the
    parameters included)."""
    import ctypes
    names = [f[0] for f in cls._fields_]
    lay = _c_layout(struct, names)
    assert lay["sizeof"] == ctypes.sizeof(cls)
    for n in names:
        assert lay[n] == getattr(cls, n).offset, n
    if struct == "lst_event_out":
        assert lst.lst_event_out.stage_ns.size == 8 * len(lst.STAGES)


def test_module_desc_layout(lib):
    lay = _c_layout("lst_module_desc", list(lst.MODULE_DTYPE.names))
    assert lay["sizeof"] == lst.MODULE_DTYPE.itemsize
    for n in lst.MODULE_DTYPE.names:
        assert lay[n] == lst.MODULE_DTYPE.fields[n][1], n


def test_connection_map_covers_the_input_contract(lib):
    """Hits at the edge of the input contract (5.4 resolutions outside their
    module's extent, across azimuth and z / r edges): every segment the
    brute-force oracle builds from them lies on a map edge."""
    import contract
    g = s.make_geometry("pu200")
    ev = s.gen_event(g, s.config_pu(200, smear=False), 4242)
    gs = contract.shrunk(g, 5.4)
    out = contract.outside_extent(gs, ev)
    assert out.max() > 5.3 and (out > 4.0).sum() > 1000
    begin, dst = lst.build_connection_map(gs)
    src = np.repeat(np.arange(g.n_mod), np.diff(begin))
    edges = set(zip(src.tolist(), dst.tolist()))
    r = oracle.run(gs, ev)
    md_mod = ev["module"][r["md"][:, 0]]
    a_out = out[r["md"][:, 0]]
    pairs = {(int(md_mod[a]), int(md_mod[b])) for a, b in r["ls"]}
    # segments whose anchors lie outside their modules are many
    edge_ls = sum(1 for a, b in r["ls"] if a_out[a] > 3.0 or a_out[b] > 3.0)
    assert edge_ls > 500
    missing = pairs - edges
    assert not missing, list(missing)[:5]
