"""GPU parity: the HIP chain against the CPU oracle, through the C ABI.

Bar: outside flagged borderline candidates (within 1e-5 relative of a cut
boundary, counted by the oracle) the object lists are identical, as sets of
expanded input-hit keys, at every stage (MD, LS, T3, T5, pT3, pT5, TC).  Also:
outputs are canonical (sorted, no duplicates), deterministic, identical
alone / in a batch / through device pointers / in the served mix, and bad
inputs return the documented error codes.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2407_18231_amd import lst, synth as s
from parity import STAGES, check_canonical, check_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def geo():
    return {k: s.make_geometry(k) for k in ("tiny", "pu200")}


@pytest.fixture(scope="module")
def ctx(geo):
    c = lst.Context()
    c.load_geometry(geo["pu200"])
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_tiny(geo):
    c = lst.Context()
    c.load_geometry(geo["tiny"])
    yield c
    c.close()


def test_parity_tiny(ctx_tiny, geo):
    g = geo["tiny"]
    ev = s.gen_event(g, s.config_tiny(), s.event_seed(1, 0))
    res = ctx_tiny.run_event(ev)
    check_canonical(res, ev)
    check_parity(g, ev, res)
    assert len(res["t5"]) > 50


@pytest.mark.parametrize("i", [0, 1])
def test_parity_pu200(ctx, geo, i):
    g = geo["pu200"]
    ev = s.gen_event(g, s.config_pu(200), s.event_seed(2, i))
    res = ctx.run_event(ev)
    check_canonical(res, ev)
    check_parity(g, ev, res)
    assert len(res["pt5"]) > 500 and len(res["ls"]) > 50_000


def test_parity_skip_layer(geo):
    """Skip-layer links (segments may bridge one surface): on a PU200 event
    (10% hit inefficiency) the lists equal the oracle's with the same links,
    the map holds the two-step edges, and a batch of three events equals the
    events run one by one."""
    g = geo["pu200"]
    with lst.Context(skip_layer=True) as c:
        c.load_geometry(g)
        ev = s.gen_event(g, s.config_pu(200), s.event_seed(2, 0))
        res = c.run_event(ev)
        check_canonical(res, ev)
        rep = check_parity(g, ev, res, oracle.Params(skip=True))
        assert rep["ls"]["got"] > 120_000
        evs = [s.gen_event(g, s.config_pu(200), s.event_seed(9, i)) for i in range(3)]
        for e, rb in zip(evs, c.run_batch(evs)):
            ra = c.run_event(e)
            for k in STAGES:
                assert np.array_equal(ra[k], rb[k]), k
        begin, dst = c.connection_map()
    begin0, dst0 = lst.build_connection_map(g)
    assert len(dst) > len(dst0)


def test_parity_pu300_stress(ctx, geo):
    g = geo["pu200"]
    ev = s.gen_event(g, s.config_pu(300, noise_frac=0.4, fake_frac=0.05), s.event_seed(5, 0))
    res = ctx.run_event(ev)
    check_canonical(res, ev)
    check_parity(g, ev, res)


def test_parity_edge_cases(ctx, geo):
    g = geo["pu200"]
    empty = dict(x=np.zeros(0, np.float32), y=np.zeros(0, np.float32), z=np.zeros(0, np.float32),
                 module=np.zeros(0, np.uint32), sensor=np.zeros(0, np.uint8),
                 pls_par=np.zeros((0, 5), np.float32), pls_cov=np.zeros((0, 15), np.float32))
    res = ctx.run_event(empty)
    assert all(len(res[k]) == 0 for k in STAGES)
    # seeds only: every seed is an unlinked track candidate
    ev = s.gen_event(g, s.config_pu(5), 77)
    seeds_only = dict(empty, pls_par=ev["pls_par"], pls_cov=ev["pls_cov"])
    res = ctx.run_event(seeds_only)
    assert len(res["tc"]) == len(ev["pls_par"])
    assert np.all(res["tc"][:, 0] == lst.TC_PLS)
    # hits only, and a single-track event, against the oracle
    hits_only = dict(ev, pls_par=np.zeros((0, 5), np.float32), pls_cov=np.zeros((0, 15), np.float32))
    check_parity(g, hits_only, ctx.run_event(hits_only))
    one = s.gen_event(g, s.config_pu(1, n_tracks=1, pt_mode="uniform", pt_lo=2, pt_hi=3, eta_max=0.5,
                                     n_pls=1, fake_frac=0.0, noise_frac=0.0, ineff=0.0), 5)
    check_parity(g, one, ctx.run_event(one))


def test_batch_matches_single_events(ctx, geo):
    g = geo["pu200"]
    evs = s.batch_events(6, g)
    evs.insert(3, dict(x=np.zeros(0, np.float32), y=np.zeros(0, np.float32), z=np.zeros(0, np.float32),
                       module=np.zeros(0, np.uint32), sensor=np.zeros(0, np.uint8),
                       pls_par=np.zeros((0, 5), np.float32), pls_cov=np.zeros((0, 15), np.float32)))
    batch = ctx.run_batch(evs)
    for ev, rb in zip(evs, batch):
        r1 = ctx.run_event(ev)
        for k in STAGES:
            assert np.array_equal(r1[k], rb[k]), k
    check_parity(g, evs[0], batch[0])


def test_deterministic(ctx, geo):
    g = geo["pu200"]
    ev = s.gen_event(g, s.config_pu(200), s.event_seed(2, 3))
    a = ctx.run_event(ev)
    for _ in range(3):
        b = ctx.run_event(ev)
        for k in STAGES:
            assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a["t3_kappa"].view(np.uint32), b["t3_kappa"].view(np.uint32))


def test_device_pointer_inputs(ctx, geo):
    torch = pytest.importorskip("torch")
    g = geo["pu200"]
    ev = s.gen_event(g, s.config_pu(100), 91)
    ref = ctx.run_event(ev)
    dev = {k: torch.from_numpy(np.ascontiguousarray(ev[k])).to("cuda:0")
           for k in ("x", "y", "z", "pls_par", "pls_cov", "sensor")}
    dev["module"] = torch.from_numpy(ev["module"].astype(np.int32)).to("cuda:0")
    torch.cuda.synchronize()
    got = ctx.run_event(dev)
    for k in STAGES:
        assert np.array_equal(ref[k], got[k]), k


def test_served_mix_matches_alone(geo):
    g = geo["pu200"]
    evs = s.batch_events(10, g, pu_lo=140, pu_hi=200, seed_base=4)
    with lst.Context(max_batch=4, n_slots=2) as c:
        c.load_geometry(g)
        alone = [c.run_event(ev) for ev in evs]
        tickets = [c.submit(ev) for ev in evs]
        outs = {}
        for t in tickets:
            outs[t] = c.poll(t, -1)
        for ev, t, a in zip(evs, tickets, alone):
            o = outs[t]
            assert o["ticket"] == t and o["latency_us"] > 0
            for k in STAGES:
                assert np.array_equal(a[k], o[k]), k
        with pytest.raises(lst.LstError) as e:
            c.poll(tickets[0], 0)
        assert e.value.name == "UNKNOWN_TICKET"


def test_error_codes(ctx, geo):
    g = geo["pu200"]
    ev = s.gen_event(g, s.config_pu(10), 3)
    bad = dict(ev, module=ev["module"].copy())
    bad["module"][7] = g.n_mod + 5
    with pytest.raises(lst.LstError) as e:
        ctx.run_event(bad)
    assert e.value.name == "BAD_MODULE"
    bad = dict(ev, x=ev["x"].copy())
    bad["x"][3] = np.nan
    with pytest.raises(lst.LstError) as e:
        ctx.run_event(bad)
    assert e.value.name == "NONFINITE"
    bad = dict(ev, pls_par=ev["pls_par"].copy())
    bad["pls_par"][0, 1] = np.inf
    with pytest.raises(lst.LstError) as e:
        ctx.run_event(bad)
    assert e.value.name == "NONFINITE"
    # the context still works after input errors
    check_parity(g, ev, ctx.run_event(ev))
    with lst.Context() as c:
        with pytest.raises(lst.LstError) as e:
            c.run_event(ev)
        assert e.value.name == "NO_GEOMETRY"


def test_regrow_after_overflow(geo):
    """A batch far larger than the first one forces the object lists to grow;
    results equal a fresh run."""
    g = geo["pu200"]
    small = s.gen_event(g, s.config_pu(20), 1)
    big = s.gen_event(g, s.config_pu(300, noise_frac=0.4), 2)
    with lst.Context() as c:
        c.load_geometry(g)
        c.run_event(small)
        r_big = c.run_event(big)
    with lst.Context() as c:
        c.load_geometry(g)
        r_ref = c.run_event(big)
    for k in STAGES:
        assert np.array_equal(r_big[k], r_ref[k]), k


def test_full_batch_sampled_parity(ctx, geo):
    """The benchmark's launch: 64 PU200-like events in one batch.  Sampled
    events match the oracle; every event matches its own per-event run."""
    g = geo["pu200"]
    evs = [s.gen_event(g, s.config_pu(200), s.event_seed(2, i)) for i in range(64)]
    with lst.Context(max_batch=64) as c:
        c.load_geometry(g)
        batch = c.run_batch(evs)
    for i in (0, 63):
        check_canonical(batch[i], evs[i])
        check_parity(g, evs[i], batch[i])
    for i in range(0, 64, 9):
        r1 = ctx.run_event(evs[i])
        for k in STAGES:
            assert np.array_equal(r1[k], batch[i][k]), (i, k)


def test_binary32_stages_bit_exact(ctx, geo):
    """MD, LS, T3 and T5 decide in binary32 on both sides with the same
    expressions, so they agree exactly -- borderline (flagged) candidates
    included, no tolerance."""
    g = geo["pu200"]
    for i in (0, 5):
        ev = s.gen_event(g, s.config_pu(200), s.event_seed(2, i))
        od = oracle.keyed(oracle.run(g, ev))
        got = lst.result_keys(ctx.run_event(ev))
        for k in ("md", "ls", "t3", "t5"):
            acc = {q for q, st in od[k].items() if st & oracle.ST_ACC}
            assert set(got[k]) == acc, (i, k, len(set(got[k]) ^ acc))


def test_graph_replay_matches_eager(geo):
    """The captured two-stream chain replayed from a hipGraph (the bench's
    graph figure) gives the eager run's lists, replay after replay, with
    eager runs in between; 16 events take the pooled large-batch kernels."""
    g = geo["pu200"]
    evs = [s.gen_event(g, s.config_pu(200), s.event_seed(2, i)) for i in range(16)]
    with lst.Context(max_batch=16) as c:
        c.load_geometry(g)
        c.batch_upload(evs)
        c.batch_execute(1, graph=False)
        eager = c.batch_download(len(evs))
        for rounds in (1, 3, 2):
            c.batch_execute(rounds, graph=True)
            got = c.batch_download(len(evs))
            for a, b in zip(eager, got):
                for k in STAGES:
                    assert np.array_equal(a[k], b[k]), (rounds, k)
            c.batch_execute(1, graph=False)
    assert sum(len(r["ls"]) for r in eager) > 16 * 50_000


@pytest.mark.parametrize("bins", [(32, 12), (128, 24)])
def test_bucket_granularity_does_not_change_lists(ctx, geo, bins):
    """The seed-lookup bucket granularity (what the tuner picks) changes only
    the speed: the lists equal those of the default setting."""
    g = geo["pu200"]
    ev = s.gen_event(g, s.config_pu(200), s.event_seed(2, 7))
    ref = ctx.run_event(ev)
    with lst.Context(n_phi_bins=bins[0], n_kappa_bins=bins[1]) as c:
        c.load_geometry(g)
        got = c.run_event(ev)
    for k in STAGES:
        assert np.array_equal(ref[k], got[k]), (bins, k)


@pytest.mark.parametrize("variant", [(4, 0), (8, 8), (6, 6)])
def test_segment_walk_variants_do_not_change_lists(geo, variant):
    """The segment walk's edge-group size and occupancy (the tuner's other
    choices) change only the speed, on the pooled large-batch walk."""
    g = geo["pu200"]
    evs = [s.gen_event(g, s.config_pu(200), s.event_seed(2, 60 + i)) for i in range(12)]
    out = []
    for group, waves in ((6, 0), variant):
        with lst.Context(max_batch=12, ls_group=group, ls_waves=waves) as c:
            c.load_geometry(g)
            c.batch_upload(evs)
            c.batch_execute(1, graph=True)
            out.append(c.batch_download(len(evs)))
    for a, b in zip(*out):
        for k in STAGES:
            assert np.array_equal(a[k], b[k]), (variant, k)


def test_parity_special_seeds(ctx, geo):
    """Seeds whose helix cannot reach the outer tracker (|r kappa / 2| >= 1
    from r = 17.5 cm on), with cot(theta) = 0 (no disk prediction) and with
    q/pT = 0 (a straight line), among ordinary ones."""
    g = geo["pu200"]
    ev = s.gen_event(g, s.config_pu(100), s.event_seed(2, 40))
    par, cov = ev["pls_par"].copy(), ev["pls_cov"].copy()
    hi_pt = np.argsort(np.abs(par[:, 0]))[:8]          # straightest seeds
    par[hi_pt[:4], 0] = 0.0
    par[hi_pt[4:], 2] = 0.0
    par[:6, 0] = np.where(par[:6, 0] < 0, -12.0, 12.0)    # pT ~ 0.08 GeV
    cov[:6, 0] = (0.015 * 12.0) ** 2
    ev2 = dict(ev, pls_par=par, pls_cov=cov)
    res = ctx.run_event(ev2)
    check_canonical(res, ev2)
    check_parity(g, ev2, res)
    linked = set(res["pt3"][:, 0].tolist()) | set(res["pt5"][:, 0].tolist())
    assert not linked & set(range(6))
    assert len(res["pt3"]) > 1000


def test_parity_disk_only(ctx, geo):
    """An event with hits on the disks only: endcap MDs, disk-to-disk
    segments and the T3 / T5 / seed links built from them."""
    g = geo["pu200"]
    ev = s.gen_event(g, s.config_pu(200), s.event_seed(2, 41))
    keep = g.kind[ev["module"]] != s.BARREL
    ev2 = {k: ev[k][keep] for k in ("x", "y", "z", "module", "sensor")}
    ev2.update(pls_par=ev["pls_par"], pls_cov=ev["pls_cov"])
    res = ctx.run_event(ev2)
    check_canonical(res, ev2)
    check_parity(g, ev2, res)
    assert len(res["t3"]) > 100 and len(res["ls"]) > 1000


def _md_pairs(key):
    """MDs (hit pairs) of a candidate key: (type, [seed,] hits...)."""
    hits = key[2:] if key[0] in (0, 1) else key[1:] if key[0] == 2 else ()
    return {(hits[i], hits[i + 1]) for i in range(0, len(hits), 2)}


def _oracle_cleaned(geom, ev, params=None):
    """The oracle's accepted candidates and the subset its duplicate cleaning
    keeps, as keys, and the candidates whose cleaning may depend on a
    borderline one: the flagged candidates and every candidate sharing an MD
    with one of them (a device that kept or dropped the flagged candidate
    may rank its neighbours differently)."""
    ores = oracle.run(geom, ev, params)
    ks = oracle.object_keys(ores["md"], ores["ls"], ores["t3"], ores["t5"], ores["pt3"], ores["pt5"],
                            ores["tc"])["tc"]
    st = ores["tc_st"]
    acc = [k for k, q in zip(ks, st) if q & oracle.ST_ACC]
    kept = [k for k, q, f in zip(ks, st, ores["tc_keep"]) if (q & oracle.ST_ACC) and f]
    flagged = [k for k, q in zip(ks, st) if q & oracle.ST_FLAG]
    fl_mds = set().union(*[_md_pairs(k) for k in flagged]) if flagged else set()
    affected = {k for k in ks if k in set(flagged) or _md_pairs(k) & fl_mds}
    return acc, kept, set(flagged), affected


def test_tc_cleaning_parity(geo):
    """Duplicate cleaning of the track candidates: the kept subset equals the
    oracle's, for single events and inside a batch; it removes most
    candidates and never a seed-only one."""
    g = geo["pu200"]
    evs = [s.gen_event(g, s.config_pu(200), s.event_seed(2, i)) for i in (0, 1)]
    evs.append(s.gen_event(g, s.config_pu(300, noise_frac=0.4, fake_frac=0.05), s.event_seed(5, 2)))
    with lst.Context(tc_clean=True, max_batch=8) as c:
        c.load_geometry(g)
        singles = [c.run_event(ev) for ev in evs]
        batch = c.run_batch(evs)
    for ev, r, rb in zip(evs, singles, batch):
        acc, kept, flagged, affected = _oracle_cleaned(g, ev)
        got = lst.result_keys(r)
        print("candidates", len(acc), "kept", len(kept), "flagged", len(flagged), "affected", len(affected), flush=True)
        assert len(affected) <= 0.01 * len(acc)
        assert set(got["tc"]) - flagged == set(acc) - flagged
        assert len(got["tcc"]) == len(set(got["tcc"]))
        assert set(got["tcc"]) - affected == set(kept) - affected
        assert np.array_equal(r["tcc"], rb["tcc"])
        assert len(kept) < 0.5 * len(acc)
        n_pls = int((r["tc"][:, 0] == lst.TC_PLS).sum())
        assert int((r["tcc"][:, 0] == lst.TC_PLS).sum()) == n_pls
    with lst.Context() as c:
        c.load_geometry(g)
        assert c.run_event(evs[0])["tcc"] is None


def test_tc_cleaning_parity_skip_layer(geo):
    """Duplicate cleaning with skip-layer links, where one track leaves tens
    of candidates on each of its MDs: the kept subset equals the oracle's
    with the same links, per event and in a batch."""
    g = geo["pu200"]
    evs = [s.gen_event(g, s.config_pu(200), s.event_seed(2, i)) for i in (3, 4)]
    with lst.Context(tc_clean=True, skip_layer=True, max_batch=4) as c:
        c.load_geometry(g)
        singles = [c.run_event(ev) for ev in evs]
        batch = c.run_batch(evs)
    for ev, r, rb in zip(evs, singles, batch):
        acc, kept, flagged, affected = _oracle_cleaned(g, ev, oracle.Params(skip=True))
        got = lst.result_keys(r)
        print("candidates", len(acc), "kept", len(kept), "flagged", len(flagged), "affected", len(affected), flush=True)
        assert len(affected) <= 0.02 * len(acc)
        assert set(got["tc"]) - flagged == set(acc) - flagged
        assert set(got["tcc"]) - affected == set(kept) - affected
        assert np.array_equal(r["tcc"], rb["tcc"])
        assert len(kept) < 0.25 * len(acc)


def _seed_set(seeds, excused):
    return set(int(v) for v in seeds) - excused


def test_seed_export(geo):
    """Exported seeds (Sec. 2, Table 1: the recovery iteration seeded by LST
    pLS quads, or quads and triplets) equal the oracle's selection from its
    own candidate list, alone, in a batch, in the served mix and from device
    pointers.  Seeds whose linking the oracle flags (a flagged pT3 or pT5, or
    a flagged seed-only candidate) may differ."""
    torch = pytest.importorskip("torch")
    g = geo["pu200"]
    evs = [s.gen_event(g, s.config_pu(200), s.event_seed(2, i)) for i in (0, 1)]
    for ev in evs:
        assert set(np.unique(ev["pls_nhits"]).tolist()) == {3, 4}
    for triplets in (False, True):
        with lst.Context(seeds_triplets=triplets, n_slots=1) as c:
            c.load_geometry(g)
            alone = [c.run_event(ev) for ev in evs]
            batch = c.run_batch(evs)
            served = [c.poll(c.submit(ev), -1) for ev in evs]
            d = {k: torch.from_numpy(np.ascontiguousarray(evs[0][k])).to("cuda:0")
                 for k in ("x", "y", "z", "sensor", "pls_par", "pls_cov", "pls_nhits")}
            d["module"] = torch.from_numpy(evs[0]["module"].astype(np.int32)).to("cuda:0")
            torch.cuda.synchronize()
            dev = c.run_event(d)
        assert np.array_equal(dev["seeds"], alone[0]["seeds"])
        for ev, a, b, v in zip(evs, alone, batch, served):
            assert np.array_equal(a["seeds"], b["seeds"]) and np.array_equal(a["seeds"], v["seeds"])
            assert np.all(np.diff(a["seeds"].astype(np.int64)) > 0)
            ores = oracle.run(g, ev)
            want, flag = oracle.export_seeds(ores, ev["pls_nhits"], triplets)
            excused = set(int(p) for p in want[flag])
            for k in ("pt3", "pt5"):
                excused |= set(int(p) for p in ores[k][ores[k + "_st"] == oracle.ST_FLAG][:, 0])
            assert _seed_set(a["seeds"], excused) == _seed_set(want, excused)
            assert len(want) > 100
            nh = ev["pls_nhits"][a["seeds"].astype(np.int64)]
            assert np.all(nh >= (3 if triplets else 4))


def test_parity_displaced(ctx, geo):
    """Displaced tracks (production radius up to 35 cm; Sec. 3, Fig. 3 right)
    on a PU50 background: the lists match the oracle, and T5 candidates find
    displaced tracks in every radius bin."""
    from paper_2407_18231_amd import metrics
    g = geo["pu200"]
    ev = s.gen_event(g, s.config_pu(50, n_displaced=400), s.event_seed(8, 0))
    res = ctx.run_event(ev)
    check_canonical(res, ev)
    check_parity(g, ev, res)
    eff = metrics.efficiency_vs_rv(ev, res)
    for b in eff["bins"]:
        assert b["n_sim"] > 0 and b["by_type"]["T5"] > 0.1, b
