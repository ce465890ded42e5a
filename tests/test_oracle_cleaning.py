"""Pins of the oracle's track-candidate duplicate cleaning (CPU).

The rule (a reading: the paper names the candidate types and measures
duplicate rates but gives no removal procedure): a candidate with
outer-tracker MDs is removed when a higher-ranked one shares more than half
of the smaller MD set.  Checked here by properties the rule implies, with MD
sets expanded from the oracle's own index lists: kept candidates never
overlap, every removed one overlaps a candidate of a type at least as high,
seed-only candidates are all kept, copies of one seed on one track collapse
to the first, and on PU200-like events the duplicate rate falls several-fold
at almost no cost in efficiency."""
import numpy as np
import pytest

import oracle
from paper_2407_18231_amd import metrics, synth as s


def md_sets(r):
    ls, t3, t5 = r["ls"].astype(np.int64), r["t3"].astype(np.int64), r["t5"].astype(np.int64)

    def t3m(u):
        return [ls[t3[u, 0], 0], ls[t3[u, 0], 1], ls[t3[u, 1], 1]]

    out = []
    for typ, idx in r["tc"].astype(np.int64):
        if typ == 0:
            v = r["pt5"][idx, 1]
            out.append(set(t3m(t5[v, 0]) + t3m(t5[v, 1])[1:]))
        elif typ == 1:
            out.append(set(t3m(r["pt3"][idx, 1])))
        elif typ == 2:
            out.append(set(t3m(t5[idx, 0]) + t3m(t5[idx, 1])[1:]))
        else:
            out.append(set())
    return out


@pytest.fixture(scope="module")
def pu200():
    g = s.make_geometry("pu200")
    ev = s.gen_event(g, s.config_pu(200), s.event_seed(2, 4))
    return g, ev, oracle.run(g, ev)


def test_kept_candidates_do_not_overlap(pu200):
    g, ev, r = pu200
    sets = md_sets(r)
    keep = r["tc_keep"]
    kept = [i for i in range(len(sets)) if keep[i] and sets[i]]
    assert len(kept) > 500
    by_md = {}
    for i in kept:
        for m in sets[i]:
            by_md.setdefault(m, []).append(i)
    for i in kept:
        for m in sets[i]:
            for j in by_md[m]:
                if j != i:
                    assert 2 * len(sets[i] & sets[j]) <= min(len(sets[i]), len(sets[j])), (i, j)


def test_removed_candidates_overlap_a_higher_type(pu200):
    g, ev, r = pu200
    sets = md_sets(r)
    keep, typ = r["tc_keep"], r["tc"][:, 0]
    removed = np.nonzero(~keep)[0]
    assert len(removed) > 1000
    by_md = {}
    for i, st in enumerate(sets):
        for m in st:
            by_md.setdefault(m, []).append(i)
    for i in removed:
        assert sets[i], "a seed-only candidate was removed"
        assert any(j != i and typ[j] <= typ[i] and 2 * len(sets[i] & sets[j]) > min(len(sets[i]), len(sets[j]))
                   for m in sets[i] for j in by_md[m])
    assert keep[typ == 3].all()


def test_copies_of_one_seed_collapse_to_the_first():
    g = s.make_geometry("pu200")
    trk = np.array([[1.0, 3.0, 0.3, 1.0, 0.0]])
    cfg = s.config_pu(1, tracks=trk, n_pls=1, fake_frac=0.0, noise_frac=0.0, ineff=0.0, pls_smear=False)
    ev = s.gen_event(g, cfg, 11)
    ev["pls_par"] = np.repeat(ev["pls_par"], 3, axis=0)
    ev["pls_cov"] = np.repeat(ev["pls_cov"], 3, axis=0)
    r = oracle.run(g, ev)
    tc, keep = r["tc"], r["tc_keep"]
    pt5 = np.nonzero(tc[:, 0] == 0)[0]
    assert len(pt5) >= 3
    kept = pt5[keep[pt5]]
    assert len(kept) == 1 and kept[0] == pt5[0]


def test_cleaning_cuts_duplicates_not_efficiency(pu200):
    g, ev, r = pu200
    res = {k: r[k] for k in ("md", "ls", "t3", "t5", "pt3", "pt5", "tc")}
    before = metrics.rates(ev, res)
    after = metrics.rates(ev, dict(res, tc=r["tc"][r["tc_keep"]]))
    assert before["duplicate_rate"] > 0.6 and after["duplicate_rate"] < before["duplicate_rate"] / 3
    assert after["efficiency"] > before["efficiency"] - 0.02
    assert after["fake_rate"] <= before["fake_rate"]


def test_seed_export_selection():
    """Seed export (Sec. 2, Table 1): only the seed-only candidates, quads by
    default, triplets too on request, in seed order; a hand-made list."""
    res = dict(tc=np.array([[0, 0], [3, 2], [1, 0], [3, 0], [3, 5], [2, 1], [3, 1]]),
               tc_st=np.array([1, 1, 1, 1, 2, 1, 1], np.uint8))
    nh = np.array([3, 2, 4, 4, 4, 5], np.uint8)
    s, f = oracle.export_seeds(res, nh)
    assert s.tolist() == [2, 5] and f.tolist() == [False, True]
    s, f = oracle.export_seeds(res, nh, triplets=True)
    assert s.tolist() == [0, 2, 5]
    s, _ = oracle.export_seeds(res)          # no hit counts: every seed a quad
    assert s.tolist() == [0, 1, 2, 5]
