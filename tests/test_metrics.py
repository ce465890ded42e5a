"""The truth-matched metrics on hand-built candidate lists (CPU): more than
75% of a candidate's hits from one track matches it; the rates follow the
definitions of the paper's Sec. 3."""
import numpy as np

from paper_2407_18231_amd import metrics


def _event():
    # two tracks, ten hits each (track 0: hits 0-9, track 1: hits 10-19), two noise hits
    lab = np.array([0] * 10 + [1] * 10 + [-1, -1], np.int32)
    tracks = np.array([[1, 2.0, 0.1, 0.0, 0.0], [-1, 1.5, -0.2, 1.0, 0.0], [1, 0.6, 0.0, 2.0, 0.0]])
    return dict(hit_track=lab, tracks=tracks, pls_track=np.array([0, 1, -1], np.int32))


def _res(t5_hits, extra_tc=()):
    """A result with one MD per hit pair (h, h+1) and one T5 per given list
    of ten hits; each T5 is a track candidate, then the extra (type, index)."""
    md, ls, t3, t5 = [], [], [], []
    for hits in t5_hits:
        m0 = len(md)
        for k in range(5):
            md.append((hits[2 * k], hits[2 * k + 1]))
        l0 = len(ls)
        for k in range(4):
            ls.append((m0 + k, m0 + k + 1))
        u0 = len(t3)
        t3 += [(l0, l0 + 1), (l0 + 2, l0 + 3)]
        t5.append((u0, u0 + 1))
    tc = [(2, i) for i in range(len(t5_hits))] + list(extra_tc)
    a = lambda v: np.array(v, np.uint32).reshape(-1, 2)
    return dict(md=a(md), ls=a(ls), t3=a(t3), t5=a(t5), pt3=a([]), pt5=a([]), tc=a(tc))


def test_perfect_candidates():
    ev = _event()
    r = metrics.rates(ev, _res([list(range(10)), list(range(10, 20))]))
    assert r["efficiency"] == 1.0 and r["fake_rate"] == 0.0 and r["duplicate_rate"] == 0.0
    assert r["n_sim"] == 2      # the third track is below the pT threshold


def test_match_needs_more_than_75_percent():
    ev = _event()
    # 8 of 10 hits from track 0 match; 7 of 10 do not
    m8 = list(range(8)) + [20, 21]
    m7 = list(range(7)) + [20, 21, 12]
    r = metrics.match(ev, _res([m8, m7]))
    assert list(r) == [0, -1]


def test_duplicates_and_seed_candidates():
    ev = _event()
    # two candidates of track 0, one seed-only candidate of track 1, one fake seed
    r = metrics.rates(ev, _res([list(range(10)), list(range(10))], extra_tc=[(3, 1), (3, 2)]))
    assert r["n_tc"] == 4
    assert r["duplicate_rate"] == 0.5 and r["fake_rate"] == 0.25 and r["efficiency"] == 1.0
    # track 1 is found by its seed only: not by an outer-tracker candidate
    assert r["efficiency_ot"] == 0.5


def test_efficiency_vs_rv_bins():
    """Efficiency per production-radius bin: track 0 (r_vertex 3 cm) is
    found by a T5, track 1 (12 cm) by nothing, track 2 (prompt, below the
    pT cut) is not counted."""
    ev = dict(_event(), track_rv=np.array([3.0, 12.0, 0.0]))
    res = _res([list(range(10))])
    r = metrics.efficiency_vs_rv(ev, res, edges=(0.0, 5.0, 20.0))
    b0, b1 = r["bins"]
    assert (b0["n_sim"], b0["efficiency"], b0["by_type"]["T5"]) == (1, 1.0, 1.0)
    assert (b1["n_sim"], b1["efficiency"]) == (1, 0.0)
    r = metrics.efficiency_vs_rv(ev, res, edges=(0.0, 5.0, 20.0), displaced_only=False, pt_min=0.5)
    assert r["bins"][0]["n_sim"] == 2
