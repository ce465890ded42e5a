"""Truth-matched physics metrics of a track-candidate list (Sec. 3 of the
paper): efficiency, fake rate and duplicate rate.

A simulated track matches a candidate when more than 75% of the
candidate's hits come from it.  The candidate's hits are the outer-tracker
hits of its mini-doublets (ten for pT5 and T5, six for pT3); a candidate
made of a pixel seed alone has no outer-tracker hit and is matched to the
track the seed came from (a fake seed matches nothing) -- the synthetic seeds
carry no pixel hits, only that label.  Efficiency is the fraction of
selected simulated tracks matched by at least one candidate; the fake rate
the fraction of candidates matched by no track; the duplicate rate the
fraction of candidates whose track is matched by more than one candidate.
This module only reads result lists and generator labels; it does no
reconstruction arithmetic.
"""
from __future__ import annotations

import numpy as np

MATCH_FRACTION = 0.75
TYPES = ("pT5", "pT3", "T5", "pLS")


def candidate_hits(res: dict):
    """Per track candidate: (type, seed index or -1, array of input hit
    indices), from a result's index lists."""
    md = res["md"].astype(np.int64)
    ls = res["ls"].astype(np.int64)
    t3 = res["t3"].astype(np.int64)
    t5 = res["t5"].astype(np.int64)

    def t3_mds(i):
        l1, l2 = t3[i]
        return [ls[l1, 0], ls[l1, 1], ls[l2, 1]]

    def t5_mds(i):
        u, w = t5[i]
        a = t3_mds(u)
        b = t3_mds(w)
        return a + b[1:]

    out = []
    for typ, idx in res["tc"].astype(np.int64):
        if typ == 0:
            p, v = res["pt5"][idx]
            mds = t5_mds(int(v))
        elif typ == 1:
            p, v = res["pt3"][idx]
            mds = t3_mds(int(v))
        elif typ == 2:
            p, mds = -1, t5_mds(int(idx))
        else:
            p, mds = int(idx), []
        hits = md[mds].reshape(-1) if mds else np.zeros(0, np.int64)
        out.append((int(typ), int(p), hits))
    return out


def match(ev: dict, res: dict) -> np.ndarray:
    """Simulated track matched by each candidate (-1: none)."""
    label = ev["hit_track"]
    seed_label = ev.get("pls_track")
    m = np.full(len(res["tc"]), -1, np.int64)
    for k, (typ, p, hits) in enumerate(candidate_hits(res)):
        if typ == 3:
            if seed_label is not None and seed_label[p] >= 0:
                m[k] = int(seed_label[p])
            continue
        lab = label[hits]
        lab = lab[lab >= 0]
        if lab.size == 0:
            continue
        vals, cnt = np.unique(lab, return_counts=True)
        j = int(np.argmax(cnt))
        if cnt[j] > MATCH_FRACTION * hits.size:
            m[k] = int(vals[j])
    return m


def rates(ev: dict, res: dict, pt_min: float = 0.8, eta_max: float = 2.4) -> dict:
    """Efficiency over simulated tracks with pT > pt_min and |eta| < eta_max;
    fake and duplicate rates over all candidates; per candidate type too."""
    m = match(ev, res)
    trk = ev["tracks"]
    sel = np.nonzero((trk[:, 1] > pt_min) & (np.abs(trk[:, 2]) < eta_max))[0]
    matched = m[m >= 0]
    n_per_track = np.bincount(matched, minlength=trk.shape[0]) if matched.size else np.zeros(trk.shape[0], np.int64)
    found = n_per_track[sel] > 0
    n = len(m)
    dup = np.array([t >= 0 and n_per_track[t] > 1 for t in m], bool)
    types = res["tc"][:, 0].astype(np.int64) if n else np.zeros(0, np.int64)
    ot = m[(m >= 0) & (types != TYPES.index("pLS"))] if n else m[:0]
    found_ot = np.bincount(ot, minlength=trk.shape[0])[sel] > 0 if ot.size else np.zeros(sel.size, bool)
    by_type = {}
    for ti, name in enumerate(TYPES):
        k = types == ti
        by_type[name] = dict(n=int(k.sum()),
                             fake=float((m[k] < 0).mean()) if k.any() else 0.0,
                             duplicate=float(dup[k].mean()) if k.any() else 0.0)
    return dict(n_tc=n, n_sim=int(sel.size),
                efficiency=float(found.mean()) if sel.size else 0.0,
                efficiency_ot=float(found_ot.mean()) if sel.size else 0.0,
                fake_rate=float((m < 0).mean()) if n else 0.0,
                duplicate_rate=float(dup.mean()) if n else 0.0,
                by_type=by_type)


def efficiency_vs_rv(ev: dict, res: dict, edges=(0.0, 1.0, 5.0, 10.0, 20.0, 35.0), pt_min: float = 0.8,
                     eta_max: float = 2.4, displaced_only: bool = True) -> dict:
    """Efficiency as a function of the production radius r_vertex (Sec. 3,
    Fig. 3 right): per bin [edges[i], edges[i+1]) of ev["track_rv"], the
    fraction of selected simulated tracks (pT > pt_min, |eta| < eta_max;
    only those with r_vertex > 0 when displaced_only) matched by at least one
    candidate, with the bin's track count; and the same for candidates of
    each type."""
    m = match(ev, res)
    trk = ev["tracks"]
    rv = ev.get("track_rv", np.zeros(trk.shape[0]))
    sel = (trk[:, 1] > pt_min) & (np.abs(trk[:, 2]) < eta_max)
    if displaced_only:
        sel &= rv > 0
    types = res["tc"][:, 0].astype(np.int64) if len(res["tc"]) else np.zeros(0, np.int64)
    found_by = {}
    for ti, name in enumerate(TYPES):
        hit = np.zeros(trk.shape[0], bool)
        t = m[(types == ti) & (m >= 0)]
        hit[t] = True
        found_by[name] = hit
    found = np.zeros(trk.shape[0], bool)
    found[m[m >= 0]] = True
    out = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        b = sel & (rv >= lo) & (rv < hi)
        n = int(b.sum())
        out.append(dict(rv_lo=lo, rv_hi=hi, n_sim=n, efficiency=float(found[b].mean()) if n else 0.0,
                        by_type={k: float(v[b].mean()) if n else 0.0 for k, v in found_by.items()}))
    return dict(bins=out)
