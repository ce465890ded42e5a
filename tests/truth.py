"""Truth objects of generated events (test helper).

From the generator's hit -> track labels, lists for each track the objects a
perfect reconstruction would build: a mini-doublet where a track left one hit
on each sensor of the same module, a line segment for consecutive
mini-doublets on consecutive surfaces, T3 / T5 for chains of three / five
consecutive mini-doublets.  Keys use input hit indices, like
``oracle.object_keys``.
"""
from __future__ import annotations

import numpy as np

from paper_2407_18231_amd.synth import BARREL


def _surface_ids(geom):
    kind, layer, side = geom.kind, geom.layer, geom.side
    nb = int(layer[kind == BARREL].max()) + 1 if (kind == BARREL).any() else 0
    nd = int(layer[kind != BARREL].max()) + 1 if (kind != BARREL).any() else 0
    sid = np.where(kind == BARREL, layer, nb + np.where(side > 0, 0, nd) + layer)
    return sid.astype(np.int64), nb, nd


def _is_next(nb, nd, s, t):
    if s < nb:
        if t == s + 1 and t < nb:
            return True
        return bool(nd) and (t == nb or t == nb + nd)
    d = (s - nb) % nd
    return d + 1 < nd and t == s + 1


def _is_linked(nb, nd, s, t, skip):
    """t is the next surface of s, or with skip the next of a next surface"""
    if _is_next(nb, nd, s, t):
        return True
    return skip and any(_is_next(nb, nd, s, u) and _is_next(nb, nd, u, t)
                        for u in range(nb + 2 * nd))


def truth_objects(geom, ev, track_mask=None, skip=False):
    """Returns dict stage -> set of keys, for tracks selected by track_mask
    (boolean array over tracks; default all).  With skip, segments may also
    join a track's mini-doublets two surfaces apart, and every chain of such
    segments is a true T3 / T5."""
    sid, nb, nd = _surface_ids(geom)
    tid = ev["hit_track"]
    mod = ev["module"].astype(np.int64)
    sen = ev["sensor"]
    n_trk = ev["tracks"].shape[0]
    if track_mask is None:
        track_mask = np.ones(n_trk, bool)
    order = np.argsort(tid, kind="stable")
    out = {k: set() for k in ("md", "ls", "t3", "t5")}
    per_track_mds = {}
    tids = tid[order]
    bounds = np.searchsorted(tids, np.arange(n_trk + 1))
    for t in range(n_trk):
        if not track_mask[t]:
            continue
        hits = order[bounds[t]:bounds[t + 1]]
        by_surf = {}
        for h in hits:
            s = int(sid[mod[h]])
            by_surf.setdefault(s, [None, None, None, None])
            e = by_surf[s]
            e[int(sen[h])] = int(h)
            e[2 + int(sen[h])] = int(mod[h])
        # surfaces in the order the track crosses them: barrel layers by radius
        # then disks by |z| (prompt outgoing tracks cross them in this order)
        mds = []
        for s in sorted(by_surf):
            lo, up, mlo, mup = by_surf[s]
            if lo is not None and up is not None and mlo == mup:
                mds.append((s, (lo, up)))
        per_track_mds[t] = mds
        for s, k in mds:
            out["md"].add(k)
        if skip:
            n = len(mds)
            nxt = [[j for j in range(i + 1, n) if _is_linked(nb, nd, mds[i][0], mds[j][0], True)]
                   for i in range(n)]
            for i in range(n):
                for j in nxt[i]:
                    out["ls"].add(mds[i][1] + mds[j][1])
                    for k in nxt[j]:
                        out["t3"].add(mds[i][1] + mds[j][1] + mds[k][1])
                        for l in nxt[k]:
                            for m in nxt[l]:
                                out["t5"].add(mds[i][1] + mds[j][1] + mds[k][1] + mds[l][1] + mds[m][1])
            continue
        # chains of consecutive MDs on consecutive surfaces
        runs = []
        cur = []
        for s, k in mds:
            if cur and not _is_next(nb, nd, cur[-1][0], s):
                runs.append(cur)
                cur = []
            cur.append((s, k))
        if cur:
            runs.append(cur)
        for run in runs:
            keys = [k for _, k in run]
            for i in range(len(keys) - 1):
                out["ls"].add(keys[i] + keys[i + 1])
            for i in range(len(keys) - 2):
                out["t3"].add(keys[i] + keys[i + 1] + keys[i + 2])
            for i in range(len(keys) - 4):
                out["t5"].add(keys[i] + keys[i + 1] + keys[i + 2] + keys[i + 3] + keys[i + 4])
    return out
