"""Parity helpers shared by the GPU tests: the library's result against the
CPU oracle on the same event, and the canonical order of its lists."""
import numpy as np

import oracle
from paper_2407_18231_amd import lst

STAGES = ("md", "ls", "t3", "t5", "pt3", "pt5", "tc")


# Flagged-candidate budget of one event: the bar over many events is 1e-4 of
# a stage's objects for candidates flagged by their own cut margin and 2.5e-4
# with the objects that inherit a flag from a constituent; one event may
# fluctuate to three times that.
OWN_BUDGET = 3e-4
ALL_BUDGET = 6e-4


def check_parity(geom, ev, res):
    ores = oracle.run(geom, ev)
    kd = oracle.keyed(ores)
    fb = oracle.flag_breakdown(ores)
    got = lst.result_keys(res)
    for k in STAGES:
        assert len(set(got[k])) == len(got[k]), f"duplicates in {k}"
    rep = oracle.compare(kd, got)
    for k in STAGES:
        r = rep[k]
        n, n_flag, n_own = fb[k]
        print(k, {q: r[q] for q in ("got", "total", "flagged", "missing", "extra")}, "own", n_own, flush=True)
        assert r["missing"] == 0 and r["extra"] == 0, (k, r)
        assert n_own <= max(3, OWN_BUDGET * n), (k, n, n_own)
        assert n_flag <= max(5, ALL_BUDGET * n), (k, n, n_flag)
    return rep


def check_canonical(res, ev):
    md = res["md"].astype(np.int64)
    if len(md) > 1:
        key = np.lexsort((md[:, 1], md[:, 0], ev["module"][md[:, 0]]))
        assert np.array_equal(key, np.arange(len(md))), "md order"
    for k in ("ls", "t3", "t5", "pt3", "pt5"):
        a = res[k].astype(np.int64)
        if len(a) > 1:
            key = a[:, 0] * (1 << 32) + a[:, 1]
            assert np.all(np.diff(key) > 0), k


