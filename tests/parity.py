"""Parity helpers shared by the GPU tests: the library's result against the
CPU oracle on the same event, and the canonical order of its lists."""
import numpy as np

import oracle
from paper_2407_18231_amd import lst

STAGES = ("md", "ls", "t3", "t5", "pt3", "pt5", "tc")


# Flagged-candidate budget of one event: the bar over many events is 1e-4 of
# a stage's objects for candidates flagged by their own cut margin (one event
# may fluctuate to three times that).  Objects that inherit a flag come in
# clusters -- every segment of a flagged mini-doublet, every T3 of a flagged
# segment -- so one event can carry ten times the average of 2.5e-4 (a
# 64-event PU200 batch holds one with LS 83 flagged of 83 286, 18 of them by
# their own margin).
OWN_BUDGET = 3e-4
ALL_BUDGET = 1.5e-3
# floors for small events, where the expected counts are a few (a PU100
# event has 2 own-margin segment flags on average; 8 is its 0.1% tail)
OWN_FLOOR = 8
ALL_FLOOR = 20


def check_parity(geom, ev, res, params=None):
    ores = oracle.run(geom, ev, params)
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
        assert n_own <= max(OWN_FLOOR, OWN_BUDGET * n), (k, n, n_own)
        assert n_flag <= max(ALL_FLOOR, ALL_BUDGET * n), (k, n, n_flag)
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


