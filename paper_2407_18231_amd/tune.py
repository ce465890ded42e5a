"""Autotuner for the speed-only parameters of the chain.

Two choices change only the speed, never the lists:
  * the seed-lookup bucket granularity: azimuth bins per (event, surface)
    row and curvature bins per resolution class (lst_params.n_phi_bins,
    n_kappa_bins) -- finer bins mean fewer candidate entries per seed but
    more bucket offsets to load, scan and clear;
  * the segment walk's tile: runs of edges per group (ls_group 4 / 6 / 8,
    i.e. how many MD ranges a lane loads per step) and its occupancy (ls_waves: the
    compiler's register choice, or at least 6 or 8 waves per SIMD).
The tuner times the bucket grid first, then the segment-walk variants at the
best grid, each on a batch on the device (hipGraph replays of the whole
chain), checks that every setting yields the same lists as the first one,
and caches the fastest per GPU architecture and workload class.
lst.Context applies the cached choice when the caller sets none of these.

Usage: python -m paper_2407_18231_amd.tune [--batch 64] [--pileup 200]
                                           [--repeats 20] [--cache FILE]
"""
from __future__ import annotations

import argparse
import json
import os
import time

from . import lst, synth

CANDIDATES = [(32, 12), (32, 16), (48, 16), (64, 12), (64, 16), (64, 24), (96, 16), (128, 16)]
LS_CANDIDATES = [(6, 0), (4, 0), (8, 0), (6, 6), (4, 6), (8, 6), (6, 8), (4, 8), (8, 8)]
TUNED = ("n_phi_bins", "n_kappa_bins", "ls_group", "ls_waves")
STAGES = ("md", "ls", "t3", "t5", "pt3", "pt5", "tc")


def default_cache() -> str:
    return os.environ.get("LST_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lst_tune.json"))


def device_arch(device: int = 0) -> str:
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def workload_class(n_events: int, pileup: int) -> str:
    return f"batch{n_events}-pu{pileup}"


def time_setting(events: list, geometry, n_phi: int, n_kappa: int, repeats: int, ls_group: int = 0,
                 ls_waves: int = 0):
    """Mean ms per batch over `repeats` graph replays, and the lists."""
    with lst.Context(max_batch=len(events), n_phi_bins=n_phi, n_kappa_bins=n_kappa, ls_group=ls_group,
                     ls_waves=ls_waves) as c:
        c.load_geometry(geometry)
        c.batch_upload(events)
        c.batch_execute(2, graph=True)            # capture, sizing, warm-up
        t0 = time.perf_counter()
        c.batch_execute(repeats, graph=True)
        ms = (time.perf_counter() - t0) * 1e3 / repeats
        return ms, c.batch_download(len(events))


def tune(events: list, geometry, candidates=CANDIDATES, ls_candidates=LS_CANDIDATES, repeats: int = 20) -> dict:
    ref = None

    def check(res, what):
        nonlocal ref
        if ref is None:
            ref = res
            return
        for a, b in zip(ref, res):
            for k in STAGES:
                if a[k].shape != b[k].shape or (a[k] != b[k]).any():
                    raise RuntimeError(f"setting {what} changed the {k} list")

    times = {}
    for n_phi, n_kappa in candidates:
        ms, res = time_setting(events, geometry, n_phi, n_kappa, repeats)
        check(res, (n_phi, n_kappa))
        times[f"{n_phi}x{n_kappa}"] = round(ms, 4)
    best = min(times, key=times.get)
    n_phi, n_kappa = (int(v) for v in best.split("x"))
    ls_times = {}
    for group, waves in ls_candidates:
        ms, res = time_setting(events, geometry, n_phi, n_kappa, repeats, group, waves)
        check(res, (group, waves))
        ls_times[f"g{group}w{waves}"] = round(ms, 4)
    best_ls = min(ls_times, key=ls_times.get)
    group, waves = (int(v) for v in best_ls[1:].split("w"))
    return {"n_phi_bins": n_phi, "n_kappa_bins": n_kappa, "ls_group": group, "ls_waves": waves,
            "ms_per_batch": times, "ms_per_batch_ls": ls_times}


def cached_choice(max_batch: int, path: str | None = None) -> dict | None:
    """The tuned parameters for this GPU and batch size, if the cache holds
    them (the PU200 workload class first, else any of that batch size)."""
    path = path or default_cache()
    if not os.path.exists(path):
        return None
    try:
        import torch
        if not torch.cuda.is_available():
            return None
        arch = device_arch()
        with open(path) as f:
            per_arch = json.load(f).get(arch, {})
    except (OSError, ValueError, RuntimeError, ImportError):
        return None
    return choice_for(per_arch, max_batch)


def choice_for(per_arch: dict, max_batch: int) -> dict | None:
    """From one architecture's cache entries: the PU200 class of this batch
    size, else any class of that batch size; only the tuned parameters."""
    ch = per_arch.get(workload_class(max_batch, 200))
    if ch is None:
        ch = next((v for k, v in sorted(per_arch.items()) if k.startswith(f"batch{max_batch}-")), None)
    return {k: ch[k] for k in TUNED if k in ch} if ch else None


def load_choice(arch: str, workload: str, path: str | None = None) -> dict | None:
    """The cached (n_phi_bins, n_kappa_bins) for this architecture and workload, if any."""
    try:
        with open(path or default_cache()) as f:
            return json.load(f).get(arch, {}).get(workload)
    except (OSError, ValueError):
        return None


def store_choice(arch: str, workload: str, choice: dict, path: str | None = None) -> None:
    path = path or default_cache()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data.setdefault(arch, {})[workload] = choice
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    with open(path, "w") as f:
        json.dump(data, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--pileup", type=int, default=200)
    ap.add_argument("--repeats", type=int, default=20)
    ap.add_argument("--cache", default=None)
    args = ap.parse_args()
    g = synth.make_geometry("pu200")
    events = [synth.gen_event(g, synth.config_pu(args.pileup), synth.event_seed(2, i)) for i in range(args.batch)]
    choice = tune(events, g, repeats=args.repeats)
    arch, wl = device_arch(), workload_class(args.batch, args.pileup)
    store_choice(arch, wl, choice, args.cache)
    print(json.dumps({"arch": arch, "workload": wl, **choice}), flush=True)


if __name__ == "__main__":
    main()
