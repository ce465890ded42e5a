"""Benchmark of the LST object-building chain on one MI355X.

Workload: PU200-like events (6 barrel layers + 2 x 5 disks, 12 800 modules,
4000 tracks with dN/dpT ~ pT^-3 above 0.5 GeV, |eta| < 2.4, 10% hit
inefficiency, 20% noise hits, 2000 pixel seeds with 2% fakes), synthetic and
seeded (event i uses seed 2000 + i).  One step = the whole chain (hit sort,
MD, LS, T3, T5, seed lookup, pT3/pT5, TC) over one batch of events already
resident in device memory.

Printed JSON line: value = events/s of the batched path (64 events per
launch); beside it the plain one-event-per-launch path (events/s, p50/p99
latency on device and end to end), a mixed-pileup batch, the roofline of the
dominant kernel (HIP events on the library's stream over the timed region),
and the CPU oracle on the host as a reported baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch 64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes of one step, per kernel name: the per-unit figures of the
# method (hit 17 B in / 20 B sorted, MD anchor 20 B, index pair 8 B, seed
# 80 B, candidate 24 B) times the units of this batch.  Candidates are what
# each stage examines; S_B is the number of outer-MD gathers one pass over the
# connection map needs (per edge leaving a module that holds MDs, the MDs of
# its destination), E_used the number of such edges.  The seed lookup walks
# bucket entries of 12 B (curvature, its resolution, anchor azimuth) and
# appends (seed, object) pairs of 8 B; the full seed cuts read each seed
# (80 B) once and, per pair, the pair, the object's anchors (2 x 20 B plus
# curvature 8 B) and write a 4 B rank.
def step_bytes(c: dict, n_hits: int, n_pls: int, n_units: int, s_b: int, e_used: int) -> dict:
    nmd, nls, nt3, nt5 = c["md"], c["ls"], c["t3"], c["t5"]
    ls = 20.0 * nmd + 20.0 * s_b + 6.0 * e_used + 4.0 * nmd
    t3 = 8.0 * nls + 8.0 * nmd + 24.0 * c["cand_t3"]
    t5 = 8.0 * nt3 + 8.0 * nmd + 24.0 * c["cand_t5"]
    out = {
        "hit_hist": 17.0 * n_hits + 8.0 * n_hits,
        "hit_scatter": 25.0 * n_hits + 16.0 * n_hits,
        "hit_gather": 16.0 * n_hits + 24.0 * n_hits,
        "md_count": 16.0 * n_hits + 12.0 * n_units + 4.0 * n_hits,
        "md_fill": 16.0 * n_hits + 12.0 * n_units + 28.0 * nmd,
        "md_walk": 16.0 * n_hits + 12.0 * n_units + 4.0 * n_hits,
        "md_place": 28.0 * nmd,
        "ls_count": ls,
        "ls_fill": ls + 8.0 * nls,
        "ls_walk": ls,
        "ls_place": 8.0 * nls,
        "t3_count": t3 + 4.0 * nls,
        "t3_fill": t3 + 8.0 * nt3 + 16.0 * nt3,
        "t3_walk": t3 + 4.0 * nls,
        "t3_place": 24.0 * nt3,
        "t5_count": t5 + 4.0 * nt3,
        "t5_fill": t5 + 16.0 * nt5,
        "t5_walk": t5 + 4.0 * nt3,
        "t5_place": 16.0 * nt5,
    }
    for k in ("3", "5"):
        out[f"pt{k}c_walk"] = 80.0 * n_pls + 12.0 * c["cand_pt" + k] + 8.0 * c["eval_pt" + k]
        out[f"pt{k}_eval"] = 80.0 * n_pls + (8.0 + 48.0 + 4.0) * c["eval_pt" + k]
    return out


def outer_gathers(events, results, begin, dst):
    """S_B and E_used of the batch from the MD lists the chain returned."""
    src = np.repeat(np.arange(begin.size - 1), np.diff(begin))
    s_b = e_used = 0
    for ev, r in zip(events, results):
        n = np.bincount(ev["module"][r["md"][:, 0]], minlength=begin.size - 1) if len(r["md"]) else \
            np.zeros(begin.size - 1, np.int64)
        has = n[src] > 0
        s_b += int(n[dst][has].sum())
        e_used += int(has.sum())
    return s_b, e_used


def kernels_digest() -> str:
    """sha256 of the kernel sources, to tie counter results to the code they
    were taken on."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "engine.h"):
        with open(os.path.join(ROOT, "paper_2407_18231_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_of(kernel: str):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE,
    WRITE_SIZE, each scaled by what the counter reads for a plain copy of
    known size), stored beside the profile summaries; null when absent or
    when the kernels have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernels_sha256") != kernels_digest():
        return None
    v = t.get("kernels", {}).get(kernel)
    return None if v is None else v.get("bytes_per_launch")


def cpu_baseline(n_events: int, budget_s: float):
    import oracle
    from paper_2407_18231_amd import synth
    g = synth.make_geometry("pu200")
    oracle.build(force=False)
    times = []
    t_all = time.perf_counter()
    for i in range(n_events):
        ev = synth.gen_event(g, synth.config_pu(200), synth.event_seed(2, i))
        t0 = time.perf_counter()
        oracle.run(g, ev)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_all > budget_s:
            break
    tot = sum(times)
    return dict(value=len(times) / tot, unit="events/s", cores=1, kind="oracle",
                sample=f"{len(times)} PU200-like events (seeds 2000..{1999 + len(times)}), "
                       f"one thread, {tot:.1f} s of oracle time")


def _oracle_one(i):
    import oracle
    from paper_2407_18231_amd import synth
    g = synth.make_geometry("pu200")
    ev = synth.gen_event(g, synth.config_pu(200), synth.event_seed(2, i))
    t0 = time.perf_counter()
    oracle.run(g, ev)
    return time.perf_counter() - t0


def cpu_baseline_all_cores(budget_s: float):
    """The oracle on every host core at once, one event per worker process
    (events are independent)."""
    import multiprocessing as mp
    import oracle
    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))
    n = cores
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        pool.map(_oracle_one, range(n))
    wall = time.perf_counter() - t0
    return dict(value=n / wall, unit="events/s", cores=cores, kind="oracle",
                sample=f"{n} PU200-like events, one per process on {cores} cores, {wall:.1f} s wall")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-events", type=int, default=32)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--quick", action="store_true", help="only the batched path (profiling runs)")
    ap.add_argument("--chain-only", type=int, default=0, metavar="N",
                    help="counter runs: upload one batch, run the chain N times, print nothing else")
    ap.add_argument("--graph", action="store_true", help="with --chain-only: replay the captured graph")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="counter calibration: one device-to-device copy of MB megabytes (torch)")
    ap.add_argument("--link-probe", action="store_true",
                    help="host link bandwidth of large pinned copies, each way and both at once")
    ap.add_argument("--served-only", type=int, default=0, metavar="N",
                    help="trace runs: N events (PU ~ U[140, 200]) submitted back to back to the served path")
    ap.add_argument("--skip-only", action="store_true",
                    help="only the skip-layer section (batch, objects, rates with and without the flag)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.link_probe:
        log("host link:", link_probe())
        return
    if args.served_only:
        from paper_2407_18231_amd import lst, synth
        pool = served_events(min(args.served_only, 512))
        g = synth.make_geometry("pu200")
        with lst.Context(max_batch=64, n_slots=2) as c:
            c.load_geometry(g)
            r = served_run(c, pool, 0.0, args.served_only, 100)
        log("served:", r)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the events of a batch shard across GPUs with no "
              f"exchange, so there is no multi-GPU path to time (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    from paper_2407_18231_amd import lst, synth

    g = synth.make_geometry("pu200")
    B = args.batch
    t0 = time.perf_counter()
    events = [synth.gen_event(g, synth.config_pu(200), synth.event_seed(2, i)) for i in range(B)]
    log(f"generated {B} events in {time.perf_counter() - t0:.1f} s")
    n_hits = int(sum(e["x"].size for e in events))
    n_pls = int(sum(e["pls_par"].shape[0] for e in events))
    if not args.quick and not args.chain_only:
        # the served workloads, generated on the host's cores before the GPU is touched
        t0 = time.perf_counter()
        pool4 = served_events(5000)
        pool5 = served_events(256, 300.0, 300.0, 5, 0.4, 0.05)
        log(f"served pools: {len(pool4)} + {len(pool5)} events in {time.perf_counter() - t0:.1f} s")

    if args.skip_only:
        log("skip-layer links:", json.dumps(skip_layer(g, events, args.steps)))
        log("physics:", json.dumps(physics(g, events[:16])))
        return

    ctx = lst.Context(max_batch=max(B, 64))
    ctx.load_geometry(g)
    begin, dst = ctx.connection_map()

    # ---- batched path: B events per launch --------------------------------
    ctx.batch_upload(events)
    if args.chain_only:
        ctx.batch_execute(args.chain_only, graph=args.graph, timing=False)
        log(f"chain run {args.chain_only} times on {B} events")
        ctx.close()
        return
    counts = ctx.batch_counts()
    log("object totals:", counts)
    for _ in range(args.warmup):
        ctx.batch_execute(1, graph=False, timing=False)
    # where a step's time goes: every launch bracketed by HIP events (a
    # diagnostic pass before the timed region; the events and the host wait
    # per step slow it down)
    ctx.time_only(None)
    ctx.batch_execute(args.steps, graph=False, timing=True)
    kdiag = ctx.kernel_times()
    step_ms = {k: v[0] / args.steps for k, v in kdiag.items()}
    launches = {k: v[1] / args.steps for k, v in kdiag.items()}
    dom = max(step_ms, key=step_ms.get)
    # timed region: K steps back to back on the library's stream; HIP events
    # bracket every launch of the dominant kernel (its durations below)
    ctx.time_only(dom)
    t0 = time.perf_counter()
    dev_ms = ctx.batch_execute(args.steps, graph=False, timing=True)
    wall = time.perf_counter() - t0
    ktimed = ctx.kernel_times()
    ctx.time_only(None)
    ms_per_step = 1e3 * wall / args.steps
    value = B / (wall / args.steps)
    log(f"batched: {ms_per_step:.3f} ms/step, {value:.1f} events/s (device {dev_ms / args.steps:.3f} ms/step)")
    # graph replay of the same chain
    ctx.batch_execute(2, graph=True)
    t0 = time.perf_counter()
    ctx.batch_execute(args.steps, graph=True)
    graph_rate = B / ((time.perf_counter() - t0) / args.steps)
    log(f"batched, graph replay: {graph_rate:.1f} events/s")

    # dominant kernel and its roofline (durations from the timed region)
    per = {k: v[0] / max(v[1], 1) for k, v in kdiag.items()}
    avg_ms = ktimed[dom][0] / max(ktimed[dom][1], 1)
    s_b, e_used = outer_gathers(events, ctx.batch_download(B), begin, dst)
    sb = step_bytes(counts, n_hits, n_pls, B * g.n_mod, s_b, e_used)
    alg = sb.get(dom, 0.0) / max(launches[dom], 1.0)     # per launch
    achieved = alg / (avg_ms * 1e-3) / 1e9 if alg else 0.0
    roofline = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic_of(dom),
                    avg_launch_ms=round(avg_ms, 4), launches_timed=int(ktimed[dom][1]),
                    algorithmic_bytes_per_launch=int(alg))
    effective = {k: round(sb[k] / max(launches[k], 1.0) / (per[k] * 1e-3) / 1e9, 1)
                 for k in sb if k in per and per[k] > 0}
    log("effective GB/s by kernel:", effective)
    stages = {k: round(v, 4) for k, v in sorted(step_ms.items(), key=lambda kv: -kv[1])}
    log("ms per step by kernel:", stages)

    result = dict(metric="events/sec at PU200-like load, batched vs per-event; p50/p99 event latency",
                  value=round(value, 2), unit="events/s", n_gpus=1, steps=args.steps,
                  warmup=args.warmup, ms_per_step=round(ms_per_step, 4), higher_is_better=True,
                  scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
                  config=dict(workload=f"{B} PU200-like events per launch (single-event PU200 shape, "
                                       f"seeds 2000+i), batched path, inputs resident in HBM",
                              events_per_step=B, pileup=200, modules=g.n_mod,
                              hits_per_event=round(n_hits / B, 1), seeds_per_event=round(n_pls / B, 1)),
                  batched_graph_events_per_s=round(graph_rate, 2),
                  roofline=roofline, kernel_ms_per_step=stages, effective_gbs_by_kernel=effective,
                  objects_per_event={k: round(counts[k] / B, 1) for k in ("md", "ls", "t3", "t5", "pt3", "pt5", "tc")})

    if not args.quick:
        # ---- batched, end to end: host inputs in, host lists out ----------------
        ins = [lst.EventIn(ev) for ev in events]
        ctx.run_batch_in(ins, fetch=False)
        t1 = time.perf_counter()
        for _ in range(5):
            ctx.run_batch_in(ins, fetch=False)
        dt = (time.perf_counter() - t1) / 5
        result["batched_e2e"] = dict(events_per_s=round(B / dt, 1), ms_per_call=round(dt * 1e3, 3),
                                     path=f"lst_run_batch, {B} events per call: host inputs in, "
                                          f"host lists out, the library call alone")
        log("batched end to end:", result["batched_e2e"])
        del ins
        # ---- plain path: one event per launch, on its own context ---------------
        ctx1 = lst.Context()
        ctx1.load_geometry(g)
        lat = []
        for i in range(min(B, 32)):
            ctx1.batch_upload([events[i]])
            ctx1.batch_execute(1, graph=True)
            for _ in range(3):
                t1 = time.perf_counter()
                ctx1.batch_execute(1, graph=True)
                lat.append(time.perf_counter() - t1)
        lat_us = np.array(lat) * 1e6
        per_event_rate = 1e6 / lat_us.mean()
        # where a single event's time goes (HIP events around each kernel)
        ctx1.batch_upload([events[0]])
        ctx1.batch_execute(10, graph=False, timing=True)
        kt1 = ctx1.kernel_times()
        per_event_kernels = {k: round(v[0] / 10, 4) for k, v in sorted(kt1.items(), key=lambda kv: -kv[1][0])[:12]}
        log("per-event kernel ms:", per_event_kernels)
        # end to end: host inputs in, host outputs back (lst_run_event), over
        # 200 events with PU ~ U[140, 200]: the library call alone, and with
        # the binding's conversion of the lists to numpy
        e2e_evs = pool4[:200]
        for ev in e2e_evs[:3]:
            ctx1.run_event(ev)
        ins = [lst.EventIn(ev) for ev in e2e_evs]
        e2e, e2e_py = [], []
        for e in ins:
            t1 = time.perf_counter()
            ctx1.run_event_in(e, fetch=False)
            e2e.append(time.perf_counter() - t1)
        for e in ins:
            t1 = time.perf_counter()
            ctx1.run_event_in(e, fetch=True)
            e2e_py.append(time.perf_counter() - t1)
        ctx1.close()
        e2e_us = np.array(e2e) * 1e6
        e2e_py_us = np.array(e2e_py) * 1e6
        result["per_event"] = dict(events_per_s=round(per_event_rate, 2),
                                   latency_us_p50=round(float(np.percentile(lat_us, 50)), 1),
                                   latency_us_p99=round(float(np.percentile(lat_us, 99)), 1),
                                   e2e_events_per_s=round(1e6 / e2e_us.mean(), 2),
                                   e2e_latency_us_p50=round(float(np.percentile(e2e_us, 50)), 1),
                                   e2e_latency_us_p99=round(float(np.percentile(e2e_us, 99)), 1),
                                   e2e_events="200, PU ~ U[140, 200]",
                                   e2e_python_latency_us_p50=round(float(np.percentile(e2e_py_us, 50)), 1),
                                   e2e_python_latency_us_p99=round(float(np.percentile(e2e_py_us, 99)), 1))
        result["per_event_kernel_ms"] = per_event_kernels
        result["batched_over_per_event"] = round(value / per_event_rate, 2)
        log("per-event:", result["per_event"])
        # ---- mixed-pileup batch: 64 events, PU ~ U[50, 250] --------------------
        mixed = synth.batch_events(64, g)
        ctx.batch_upload(mixed)
        ctx.batch_execute(2, graph=True)
        t1 = time.perf_counter()
        ctx.batch_execute(args.steps, graph=True)
        result["mixed_pu50_250_batch64_events_per_s"] = round(64 / ((time.perf_counter() - t1) / args.steps), 2)
        log("mixed batch:", result["mixed_pu50_250_batch64_events_per_s"])
        # ---- cost of a stage boundary: launches vs a persistent kernel ---------
        result["stage_boundary_probe"] = sync_probe()
        log("stage boundary probe:", result["stage_boundary_probe"])
        # ---- served path: Poisson arrivals, then saturation ---------------------
        result["served"] = served(g, pool4)
        result["served_pu300_stress"] = served_stress(g, pool5)
        log("served stress:", result["served_pu300_stress"])
        # what the served path moves per event crosses this link both ways
        result["host_link"] = link_probe()
        log("host link:", result["host_link"])
        # ---- physics: truth-matched rates of the candidates --------------------
        result["physics"] = physics(g, events[:16])
        log("physics:", result["physics"])
        result["skip_layer"] = skip_layer(g, events, args.steps)
        log("skip-layer links:", result["skip_layer"])
    ctx.close()

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(args.cpu_events, args.cpu_budget)
        log("cpu baseline:", result["cpu_baseline"])
        result["cpu_baseline_all_cores"] = cpu_baseline_all_cores(args.cpu_budget)
        log("cpu baseline, all cores:", result["cpu_baseline_all_cores"])
    print(json.dumps(result), flush=True)


def sync_probe(iters: int = 200):
    """Microseconds per stage boundary for the chain's grid shape, crossed by
    launches (graph replay, eager) or by grid barriers in one persistent
    cooperative kernel (paper_2407_18231_amd/csrc/sync_probe.hip), run as a
    separate process."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2407_18231_amd", "sync_probe")
    if not os.path.exists(exe):
        return None
    out = subprocess.run([exe, str(iters)], capture_output=True, text=True, timeout=120)
    if out.returncode != 0:
        return {"error": out.stderr.strip()[-200:]}
    return json.loads(out.stdout.strip().splitlines()[-1])


def copy_probe(mb: int):
    """A plain copy kernel of known size: reads and writes mb * 2^20 bytes."""
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {mb} MiB")


def physics(g, events, n_displaced_events: int = 8):
    """Truth-matched efficiency, fake and duplicate rates (Sec. 3: a track is
    found by a candidate with more than 75% of its hits) of the benchmark's
    PU200 events, for the candidate list and for the list after duplicate
    cleaning; and the efficiency vs production radius of displaced tracks
    (400 per event on a PU50 background, r_vertex up to 35 cm; Sec. 3,
    Fig. 3 right), without and with skip-layer links."""
    from paper_2407_18231_amd import lst, metrics, synth
    with lst.Context(max_batch=len(events), tc_clean=True) as c:
        c.load_geometry(g)
        res = c.run_batch(events)
        disp = [synth.gen_event(g, synth.config_pu(50, n_displaced=400), synth.event_seed(8, i))
                for i in range(n_displaced_events)]
        dres = c.run_batch(disp) if disp else []
    with lst.Context(max_batch=max(len(disp), 1), skip_layer=True) as c:
        c.load_geometry(g)
        dres_skip = c.run_batch(disp) if disp else []

    def rv_bins(results):
        bins = []
        for ev, r in zip(disp, results):
            e = metrics.efficiency_vs_rv(ev, r)["bins"]
            if not bins:
                bins = [dict(rv_cm=[b["rv_lo"], b["rv_hi"]], n_sim=0, found=0.0) for b in e]
            for acc_b, b in zip(bins, e):
                acc_b["n_sim"] += b["n_sim"]
                acc_b["found"] += b["efficiency"] * b["n_sim"]
        for b in bins:
            b["efficiency"] = round(b.pop("found") / max(b["n_sim"], 1), 4)
        return bins
    return dict(events=f"{len(events)} PU200-like events of the benchmark batch",
                candidates=_rates(events, res),
                displaced=dict(events=f"{n_displaced_events} events: PU50 + 400 displaced tracks "
                                      f"(pT 1-10 GeV, |eta| < 2, seeds 8000+i)",
                               efficiency_vs_rv=rv_bins(dres),
                               efficiency_vs_rv_skip_layer=rv_bins(dres_skip)))


def _rates(events, res):
    """Mean truth-matched rates over events, for the candidate list and the
    list after duplicate cleaning; efficiency_ot counts a track found only
    by a candidate with outer-tracker objects (pT5, pT3, T5)."""
    from paper_2407_18231_amd import metrics
    keys = ("efficiency", "efficiency_ot", "fake_rate", "duplicate_rate")
    out = {}
    for name, col in (("all", "tc"), ("cleaned", "tcc")):
        acc, n_tc = dict.fromkeys(keys, 0.0), 0
        for ev, r in zip(events, res):
            q = metrics.rates(ev, dict(r, tc=r[col]))
            n_tc += q["n_tc"]
            for k in keys:
                acc[k] += q[k] / len(events)
        out[name] = dict({k: round(v, 4) for k, v in acc.items()},
                         candidates_per_event=round(n_tc / len(events), 1))
    return out


def skip_layer(g, events, steps: int, n_physics: int = 16):
    """Skip-layer links (segments may also bridge one surface): the benchmark
    batch through a context with LST_FLAG_SKIP_LAYER, timed with hipGraph
    replay as the batched path without the flag is (no duplicate cleaning),
    its objects per event, and the truth-matched rates of its first n_physics
    events with cleaning (compare physics.candidates, the same events without
    the flag)."""
    from paper_2407_18231_amd import lst
    with lst.Context(max_batch=len(events), skip_layer=True) as c:
        c.load_geometry(g)
        c.batch_upload(events)
        c.batch_execute(2, graph=True)
        t1 = time.perf_counter()
        c.batch_execute(steps, graph=True)
        dt = (time.perf_counter() - t1) / steps
    with lst.Context(max_batch=n_physics, tc_clean=True, skip_layer=True) as c:
        c.load_geometry(g)
        res = c.run_batch(events[:n_physics])
    objs = {k: round(float(np.mean([len(r[k]) for r in res])), 1) for k in ("ls", "t3", "t5", "pt3", "pt5", "tc")}
    return dict(batch=len(events), events_per_s=round(len(events) / dt, 1), ms_per_step=round(dt * 1e3, 4),
                objects_per_event=objs, candidates=_rates(events[:n_physics], res))


def link_probe():
    """Host link bandwidth (GB/s) between pinned host memory and the device
    as the served path uses it (paper_2407_18231_amd/csrc/link_probe.hip, run
    as a separate process): one 96 MiB copy and the same bytes in 1100 KiB
    pieces, host to device, device to host, and both directions at once."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2407_18231_amd", "link_probe")
    if not os.path.exists(exe):
        return None
    out = subprocess.run([exe, "96", "1100"], capture_output=True, text=True, timeout=120)
    if out.returncode != 0:
        return None
    return json.loads(out.stdout.strip().splitlines()[-1])


_INPUT_KEYS = ("x", "y", "z", "module", "sensor", "pls_par", "pls_cov", "pls_nhits")


def _served_event(args):
    """One event of the served workload: PU ~ U[pu_lo, pu_hi] drawn for it."""
    from paper_2407_18231_amd import synth
    i, pu_lo, pu_hi, cfg_index, noise, fakes = args
    g = synth.make_geometry("pu200")
    rng = np.random.default_rng(synth.event_seed(cfg_index, i) + 700_000)
    pu = float(rng.uniform(pu_lo, pu_hi))
    ev = synth.gen_event(g, synth.config_pu(pu, noise_frac=noise, fake_frac=fakes), synth.event_seed(cfg_index, i))
    return {k: ev[k] for k in _INPUT_KEYS}


def served_events(n, pu_lo=140.0, pu_hi=200.0, cfg_index=4, noise=0.2, fakes=0.02):
    """n distinct events, generated on the host's cores."""
    import multiprocessing as mp
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    args = [(i, pu_lo, pu_hi, cfg_index, noise, fakes) for i in range(n)]
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(_served_event, args, chunksize=8)


def served_run(ctx, pool, rate_hz, n, seed, submitters=4):
    """Poisson arrivals at rate_hz (rate_hz = 0: back to back), each arrival a
    random event of the pool; several submitting threads follow the arrival
    schedule and one thread polls.  Latency = completion - submission,
    measured by the library; events/s = n / (last completion - first
    arrival)."""
    import threading
    from paper_2407_18231_amd import lst
    rng = np.random.default_rng(seed)
    t_arr = np.cumsum(rng.exponential(1.0 / rate_hz, n)) if rate_hz > 0 else np.zeros(n)
    pick = rng.integers(0, len(pool), n)
    ins = [lst.EventIn(ev) for ev in pool]
    tickets = [None] * n
    posted = [threading.Event() for _ in range(n)]
    rejected = [0]
    lat = np.zeros(n)
    batch = np.zeros(n, np.int64)
    t0 = time.perf_counter() + 0.05

    def submit(k):
        for i in range(k, n, submitters):
            while True:
                d = t0 + t_arr[i] - time.perf_counter()
                if d <= 0:
                    break
                if d > 3e-4:
                    time.sleep(d - 2e-4)
            while True:
                try:
                    tickets[i] = ctx.submit_in(ins[pick[i]])
                    break
                except lst.LstError as e:
                    if e.name != "QUEUE_FULL":
                        raise
                    rejected[0] += 1
                    time.sleep(50e-6)
            posted[i].set()

    def drain():
        for i in range(n):
            posted[i].wait()
            o = ctx.poll(tickets[i], -1, fetch=False)
            lat[i] = o["latency_us"]
            batch[i] = o["batch_events"]

    th = [threading.Thread(target=submit, args=(k,)) for k in range(submitters)]
    dr = threading.Thread(target=drain)
    sw = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)        # hand the interpreter between the threads often
    for t in th:
        t.start()
    dr.start()
    for t in th:
        t.join()
    dr.join()
    wall = time.perf_counter() - t0
    sys.setswitchinterval(sw)
    return dict(rate_hz=rate_hz if rate_hz > 0 else "back-to-back", events=n,
                events_per_s=round(n / wall, 1),
                latency_us_p50=round(float(np.percentile(lat, 50)), 1),
                latency_us_p99=round(float(np.percentile(lat, 99)), 1),
                mean_batch=round(float(batch.mean()), 2), queue_full_retries=rejected[0])


def served(g, pool, n_poisson=5000):
    """Served path (continuous batching, two device slots, 64 events per
    micro-batch at most): n_poisson Poisson arrivals at 500 Hz, then offered
    rates up to back-to-back submission to find saturation; events have
    PU ~ U[140, 200] drawn per event (distinct events of the pool, seeds
    4000+i, each arrival a random one of them)."""
    from paper_2407_18231_amd import lst
    out = []
    with lst.Context(max_batch=64, n_slots=2) as c:
        c.load_geometry(g)
        served_run(c, pool[:256], 0, 512, 98)            # warm-up: sizes the slots
        out.append(served_run(c, pool, 500.0, n_poisson, 99))
        log("served:", out[-1])
        for rate in (4000.0, 16000.0, 0.0):
            out.append(served_run(c, pool, rate, 8000, 100 + int(rate)))
            log("served:", out[-1])
    # saturation with four device slots instead of two
    with lst.Context(max_batch=64, n_slots=4) as c:
        c.load_geometry(g)
        served_run(c, pool[:256], 0, 512, 98)
        r = served_run(c, pool, 0.0, 8000, 100)
        r["slots"] = 4
        out.append(r)
        log("served:", out[-1])
    return out


def served_stress(g, pool, n=2048):
    """PU300 stress events (6000 tracks, 40% noise, 3000 seeds with 5% fakes)
    through the serving loop, 32 events per micro-batch at most, submitted
    back to back."""
    from paper_2407_18231_amd import lst
    with lst.Context(max_batch=32, n_slots=2) as c:
        c.load_geometry(g)
        served_run(c, pool[:64], 0, 128, 97)
        r = served_run(c, pool, 0, n, 101)
    r["workload"] = "PU300 stress, 32 per micro-batch"
    return r


if __name__ == "__main__":
    main()
