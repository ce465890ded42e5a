/*
 * lst.h -- C ABI of the MI355X Line Segment Tracking object-building engine.
 *
 * The engine takes the hits of a double-sensor outer tracker plus inner-tracker
 * track seeds ("pixel line segments", pLS) and returns the objects of the Line
 * Segment Tracking chain (Sec. 1 of the paper): mini-doublets (MD, one hit on
 * each sensor of a module), line segments (LS, two MDs on connected modules,
 * linked over a precomputed module connection map), T3 (two LSs sharing an MD),
 * T5 (two T3s sharing an MD), pT3 / pT5 (a pLS linked to a T3 / T5) and the
 * track candidates (TC): pT5s, pT3s, T5s and unlinked pLSs (Sec. 1, list of
 * propagated objects).
 *
 * Conventions
 *   - Every function returns lst_status: 0 = OK, 1 = PENDING, < 0 = error.
 *     No C++ exception crosses this interface.
 *   - After a device (HIP) error a context is failed for good: every later
 *     call on it returns LST_ERR_DEVICE; destroy it.
 *   - Units: cm, GeV, T.  Azimuth in radians.  Hit coordinates are IEEE
 *     binary32.  Geometry is binary64.
 *   - Object lists are in canonical order -- MDs by (module, lower hit, upper
 *     hit), every other list lexicographic in its constituent indices -- and
 *     every index is local to its event: hit indices refer to the
 *     caller's input order, MD/LS/T3/T5/pLS indices to the lists of the same
 *     output.  A result is therefore identical whether the event ran alone, in
 *     a batch or in the served mix.
 *   - lst_run_event / lst_run_batch / lst_batch_* are serialised per context
 *     (do not call them concurrently on one context); lst_submit / lst_poll
 *     are thread-safe.
 */
#ifndef LST_H
#define LST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lst_status;
#define LST_OK 0
#define LST_PENDING 1
#define LST_ERR_INVALID_ARG -1
#define LST_ERR_DEVICE -2
#define LST_ERR_NO_GEOMETRY -3
#define LST_ERR_BAD_GEOMETRY -4
#define LST_ERR_BAD_MODULE -5
#define LST_ERR_NONFINITE -6
#define LST_ERR_OOM -7
#define LST_ERR_TOO_LARGE -8
#define LST_ERR_QUEUE_FULL -9
#define LST_ERR_UNKNOWN_TICKET -10
#define LST_ERR_HIT_OUTSIDE -11   /* a hit breaks the input contract of lst_event_in */

typedef struct lst_ctx lst_ctx;

/* Engine parameters.  The window constants derive from a prompt helix with
 * curvature up to kappa_max = 0.299792458e-2 * B / pt_min (the pT threshold
 * that tunes the hit-pair search windows, Sec. 1) and a vertex within +/- L
 * along the beam, widened by n_sigma times the hit resolutions. */
typedef struct {
    int32_t device;          /* HIP device ordinal */
    double B;                /* field along +z [T] (default 3.8) */
    double pt_min;           /* pT threshold [GeV] (default 0.8) */
    double L;                /* luminous-region half length [cm] (default 15) */
    double sig_rphi;         /* hit resolution along r-phi [cm] (default 30e-4) */
    double sig_c;            /* z (barrel) / r (endcap) resolution [cm] (default 0.1) */
    double n_sigma;          /* window width in resolutions (default 3) */
    uint32_t flags;          /* LST_FLAG_* (default LST_FLAG_BEND) */
    uint32_t max_batch;      /* largest number of events per launch (default 64) */
    uint32_t n_slots;        /* served path: device arenas / streams working in parallel (default 2) */
    uint32_t queue_depth;    /* served path: most events waiting or in flight (default 1024) */
    uint64_t mem_budget;     /* device bytes the served path may hold (0 = 32 GiB) */
    /* Seed-lookup bucket granularity: azimuth bins per (event, surface) row
     * (0 = 64, else 4..4096) and curvature bins per resolution class (0 = 16,
     * else 2..128).  The object lists do not depend on them, only the speed;
     * paper_2407_18231_amd.tune picks them by measurement. */
    uint32_t n_phi_bins;
    uint32_t n_kappa_bins;
    /* Segment walk: runs of a module's edges (edges to consecutive modules of
     * one class) taken per group (0 = 6, else 4, 6 or 8)
     * and the minimum number of waves per SIMD its registers allow (0 = the
     * compiler's choice, else 6 or 8).  Speed only; picked by the tuner. */
    uint32_t ls_group;
    uint32_t ls_waves;
    /* hipStream_t the per-event and batched paths (lst_run_event,
     * lst_run_batch, lst_batch_*) enqueue their work on; NULL: a stream of the
     * library's own.  Borrowed: it must outlive the context and is never
     * destroyed by the library; the calls still return only once their work
     * on it is complete.  The served path always uses its own streams. */
    void *stream;
} lst_params;

#define LST_FLAG_BEND 1u     /* line segments: MD bend consistent with the segment's (barrel pairs) */
/* lst_run_event / lst_run_batch fill lst_event_out.stage_ns: the chain then
 * runs on one stream with a HIP event pair around every launch (slower; for
 * diagnosis).  Without it stage_ns is all zero. */
#define LST_FLAG_STAGE_TIMES 2u
/* Duplicate cleaning of the track candidates: lst_event_out.tcc lists the
 * candidates that survive it.  The paper names the candidate types (Sec. 1)
 * and measures duplicate rates (Sec. 3) but does not describe the removal;
 * this library's rule: a candidate with outer-tracker MDs (pT5 and T5: 5,
 * pT3: 3) is removed when another one that ranks higher shares more than
 * half of the smaller of the two MD sets.  Rank: type (pT5, pT3, T5), then
 * the smaller curvature disagreement (seed against object for pT5 / pT3,
 * inner against outer T3 for a T5, relative to the summed resolutions),
 * then the smaller index in its own list.  Seed-only candidates are kept. */
#define LST_FLAG_TC_CLEAN 4u
/* Seed export (lst_event_out.seeds): besides the quads, the triplets (the
 * "quads + triplets" configuration of the recovery iteration, Sec. 2). */
#define LST_FLAG_SEEDS_TRIPLETS 8u
/* Skip-layer links: the connection map (Sec. 1: module pairs that charged
 * particles cross in turn) also pairs each module with the modules of the
 * surfaces two steps out -- the next surfaces of its next surfaces -- so a
 * line segment may bridge a surface on which the track left no mini-doublet.
 * Without it a module is paired with the next barrel layer, the first disk of
 * either side (barrel) or the next disk of its side (endcap).  More segments,
 * T3s and T5s, and candidates that the cleaning (LST_FLAG_TC_CLEAN) merges. */
#define LST_FLAG_SKIP_LAYER 16u

/* Stages of the chain (Sec. 1: hits -> MD -> LS -> T3 -> T5; pLS linked into
 * pT3 / pT5; track candidates), the index of each in stage_ns */
#define LST_STAGE_INGEST 0       /* validation and sort of the hits by (module, sensor) */
#define LST_STAGE_MD 1
#define LST_STAGE_LS 2
#define LST_STAGE_T3 3
#define LST_STAGE_T5 4
#define LST_STAGE_SEED_LOOKUP 5  /* seed quantities, roads, object buckets, seed-object candidate walk */
#define LST_STAGE_PT 6           /* seed cuts of the candidate pairs, pT3 / pT5 lists */
#define LST_STAGE_TC 7
#define LST_N_STAGES 8

/* One double-sensor module.  Modules must be listed with consecutive ids
 * 0..n-1 in this array.  Barrel modules are cylinder patches, endcap modules
 * are annulus sectors on planes z = const.  "Lower" is the sensor nearer the
 * interaction point. */
typedef struct {
    uint32_t kind;           /* LST_BARREL or LST_ENDCAP */
    uint32_t layer;          /* barrel layer / disk index, increasing outward from 0 */
    int32_t side;            /* 0 for barrel; +1 / -1 for the endcap at +z / -z */
    uint32_t pad;
    double s_lo, s_hi;       /* sensor radii (barrel) or signed plane z (endcap) */
    double c_min, c_max;     /* z extent (barrel) or r extent (endcap) */
    double phi_min, phi_max; /* azimuth range [phi_min, phi_max), within [0, 2 pi] */
} lst_module_desc;

#define LST_BARREL 0u
#define LST_ENDCAP 1u

/* Input of one event: the hits of the outer tracker and the inner-tracker
 * seeds (Sec. 1: outer-tracker hits are the input, and the objects built from
 * them are linked to inner-tracker tracks).  Host pointers unless flags &
 * LST_DEVICE_PTRS (device pointers, e.g. from torch tensors on the context's
 * device).  Borrowed for the duration of the call (lst_submit copies them
 * before returning).
 *
 * Input contract, checked for every hit at ingest (LST_ERR_HIT_OUTSIDE
 * otherwise; BAD_MODULE for a module id >= n or sensor > 1, NONFINITE for a
 * NaN or infinite coordinate or seed value): the hit lies on its sensor --
 * radius (barrel) or plane z (endcap) within 0.008 cm of that sensor's
 * s_lo / s_hi -- and inside its module's extent widened by 5.5 resolutions:
 * z (barrel) or r (endcap) within [c_min - 5.5 sig_c, c_max + 5.5 sig_c],
 * azimuth within [phi_min - w, phi_max + w] with w = 5.5 sig_rphi over the
 * module's inner radius.  The connection map and the seed roads cover hits up
 * to 6 resolutions out, so every hit that passes the check is searched as
 * widely as a search without the map would. */
typedef struct {
    uint32_t n_hits;
    uint32_t n_pls;
    const float *x, *y, *z;  /* hit positions */
    const uint32_t *module;  /* module id of each hit */
    const uint8_t *sensor;   /* 0 = lower, 1 = upper sensor */
    const float *pls_par;    /* 5 per seed: q/pT [1/GeV], phi0, cot(theta), d0 [cm], z0 [cm] */
    const float *pls_cov;    /* 15 per seed: upper triangle of the 5x5 covariance, row major */
    uint32_t flags;          /* LST_DEVICE_PTRS */
    uint32_t pad;
    /* pixel hits of each seed (3: triplet, >= 4: quad); NULL: every seed is a
     * quad.  Used only to select the seeds the event exports (seeds in
     * lst_event_out). */
    const uint8_t *pls_nhits;
} lst_event_in;

#define LST_DEVICE_PTRS 1u

/* Track-candidate types, in output order */
#define LST_TC_PT5 0u
#define LST_TC_PT3 1u
#define LST_TC_T5 2u
#define LST_TC_PLS 3u

/* Result of one event, owned by the library (free with lst_free_output):
 * the objects of every stage and the track candidates (Sec. 1, list of
 * propagated objects).  Pairs are stored flat: element 2*i and 2*i+1.
 * The lists of all events of one batch (or served micro-batch) lie in one
 * pinned host buffer, copied from the device in one transfer; it is released
 * when the last output pointing into it is freed, which may be after
 * lst_destroy.  Holding one output keeps its batch's buffer. */
typedef struct {
    uint32_t n_md, n_ls, n_t3, n_t5, n_pt3, n_pt5, n_tc;
    uint32_t status;         /* lst_status of this event (served path) */
    uint32_t *md;            /* (hit on lower sensor, hit on upper sensor) */
    uint32_t *ls;            /* (inner MD, outer MD) */
    uint32_t *t3;            /* (inner LS, outer LS); inner LS's outer MD = outer LS's inner MD */
    uint32_t *t5;            /* (inner T3, outer T3); inner T3's outer MD = outer T3's inner MD */
    uint32_t *pt3;           /* (pLS, T3) */
    uint32_t *pt5;           /* (pLS, T5) */
    uint32_t *tc;            /* (type LST_TC_*, index into pt5 / pt3 / t5 / pLS) */
    float *t3_kappa;         /* signed transverse curvature of each T3 [1/cm] */
    double latency_us;       /* served path: completion minus submission */
    uint64_t ticket;
    /* times the chain was re-run with larger object lists because one
     * overflowed (regrow and re-run; 0 when the first run fit) */
    uint32_t n_flag_regrow;
    uint32_t n_stage;        /* LST_N_STAGES */
    /* with LST_FLAG_STAGE_TIMES: device nanoseconds per stage (LST_STAGE_*)
     * of the launch that produced this event -- for a batch, of the whole
     * batch; their sum does not exceed the call's duration */
    uint64_t stage_ns[LST_N_STAGES];
    uint32_t batch_events;   /* events in the launch that produced this output */
    uint32_t n_tcc;          /* with LST_FLAG_TC_CLEAN: candidates kept by the duplicate cleaning */
    uint64_t footprint;      /* served path: predicted device bytes the event was admitted with */
    uint32_t *tcc;           /* (type, index) as in tc, the kept subset in tc order; NULL without the flag */
    /* Seeds exported for a downstream seeded track finder (Sec. 2, Table 1:
     * the recovery iteration seeded by LST pLS quads, or quads and
     * triplets): the seeds that are track candidates on their own (linked to
     * no T3 or T5), in increasing order, those with at least 4 pixel hits,
     * and with LST_FLAG_SEEDS_TRIPLETS also those with 3. */
    uint32_t n_seeds;
    uint32_t *seeds;
} lst_event_out;

void lst_default_params(lst_params *p);

/* Create a context on p->device (p = NULL: defaults).  Errors: INVALID_ARG,
 * DEVICE. */
lst_status lst_create(const lst_params *p, lst_ctx **out);

/* Load the detector: validates the module table, derives per-module and
 * per-module-pair window constants in binary64 (rounded once to binary32),
 * builds the module connection map (Sec. 1: "precomputed connection maps")
 * and the seed-lookup surface table, and uploads them.  m is borrowed for the
 * call.  Errors: INVALID_ARG, BAD_GEOMETRY, OOM, DEVICE. */
lst_status lst_load_geometry(lst_ctx *ctx, const lst_module_desc *m, uint32_t n);

/* Cache of the host-side tables lst_load_geometry builds (window constants,
 * connection map, segment-walk runs, seed-lookup surfaces; ≈ 1 s for 12 800
 * modules): with a directory set, a load reads them from a blob there that
 * was built from exactly the same module table and parameters, and
 * otherwise builds them and writes such a blob (named by a hash of the
 * inputs; the blob holds the inputs and is used only when they match byte
 * for byte).  dir NULL or "": no cache.  A blob that cannot be read or
 * written is ignored.  Errors: INVALID_ARG. */
lst_status lst_set_geometry_cache(lst_ctx *ctx, const char *dir);
/* 1 when the geometry loaded last came from the cache, else 0. */
int32_t lst_geometry_from_cache(const lst_ctx *ctx);

/* The connection map in CSR form: module A connects to dst[begin[A] ..
 * begin[A+1]).  Pointers into library-owned host memory, valid until the next
 * lst_load_geometry or lst_destroy.  Errors: NO_GEOMETRY. */
lst_status lst_get_connection_map(lst_ctx *ctx, const uint32_t **begin,
                                  const uint32_t **dst, uint32_t *n_edges);

/* Host-only variant (no device needed): builds the connection map of a module
 * table with parameters p into newly allocated arrays; release with
 * lst_free_map.  Errors: INVALID_ARG, BAD_GEOMETRY, OOM. */
lst_status lst_build_connection_map(const lst_params *p, const lst_module_desc *m, uint32_t n,
                                    uint32_t **begin, uint32_t **dst, uint32_t *n_edges);
void lst_free_map(uint32_t *begin, uint32_t *dst);

/* Run one event synchronously (the plain per-event path): hits and seeds in,
 * the object lists of every stage and the track candidates out (Sec. 1: the
 * candidates either combine a seed with outer-tracker objects or use the
 * outer tracker alone).  *out is allocated by the library.
 * Errors: NO_GEOMETRY, BAD_MODULE (module id out of range or sensor > 1),
 * NONFINITE (NaN/inf coordinate or seed parameter), HIT_OUTSIDE (a hit
 * breaks the input contract), OOM, TOO_LARGE (event above the device memory
 * budget), DEVICE. */
lst_status lst_run_event(lst_ctx *ctx, const lst_event_in *ev, lst_event_out **out);

/* Run n events in one launch of the chain (the batched path); outs[i] receives
 * event i.  Every object of a stage depends only on objects of its own event
 * (Sec. 1: objects of one kind are built independently, so they can be
 * created concurrently), so a batch is one flat index space and each output
 * equals the event's lst_run_event output.  Same errors as lst_run_event
 * (an input error in any event fails the call); INVALID_ARG if
 * n > max_batch. */
lst_status lst_run_batch(lst_ctx *ctx, const lst_event_in *evs, uint32_t n, lst_event_out **outs);

/* Served path.  lst_submit copies the event and returns a ticket at once;
 * a scheduler admits waiting events into free device slots by their predicted
 * device-memory footprint, forms micro-batches and runs them on parallel
 * streams (the paper's throughput runs keep two streams of events on one GPU,
 * Sec. 3).  lst_poll returns LST_OK and hands over the output once (the ticket
 * is then consumed) or LST_PENDING; timeout_us = 0 does not wait, -1 waits.
 * An input error fails only its own ticket (lst_poll returns the error);
 * the other events of its micro-batch are unaffected.
 * Errors: lst_submit: QUEUE_FULL (queue_depth events waiting or in flight),
 * TOO_LARGE (predicted footprint above mem_budget), INVALID_ARG (device
 * pointers); lst_poll: UNKNOWN_TICKET, DEVICE, the input errors of
 * lst_run_event. */
lst_status lst_submit(lst_ctx *ctx, const lst_event_in *ev, uint64_t *ticket);
lst_status lst_poll(lst_ctx *ctx, uint64_t ticket, int64_t timeout_us, lst_event_out **out);

/* Device-resident benchmarking path: lst_batch_upload copies n events into the
 * plain path's device arena (sizing it); lst_batch_execute runs the whole chain
 * on them `repeats` times (use_graph: replay a captured hipGraph) and returns
 * the device time of all repeats in *ms; with timing on it also accumulates
 * per-kernel durations, read by lst_kernel_times (names, total ms, launches;
 * arrays of length at least *n on input, number written on output);
 * lst_batch_download returns the outputs of the last execute.
 * Errors: as lst_run_batch. */
lst_status lst_batch_upload(lst_ctx *ctx, const lst_event_in *evs, uint32_t n);
lst_status lst_batch_execute(lst_ctx *ctx, uint32_t repeats, int32_t use_graph, int32_t timing,
                             double *ms);
lst_status lst_kernel_times(lst_ctx *ctx, const char **names, double *total_ms,
                            uint32_t *launches, uint32_t *n);
/* Restrict the timing of later lst_batch_execute calls to the launches named
 * name (as reported by lst_kernel_times); NULL or "" times every launch.
 * With a restriction the repeats run back to back (no host wait between
 * them).  Errors: INVALID_ARG. */
lst_status lst_time_only(lst_ctx *ctx, const char *name);
lst_status lst_batch_download(lst_ctx *ctx, lst_event_out **outs);
/* Object totals of the last execute over the whole batch: md, ls, t3, t5,
 * pt3, pt5, tc; candidates examined by the md, ls, t3, t5, pt3 and pt5
 * stages (for pt3 / pt5: bucket entries walked by the seed lookup); and the
 * pt3 / pt5 candidates that reach the full seed cuts (15 values). */
lst_status lst_batch_counts(lst_ctx *ctx, uint64_t counts[15]);

/* Output of lst_run_event_noalloc: the lists of lst_event_out (same pairs,
 * same canonical order) written into device buffers the caller owns, each
 * holding 2 x cap_* uint32 (t3_kappa: cap_t3 floats, or NULL).  The library
 * sets the n_* fields. */
typedef struct {
    uint32_t *md, *ls, *t3, *t5, *pt3, *pt5, *tc;
    float *t3_kappa;
    uint32_t cap_md, cap_ls, cap_t3, cap_t5, cap_pt3, cap_pt5, cap_tc;
    uint32_t n_md, n_ls, n_t3, n_t5, n_pt3, n_pt5, n_tc;
} lst_event_dev_out;

#define LST_NOALLOC_MAX_HITS 131072u
#define LST_NOALLOC_MAX_PLS 8192u
#define LST_NOALLOC_WORKSPACE_BYTES (128ull << 20)

/* lst_run_event for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, hosts that forbid allocation): the
 * call makes no device or pinned-host allocation.  Every intermediate buffer
 * lives in a fixed workspace of LST_NOALLOC_WORKSPACE_BYTES that the library
 * holds on each GPU it runs on (a static device array, kept until the process
 * ends); inputs must be device pointers (LST_DEVICE_PTRS) of at most
 * LST_NOALLOC_MAX_HITS hits and LST_NOALLOC_MAX_PLS seeds, and the outputs go
 * to the caller's device buffers in *out.  The work runs on `stream`
 * (hipStream_t; NULL: the null stream) and is complete when the call returns.
 * Calls on one GPU share its workspace, which keeps the last call's contents:
 * the library serialises them within a process (concurrent callers wait).
 * Errors: as lst_run_event; INVALID_ARG (host pointers, a null output buffer
 * that the event needs); TOO_LARGE (inputs above the limits, object lists that
 * do not fit the workspace, or an output buffer below the event's count -- the
 * n_* fields then give the sizes needed; nothing is written). */
lst_status lst_run_event_noalloc(lst_ctx *ctx, const lst_event_in *ev, lst_event_dev_out *out, void *stream);

/* Frees an output of lst_run_event, lst_run_batch, lst_batch_download or
 * lst_poll (NULL: nothing); thread-safe, also after lst_destroy. */
void lst_free_output(lst_event_out *out);

/* Drains in-flight served events, then frees everything. */
void lst_destroy(lst_ctx *ctx);

const char *lst_status_str(lst_status s);
const char *lst_last_error(const lst_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LST_H */
