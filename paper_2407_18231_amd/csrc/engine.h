// engine.h -- device-side data layout of liblst (library-internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <cstring>
#include <vector>

#include "lst_internal.h"

namespace lst {

constexpr uint32_t kInvalid = 0xFFFFFFFFu;
constexpr uint32_t kDiskBit = 0x80000000u;   // md_u: anchor on an endcap module
constexpr uint32_t kUnitMask = 0x7FFFFFFFu;  // md_u: (event, module) unit
constexpr uint32_t kErrBadModule = 1u;
constexpr uint32_t kErrNonFinite = 2u;
constexpr uint32_t kErrOutside = 4u;   // hit outside its module's extent or off its sensor
constexpr int kScanGrid = 2048;   // blocks (and partial sums) of the device-wide scan
constexpr unsigned kMaxGrid = 2048;
constexpr int kEvTabCols = 12;
// survivors a count pass records per unit, so that the fill pass copies them
// instead of walking the candidates again (units with more walk again)
constexpr uint32_t kKeepLs = 8;
// Lists that a walk appends to in no particular order (segments, T3s,
// seed-object pairs) are split into one equal region per block of the walk
// (at most kSubLists): a block counts its appends in LDS and publishes the
// count when it ends, so appends never wait on a global atomic.
constexpr uint32_t kSubLists = kMaxGrid;
// Entries per walk block in those regions beyond an even share of the
// list's capacity: the blocks of a small batch take one tile of 256 owners
// each, and a dense tile holds a few times the average (a PU200 event's
// densest tile of 256 T3s has up to ≈ 530 T5s against an average of 20).
constexpr uint32_t kRegionSlack = 256;       // MD and LS regions
constexpr uint32_t kRegionSlackT3 = 512;
constexpr uint32_t kRegionSlackT5 = 1024;

// blocks of a walk over `units` owners (256 per block, at most kMaxGrid)
inline uint32_t walk_blocks(uint64_t units)
{
    const uint64_t g = (units + 255) / 256;
    return (uint32_t)(g < 1 ? 1 : (g > kMaxGrid ? kMaxGrid : g));
}

// Device copy of the geometry (read-only).
// Device copy of a line-segment class (LsClass), 32 bytes:
//   a = (S, p0, p1, p2), b = (p3, p4, reach, type bits) with reach the
//   largest azimuth difference of the anchors (asin S, plus margin) and
//   barrel -> barrel: p0..p4 = rho_lo, rho_hi, lam_lo, lam_hi, tau;
//   endcap -> endcap: p0, p1 = lo_fac, hi_fac;
//   barrel -> endcap: p0..p3 = cf, zs, zbpl, zbml.
struct LsK {
    float4 a, b;
};

struct DevGeom {
    const uint32_t *mod_kind;   // n_mod
    const uint32_t *mod_surf;   // n_mod
    const float4 *mdc;          // n_mod: (S, G, K, D)
    const uint32_t *edge_begin; // n_mod + 1
    const uint2 *edge;          // (destination module, class)
    const LsK *cls;
    const Surface *surf;        // n_surf
    const float2 *mod_phi;      // n_mod: azimuth centre and half-width (with margin)
    const float4 *mod_ext;      // 2 per module: accepted extent of a hit, sensor positions
    const uint32_t *run_begin;  // n_mod + 1: segment-walk runs of each module's edges
    const uint4 *run;           // (first destination, class | length << 24, azimuth centre, 1 / pitch)
    const float *run_win;       // window of each run (radians; module indices for runs of several modules)
    uint32_t hist_slice;        // hit histogram in LDS: (module, sensor) bins per slice
};

// Counters of one batch in device memory.  n_ev / n_hits / n_pls are written
// by the host before the chain runs; every other count by the chain itself.
struct Totals {
    uint32_t n_ev, n_hits, n_pls;
    uint32_t n_bins, n_md_units, n_bk, n_sorted, n_rows, n_pt_units;
    uint32_t n_md, n_ls, n_t3, n_t5, n_pt3, n_pt5;
    uint32_t n_bk3, n_bk5, n_tcu, n_tc;
    uint32_t n_ptc3, n_ptc5;      // seed-object candidate pairs (or, after a sub-list overflow, the capacity needed)
    uint32_t n_mds;               // MDs in the unordered MD regions (likewise)
    uint32_t n_lss;               // segments in the unordered segment sub-lists (likewise)
    uint32_t n_t3s;               // T3s in the unordered T3 sub-lists (likewise)
    uint32_t n_t5s;               // T5s in the unordered T5 regions (likewise)
    uint32_t n_tccm;              // (MD, candidate) entries of the track-candidate cleaning
    uint32_t err;
    unsigned long long cand[6];  // candidates examined: md, ls, t3, t5, pt3, pt5
};

// Device arena of one slot: inputs, intermediate and output lists of a batch.
// Capacities bound every list; a stage whose total exceeds its capacity writes
// nothing past it and the host re-runs the batch with larger arrays.
struct Batch {
    uint32_t cap_ev, cap_hits, cap_pls, cap_md, cap_ls, cap_t3, cap_t5, cap_pt3, cap_pt5, cap_tc;
    // the walks' unordered sub-lists (one region of cap / blocks per walk block)
    uint32_t cap_mds, cap_lss, cap_t3s, cap_t5s;
    uint32_t cap_ptc3, cap_ptc5;
    // inputs (event-major concatenation)
    float *in_x, *in_y, *in_z;
    uint32_t *in_mod;
    uint8_t *in_sen;
    float *in_par, *in_cov;
    uint8_t *in_nhit;                   // pixel hits of each seed (seed export)
    uint32_t *ev_hit_off, *ev_pls_off;  // cap_ev + 1
    // a1: hits sorted by (event, module, sensor)
    uint32_t *bin_cnt, *bin_off, *hbin, *hrank;
    float4 *hrec;                       // (x, y, z, input index bits) scattered by bin
    float4 *hpos;                       // (x, y, z, r) of each sorted hit
    uint32_t *hin;                      // event-local input index of each sorted hit
    uint32_t *hbin_s;                   // bin of each sorted hit
    // a2: mini-doublets (anchor = hit on the lower sensor)
    uint32_t *md_cnt, *md_hoff;         // per sorted hit (MDs of a lower-sensor hit)
    // MDs in the block regions of an unordered list before placement:
    // (lower hit's sorted position, place in its list, upper hit's sorted position, beta)
    uint4 *mds;
    uint32_t *mds_sub, *mds_soff;
    uint32_t *md_off;                   // per (event, module) unit
    float4 *md_pos;                     // anchor (x, y, z, r)
    float *md_beta;
    uint32_t *md_u, *md_hlo, *md_hup;
    // a3: line segments
    uint32_t *ls_cnt, *ls_off;          // per inner MD
    uint32_t *ls_a, *ls_b;
    uint32_t *ls_keep;                  // kKeepLs outer MDs per inner MD (small batches)
    // large batches: segments in the block sub-lists of an unordered list,
    // (inner MD, outer MD, place in the inner MD's list), before placement
    uint32_t *lss_a, *lss_b, *lss_j, *lss_sub, *lss_soff;
    // a4: T3
    uint32_t *t3_cnt, *t3_off;          // per inner LS
    uint32_t *t3_l1, *t3_l2;
    // T3s in the block sub-lists of an unordered list before placement:
    // (inner LS, outer LS, place in the inner LS's list, anchors, curvature)
    uint32_t *t3s_l1, *t3s_l2, *t3s_j, *t3s_sub, *t3s_soff;
    uint2 *t3s_ac;
    float2 *t3s_ks;
    uint2 *t3_ac;                       // inner and outer MD
    float2 *t3_ks;                      // curvature and its resolution
    // a5: T5
    uint32_t *t5_cnt, *t5_off;          // per inner T3
    uint32_t *t5_u, *t5_w;
    float2 *t5_ks;                      // curvature through (A, C, E) and its resolution
    // T5s in the block regions of an unordered list before placement:
    // (inner T3, outer T3, place in the inner T3's list, curvature)
    uint32_t *t5s_u, *t5s_w, *t5s_j, *t5s_sub, *t5s_soff;
    float2 *t5s_ks;
    // a6: seed lookup buckets of T3s / T5s by (event, surface, azimuth bin,
    // resolution class, curvature bin); the last bucket of a row holds the
    // objects with a wide curvature resolution
    uint32_t *bk3_cnt, *bk3_off, *bk3_id, *bk3_rank;
    uint32_t *bk5_cnt, *bk5_off, *bk5_id, *bk5_rank;
    float4 *bk3_ks, *bk5_ks;            // (curvature, resolution, inner-anchor azimuth, object index bits)
    // a7: road of each (seed, surface) unit: x = first azimuth bin | bin count
    // << 16; y, z = curvature bin ranges of the resolution classes (k0 | k1 << 8
    // per class, class 2 in z), valid << 31 in z
    uint4 *road;
    float2 *road_phi;                   // azimuth window of the road: (start in [0, 2 pi), width)
    // seed-object candidate pairs (unordered) and, per pair, its rank among
    // the accepted pairs of its seed (kInvalid: rejected); accepted pairs
    // per seed and their offsets; the pT3 / pT5 lists (seed, object) before
    // (tp, to) and after (p, o) the per-seed order by object
    uint32_t *ptc3_p, *ptc3_o, *ptc3_rank;
    uint32_t *ptc5_p, *ptc5_o, *ptc5_rank;
    uint32_t *ptc3_sub, *ptc5_sub;      // appends per block region
    uint32_t *ptc3_soff, *ptc5_soff;    // dense offsets of the regions (kSubLists + 1)
    uint32_t *pt3_cnt, *pt3_off, *pt5_cnt, *pt5_off;
    uint32_t *pt3_tp, *pt3_to, *pt5_tp, *pt5_to;
    uint32_t *pt3_p, *pt3_o;
    uint32_t *pt5_p, *pt5_o;
    // a8: track candidates over [pT3 | T5 | pLS]
    uint8_t *pls_used5, *pls_used3, *t5_used;
    uint32_t *pls_ev;                   // event of each seed
    double *pls_seed;                   // derived binary64 quantities of each seed (10 words)
    uint32_t *tc_cnt, *tc_off, *tc_type, *tc_idx;
    // duplicate cleaning of the track candidates (pT5 list, then the kept
    // [pT3 | T5 | pLS] entries): MD set (5 per candidate, 3 or 5 used),
    // rank quality, each candidate's slot in the list of every one of its
    // MDs, the candidates of each MD (offsets by MD), keep flags
    uint32_t *tcc_md, *tcc_nm, *tcc_rank, *md_tcc_cnt, *md_tcc_off, *md_tcc;
    double *tcc_q;
    uint8_t *tcc_keep;
    uint32_t *ev_tab;                   // (cap_ev + 1) x kEvTabCols
    uint32_t *ev_err;                   // input error bits of each event (kErr*)
};

// Launches kernels on one stream; optionally brackets each launch with HIP
// events to time it.
struct Launcher {
    hipStream_t stream = nullptr;       // the slot's stream
    hipStream_t side = nullptr;         // second stream for branches of the chain that run alongside
    hipStream_t cur = nullptr;          // stream the next launches go to
    uint32_t *part = nullptr;           // scan partials of each stream, kScanGrid entries
    uint32_t *part_side = nullptr;
    hipEvent_t ev_fork[2] = {nullptr, nullptr}, ev_join[2] = {nullptr, nullptr};
    bool timing = false;
    const char *only = nullptr;         // with timing: time only the launches of this name (nullptr: all)
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int stage = 0;                      // stage of the chain the next launches belong to (LST_STAGE_*)
    bool range_open = false;            // a tracing range for the stage being enqueued is open
    struct Rec {
        const char *name;
        int stage;
        hipEvent_t e0, e1;
    };
    std::vector<Rec> recs;
    hipError_t err = hipSuccess;

    hipEvent_t next_event()
    {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }

    // the side stream starts after what the slot's stream has queued so far
    void fork(int k)
    {
        if (!side) return;
        hipError_t e = hipEventRecord(ev_fork[k], stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, ev_fork[k], 0);
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
    // a point on the side stream (after what it has queued so far) ...
    void mark(int k)
    {
        if (!side) return;
        hipError_t e = hipEventRecord(ev_join[k], side);
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
    // ... that the slot's stream waits for from here on
    void wait(int k)
    {
        if (!side) return;
        hipError_t e = hipStreamWaitEvent(stream, ev_join[k], 0);
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
    void on_side(bool s) { cur = (s && side) ? side : stream; }
    // the stage the next launches belong to; a host-side tracing range
    // (rocprofv3 --marker-trace) brackets the enqueueing of each stage
    void set_stage(int st);
    void end_stages();

    template <typename... KArgs, typename... Args>
    void launch(const char *name, void (*kernel)(KArgs...), dim3 grid, dim3 block, Args... args)
    {
        launch_lds(name, kernel, grid, block, 0u, args...);
    }

    // with dynamic LDS of lds bytes per block
    template <typename... KArgs, typename... Args>
    void launch_lds(const char *name, void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t lds, Args... args)
    {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const hipStream_t st = cur ? cur : stream;
        const bool timed = timing && (only == nullptr || std::strcmp(only, name) == 0);
        if (timed) {
            e0 = next_event();
            e1 = next_event();
            if (e0) (void)hipEventRecord(e0, st);
        }
        kernel<<<grid, block, lds, st>>>(args...);
        hipError_t le = hipGetLastError();
        if (le != hipSuccess && err == hipSuccess) err = le;
        if (timed && e1) {
            (void)hipEventRecord(e1, st);
            recs.push_back({name, stage, e0, e1});
        }
    }

    void scan(const uint32_t *in, uint32_t *out, const uint32_t *n_ptr, uint32_t cap, uint32_t *total,
              const char *name);
    // scan() whose first pass also turns a walk's sub-list sizes into region
    // offsets (soff[0..nsub], need: the capacity the sub-lists needed)
    void scan_sub(const uint32_t *in, uint32_t *out, const uint32_t *n_ptr, uint32_t cap, uint32_t *total,
                  const char *name, const uint32_t *sub, uint32_t *soff, uint32_t cap_total, uint32_t nsub,
                  uint32_t *need);
};

void launch_setup(Launcher &L, const Batch &b, Totals *t, const Consts &c);

// Object lists of a one-event batch written as the pairs of lst_event_out,
// into buffers the caller owns (device memory).
struct EventOut {
    uint32_t *md, *ls, *t3, *t5, *pt3, *pt5, *tc;
    float *t3_kappa;         // may be null
};
// One event staged by kernel arguments alone: n_ev = 1 and the event's hit
// and seed offsets written on the device (no host copy).
void launch_event_init(Launcher &L, const Batch &b, Totals *t, uint32_t n_hits, uint32_t n_pls);

// Bytes of one served event's host block and the offsets of its parts
// (x, y, z, module, sensor, seed parameters, seed covariance, seed pixel
// hits), every part aligned to 16 bytes; k_unpack reads the same layout.
struct BlockLayout {
    size_t off[8];
    size_t bytes;
};
inline BlockLayout served_block_layout(uint32_t n_hits, uint32_t n_pls)
{
    auto pad = [](size_t v) { return (v + 15) & ~(size_t)15; };
    BlockLayout l;
    const size_t sz[8] = {4ull * n_hits, 4ull * n_hits, 4ull * n_hits, 4ull * n_hits, n_hits, 20ull * n_pls,
                          60ull * n_pls, n_pls};
    size_t at = 0;
    for (int i = 0; i < 8; i++) {
        l.off[i] = at;
        at += pad(sz[i]);
    }
    l.bytes = at;
    return l;
}
void launch_unpack(Launcher &L, const Batch &b, const Totals *t, const char *raw, const unsigned long long *raw_off);
// the output image of the staged batch (event table, cleaning and seed
// counts, then every event's lists in the layout of lst_event_out) at img,
// head words of table and counts first; nothing is written at or past cap
// words
void launch_pack(Launcher &L, const Batch &b, const Totals *t, uint32_t *img, uint32_t n_ev, uint64_t head,
                 uint64_t cap, bool clean, bool triplets, uint64_t n_items);
void launch_event_out(Launcher &L, const Batch &b, const Totals *t, const EventOut &o, uint64_t n_items);
void enqueue_chain(Launcher &L, const Batch &b, Totals *t, const DevGeom &g, const Consts &c, int stats);

}  // namespace lst
