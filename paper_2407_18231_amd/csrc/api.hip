// api.hip -- the C ABI of liblst: contexts, device arenas, the per-event,
// batched and device-resident paths, output assembly, and the served path
// (submit / poll with a scheduler thread and parallel device slots).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "engine.h"
#include "lst.h"

namespace lst {
namespace {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Caps {
    uint32_t ev = 0, hits = 0, pls = 0, md = 0, ls = 0, t3 = 0, t5 = 0, pt3 = 0, pt5 = 0, ptc3 = 0, ptc5 = 0;
};

uint32_t clamp32(uint64_t v) { return v > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)v; }

// Initial capacities from the batch size; measured ratios at PU200-PU300 are
// MD ~0.25, LS ~1.5-2.5, T3 ~0.6-1 per hit, pT3 ~3 and pT5 ~1 per seed.
Caps plan_caps(uint32_t n_ev, uint64_t hits, uint64_t pls)
{
    Caps c;
    c.ev = n_ev;
    c.hits = clamp32(hits);
    c.pls = clamp32(pls);
    c.md = clamp32(hits / 2 + 1024);
    c.ls = clamp32(3 * hits + 4096);
    c.t3 = clamp32(2 * hits + 4096);
    c.t5 = clamp32(hits / 2 + 4096);
    c.pt3 = clamp32(8 * pls + 4096);
    c.pt5 = clamp32(4 * pls + 4096);
    c.ptc3 = clamp32(64 * pls + 4096);
    c.ptc5 = clamp32(16 * pls + 4096);
    return c;
}

// Capacities of the walks' sub-lists: an even share of the list's capacity
// per walk block plus the slack of that walk (never smaller than before).
void plan_sublists(Batch &b)
{
    auto at_least = [](uint32_t &cap, uint64_t want) { cap = std::max(cap, clamp32(want)); };
    at_least(b.cap_mds, (uint64_t)b.cap_md + (uint64_t)walk_blocks(b.cap_hits) * kRegionSlack);
    at_least(b.cap_lss, (uint64_t)b.cap_ls + (uint64_t)walk_blocks(b.cap_md) * kRegionSlack);
    at_least(b.cap_t3s, (uint64_t)b.cap_t3 + (uint64_t)walk_blocks(b.cap_ls) * kRegionSlackT3);
    at_least(b.cap_t5s, (uint64_t)b.cap_t5 + (uint64_t)walk_blocks(b.cap_t3) * kRegionSlackT5);
}

// After a run: a quarter more room for every list (or sub-list) whose
// count (or largest region, times the regions) exceeded its capacity.
// True when anything grew (the batch must run again).
bool grow_caps(Batch &b, const Totals &t)
{
    auto grow = [](uint32_t need, uint32_t &cap) {
        if (need <= cap) return false;
        cap = clamp32((uint64_t)need + need / 4 + 1024);
        return true;
    };
    bool g = false;
    g |= grow(t.n_md, b.cap_md);
    g |= grow(t.n_ls, b.cap_ls);
    g |= grow(t.n_t3, b.cap_t3);
    g |= grow(t.n_t5, b.cap_t5);
    g |= grow(t.n_mds, b.cap_mds);
    g |= grow(t.n_lss, b.cap_lss);
    g |= grow(t.n_t3s, b.cap_t3s);
    g |= grow(t.n_t5s, b.cap_t5s);
    g |= grow(t.n_pt3, b.cap_pt3);
    g |= grow(t.n_pt5, b.cap_pt5);
    g |= grow(t.n_ptc3, b.cap_ptc3);
    g |= grow(t.n_ptc5, b.cap_ptc5);
    if (g) plan_sublists(b);
    return g;
}

// Sub-allocates the device arena; with base == nullptr only sums the sizes.
struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t n)
    {
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += align_up(n * sizeof(T) + 16);
        return p;
    }
};

void carve_inputs(Carver &cv, Batch &b)
{
    b.in_x = cv.take<float>(b.cap_hits);
    b.in_y = cv.take<float>(b.cap_hits);
    b.in_z = cv.take<float>(b.cap_hits);
    b.in_mod = cv.take<uint32_t>(b.cap_hits);
    b.in_sen = cv.take<uint8_t>(b.cap_hits);
    b.in_par = cv.take<float>(5ull * b.cap_pls);
    b.in_cov = cv.take<float>(15ull * b.cap_pls);
    b.in_nhit = cv.take<uint8_t>(b.cap_pls);
    b.ev_hit_off = cv.take<uint32_t>(b.cap_ev + 1);
    b.ev_pls_off = cv.take<uint32_t>(b.cap_ev + 1);
}

void carve_work(Carver &cv, Batch &b, uint32_t n_mod, uint32_t n_surf, uint32_t nphi, uint32_t nkb)
{
    const size_t bins = (size_t)b.cap_ev * 2 * n_mod;
    const size_t units = (size_t)b.cap_ev * n_mod;
    const size_t rows = (size_t)b.cap_ev * n_surf * nphi;
    const size_t bk = rows * (3 * nkb + 1);
    const size_t pt_units = (size_t)b.cap_pls * n_surf;
    const size_t tcu = (size_t)b.cap_pt3 + b.cap_t5 + b.cap_pls;
    b.bin_cnt = cv.take<uint32_t>(bins + 1);
    b.bin_off = cv.take<uint32_t>(bins + 1);
    b.hbin = cv.take<uint32_t>(b.cap_hits);
    b.hrank = cv.take<uint32_t>(b.cap_hits);
    b.hrec = cv.take<float4>(b.cap_hits);
    b.hpos = cv.take<float4>(b.cap_hits);
    b.hin = cv.take<uint32_t>(b.cap_hits);
    b.hbin_s = cv.take<uint32_t>(b.cap_hits);
    b.md_cnt = cv.take<uint32_t>((size_t)b.cap_hits + 1);
    b.md_hoff = cv.take<uint32_t>((size_t)b.cap_hits + 1);
    b.mds = cv.take<uint4>(b.cap_mds);
    b.mds_sub = cv.take<uint32_t>(kSubLists);
    b.mds_soff = cv.take<uint32_t>(kSubLists + 1);
    b.md_off = cv.take<uint32_t>(units + 1);
    b.md_pos = cv.take<float4>(b.cap_md);
    b.md_beta = cv.take<float>(b.cap_md);
    b.md_u = cv.take<uint32_t>(b.cap_md);
    b.md_hlo = cv.take<uint32_t>(b.cap_md);
    b.md_hup = cv.take<uint32_t>(b.cap_md);
    b.ls_cnt = cv.take<uint32_t>((size_t)b.cap_md + 1);
    b.ls_off = cv.take<uint32_t>((size_t)b.cap_md + 1);
    b.ls_a = cv.take<uint32_t>(b.cap_ls);
    b.ls_b = cv.take<uint32_t>(b.cap_ls);
    b.ls_keep = cv.take<uint32_t>((size_t)b.cap_md * kKeepLs);
    b.lss_a = cv.take<uint32_t>(b.cap_lss);
    b.lss_b = cv.take<uint32_t>(b.cap_lss);
    b.lss_j = cv.take<uint32_t>(b.cap_lss);
    b.lss_sub = cv.take<uint32_t>(kSubLists);
    b.lss_soff = cv.take<uint32_t>(kSubLists + 1);
    b.t3_cnt = cv.take<uint32_t>((size_t)b.cap_ls + 1);
    b.t3_off = cv.take<uint32_t>((size_t)b.cap_ls + 1);
    b.t3_l1 = cv.take<uint32_t>(b.cap_t3);
    b.t3_l2 = cv.take<uint32_t>(b.cap_t3);
    b.t3s_l1 = cv.take<uint32_t>(b.cap_t3s);
    b.t3s_l2 = cv.take<uint32_t>(b.cap_t3s);
    b.t3s_j = cv.take<uint32_t>(b.cap_t3s);
    b.t3s_ac = cv.take<uint2>(b.cap_t3s);
    b.t3s_ks = cv.take<float2>(b.cap_t3s);
    b.t3s_sub = cv.take<uint32_t>(kSubLists);
    b.t3s_soff = cv.take<uint32_t>(kSubLists + 1);
    b.t3_ac = cv.take<uint2>(b.cap_t3);
    b.t3_ks = cv.take<float2>(b.cap_t3);
    b.t5_cnt = cv.take<uint32_t>((size_t)b.cap_t3 + 1);
    b.t5_off = cv.take<uint32_t>((size_t)b.cap_t3 + 1);
    b.t5_u = cv.take<uint32_t>(b.cap_t5);
    b.t5_w = cv.take<uint32_t>(b.cap_t5);
    b.t5_ks = cv.take<float2>(b.cap_t5);
    b.t5s_u = cv.take<uint32_t>(b.cap_t5s);
    b.t5s_w = cv.take<uint32_t>(b.cap_t5s);
    b.t5s_j = cv.take<uint32_t>(b.cap_t5s);
    b.t5s_ks = cv.take<float2>(b.cap_t5s);
    b.t5s_sub = cv.take<uint32_t>(kSubLists);
    b.t5s_soff = cv.take<uint32_t>(kSubLists + 1);
    b.bk3_cnt = cv.take<uint32_t>(bk + 1);
    b.bk3_off = cv.take<uint32_t>(bk + 1);
    b.bk3_id = cv.take<uint32_t>(b.cap_t3);
    b.bk3_rank = cv.take<uint32_t>(b.cap_t3);
    b.bk3_ks = cv.take<float4>(b.cap_t3);
    b.bk5_cnt = cv.take<uint32_t>(bk + 1);
    b.bk5_off = cv.take<uint32_t>(bk + 1);
    b.bk5_id = cv.take<uint32_t>(b.cap_t5);
    b.bk5_rank = cv.take<uint32_t>(b.cap_t5);
    b.bk5_ks = cv.take<float4>(b.cap_t5);
    b.road = cv.take<uint4>(pt_units);
    b.road_phi = cv.take<float2>(pt_units);
    b.ptc3_p = cv.take<uint32_t>(b.cap_ptc3);
    b.ptc3_o = cv.take<uint32_t>(b.cap_ptc3);
    b.ptc3_rank = cv.take<uint32_t>(b.cap_ptc3);
    b.ptc5_p = cv.take<uint32_t>(b.cap_ptc5);
    b.ptc5_o = cv.take<uint32_t>(b.cap_ptc5);
    b.ptc5_rank = cv.take<uint32_t>(b.cap_ptc5);
    b.ptc3_sub = cv.take<uint32_t>(kSubLists);
    b.ptc5_sub = cv.take<uint32_t>(kSubLists);
    b.ptc3_soff = cv.take<uint32_t>(kSubLists + 1);
    b.ptc5_soff = cv.take<uint32_t>(kSubLists + 1);
    b.pt3_cnt = cv.take<uint32_t>((size_t)b.cap_pls + 1);
    b.pt3_off = cv.take<uint32_t>((size_t)b.cap_pls + 1);
    b.pt5_cnt = cv.take<uint32_t>((size_t)b.cap_pls + 1);
    b.pt5_off = cv.take<uint32_t>((size_t)b.cap_pls + 1);
    b.pt3_tp = cv.take<uint32_t>(b.cap_pt3);
    b.pt3_to = cv.take<uint32_t>(b.cap_pt3);
    b.pt5_tp = cv.take<uint32_t>(b.cap_pt5);
    b.pt5_to = cv.take<uint32_t>(b.cap_pt5);
    b.pt3_p = cv.take<uint32_t>(b.cap_pt3);
    b.pt3_o = cv.take<uint32_t>(b.cap_pt3);
    b.pt5_p = cv.take<uint32_t>(b.cap_pt5);
    b.pt5_o = cv.take<uint32_t>(b.cap_pt5);
    b.pls_ev = cv.take<uint32_t>(b.cap_pls);
    b.pls_seed = cv.take<double>(10ull * b.cap_pls);
    b.pls_used5 = cv.take<uint8_t>(b.cap_pls);
    b.pls_used3 = cv.take<uint8_t>(b.cap_pls);
    b.t5_used = cv.take<uint8_t>(b.cap_t5);
    b.tc_cnt = cv.take<uint32_t>(tcu + 1);
    b.tc_off = cv.take<uint32_t>(tcu + 1);
    b.tc_type = cv.take<uint32_t>(tcu);
    b.tc_idx = cv.take<uint32_t>(tcu);
    const size_t tcc = (size_t)b.cap_pt5 + tcu;
    b.tcc_md = cv.take<uint32_t>(5 * tcc);
    b.tcc_nm = cv.take<uint32_t>(tcc);
    b.tcc_rank = cv.take<uint32_t>(5 * tcc);
    b.md_tcc_cnt = cv.take<uint32_t>((size_t)b.cap_md + 1);
    b.md_tcc_off = cv.take<uint32_t>((size_t)b.cap_md + 1);
    b.md_tcc = cv.take<uint32_t>(5 * tcc);
    b.tcc_q = cv.take<double>(tcc);
    b.tcc_keep = cv.take<uint8_t>(tcc);
    b.ev_tab = cv.take<uint32_t>(((size_t)b.cap_ev + 1) * kEvTabCols);
    b.ev_err = cv.take<uint32_t>((size_t)b.cap_ev + 1);
}

}  // namespace

// One device slot: a stream, the arenas of one batch and its captured graph.
struct Slot {
    int device = 0;
    hipStream_t stream = nullptr;
    void *in_arena = nullptr, *work_arena = nullptr;
    size_t in_bytes = 0, work_bytes = 0;
    Batch b{};
    Totals *d_tot = nullptr, *h_tot = nullptr;
    uint32_t *d_part = nullptr;          // scan partials of the stream and of the side stream
    hipStream_t side = nullptr;
    char *h_stage = nullptr;
    size_t stage_bytes = 0;
    size_t img_words = 0;               // largest output image the list capacities allow
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_valid = false;
    Launcher L;
    // host view of the staged batch
    uint32_t n_ev = 0;
    std::vector<uint32_t> hit_off, pls_off;
    hipEvent_t done = nullptr;
    bool own_stream = true;          // false: the caller's stream (lst_params.stream), not destroyed here
    // served path: the events' host blocks as copied to the device, and the
    // offset of each block (device and pinned host copies)
    char *raw = nullptr;
    size_t raw_cap = 0;
    unsigned long long *d_rawoff = nullptr, *h_rawoff = nullptr;
    uint32_t rawoff_cap = 0;
    uint32_t n_regrow = 0;           // re-runs of the last batch after an overflow
    uint64_t stage_ns[LST_N_STAGES] = {};   // stage times of the last batch (stage timing only)
    std::vector<uint64_t> tickets;   // served path
    std::vector<std::chrono::steady_clock::time_point> t_submit;
};

}  // namespace lst

// Workspace of lst_run_event_noalloc: every device buffer that call needs
// beyond its inputs and outputs (counters, scan partials, sorted hits, the
// object lists of every stage) is carved from this array, so the call makes
// no device allocation.  Each GPU the library runs on holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (noalloc_ws).
namespace {
constexpr size_t kScratchBytes = LST_NOALLOC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_ws_mu;                          // guards g_ws
void *g_ws[kMaxDevices] = {};                // address of scratch on each device
std::mutex g_ws_run_mu[kMaxDevices];         // serialises the calls on one device
}  // namespace
static __device__ __align__(256) char scratch[kScratchBytes];

// Pinned host blocks that hold submitted events until their micro-batch is
// copied to the device; freed blocks are kept per size class and reused.
struct PinnedPool {
    std::mutex mu;
    std::map<size_t, std::vector<char *>> free_blocks;
    std::vector<char *> all;
    unsigned flags = hipHostMallocDefault;   // hipHostMalloc flags of new blocks
    static size_t size_class(size_t bytes)
    {
        size_t c = 64 << 10;
        while (c < bytes) c += c / 2;   // classes 64 KiB x 1.5^k
        return c;
    }
    // the smallest free block of this size class or up to four classes
    // larger, else a new block of the class of bytes + headroom
    char *get(size_t bytes, size_t &cls, size_t headroom = 0)
    {
        cls = size_class(bytes);
        {
            std::lock_guard<std::mutex> g(mu);
            const size_t limit = 5 * cls + 1;
            for (auto it = free_blocks.lower_bound(cls); it != free_blocks.end() && it->first <= limit; ++it) {
                if (it->second.empty()) continue;
                char *p = it->second.back();
                it->second.pop_back();
                cls = it->first;
                return p;
            }
        }
        char *p = nullptr;
        cls = size_class(bytes + headroom);
        if (hipHostMalloc((void **)&p, cls, flags) != hipSuccess) return nullptr;
        std::lock_guard<std::mutex> g(mu);
        all.push_back(p);
        return p;
    }
    void put(char *p, size_t cls)
    {
        if (!p) return;
        std::lock_guard<std::mutex> g(mu);
        free_blocks[cls].push_back(p);
    }
    void release()
    {
        for (char *p : all) (void)hipHostFree(p);
        all.clear();
        free_blocks.clear();
    }
    ~PinnedPool() { release(); }
};

// The outputs of one batch: a pinned buffer that holds every event's lists
// (the output image, copied from the device in one transfer) and the number
// of outputs that point into it; the last lst_free_output gives it back to
// the pool, which each buffer keeps alive (outputs may outlive the context).
struct OutBatch {
    std::shared_ptr<PinnedPool> pool;
    char *buf = nullptr;
    size_t cls = 0;
    std::atomic<uint32_t> refs{0};
    void unref()
    {
        if (refs.fetch_sub(1, std::memory_order_acq_rel) == 1) {
            pool->put(buf, cls);
            delete this;
        }
    }
};

// What an lst_event_out pointer handed to the caller points to.
struct OutBox {
    lst_event_out pub;       // first member: the caller's pointer is its address
    OutBatch *batch;         // buffer the lists point into (null: no lists)
};

// A host-side range for tracing tools (rocprofv3 --marker-trace) around a
// call that enqueues or collects device work; nearly free without a tool.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

lst_event_out *new_out()
{
    OutBox *b = (OutBox *)std::calloc(1, sizeof(OutBox));
    return b ? &b->pub : nullptr;
}

// Pinned chunks that submitted events are appended to, one after the other,
// so that the events of a micro-batch lie (nearly) back to back and reach the
// device in a few large copies instead of one copy per event.  A chunk goes
// back to the free list once none of its events is held and it is no longer
// the one being appended to; an event larger than a chunk gets one of its
// own.
struct InChunk {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    uint32_t live = 0;       // events in the chunk not yet released
};

struct InChunks {
    static constexpr size_t kChunk = 64ull << 20;
    static constexpr size_t kAlign = 256;
    std::mutex mu;
    std::vector<InChunk *> all, free_list;
    InChunk *open = nullptr;
    // room for an event block: its chunk and offset; false if pinned memory
    // cannot be had
    bool get(size_t bytes, InChunk *&c, size_t &off)
    {
        std::lock_guard<std::mutex> g(mu);
        const size_t need = (bytes + kAlign - 1) / kAlign * kAlign;
        if (!open || open->used + need > open->cap) {
            InChunk *old = open;
            open = nullptr;
            if (old && old->live == 0) { old->used = 0; free_list.push_back(old); }
            const size_t cap = std::max(kChunk, need);
            for (size_t i = 0; i < free_list.size(); i++)
                if (free_list[i]->cap >= cap) {
                    open = free_list[i];
                    free_list.erase(free_list.begin() + (long)i);
                    break;
                }
            if (!open) {
                InChunk *n = new (std::nothrow) InChunk;
                if (!n) return false;
                if (hipHostMalloc((void **)&n->base, cap, hipHostMallocDefault) != hipSuccess) {
                    delete n;
                    return false;
                }
                n->cap = cap;
                all.push_back(n);
                open = n;
            }
            open->used = 0;
        }
        c = open;
        off = open->used;
        open->used += need;
        open->live++;
        return true;
    }
    void put(InChunk *c)
    {
        if (!c) return;
        std::lock_guard<std::mutex> g(mu);
        if (--c->live == 0 && c != open) {
            c->used = 0;
            free_list.push_back(c);
        }
    }
    void release()
    {
        for (InChunk *c : all) {
            (void)hipHostFree(c->base);
            delete c;
        }
        all.clear();
        free_list.clear();
        open = nullptr;
    }
    ~InChunks() { release(); }
};

struct ServedEvent {
    uint64_t ticket;
    uint32_t n_hits = 0, n_pls = 0;
    InChunk *chunk = nullptr;   // pinned chunk holding the event's block (served_block_layout)
    size_t blk_off = 0;         // the block's offset in the chunk
    size_t blk_bytes = 0;
    uint64_t footprint;
    std::chrono::steady_clock::time_point t_submit;
};

struct lst_ctx {
    lst_params p{};
    int device = 0;
    void *ws = nullptr;                 // this device's copy of scratch (lst_run_event_noalloc)
    std::atomic<bool> failed{false};
    mutable std::mutex err_mu;
    std::string last_error;
    bool has_geom = false;
    lst::Geometry geom;
    std::string geom_cache;             // directory of the geometry cache (empty: none)
    bool geom_from_cache = false;       // the loaded tables came from the cache
    lst::DevGeom dg{};
    void *geom_mem = nullptr;
    std::unique_ptr<lst::Slot> plain;   // per-event / batched / device-resident path
    std::map<std::string, std::pair<double, uint32_t>> ktimes;
    std::string time_only;          // launch name that timing is restricted to (empty: all)
    std::mutex run_mu;                  // serialises the plain path
    // served path
    std::vector<std::unique_ptr<lst::Slot>> slots;
    std::mutex q_mu;
    // q_cv: the admission thread (new events, a slot freed); slot_cv: the
    // completion threads (a slot launched); done_cv: pollers (outputs ready)
    std::condition_variable q_cv, slot_cv, done_cv;
    std::deque<std::unique_ptr<ServedEvent>> waiting;
    InChunks in_chunks;                 // submitted events
    // output batches: mapped and coherent, so that the pack kernel writes
    // them over the host link itself (no device-to-host copy)
    std::shared_ptr<PinnedPool> out_pool = [] {
        auto p = std::make_shared<PinnedPool>();
        p->flags = hipHostMallocMapped | hipHostMallocCoherent;
        return p;
    }();
    std::vector<int> slot_state;        // 0 free, 1 being staged, 2 launched
    std::vector<uint64_t> slot_mem;
    std::vector<std::vector<std::unique_ptr<ServedEvent>>> held;
    std::vector<std::thread> completers;
    bool stop_completers = false;
    std::unordered_map<uint64_t, lst_event_out *> finished;
    std::unordered_map<uint64_t, int> state;   // 1 waiting / running, 2 finished
    uint64_t next_ticket = 1;
    size_t in_system = 0;
    uint64_t mem_in_use = 0;
    std::thread worker;
    bool stop = false;
    bool worker_started = false;
};

using lst::Batch;
using lst::Slot;

namespace {

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            fail(ctx, std::string(#expr) + ": " + hipGetErrorString(e_));              \
            return LST_ERR_DEVICE;                                                     \
        }                                                                              \
    } while (0)

void fail(lst_ctx *ctx, const std::string &msg)
{
    std::lock_guard<std::mutex> g(ctx->err_mu);
    ctx->failed = true;
    ctx->last_error = msg;
}

lst_status set_err(lst_ctx *ctx, lst_status s, const std::string &msg)
{
    std::lock_guard<std::mutex> g(ctx->err_mu);
    ctx->last_error = msg;
    return s;
}

void free_slot_arenas(Slot &s)
{
    if (s.gexec) { (void)hipGraphExecDestroy(s.gexec); s.gexec = nullptr; }
    if (s.graph) { (void)hipGraphDestroy(s.graph); s.graph = nullptr; }
    s.graph_valid = false;
    if (s.in_arena) { (void)hipFree(s.in_arena); s.in_arena = nullptr; }
    if (s.work_arena) { (void)hipFree(s.work_arena); s.work_arena = nullptr; }
    if (s.h_stage) { (void)hipHostFree(s.h_stage); s.h_stage = nullptr; }
    s.in_bytes = s.work_bytes = s.stage_bytes = s.img_words = 0;
}

void destroy_slot(Slot &s)
{
    free_slot_arenas(s);
    if (s.raw) (void)hipFree(s.raw);
    if (s.d_rawoff) (void)hipFree(s.d_rawoff);
    if (s.h_rawoff) (void)hipHostFree(s.h_rawoff);
    if (s.d_tot) (void)hipFree(s.d_tot);
    if (s.h_tot) (void)hipHostFree(s.h_tot);
    if (s.d_part) (void)hipFree(s.d_part);
    for (hipEvent_t e : s.L.pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : s.L.ev_fork) if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : s.L.ev_join) if (e) (void)hipEventDestroy(e);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.side) (void)hipStreamDestroy(s.side);
    if (s.stream && s.own_stream) (void)hipStreamDestroy(s.stream);
}

lst_status make_slot(lst_ctx *ctx, std::unique_ptr<Slot> &out, hipStream_t caller = nullptr)
{
    auto s = std::make_unique<Slot>();
    s->device = ctx->device;
    if (caller) {
        s->stream = caller;
        s->own_stream = false;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    }
    HIP_TRY(hipMalloc(&s->d_tot, sizeof(lst::Totals)));
    HIP_TRY(hipHostMalloc((void **)&s->h_tot, sizeof(lst::Totals), hipHostMallocDefault));
    HIP_TRY(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
    HIP_TRY(hipMalloc(&s->d_part, 2 * sizeof(uint32_t) * lst::kScanGrid));
    HIP_TRY(hipEventCreateWithFlags(&s->done, hipEventDisableTiming | hipEventBlockingSync));
    for (int k = 0; k < 2; k++) {
        HIP_TRY(hipEventCreateWithFlags(&s->L.ev_fork[k], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&s->L.ev_join[k], hipEventDisableTiming));
    }
    s->L.stream = s->stream;
    s->L.side = s->side;
    s->L.cur = s->stream;
    s->L.part = s->d_part;
    s->L.part_side = s->d_part + lst::kScanGrid;
    out = std::move(s);
    return LST_OK;
}

// Ensure the slot's arenas hold a batch with these capacities (inputs and
// work are separate so that growing the work arena keeps staged inputs).
lst_status ensure_inputs(lst_ctx *ctx, Slot &s, uint32_t n_ev, uint64_t hits, uint64_t pls)
{
    Batch &b = s.b;
    if (s.in_arena && n_ev <= b.cap_ev && hits <= b.cap_hits && pls <= b.cap_pls) return LST_OK;
    // a quarter of headroom: events of similar size that follow reuse the
    // arenas (and the captured graph) instead of reallocating them one after
    // another
    lst::Caps c = lst::plan_caps(std::max(n_ev, b.cap_ev), std::max<uint64_t>(hits + hits / 4 + 1024, b.cap_hits),
                                 std::max<uint64_t>(pls + pls / 4 + 64, b.cap_pls));
    // keep work capacities at least as large as before
    c.md = std::max(c.md, b.cap_md); c.ls = std::max(c.ls, b.cap_ls); c.t3 = std::max(c.t3, b.cap_t3);
    c.t5 = std::max(c.t5, b.cap_t5); c.pt3 = std::max(c.pt3, b.cap_pt3); c.pt5 = std::max(c.pt5, b.cap_pt5);
    c.ptc3 = std::max(c.ptc3, b.cap_ptc3); c.ptc5 = std::max(c.ptc5, b.cap_ptc5);
    // (seed, surface) units are 32-bit indices on the device
    if ((uint64_t)std::max<uint32_t>(c.pls, 1) * ctx->geom.c.n_surf > 0xFFFFFFF0ull)
        return set_err(ctx, LST_ERR_TOO_LARGE, "too many seeds for 32-bit (seed, surface) indexing");
    free_slot_arenas(s);
    b.cap_ev = c.ev; b.cap_hits = std::max<uint32_t>(c.hits, 1); b.cap_pls = std::max<uint32_t>(c.pls, 1);
    b.cap_md = c.md; b.cap_ls = c.ls; b.cap_t3 = c.t3; b.cap_t5 = c.t5; b.cap_pt3 = c.pt3; b.cap_pt5 = c.pt5;
    b.cap_ptc3 = c.ptc3; b.cap_ptc5 = c.ptc5;
    lst::plan_sublists(b);
    b.cap_tc = b.cap_pt3 + b.cap_t5 + b.cap_pls;
    lst::Carver ci{nullptr};
    lst::carve_inputs(ci, b);
    s.in_bytes = ci.off;
    hipError_t e = hipMalloc(&s.in_arena, s.in_bytes);
    if (e != hipSuccess) { s.in_arena = nullptr; return set_err(ctx, LST_ERR_OOM, "input arena allocation failed"); }
    lst::Carver ci2{(char *)s.in_arena};
    lst::carve_inputs(ci2, b);
    s.stage_bytes = s.in_bytes;
    HIP_TRY(hipHostMalloc((void **)&s.h_stage, s.stage_bytes, hipHostMallocDefault));
    return LST_OK;
}

lst_status ensure_work(lst_ctx *ctx, Slot &s)
{
    if (s.work_arena) return LST_OK;
    Batch &b = s.b;
    b.cap_tc = b.cap_pt3 + b.cap_t5 + b.cap_pls;
    const lst::Consts &c = ctx->geom.c;
    lst::Carver cw{nullptr};
    lst::carve_work(cw, b, c.n_mod, c.n_surf, c.nphi, c.nkb);
    // the largest output image the list capacities allow (download checks
    // the image it writes against it)
    const bool clean = (c.flags & LST_FLAG_TC_CLEAN) != 0u;
    const uint64_t img_words = (uint64_t)(b.cap_ev + 1) * lst::kEvTabCols + 2ull * b.cap_ev +
                               2ull * ((uint64_t)b.cap_md + b.cap_ls + b.cap_t3 + b.cap_t5 + b.cap_pt3 +
                                       2ull * b.cap_pt5 + b.cap_tc) +
                               b.cap_t3 + (clean ? 2ull * ((uint64_t)b.cap_pt5 + b.cap_tc) : 0ull) + b.cap_tc;
    s.work_bytes = cw.off;
    hipError_t e = hipMalloc(&s.work_arena, s.work_bytes);
    if (e != hipSuccess) {
        s.work_arena = nullptr;
        return set_err(ctx, LST_ERR_OOM,
                       "work arena allocation failed (" + std::to_string(s.work_bytes >> 20) + " MiB; capacities md " +
                           std::to_string(b.cap_md) + " ls " + std::to_string(b.cap_ls) + " t3 " +
                           std::to_string(b.cap_t3) + " t5 " + std::to_string(b.cap_t5) + " pt3 " +
                           std::to_string(b.cap_pt3) + " pt5 " + std::to_string(b.cap_pt5) + " pairs " +
                           std::to_string(b.cap_ptc3) + "/" + std::to_string(b.cap_ptc5) + ")");
    }
    lst::Carver cw2{(char *)s.work_arena};
    lst::carve_work(cw2, b, c.n_mod, c.n_surf, c.nphi, c.nkb);
    s.img_words = img_words;
    s.graph_valid = false;
    return LST_OK;
}

lst_status check_event(lst_ctx *ctx, const lst_event_in &ev)
{
    if (ev.n_hits && (!ev.x || !ev.y || !ev.z || !ev.module || !ev.sensor))
        return set_err(ctx, LST_ERR_INVALID_ARG, "null hit array");
    if (ev.n_pls && (!ev.pls_par || !ev.pls_cov)) return set_err(ctx, LST_ERR_INVALID_ARG, "null seed array");
    return LST_OK;
}

// Stage n events into the slot's input arena (async on the slot stream).
// Copies of host-pointer inputs into the pinned stage.  A batch of 64
// PU200-like events moves about 70 MB this way, which one thread copies out
// of pageable memory at a fraction of what the host's memory gives, so
// copies of more than 8 MiB in all are split by bytes over up to 8 threads
// (the calling thread takes the first share).
struct HostCopy { char *dst; const char *src; size_t n; };

static void parallel_copy(const std::vector<HostCopy> &jobs)
{
    size_t total = 0;
    for (const HostCopy &j : jobs) total += j.n;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned nt = total < (size_t(8) << 20) ? 1u : std::min(8u, hw);
    auto work = [&jobs, total, nt](unsigned t) {
        const size_t share = (total + nt - 1) / nt;
        const size_t lo = std::min(total, t * share), hi = std::min(total, lo + share);
        size_t pos = 0;
        for (const HostCopy &j : jobs) {
            const size_t a = std::max(lo, pos), b = std::min(hi, pos + j.n);
            if (a < b) std::memcpy(j.dst + (a - pos), j.src + (a - pos), b - a);
            pos += j.n;
            if (pos >= hi) break;
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; t++) {
        try {
            th.emplace_back(work, t);
        } catch (...) {
            work(t);   // no thread to be had: copy this share here
        }
    }
    work(0);
    for (std::thread &x : th) x.join();
}

lst_status stage_inputs(lst_ctx *ctx, Slot &s, const lst_event_in *evs, uint32_t n)
{
    uint64_t hits = 0, pls = 0;
    for (uint32_t i = 0; i < n; i++) {
        lst_status st = check_event(ctx, evs[i]);
        if (st != LST_OK) return st;
        hits += evs[i].n_hits;
        pls += evs[i].n_pls;
    }
    if (hits > 0x7FFFFFFFull || pls > 0x7FFFFFFFull) return set_err(ctx, LST_ERR_TOO_LARGE, "batch too large");
    lst_status st = ensure_inputs(ctx, s, n, hits, pls);
    if (st != LST_OK) return st;
    st = ensure_work(ctx, s);
    if (st != LST_OK) return st;
    Batch &b = s.b;
    s.n_ev = n;
    s.hit_off.assign(n + 1, 0);
    s.pls_off.assign(n + 1, 0);
    for (uint32_t i = 0; i < n; i++) {
        s.hit_off[i + 1] = s.hit_off[i] + evs[i].n_hits;
        s.pls_off[i + 1] = s.pls_off[i] + evs[i].n_pls;
    }
    // host-pointer events go through the pinned stage, laid out like the arena
    char *hs = s.h_stage;
    struct Arr { void *dev; size_t elt; int which; };
    const Arr arrs[] = {{b.in_x, 4, 0}, {b.in_y, 4, 1}, {b.in_z, 4, 2}, {b.in_mod, 4, 3},
                        {b.in_sen, 1, 4}, {b.in_par, 20, 5}, {b.in_cov, 60, 6}, {b.in_nhit, 1, 7}};
    std::vector<HostCopy> jobs;
    for (const Arr &a : arrs) {
        size_t base_off = (char *)a.dev - (char *)s.in_arena;
        const std::vector<uint32_t> &offs = a.which < 5 ? s.hit_off : s.pls_off;
        for (uint32_t i = 0; i < n; i++) {
            const lst_event_in &ev = evs[i];
            size_t cnt = a.which < 5 ? ev.n_hits : ev.n_pls;
            if (!cnt) continue;
            const void *src = a.which == 0 ? (const void *)ev.x : a.which == 1 ? (const void *)ev.y
                            : a.which == 2 ? (const void *)ev.z : a.which == 3 ? (const void *)ev.module
                            : a.which == 4 ? (const void *)ev.sensor : a.which == 5 ? (const void *)ev.pls_par
                            : a.which == 6 ? (const void *)ev.pls_cov : (const void *)ev.pls_nhits;
            size_t at = (size_t)offs[i] * a.elt;
            if (a.which == 7 && !src) {
                // no hit counts given: every seed is a quad
                if (ev.flags & LST_DEVICE_PTRS)
                    HIP_TRY(hipMemsetAsync((char *)a.dev + at, 4, cnt, s.stream));
                else
                    std::memset(hs + base_off + at, 4, cnt);
                continue;
            }
            if (ev.flags & LST_DEVICE_PTRS) {
                HIP_TRY(hipMemcpyAsync((char *)a.dev + at, src, cnt * a.elt, hipMemcpyDeviceToDevice, s.stream));
            } else {
                jobs.push_back({hs + base_off + at, (const char *)src, cnt * a.elt});
            }
        }
    }
    parallel_copy(jobs);
    // one host->device copy per array for the host-pointer events
    for (const Arr &a : arrs) {
        size_t base_off = (char *)a.dev - (char *)s.in_arena;
        const std::vector<uint32_t> &offs = a.which < 5 ? s.hit_off : s.pls_off;
        // copy contiguous runs of host-pointer events
        uint32_t i = 0;
        while (i < n) {
            if (evs[i].flags & LST_DEVICE_PTRS) { i++; continue; }
            uint32_t j = i;
            while (j < n && !(evs[j].flags & LST_DEVICE_PTRS)) j++;
            size_t lo = (size_t)offs[i] * a.elt, hi = (size_t)offs[j] * a.elt;
            if (hi > lo)
                HIP_TRY(hipMemcpyAsync((char *)a.dev + lo, hs + base_off + lo, hi - lo, hipMemcpyHostToDevice,
                                       s.stream));
            i = j;
        }
    }
    // event offsets and the host-written counters
    size_t hoff_at = (char *)b.ev_hit_off - (char *)s.in_arena;
    size_t poff_at = (char *)b.ev_pls_off - (char *)s.in_arena;
    std::memcpy(hs + hoff_at, s.hit_off.data(), (n + 1) * 4);
    std::memcpy(hs + poff_at, s.pls_off.data(), (n + 1) * 4);
    HIP_TRY(hipMemcpyAsync(b.ev_hit_off, hs + hoff_at, (n + 1) * 4, hipMemcpyHostToDevice, s.stream));
    HIP_TRY(hipMemcpyAsync(b.ev_pls_off, hs + poff_at, (n + 1) * 4, hipMemcpyHostToDevice, s.stream));
    s.h_tot->n_ev = n;
    s.h_tot->n_hits = (uint32_t)hits;
    s.h_tot->n_pls = (uint32_t)pls;
    HIP_TRY(hipMemcpyAsync(s.d_tot, s.h_tot, 3 * sizeof(uint32_t), hipMemcpyHostToDevice, s.stream));
    return LST_OK;
}

lst_status enqueue(lst_ctx *ctx, Slot &s, bool use_graph, bool timing, bool stats)
{
    if (use_graph && !timing && !stats) {
        if (!s.graph_valid) {
            if (s.gexec) { (void)hipGraphExecDestroy(s.gexec); s.gexec = nullptr; }
            if (s.graph) { (void)hipGraphDestroy(s.graph); s.graph = nullptr; }
            HIP_TRY(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
            s.L.timing = false;
            s.L.err = hipSuccess;
            lst::enqueue_chain(s.L, s.b, s.d_tot, ctx->dg, ctx->geom.c, 0);
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamEndCapture(s.stream, &g));
            s.graph = g;
            if (s.L.err != hipSuccess) {
                fail(ctx, std::string("kernel launch during capture: ") + hipGetErrorString(s.L.err));
                return LST_ERR_DEVICE;
            }
            HIP_TRY(hipGraphInstantiate(&s.gexec, s.graph, nullptr, nullptr, 0));
            s.graph_valid = true;
        }
        HIP_TRY(hipGraphLaunch(s.gexec, s.stream));
        return LST_OK;
    }
    s.L.timing = timing;
    s.L.err = hipSuccess;
    lst::enqueue_chain(s.L, s.b, s.d_tot, ctx->dg, ctx->geom.c, stats ? 1 : 0);
    if (s.L.err != hipSuccess) {
        fail(ctx, std::string("kernel launch: ") + hipGetErrorString(s.L.err));
        return LST_ERR_DEVICE;
    }
    return LST_OK;
}

// After the chain: fetch the counters; grow the work arena where a list
// overflowed (the caller re-runs).  Returns 1 when a re-run is needed.
int overflowed(Slot &s) { return lst::grow_caps(s.b, *s.h_tot) ? 1 : 0; }

// Elapsed times of the timed launches since the last drain: per launch name
// into the context's kernel table, per stage into the slot's stage times.
void drain_records(lst_ctx *ctx, Slot &s)
{
    for (auto &r : s.L.recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
            auto &kt = ctx->ktimes[r.name];
            kt.first += ms;
            kt.second += 1;
            if (r.stage >= 0 && r.stage < LST_N_STAGES) s.stage_ns[r.stage] += (uint64_t)(ms * 1e6 + 0.5);
        }
    }
    s.L.recs.clear();
    s.L.used = 0;
}

lst_status input_error(lst_ctx *ctx, uint32_t bits)
{
    if (bits & lst::kErrBadModule) return set_err(ctx, LST_ERR_BAD_MODULE, "hit with module id out of range or sensor > 1");
    if (bits & lst::kErrNonFinite) return set_err(ctx, LST_ERR_NONFINITE, "non-finite hit coordinate or seed parameter");
    if (bits & lst::kErrOutside)
        return set_err(ctx, LST_ERR_HIT_OUTSIDE, "hit off its sensor or outside its module's extent (input contract)");
    return LST_OK;
}

// After the chain: fetch the counters (and the stage times of a timed run).
// batch_errors: an input error of any event fails the batch; otherwise input
// errors are left to the per-event status (served path).
lst_status finish_run(lst_ctx *ctx, Slot &s, bool batch_errors)
{
    HIP_TRY(hipMemcpyAsync(s.h_tot, s.d_tot, sizeof(lst::Totals), hipMemcpyDeviceToHost, s.stream));
    HIP_TRY(hipStreamSynchronize(s.stream));
    if (s.L.timing) drain_records(ctx, s);
    if (batch_errors) return input_error(ctx, s.h_tot->err);
    return LST_OK;
}

// Run the staged batch to completion, growing arenas on overflow.  With
// stage_times the chain runs eagerly on the slot's stream alone, every launch
// timed.
lst_status run_staged(lst_ctx *ctx, Slot &s, bool use_graph, bool stage_times, bool batch_errors)
{
    s.n_regrow = 0;
    hipStream_t side = s.L.side;
    for (int attempt = 0; attempt < 12; attempt++) {
        std::memset(s.stage_ns, 0, sizeof s.stage_ns);
        if (stage_times) {
            s.L.side = nullptr;
            s.L.only = nullptr;
        }
        lst_status st = enqueue(ctx, s, use_graph && !stage_times, stage_times, false);
        if (st == LST_OK) st = finish_run(ctx, s, batch_errors);
        s.L.side = side;
        s.L.timing = false;
        if (st != LST_OK) return st;
        if (!overflowed(s)) return LST_OK;
        // grow the work arena; staged inputs stay valid
        s.n_regrow++;
        if (s.gexec) { (void)hipGraphExecDestroy(s.gexec); s.gexec = nullptr; }
        if (s.graph) { (void)hipGraphDestroy(s.graph); s.graph = nullptr; }
        s.graph_valid = false;
        if (s.work_arena) { (void)hipFree(s.work_arena); s.work_arena = nullptr; }
        st = ensure_work(ctx, s);
        if (st != LST_OK) return st;
    }
    return set_err(ctx, LST_ERR_OOM, "object lists kept overflowing");
}

// Copy the results of the staged batch to host memory, one output per event:
// the device writes the batch's output image (every event's lists with
// event-local indices, in the layout of lst_event_out), one transfer brings it
// into a pinned buffer, and each event's output points into that buffer.
lst_status download(lst_ctx *ctx, Slot &s, lst_event_out **outs)
{
    TraceRange trace_("lst: outputs to host");
    const uint32_t n = s.n_ev;
    for (uint32_t e = 0; e < n; e++) outs[e] = nullptr;
    const lst::Totals &t = *s.h_tot;
    const bool clean = (ctx->geom.c.flags & LST_FLAG_TC_CLEAN) != 0u;
    const bool triplets = (ctx->geom.c.flags & LST_FLAG_SEEDS_TRIPLETS) != 0u;
    const uint64_t n_tab = (uint64_t)(n + 1) * lst::kEvTabCols;
    const uint64_t head = n_tab + 2ull * n;   // table, cleaning counts, seed counts
    const uint64_t pairs = (uint64_t)t.n_md + t.n_ls + t.n_t3 + t.n_t5 + t.n_pt3 + 2ull * t.n_pt5 + t.n_tc;
    // the seed-only candidates (room for the exported seeds) are some of
    // the n_tc candidates: the image's size is known exactly only from its
    // table, so the buffer is sized with all of them
    const uint64_t words = head + 2 * pairs + t.n_t3 + (clean ? 2ull * ((uint64_t)t.n_pt5 + t.n_tc) : 0ull) + t.n_tc;
    if (words > s.img_words) {
        fail(ctx, "output image larger than the list capacities");
        return LST_ERR_DEVICE;
    }
    OutBatch *ob = new (std::nothrow) OutBatch;
    if (!ob) return set_err(ctx, LST_ERR_OOM, "host allocation of outputs failed");
    ob->pool = ctx->out_pool;
    // a new block gets room for batches half as large again (sizes vary
    // from batch to batch; larger free blocks serve smaller ones)
    ob->buf = ob->pool->get(4 * words, ob->cls, 4 * words / 2);
    if (!ob->buf) {
        delete ob;
        return set_err(ctx, LST_ERR_OOM, "pinned allocation of outputs failed");
    }
    ob->refs = 1;   // held while the outputs are made
    // the pack kernel writes the image straight into the mapped host buffer
    void *dimg = nullptr;
    hipError_t he = hipHostGetDevicePointer(&dimg, ob->buf, 0);
    s.L.on_side(false);
    s.L.timing = false;
    s.L.err = hipSuccess;
    const uint64_t items = n_tab + pairs + t.n_t3;   // one per pair, curvature and table word
    if (he == hipSuccess) {
        lst::launch_pack(s.L, s.b, s.d_tot, (uint32_t *)dimg, n, head, words, clean, triplets, items);
        he = s.L.err;
    }
    if (he == hipSuccess) he = hipStreamSynchronize(s.stream);
    if (he != hipSuccess) {
        ob->unref();
        fail(ctx, std::string("output copy: ") + hipGetErrorString(he));
        return LST_ERR_DEVICE;
    }
    uint32_t *img = (uint32_t *)ob->buf;
    const uint32_t *tab = img;
    // the image's size from the copied table must be the one the totals gave
    auto before = [&](const uint32_t *r) {
        const uint64_t p = (uint64_t)r[2] + r[3] + r[4] + r[5] + r[6] + 2ull * r[7] + r[8] + r[9] + r[10];
        return 2 * p + r[4] + (clean ? 2ull * ((uint64_t)r[7] + r[8] + r[9] + r[10]) : 0ull) + r[10];
    };
    if (head + before(tab + n_tab - lst::kEvTabCols) - before(tab) > words) {
        ob->unref();
        fail(ctx, "output image larger than the list totals allow");
        return LST_ERR_DEVICE;
    }
    uint32_t *lists = img + head;
    bool failed = false;
    for (uint32_t e = 0; e < n; e++) {
        const uint32_t *r0 = &tab[(size_t)e * lst::kEvTabCols], *r1 = r0 + lst::kEvTabCols;
        lst_event_out *o = new_out();
        if (!o) { failed = true; break; }
        outs[e] = o;
        o->n_flag_regrow = s.n_regrow;
        o->n_stage = LST_N_STAGES;
        o->batch_events = n;
        if (r0[11]) {
            // an input error of this event: its status only, no lists
            o->status = (uint32_t)(r0[11] & lst::kErrBadModule ? LST_ERR_BAD_MODULE
                                   : r0[11] & lst::kErrNonFinite ? LST_ERR_NONFINITE
                                                                 : LST_ERR_HIT_OUTSIDE);
            continue;
        }
        const uint32_t cmd = r1[2] - r0[2], cls = r1[3] - r0[3], ct3 = r1[4] - r0[4], ct5 = r1[5] - r0[5];
        const uint32_t cp3 = r1[6] - r0[6], cp5 = r1[7] - r0[7];
        const uint32_t ctc = cp5 + (r1[8] - r0[8]) + (r1[9] - r0[9]) + (r1[10] - r0[10]);
        uint32_t *w = lists + (before(r0) - before(tab));
        o->n_md = cmd; o->n_ls = cls; o->n_t3 = ct3; o->n_t5 = ct5; o->n_pt3 = cp3; o->n_pt5 = cp5; o->n_tc = ctc;
        o->md = w; w += 2 * cmd;
        o->ls = w; w += 2 * cls;
        o->t3 = w; w += 2 * ct3;
        o->t5 = w; w += 2 * ct5;
        o->pt3 = w; w += 2 * cp3;
        o->pt5 = w; w += 2 * cp5;
        o->tc = w; w += 2 * ctc;
        o->t3_kappa = (float *)w;
        w += ct3;
        if (clean) {
            o->tcc = w;
            o->n_tcc = img[n_tab + e];
            if (o->n_tcc > ctc) { failed = true; break; }
            w += 2 * ctc;
        }
        o->seeds = w;
        o->n_seeds = img[n_tab + n + e];
        if (o->n_seeds > r1[10] - r0[10]) { failed = true; break; }
        o->status = LST_OK;
        std::memcpy(o->stage_ns, s.stage_ns, sizeof o->stage_ns);
        ob->refs.fetch_add(1, std::memory_order_relaxed);
        ((OutBox *)o)->batch = ob;
    }
    ob->unref();
    if (failed) {
        for (uint32_t e = 0; e < n; e++) { lst_free_output(outs[e]); outs[e] = nullptr; }
        return set_err(ctx, LST_ERR_OOM, "host allocation of outputs failed");
    }
    return LST_OK;
}

lst_status check_ctx(lst_ctx *ctx, bool need_geom)
{
    if (!ctx) return LST_ERR_INVALID_ARG;
    if (ctx->failed) return LST_ERR_DEVICE;
    if (need_geom && !ctx->has_geom) return set_err(ctx, LST_ERR_NO_GEOMETRY, "no geometry loaded");
    return LST_OK;
}

lst_status ensure_plain(lst_ctx *ctx)
{
    if (ctx->plain) return LST_OK;
    return make_slot(ctx, ctx->plain, (hipStream_t)ctx->p.stream);
}

}  // namespace

// ======================================================================
// served path: scheduler thread
// ======================================================================
namespace {

uint64_t predict_footprint(uint64_t hits, uint64_t pls, const lst::Consts &k)
{
    // device bytes of one event in a slot: inputs + work lists at planned
    // capacity + the per-event bins of the sort and of the seed lookup
    lst::Caps c = lst::plan_caps(1, hits, pls);
    uint64_t b = 0;
    b += 73ull * c.hits + 160ull * c.pls + 24ull * k.n_mod;
    b += (56ull + 4ull * lst::kKeepLs) * c.md + 28ull * c.ls + 88ull * c.t3 + 64ull * c.t5;
    b += 16ull * (c.pt3 + c.pt5) + 24ull * c.pls * k.n_surf + 19ull * c.pls + 16ull * (c.pt3 + c.t5 + c.pls);
    b += 12ull * (c.ptc3 + c.ptc5);
    b += 2ull * 8ull * k.n_surf * k.nphi * (3 * k.nkb + 1);
    return b;
}

void admit_main(lst_ctx *ctx);
void complete_main(lst_ctx *ctx, uint32_t i);

}  // namespace

namespace {

// Copy a micro-batch of served events to slot s and launch the chain: one
// host-to-device copy per event block (pinned at submission), the unpack
// kernel, then the captured chain.
lst_status stage_served(lst_ctx *ctx, Slot &s, const std::vector<std::unique_ptr<ServedEvent>> &evs)
{
    TraceRange trace_("lst: stage served micro-batch");
    const uint32_t n = (uint32_t)evs.size();
    uint64_t hits = 0, pls = 0, raw = 0;
    for (const auto &e : evs) {
        hits += e->n_hits;
        pls += e->n_pls;
        raw += e->blk_bytes;
    }
    if (hits > 0x7FFFFFFFull || pls > 0x7FFFFFFFull) return set_err(ctx, LST_ERR_TOO_LARGE, "batch too large");
    lst_status st = ensure_inputs(ctx, s, n, hits, pls);
    if (st == LST_OK) st = ensure_work(ctx, s);
    if (st != LST_OK) return st;
    // one copy per chunk the batch touches: the span from its first to the
    // end of its last block there (blocks of other batches in between are
    // copied along and not used)
    struct Span { InChunk *c; size_t lo, hi, at; };
    std::vector<Span> spans;
    for (const auto &e : evs) {
        if (!e->blk_bytes) continue;
        Span *sp = nullptr;
        for (Span &x : spans)
            if (x.c == e->chunk) sp = &x;
        if (!sp) {
            spans.push_back(Span{e->chunk, e->blk_off, e->blk_off + e->blk_bytes, 0});
        } else {
            sp->lo = std::min(sp->lo, e->blk_off);
            sp->hi = std::max(sp->hi, e->blk_off + e->blk_bytes);
        }
    }
    raw = 0;
    for (Span &x : spans) {
        x.at = raw;
        raw += (x.hi - x.lo + 255) / 256 * 256;
    }
    if (raw > s.raw_cap) {
        if (s.raw) (void)hipFree(s.raw);
        s.raw = nullptr;
        s.raw_cap = 0;
        const size_t want = raw + raw / 4 + (1 << 20);
        if (hipMalloc(&s.raw, want) != hipSuccess) { s.raw = nullptr; return set_err(ctx, LST_ERR_OOM, "served input allocation failed"); }
        s.raw_cap = want;
    }
    if (n + 1 > s.rawoff_cap) {
        if (s.d_rawoff) (void)hipFree(s.d_rawoff);
        if (s.h_rawoff) (void)hipHostFree(s.h_rawoff);
        s.d_rawoff = s.h_rawoff = nullptr;
        s.rawoff_cap = 0;
        const uint32_t cap = std::max<uint32_t>(ctx->p.max_batch, n) + 1;
        HIP_TRY(hipMalloc((void **)&s.d_rawoff, 8ull * cap));
        HIP_TRY(hipHostMalloc((void **)&s.h_rawoff, 8ull * cap, hipHostMallocDefault));
        s.rawoff_cap = cap;
    }
    Batch &b = s.b;
    s.n_ev = n;
    s.hit_off.assign(n + 1, 0);
    s.pls_off.assign(n + 1, 0);
    for (const Span &x : spans)
        HIP_TRY(hipMemcpyAsync(s.raw + x.at, x.c->base + x.lo, x.hi - x.lo, hipMemcpyHostToDevice, s.stream));
    for (uint32_t i = 0; i < n; i++) {
        s.hit_off[i + 1] = s.hit_off[i] + evs[i]->n_hits;
        s.pls_off[i + 1] = s.pls_off[i] + evs[i]->n_pls;
        s.h_rawoff[i] = 0;
        if (evs[i]->blk_bytes)
            for (const Span &x : spans)
                if (x.c == evs[i]->chunk) s.h_rawoff[i] = x.at + (evs[i]->blk_off - x.lo);
    }
    s.h_rawoff[n] = raw;
    HIP_TRY(hipMemcpyAsync(s.d_rawoff, s.h_rawoff, 8ull * (n + 1), hipMemcpyHostToDevice, s.stream));
    char *hs = s.h_stage;
    const size_t hoff_at = (char *)b.ev_hit_off - (char *)s.in_arena;
    const size_t poff_at = (char *)b.ev_pls_off - (char *)s.in_arena;
    std::memcpy(hs + hoff_at, s.hit_off.data(), (n + 1) * 4);
    std::memcpy(hs + poff_at, s.pls_off.data(), (n + 1) * 4);
    HIP_TRY(hipMemcpyAsync(b.ev_hit_off, hs + hoff_at, (n + 1) * 4, hipMemcpyHostToDevice, s.stream));
    HIP_TRY(hipMemcpyAsync(b.ev_pls_off, hs + poff_at, (n + 1) * 4, hipMemcpyHostToDevice, s.stream));
    s.h_tot->n_ev = n;
    s.h_tot->n_hits = (uint32_t)hits;
    s.h_tot->n_pls = (uint32_t)pls;
    HIP_TRY(hipMemcpyAsync(s.d_tot, s.h_tot, 3 * sizeof(uint32_t), hipMemcpyHostToDevice, s.stream));
    s.L.on_side(false);
    s.L.timing = false;
    s.L.err = hipSuccess;
    lst::launch_unpack(s.L, b, s.d_tot, s.raw, s.d_rawoff);
    if (s.L.err != hipSuccess) {
        fail(ctx, std::string("kernel launch: ") + hipGetErrorString(s.L.err));
        return LST_ERR_DEVICE;
    }
    st = enqueue(ctx, s, true, false, false);
    if (st != LST_OK) return st;
    HIP_TRY(hipEventRecord(s.done, s.stream));
    return LST_OK;
}

// Admission: whenever events wait and a slot is free, take the events at the
// front of the queue that fit the memory budget beside what is in flight (up
// to max_batch) into that slot and launch them; completion runs on the
// slot's own thread, so staging one slot overlaps the device work and the
// result assembly of the others.
void admit_main(lst_ctx *ctx)
{
    (void)hipSetDevice(ctx->device);
    const uint32_t n_slots = (uint32_t)ctx->slots.size();
    const uint64_t budget = ctx->p.mem_budget ? ctx->p.mem_budget : (32ull << 30);
    std::unique_lock<std::mutex> lk(ctx->q_mu);
    while (true) {
        int slot = -1;
        auto ready = [&] {
            slot = -1;
            if (ctx->waiting.empty()) return ctx->stop;
            if (ctx->mem_in_use + ctx->waiting.front()->footprint > budget) return false;
            for (uint32_t i = 0; i < n_slots; i++)
                if (ctx->slot_state[i] == 0) { slot = (int)i; return true; }
            return false;
        };
        ctx->q_cv.wait(lk, ready);
        if (slot < 0) break;     // stopping with nothing left to admit
        std::vector<std::unique_ptr<ServedEvent>> take;
        uint64_t mem = 0;
        while (!ctx->waiting.empty() && take.size() < ctx->p.max_batch) {
            // every admitted event fits the budget with what is in flight
            // (an event alone always fits: submit refuses larger ones)
            const uint64_t f = ctx->waiting.front()->footprint;
            if (ctx->mem_in_use + mem + f > budget) break;
            mem += f;
            take.push_back(std::move(ctx->waiting.front()));
            ctx->waiting.pop_front();
        }
        ctx->mem_in_use += mem;
        ctx->slot_state[slot] = 1;
        lk.unlock();
        Slot &s = *ctx->slots[slot];
        s.tickets.resize(take.size());
        s.t_submit.resize(take.size());
        for (size_t k = 0; k < take.size(); k++) {
            s.tickets[k] = take[k]->ticket;
            s.t_submit[k] = take[k]->t_submit;
        }
        const lst_status st = stage_served(ctx, s, take);
        lk.lock();
        if (st != LST_OK) {
            for (auto &se : take) {
                ctx->in_chunks.put(se->chunk);
                lst_event_out *o = new_out();
                if (o) { o->status = (uint32_t)st; o->ticket = se->ticket; }
                ctx->finished[se->ticket] = o;
                ctx->state[se->ticket] = 2;
            }
            ctx->in_system -= take.size();
            ctx->mem_in_use -= mem;
            ctx->slot_state[slot] = 0;
            ctx->done_cv.notify_all();
            continue;
        }
        ctx->slot_mem[slot] = mem;
        ctx->held[slot] = std::move(take);
        ctx->slot_state[slot] = 2;
        ctx->slot_cv.notify_all();
    }
}

// Completion of slot i: wait for its launch (a blocking-sync event, no
// polling), re-run with larger lists if one overflowed, copy the results
// back and hand each event its output.
void complete_main(lst_ctx *ctx, uint32_t i)
{
    (void)hipSetDevice(ctx->device);
    Slot &s = *ctx->slots[i];
    std::unique_lock<std::mutex> lk(ctx->q_mu);
    while (true) {
        ctx->slot_cv.wait(lk, [&] { return ctx->stop_completers || ctx->slot_state[i] == 2; });
        if (ctx->slot_state[i] != 2) break;
        lk.unlock();
        lst_status st = LST_OK;
        const hipError_t he = hipEventSynchronize(s.done);
        if (he != hipSuccess) {
            fail(ctx, std::string("served batch: ") + hipGetErrorString(he));
            st = LST_ERR_DEVICE;
        }
        if (st == LST_OK) st = finish_run(ctx, s, false);
        s.n_regrow = 0;
        std::vector<lst_event_out *> outs(s.n_ev, nullptr);
        if (st == LST_OK && overflowed(s)) {
            if (s.work_arena) { (void)hipFree(s.work_arena); s.work_arena = nullptr; }
            if (s.gexec) { (void)hipGraphExecDestroy(s.gexec); s.gexec = nullptr; }
            if (s.graph) { (void)hipGraphDestroy(s.graph); s.graph = nullptr; }
            s.graph_valid = false;
            st = ensure_work(ctx, s);
            if (st == LST_OK) {
                st = run_staged(ctx, s, true, false, false);
                s.n_regrow++;
            }
        }
        if (st == LST_OK) st = download(ctx, s, outs.data());
        const auto now = std::chrono::steady_clock::now();
        auto &held = ctx->held[i];
        for (auto &se : held) {
            ctx->in_chunks.put(se->chunk);
            se->chunk = nullptr;
        }
        lk.lock();
        for (uint32_t e = 0; e < s.n_ev; e++) {
            lst_event_out *o = outs[e];
            if (!o) {
                o = new_out();
                if (o) o->status = (uint32_t)(st == LST_OK ? LST_ERR_DEVICE : st);
            }
            if (o) {
                o->ticket = s.tickets[e];
                o->footprint = e < held.size() ? held[e]->footprint : 0;
                o->latency_us = std::chrono::duration<double, std::micro>(now - s.t_submit[e]).count();
            }
            ctx->finished[s.tickets[e]] = o;
            ctx->state[s.tickets[e]] = 2;
        }
        ctx->in_system -= s.n_ev;
        ctx->mem_in_use -= ctx->slot_mem[i];
        ctx->slot_mem[i] = 0;
        held.clear();
        ctx->slot_state[i] = 0;
        ctx->q_cv.notify_all();
        ctx->done_cv.notify_all();
    }
}

}  // namespace

// ======================================================================
// C ABI
// ======================================================================
extern "C" {

void lst_default_params(lst_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->device = 0;
    p->B = 3.8;
    p->pt_min = 0.8;
    p->L = 15.0;
    p->sig_rphi = 30e-4;
    p->sig_c = 0.1;
    p->n_sigma = 3.0;
    p->flags = LST_FLAG_BEND;
    p->max_batch = 64;
    p->n_slots = 2;
    p->queue_depth = 1024;
    p->mem_budget = 0;
}

lst_status lst_create(const lst_params *p, lst_ctx **out)
{
    if (!out) return LST_ERR_INVALID_ARG;
    *out = nullptr;
    lst_params prm;
    if (p) prm = *p;
    else lst_default_params(&prm);
    if (prm.max_batch == 0 || prm.max_batch > 4096 || prm.n_slots == 0 || prm.n_slots > 8 ||
        prm.queue_depth == 0)
        return LST_ERR_INVALID_ARG;
    if ((prm.n_phi_bins != 0 && (prm.n_phi_bins < 4 || prm.n_phi_bins > 4096)) ||
        (prm.n_kappa_bins != 0 && (prm.n_kappa_bins < 2 || prm.n_kappa_bins > 128)))
        return LST_ERR_INVALID_ARG;
    if ((prm.ls_group != 0 && prm.ls_group != 4 && prm.ls_group != 6 && prm.ls_group != 8) ||
        (prm.ls_waves != 0 && prm.ls_waves != 6 && prm.ls_waves != 8))
        return LST_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || prm.device < 0 || prm.device >= ndev) return LST_ERR_DEVICE;
    if (hipSetDevice(prm.device) != hipSuccess) return LST_ERR_DEVICE;
    lst_ctx *ctx = new (std::nothrow) lst_ctx();
    if (!ctx) return LST_ERR_OOM;
    ctx->p = prm;
    ctx->device = prm.device;
    // the device address of the no-allocation workspace, once per device
    // (with the device current); a failure leaves only that entry point
    // unusable
    if (prm.device < kMaxDevices) {
        std::lock_guard<std::mutex> g(g_ws_mu);
        if (!g_ws[prm.device]) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e == hipSuccess && ptr) g_ws[prm.device] = ptr;
            else (void)hipGetLastError();
        }
        ctx->ws = g_ws[prm.device];
    }
    *out = ctx;
    return LST_OK;
}

lst_status lst_load_geometry(lst_ctx *ctx, const lst_module_desc *m, uint32_t n)
{
    TraceRange trace_("lst_load_geometry");
    lst_status st = check_ctx(ctx, false);
    if (st != LST_OK) return st;
    std::lock_guard<std::mutex> g(ctx->run_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    lst::Geometry geom;
    std::string err;
    bool from_cache = false;
    st = lst::build_geometry_cached(ctx->p, m, n, ctx->geom_cache, geom, err, from_cache);
    if (st != LST_OK) return set_err(ctx, st, err);
    // every bin, unit and bucket index of a batch of max_batch events is a
    // 32-bit number on the device
    {
        const lst::Consts &k = geom.c;
        const uint64_t bins = (uint64_t)ctx->p.max_batch * 2u * k.n_mod + 1u;
        const uint64_t bk = (uint64_t)ctx->p.max_batch * k.n_surf * k.nphi * (3u * k.nkb + 1u) + 1u;
        if (bins > 0xFFFFFFF0ull || bk > 0xFFFFFFF0ull)
            return set_err(ctx, LST_ERR_INVALID_ARG,
                           "max_batch x modules or x seed-lookup buckets exceeds 32-bit indexing");
    }
    // the served slots and the staged batch of the plain path hold arenas
    // sized for the old geometry: refuse while served events are in flight,
    // otherwise wait for the streams and drop the staged batch
    std::lock_guard<std::mutex> q(ctx->q_mu);
    if (ctx->in_system > 0)
        return set_err(ctx, LST_ERR_INVALID_ARG, "served events in flight: poll them before reloading the geometry");
    if (ctx->plain) {
        HIP_TRY(hipStreamSynchronize(ctx->plain->stream));
        HIP_TRY(hipStreamSynchronize(ctx->plain->side));
        ctx->plain->n_ev = 0;
    }
    for (auto &sl : ctx->slots) {
        HIP_TRY(hipStreamSynchronize(sl->stream));
        HIP_TRY(hipStreamSynchronize(sl->side));
        sl->n_ev = 0;
    }
    // device copy: one allocation
    const size_t nm = geom.n_mod, ne = geom.edge_dst.size(), nc = std::max<size_t>(geom.classes.size(), 1);
    const size_t ns = geom.surfaces.size();
    size_t off_kind = 0;
    size_t off_surf = lst::align_up(off_kind + 4 * nm);
    size_t off_mdc = lst::align_up(off_surf + 4 * nm);
    size_t off_eb = lst::align_up(off_mdc + 16 * nm);
    size_t off_edge = lst::align_up(off_eb + 4 * (nm + 1));
    size_t off_cls = lst::align_up(off_edge + 8 * std::max<size_t>(ne, 1));
    size_t off_sf = lst::align_up(off_cls + sizeof(lst::LsK) * nc);
    size_t off_phi = lst::align_up(off_sf + sizeof(lst::Surface) * std::max<size_t>(ns, 1));
    size_t off_ext = lst::align_up(off_phi + 8 * nm);
    const size_t nr = geom.run_win.size();
    size_t off_rb = lst::align_up(off_ext + 32 * nm);
    size_t off_run = lst::align_up(off_rb + 4 * (nm + 1));
    size_t off_rw = lst::align_up(off_run + 16 * std::max<size_t>(nr, 1));
    size_t total = lst::align_up(off_rw + 4 * std::max<size_t>(nr, 1));
    std::vector<char> host(total, 0);
    std::memcpy(&host[off_kind], geom.kind.data(), 4 * nm);
    std::memcpy(&host[off_surf], geom.surf.data(), 4 * nm);
    std::memcpy(&host[off_mdc], geom.mdc.data(), 16 * nm);
    std::memcpy(&host[off_eb], geom.edge_begin.data(), 4 * (nm + 1));
    for (size_t i = 0; i < ne; i++) {
        uint32_t v[2] = {geom.edge_dst[i], geom.edge_cls[i]};
        std::memcpy(&host[off_edge + 8 * i], v, 8);
    }
    for (size_t i = 0; i < geom.classes.size(); i++) {
        const lst::LsClass &k = geom.classes[i];
        // v[6]: the largest azimuth difference of the anchors, asin(S), plus
        // the map's margin and room for the binary32 arithmetic of the
        // per-segment reach test
        float v[8] = {k.S, 0.f, 0.f, 0.f, 0.f, 0.f, lst::ls_reach(k), 0.f};
        if (k.type == 0u) {
            v[1] = k.rho_lo; v[2] = k.rho_hi; v[3] = k.lam_lo; v[4] = k.lam_hi; v[5] = k.tau;
        } else if (k.type == 1u) {
            v[1] = k.lo_fac; v[2] = k.hi_fac;
        } else {
            v[1] = k.cf; v[2] = k.zs; v[3] = k.zbpl; v[4] = k.zbml;
        }
        std::memcpy(&v[7], &k.type, 4);
        std::memcpy(&host[off_cls + sizeof(lst::LsK) * i], v, sizeof v);
    }
    if (ns) std::memcpy(&host[off_sf], geom.surfaces.data(), sizeof(lst::Surface) * ns);
    std::memcpy(&host[off_phi], geom.mod_phi.data(), 8 * nm);
    std::memcpy(&host[off_ext], geom.mod_ext.data(), 32 * nm);
    std::memcpy(&host[off_rb], geom.run_begin.data(), 4 * (nm + 1));
    if (nr) {
        std::memcpy(&host[off_run], geom.run_rec.data(), 16 * nr);
        std::memcpy(&host[off_rw], geom.run_win.data(), 4 * nr);
    }
    void *dmem = nullptr;
    if (hipMalloc(&dmem, total) != hipSuccess) return set_err(ctx, LST_ERR_OOM, "geometry allocation failed");
    hipError_t e = hipMemcpy(dmem, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dmem);
        fail(ctx, std::string("geometry upload: ") + hipGetErrorString(e));
        return LST_ERR_DEVICE;
    }
    if (ctx->geom_mem) (void)hipFree(ctx->geom_mem);
    ctx->geom_mem = dmem;
    char *d = (char *)dmem;
    ctx->dg.mod_kind = (const uint32_t *)(d + off_kind);
    ctx->dg.mod_surf = (const uint32_t *)(d + off_surf);
    ctx->dg.mdc = (const float4 *)(d + off_mdc);
    ctx->dg.edge_begin = (const uint32_t *)(d + off_eb);
    ctx->dg.edge = (const uint2 *)(d + off_edge);
    ctx->dg.cls = (const lst::LsK *)(d + off_cls);
    ctx->dg.surf = (const lst::Surface *)(d + off_sf);
    ctx->dg.mod_phi = (const float2 *)(d + off_phi);
    ctx->dg.mod_ext = (const float4 *)(d + off_ext);
    ctx->dg.run_begin = (const uint32_t *)(d + off_rb);
    ctx->dg.run = (const uint4 *)(d + off_run);
    ctx->dg.run_win = (const float *)(d + off_rw);
    // the hit histogram runs per event in LDS, in slices of the event's
    // (module, sensor) bins that fit one block's LDS
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) != hipSuccess ||
        lds_max < 65536)
        lds_max = 65536;   // every CDNA workgroup has at least 64 KiB of LDS
    ctx->dg.hist_slice =
        (uint32_t)std::min<int64_t>((int64_t)lds_max / 4 / 256 * 256, 2 * (int64_t)geom.n_mod);
    ctx->geom = std::move(geom);
    ctx->has_geom = true;
    ctx->geom_from_cache = from_cache;
    // arenas depend on the module count
    if (ctx->plain) free_slot_arenas(*ctx->plain);
    for (auto &s : ctx->slots) free_slot_arenas(*s);
    return LST_OK;
}

lst_status lst_get_connection_map(lst_ctx *ctx, const uint32_t **begin, const uint32_t **dst, uint32_t *n_edges)
{
    if (!ctx || !begin || !dst || !n_edges) return LST_ERR_INVALID_ARG;
    if (!ctx->has_geom) return set_err(ctx, LST_ERR_NO_GEOMETRY, "no geometry loaded");
    *begin = ctx->geom.edge_begin.data();
    *dst = ctx->geom.edge_dst.data();
    *n_edges = (uint32_t)ctx->geom.edge_dst.size();
    return LST_OK;
}

lst_status lst_set_geometry_cache(lst_ctx *ctx, const char *dir)
{
    if (!ctx) return LST_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(ctx->run_mu);
    ctx->geom_cache = dir ? dir : "";
    return LST_OK;
}

int32_t lst_geometry_from_cache(const lst_ctx *ctx) { return ctx && ctx->geom_from_cache ? 1 : 0; }

lst_status lst_build_connection_map(const lst_params *p, const lst_module_desc *m, uint32_t n,
                                    uint32_t **begin, uint32_t **dst, uint32_t *n_edges)
{
    if (!begin || !dst || !n_edges) return LST_ERR_INVALID_ARG;
    lst_params prm;
    if (p) prm = *p;
    else lst_default_params(&prm);
    lst::Geometry g;
    std::string err;
    lst_status st = lst::build_geometry(prm, m, n, g, err);
    if (st != LST_OK) return st;
    *begin = (uint32_t *)std::malloc(4 * (g.n_mod + 1));
    *dst = (uint32_t *)std::malloc(4 * std::max<size_t>(g.edge_dst.size(), 1));
    if (!*begin || !*dst) {
        std::free(*begin); std::free(*dst);
        *begin = *dst = nullptr;
        return LST_ERR_OOM;
    }
    std::memcpy(*begin, g.edge_begin.data(), 4 * (g.n_mod + 1));
    if (!g.edge_dst.empty()) std::memcpy(*dst, g.edge_dst.data(), 4 * g.edge_dst.size());
    *n_edges = (uint32_t)g.edge_dst.size();
    return LST_OK;
}

void lst_free_map(uint32_t *begin, uint32_t *dst)
{
    std::free(begin);
    std::free(dst);
}

lst_status lst_run_batch(lst_ctx *ctx, const lst_event_in *evs, uint32_t n, lst_event_out **outs)
{
    TraceRange trace_("lst_run_batch");
    lst_status st = check_ctx(ctx, true);
    if (st != LST_OK) return st;
    if (!evs || !outs || n == 0) return set_err(ctx, LST_ERR_INVALID_ARG, "no events");
    if (n > ctx->p.max_batch) return set_err(ctx, LST_ERR_INVALID_ARG, "more events than max_batch");
    std::lock_guard<std::mutex> g(ctx->run_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    st = ensure_plain(ctx);
    if (st != LST_OK) return st;
    Slot &s = *ctx->plain;
    st = stage_inputs(ctx, s, evs, n);
    if (st != LST_OK) return st;
    st = run_staged(ctx, s, true, (ctx->p.flags & LST_FLAG_STAGE_TIMES) != 0, true);
    if (st != LST_OK) return st;
    for (uint32_t i = 0; i < n; i++) outs[i] = nullptr;
    st = download(ctx, s, outs);
    if (st != LST_OK) {
        for (uint32_t i = 0; i < n; i++) { lst_free_output(outs[i]); outs[i] = nullptr; }
    }
    return st;
}

lst_status lst_run_event(lst_ctx *ctx, const lst_event_in *ev, lst_event_out **out)
{
    if (!ev || !out) return LST_ERR_INVALID_ARG;
    return lst_run_batch(ctx, ev, 1, out);
}

lst_status lst_batch_upload(lst_ctx *ctx, const lst_event_in *evs, uint32_t n)
{
    lst_status st = check_ctx(ctx, true);
    if (st != LST_OK) return st;
    if (!evs || n == 0) return set_err(ctx, LST_ERR_INVALID_ARG, "no events");
    if (n > ctx->p.max_batch) return set_err(ctx, LST_ERR_INVALID_ARG, "more events than max_batch");
    std::lock_guard<std::mutex> g(ctx->run_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    st = ensure_plain(ctx);
    if (st != LST_OK) return st;
    Slot &s = *ctx->plain;
    st = stage_inputs(ctx, s, evs, n);
    if (st != LST_OK) return st;
    HIP_TRY(hipStreamSynchronize(s.stream));
    // size the work arena with one untimed run
    return run_staged(ctx, s, false, false, true);
}

lst_status lst_batch_execute(lst_ctx *ctx, uint32_t repeats, int32_t use_graph, int32_t timing, double *ms)
{
    TraceRange trace_("lst_batch_execute");
    lst_status st = check_ctx(ctx, true);
    if (st != LST_OK) return st;
    if (!ctx->plain || !ctx->plain->n_ev) return set_err(ctx, LST_ERR_INVALID_ARG, "no staged batch");
    std::lock_guard<std::mutex> g(ctx->run_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    Slot &s = *ctx->plain;
    if (timing) ctx->ktimes.clear();
    s.L.only = ctx->time_only.empty() ? nullptr : ctx->time_only.c_str();
    auto drain = [&]() { drain_records(ctx, s); };
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s.stream));
    for (uint32_t r = 0; r < repeats; r++) {
        st = enqueue(ctx, s, use_graph != 0, timing != 0, false);
        if (st != LST_OK) break;
        if (timing && !s.L.only) {
            // every launch timed: drain each repeat so the event pool stays small
            HIP_TRY(hipStreamSynchronize(s.stream));
            drain();
        }
    }
    HIP_TRY(hipEventRecord(e1, s.stream));
    HIP_TRY(hipEventSynchronize(e1));
    if (timing) drain();
    s.L.only = nullptr;
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms) *ms = t;
    if (st != LST_OK) return st;
    s.L.timing = false;
    st = finish_run(ctx, s, true);
    if (st != LST_OK) return st;
    if (overflowed(s)) return set_err(ctx, LST_ERR_OOM, "object list overflow during execute");
    return LST_OK;
}

lst_status lst_time_only(lst_ctx *ctx, const char *name)
{
    if (!ctx) return LST_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(ctx->run_mu);
    ctx->time_only = name ? name : "";
    return LST_OK;
}

lst_status lst_kernel_times(lst_ctx *ctx, const char **names, double *total_ms, uint32_t *launches, uint32_t *n)
{
    if (!ctx || !n) return LST_ERR_INVALID_ARG;
    uint32_t cap = *n, k = 0;
    for (auto &kv : ctx->ktimes) {
        if (k < cap) {
            if (names) {
                // names point at string literals of the launch sites
                static thread_local std::vector<std::string> keep;
                if (keep.size() < cap) keep.resize(cap);
                keep[k] = kv.first;
                names[k] = keep[k].c_str();
            }
            if (total_ms) total_ms[k] = kv.second.first;
            if (launches) launches[k] = kv.second.second;
        }
        k++;
    }
    *n = std::min(k, cap);
    return LST_OK;
}

lst_status lst_batch_download(lst_ctx *ctx, lst_event_out **outs)
{
    lst_status st = check_ctx(ctx, true);
    if (st != LST_OK) return st;
    if (!outs || !ctx->plain || !ctx->plain->n_ev) return set_err(ctx, LST_ERR_INVALID_ARG, "no staged batch");
    std::lock_guard<std::mutex> g(ctx->run_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    return download(ctx, *ctx->plain, outs);
}

lst_status lst_batch_counts(lst_ctx *ctx, uint64_t counts[15])
{
    if (!ctx || !counts) return LST_ERR_INVALID_ARG;
    if (!ctx->plain || !ctx->plain->n_ev) return set_err(ctx, LST_ERR_INVALID_ARG, "no staged batch");
    std::lock_guard<std::mutex> g(ctx->run_mu);
    Slot &s = *ctx->plain;
    // re-run once with candidate statistics
    HIP_TRY(hipSetDevice(ctx->device));
    lst_status st = enqueue(ctx, s, false, false, true);
    if (st != LST_OK) return st;
    st = finish_run(ctx, s, true);
    if (st != LST_OK) return st;
    const lst::Totals &t = *s.h_tot;
    const uint64_t v[15] = {t.n_md, t.n_ls, t.n_t3, t.n_t5, t.n_pt3, t.n_pt5, t.n_tc + t.n_pt5,
                            t.cand[0], t.cand[1], t.cand[2], t.cand[3], t.cand[4], t.cand[5],
                            t.n_ptc3, t.n_ptc5};
    std::memcpy(counts, v, sizeof v);
    return LST_OK;
}

lst_status lst_submit(lst_ctx *ctx, const lst_event_in *ev, uint64_t *ticket)
{
    TraceRange trace_("lst_submit");
    lst_status st = check_ctx(ctx, true);
    if (st != LST_OK) return st;
    if (!ev || !ticket) return LST_ERR_INVALID_ARG;
    st = check_event(ctx, *ev);
    if (st != LST_OK) return st;
    if (ev->flags & LST_DEVICE_PTRS) return set_err(ctx, LST_ERR_INVALID_ARG, "served events take host pointers");
    if (ev->n_hits >= (1u << 28) || ev->n_pls >= (1u << 26))
        return set_err(ctx, LST_ERR_TOO_LARGE, "event above the served path's size limits");
    // the event is copied once, into a pinned block that the device reads
    auto se = std::make_unique<ServedEvent>();
    se->n_hits = ev->n_hits;
    se->n_pls = ev->n_pls;
    const lst::BlockLayout lay = lst::served_block_layout(ev->n_hits, ev->n_pls);
    se->blk_bytes = lay.bytes;
    if (lay.bytes) {
        if (!ctx->in_chunks.get(lay.bytes, se->chunk, se->blk_off))
            return set_err(ctx, LST_ERR_OOM, "pinned host allocation failed");
        char *blk = se->chunk->base + se->blk_off;
        const void *src[8] = {ev->x, ev->y, ev->z, ev->module, ev->sensor, ev->pls_par, ev->pls_cov, ev->pls_nhits};
        const size_t sz[8] = {4ull * ev->n_hits, 4ull * ev->n_hits, 4ull * ev->n_hits, 4ull * ev->n_hits,
                              ev->n_hits, 20ull * ev->n_pls, 60ull * ev->n_pls, ev->n_pls};
        for (int i = 0; i < 7; i++)
            if (sz[i]) std::memcpy(blk + lay.off[i], src[i], sz[i]);
        // seed hit counts, or every seed a quad
        if (sz[7]) {
            if (src[7]) std::memcpy(blk + lay.off[7], src[7], sz[7]);
            else std::memset(blk + lay.off[7], 4, sz[7]);
        }
    }
    se->t_submit = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> g(ctx->q_mu);
    auto give_back = [&] { ctx->in_chunks.put(se->chunk); se->chunk = nullptr; };
    const uint64_t budget = ctx->p.mem_budget ? ctx->p.mem_budget : (32ull << 30);
    const uint64_t f = predict_footprint(ev->n_hits, ev->n_pls, ctx->geom.c);
    if (f > budget) { give_back(); return set_err(ctx, LST_ERR_TOO_LARGE, "event above the device memory budget"); }
    se->footprint = f;
    if (ctx->in_system >= ctx->p.queue_depth) { give_back(); return set_err(ctx, LST_ERR_QUEUE_FULL, "queue full"); }
    if (!ctx->worker_started) {
        ctx->slots.clear();
        for (uint32_t i = 0; i < ctx->p.n_slots; i++) {
            std::unique_ptr<Slot> sl;
            st = make_slot(ctx, sl);
            if (st != LST_OK) { give_back(); return st; }
            ctx->slots.push_back(std::move(sl));
        }
        ctx->slot_state.assign(ctx->p.n_slots, 0);
        ctx->slot_mem.assign(ctx->p.n_slots, 0);
        ctx->held.clear();
        ctx->held.resize(ctx->p.n_slots);
        ctx->worker = std::thread(admit_main, ctx);
        for (uint32_t i = 0; i < ctx->p.n_slots; i++) ctx->completers.emplace_back(complete_main, ctx, i);
        ctx->worker_started = true;
    }
    se->ticket = ctx->next_ticket++;
    *ticket = se->ticket;
    ctx->state[se->ticket] = 1;
    ctx->in_system++;
    ctx->waiting.push_back(std::move(se));
    ctx->q_cv.notify_all();
    return LST_OK;
}

lst_status lst_poll(lst_ctx *ctx, uint64_t ticket, int64_t timeout_us, lst_event_out **out)
{
    if (!ctx || !out) return LST_ERR_INVALID_ARG;
    *out = nullptr;
    std::unique_lock<std::mutex> lk(ctx->q_mu);
    auto it = ctx->state.find(ticket);
    if (it == ctx->state.end()) return set_err(ctx, LST_ERR_UNKNOWN_TICKET, "unknown or consumed ticket");
    auto ready = [&] { return ctx->state[ticket] == 2; };
    if (!ready()) {
        if (timeout_us == 0) return LST_PENDING;
        if (timeout_us < 0) ctx->done_cv.wait(lk, ready);
        else if (!ctx->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return LST_PENDING;
    }
    lst_event_out *o = ctx->finished[ticket];
    ctx->finished.erase(ticket);
    ctx->state.erase(ticket);
    *out = o;
    if (!o) return LST_ERR_OOM;
    if (o->status != (uint32_t)LST_OK) return (lst_status)(int32_t)o->status;
    return LST_OK;
}

lst_status lst_run_event_noalloc(lst_ctx *ctx, const lst_event_in *ev, lst_event_dev_out *out, void *stream)
{
    TraceRange trace_("lst_run_event_noalloc");
    lst_status st = check_ctx(ctx, true);
    if (st != LST_OK) return st;
    if (!ev || !out) return set_err(ctx, LST_ERR_INVALID_ARG, "null event or output");
    if (!(ev->flags & LST_DEVICE_PTRS)) return set_err(ctx, LST_ERR_INVALID_ARG, "inputs must be device pointers");
    st = check_event(ctx, *ev);
    if (st != LST_OK) return st;
    if (!ctx->ws) return set_err(ctx, LST_ERR_DEVICE, "no-allocation workspace unavailable on this device");
    if (ev->n_hits > LST_NOALLOC_MAX_HITS || ev->n_pls > LST_NOALLOC_MAX_PLS)
        return set_err(ctx, LST_ERR_TOO_LARGE, "event above the no-allocation workspace's limits");
    std::lock_guard<std::mutex> run(g_ws_run_mu[ctx->device]);
    HIP_TRY(hipSetDevice(ctx->device));
    const hipStream_t sm = (hipStream_t)stream;
    const lst::Consts &k = ctx->geom.c;
    // fixed part of the workspace: counters, scan partials, event offsets
    char *ws = (char *)ctx->ws;
    lst::Totals *d_tot = (lst::Totals *)ws;
    uint32_t *part = (uint32_t *)(ws + lst::align_up(sizeof(lst::Totals)));
    uint32_t *offs = part + lst::kScanGrid;
    const size_t fixed = lst::align_up(sizeof(lst::Totals)) + lst::align_up(4ull * lst::kScanGrid + 16);
    Batch b{};
    b.cap_ev = 1;
    b.cap_hits = std::max<uint32_t>(ev->n_hits, 1);
    b.cap_pls = std::max<uint32_t>(ev->n_pls, 1);
    b.in_x = const_cast<float *>(ev->x);
    b.in_y = const_cast<float *>(ev->y);
    b.in_z = const_cast<float *>(ev->z);
    b.in_mod = const_cast<uint32_t *>(ev->module);
    b.in_sen = const_cast<uint8_t *>(ev->sensor);
    b.in_par = const_cast<float *>(ev->pls_par);
    b.in_cov = const_cast<float *>(ev->pls_cov);
    b.ev_hit_off = offs;
    b.ev_pls_off = offs + 2;
    lst::Caps c = lst::plan_caps(1, ev->n_hits, ev->n_pls);
    b.cap_md = c.md; b.cap_ls = c.ls; b.cap_t3 = c.t3; b.cap_t5 = c.t5;
    b.cap_pt3 = c.pt3; b.cap_pt5 = c.pt5; b.cap_ptc3 = c.ptc3; b.cap_ptc5 = c.ptc5;
    lst::plan_sublists(b);
    lst::Launcher L;
    L.stream = sm;
    L.side = nullptr;
    L.cur = sm;
    L.part = part;
    lst::Totals tot{};
    for (int attempt = 0;; attempt++) {
        b.cap_tc = b.cap_pt3 + b.cap_t5 + b.cap_pls;
        lst::Carver cw{nullptr};
        lst::carve_work(cw, b, k.n_mod, k.n_surf, k.nphi, k.nkb);
        if (fixed + cw.off > kScratchBytes || attempt >= 6)
            return set_err(ctx, LST_ERR_TOO_LARGE,
                           "object lists of this event do not fit the no-allocation workspace (" +
                               std::to_string((fixed + cw.off) >> 20) + " MiB needed)");
        lst::Carver cw2{ws + fixed};
        lst::carve_work(cw2, b, k.n_mod, k.n_surf, k.nphi, k.nkb);
        lst::launch_event_init(L, b, d_tot, ev->n_hits, ev->n_pls);
        lst::enqueue_chain(L, b, d_tot, ctx->dg, k, 0);
        if (L.err != hipSuccess) {
            fail(ctx, std::string("kernel launch: ") + hipGetErrorString(L.err));
            return LST_ERR_DEVICE;
        }
        HIP_TRY(hipMemcpyAsync(&tot, d_tot, sizeof tot, hipMemcpyDeviceToHost, sm));
        HIP_TRY(hipStreamSynchronize(sm));
        st = input_error(ctx, tot.err);
        if (st != LST_OK) return st;
        // a list that overflowed: larger capacities inside the same workspace
        if (!lst::grow_caps(b, tot)) break;
    }
    out->n_md = tot.n_md; out->n_ls = tot.n_ls; out->n_t3 = tot.n_t3; out->n_t5 = tot.n_t5;
    out->n_pt3 = tot.n_pt3; out->n_pt5 = tot.n_pt5; out->n_tc = tot.n_pt5 + tot.n_tc;
    if (out->n_md > out->cap_md || out->n_ls > out->cap_ls || out->n_t3 > out->cap_t3 ||
        out->n_t5 > out->cap_t5 || out->n_pt3 > out->cap_pt3 || out->n_pt5 > out->cap_pt5 ||
        out->n_tc > out->cap_tc)
        return set_err(ctx, LST_ERR_TOO_LARGE, "output buffers too small (the counts give the sizes needed)");
    const uint64_t items = (uint64_t)out->n_md + out->n_ls + out->n_t3 + out->n_t5 + out->n_pt3 + out->n_pt5 +
                           out->n_tc;
    if ((out->n_md && !out->md) || (out->n_ls && !out->ls) || (out->n_t3 && !out->t3) || (out->n_t5 && !out->t5) ||
        (out->n_pt3 && !out->pt3) || (out->n_pt5 && !out->pt5) || (out->n_tc && !out->tc))
        return set_err(ctx, LST_ERR_INVALID_ARG, "null output buffer");
    if (items) {
        const lst::EventOut o{out->md, out->ls, out->t3, out->t5, out->pt3, out->pt5, out->tc, out->t3_kappa};
        lst::launch_event_out(L, b, d_tot, o, items);
        if (L.err != hipSuccess) {
            fail(ctx, std::string("kernel launch: ") + hipGetErrorString(L.err));
            return LST_ERR_DEVICE;
        }
        HIP_TRY(hipStreamSynchronize(sm));
    }
    return LST_OK;
}

void lst_free_output(lst_event_out *out)
{
    if (!out) return;
    OutBox *b = (OutBox *)out;
    if (b->batch) b->batch->unref();
    std::free(b);
}

void lst_destroy(lst_ctx *ctx)
{
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> g(ctx->q_mu);
        ctx->stop = true;
        ctx->q_cv.notify_all();
    }
    // the admission thread ends once nothing waits; the completion threads
    // once every slot has been handed back
    if (ctx->worker.joinable()) ctx->worker.join();
    {
        std::unique_lock<std::mutex> lk(ctx->q_mu);
        ctx->done_cv.wait(lk, [&] {
            return std::all_of(ctx->slot_state.begin(), ctx->slot_state.end(), [](int v) { return v == 0; });
        });
        ctx->stop_completers = true;
        ctx->slot_cv.notify_all();
    }
    for (auto &th : ctx->completers)
        if (th.joinable()) th.join();
    for (auto &kv : ctx->waiting) ctx->in_chunks.put(kv->chunk);
    for (auto &kv : ctx->finished) lst_free_output(kv.second);
    (void)hipSetDevice(ctx->device);
    for (auto &s : ctx->slots) destroy_slot(*s);
    if (ctx->plain) destroy_slot(*ctx->plain);
    if (ctx->geom_mem) (void)hipFree(ctx->geom_mem);
    ctx->in_chunks.release();
    delete ctx;
}

const char *lst_status_str(lst_status s)
{
    switch (s) {
    case LST_OK: return "ok";
    case LST_PENDING: return "pending";
    case LST_ERR_INVALID_ARG: return "invalid argument";
    case LST_ERR_DEVICE: return "device error";
    case LST_ERR_NO_GEOMETRY: return "no geometry loaded";
    case LST_ERR_BAD_GEOMETRY: return "bad geometry";
    case LST_ERR_BAD_MODULE: return "hit with bad module id or sensor";
    case LST_ERR_NONFINITE: return "non-finite input";
    case LST_ERR_OOM: return "out of memory";
    case LST_ERR_TOO_LARGE: return "event too large";
    case LST_ERR_QUEUE_FULL: return "queue full";
    case LST_ERR_UNKNOWN_TICKET: return "unknown ticket";
    case LST_ERR_HIT_OUTSIDE: return "hit outside its module or off its sensor";
    default: return "unknown status";
    }
}

const char *lst_last_error(const lst_ctx *ctx)
{
    if (!ctx) return "null context";
    static thread_local std::string copy;
    std::lock_guard<std::mutex> g(ctx->err_mu);
    copy = ctx->last_error;
    return copy.c_str();
}

}  // extern "C"
