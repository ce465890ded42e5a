// kernels.hip -- gfx950 kernels of the Line Segment Tracking chain.
//
// Every stage follows count -> device-wide exclusive scan -> fill, so each
// object list comes out compacted and in canonical order without global
// atomics on the output path, and a stage's scan doubles as the CSR index the
// next stage walks:
//   hits sorted by (event, module, sensor)          -> per-module hit ranges
//   MDs per (event, module)                          -> per-module MD ranges
//   LSs per inner MD                                 -> "segments starting at MD b"
//   T3s per inner LS (hence grouped by inner MD)     -> "T3s starting at MD c"
//   T5s per inner T3; pT3 / pT5 per pixel seed.
// A batch of events is one flat index space (event-major), so one launch of
// the chain serves any number of events.  Unit counts live in device memory
// (struct Totals) and kernels walk them with grid-stride loops: the launch
// sequence is independent of the data and can be captured in a hipGraph.
//
// Cut arithmetic: IEEE binary32 with the expression order written out below
// (no contraction: built with -ffp-contract=off), pixel-seed cuts in binary64.
#include <hip/hip_runtime.h>

#include <functional>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "engine.h"

namespace lst {

// ------------------------------------------------------------------ scan ---

constexpr int kScanBlock = 256;
constexpr int kScanTile = 4 * kScanBlock;
constexpr float kPiF = 3.14159265358979f;
constexpr double kPiD = 3.14159265358979323846;

// inclusive prefix sum across a wave: row shifts by 1, 2, 4, 8 within each
// row of 16 lanes, then the last lane of rows 0 / 2 broadcast into rows 1 / 3
// and the last lane of row 1 into rows 2 and 3 (register-to-register, no
// LDS round trip; lanes a shift cannot reach add 0)
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
    return v;
}

// the value of lane 63 in every lane (a scalar read, no LDS)
__device__ inline uint32_t wave_last(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 63); }

// exclusive scan of one value per thread across a 256-thread block
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t &total)
{
    __shared__ uint32_t ws[kScanBlock / 64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kScanBlock / 64; i++) {
        uint32_t t = ws[i];
        off += (i < w) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

// values per block: whole tiles, nb blocks covering n
__device__ inline uint32_t scan_chunk(uint32_t n, uint32_t nb)
{
    uint32_t per = (n + nb - 1) / nb;
    return (per + kScanTile - 1) / kScanTile * kScanTile;
}

// Two-kernel scan: every block sums a chunk (whole tiles of kScanTile
// values, four per thread as one 16-byte load); then every block sums the
// partial sums of the blocks before it (at most kScanGrid, from L2) for its
// carry and scans its chunk again, and the last block writes the total.
__device__ inline void scan_up_block(const uint32_t *__restrict__ in, const uint32_t *n_ptr, uint32_t cap,
                                     uint32_t *__restrict__ part, uint32_t nblocks, uint32_t bid)
{
    const uint32_t n = min(*n_ptr, cap);
    const uint32_t chunk = scan_chunk(n, nblocks);
    const uint32_t start = min(bid * chunk, n);
    const uint32_t end = min(start + chunk, n);
    uint32_t s = 0;
    for (uint32_t base = start; base < end; base += kScanTile) {
        const uint32_t i = base + 4 * threadIdx.x;
        if (i + 3 < end) {
            const uint4 v = *reinterpret_cast<const uint4 *>(in + i);
            s += (v.x + v.y) + (v.z + v.w);
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (i + k < end) s += in[i + k];
        }
    }
    uint32_t tot;
    block_excl_scan(s, tot);
    if (threadIdx.x == 0) part[bid] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_up(const uint32_t *__restrict__ in,
                                                        const uint32_t *n_ptr, uint32_t cap,
                                                        uint32_t *__restrict__ part)
{
    scan_up_block(in, n_ptr, cap, part, gridDim.x, blockIdx.x);
}

__global__ __launch_bounds__(kScanBlock) void k_scan_down(const uint32_t *__restrict__ in,
                                                          const uint32_t *n_ptr, uint32_t cap,
                                                          const uint32_t *__restrict__ part,
                                                          uint32_t *__restrict__ out,
                                                          uint32_t *total_out)
{
    const uint32_t n = min(*n_ptr, cap);
    const uint32_t chunk = scan_chunk(n, gridDim.x);
    const uint32_t start = min(blockIdx.x * chunk, n);
    const uint32_t end = min(start + chunk, n);
    uint32_t before = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanBlock) before += part[i];
    uint32_t carry;
    block_excl_scan(before, carry);
    for (uint32_t base = start; base < end; base += kScanTile) {
        const uint32_t i = base + 4 * threadIdx.x;
        const bool full = i + 3 < end;
        uint32_t v[4];
        if (full) {
            const uint4 q = *reinterpret_cast<const uint4 *>(in + i);
            v[0] = q.x;
            v[1] = q.y;
            v[2] = q.z;
            v[3] = q.w;
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++) v[k] = (i + k < end) ? in[i + k] : 0u;
        }
        const uint32_t s = (v[0] + v[1]) + (v[2] + v[3]);
        uint32_t tot;
        uint32_t ex = block_excl_scan(s, tot) + carry;
        uint32_t o[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            o[k] = ex;
            ex += v[k];
        }
        if (full) {
            *reinterpret_cast<uint4 *>(out + i) = make_uint4(o[0], o[1], o[2], o[3]);
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (i + k < end) out[i + k] = o[k];
        }
        carry += tot;
    }
    if (blockIdx.x == gridDim.x - 1u && threadIdx.x == 0) {
        out[n] = carry;
        *total_out = carry;
    }
}

// --------------------------------------------------------------- helpers ---

#define GRID_STRIDE(i, n) \
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += gridDim.x * blockDim.x)

// Grid-stride loop over [0, n) in which the blocks of each XCD take one
// contiguous eighth (workgroups are dealt to the eight XCDs in turn), so
// that the region of the output a kernel scatters into from that eighth
// stays in one XCD's L2, where partial lines are merged before they go to
// HBM.  Grids that are not a multiple of eight stride as usual.
constexpr uint32_t kXcds = 8;
struct XcdRange {
    uint32_t first, end, stride;
};
__device__ inline XcdRange xcd_range(uint32_t n)
{
    const uint32_t g = gridDim.x;
    if (g < kXcds || g % kXcds != 0u)
        return {blockIdx.x * blockDim.x + threadIdx.x, n, g * blockDim.x};
    const uint32_t x = blockIdx.x % kXcds;
    const uint32_t part = (n + kXcds - 1u) / kXcds;
    const uint32_t lo = min(x * part, n), hi = min(lo + part, n);
    return {lo + (blockIdx.x / kXcds) * blockDim.x + threadIdx.x, hi, (g / kXcds) * blockDim.x};
}
#define XCD_STRIDE(i, n) \
    for (XcdRange xr_ = xcd_range(n); xr_.first < xr_.end; xr_.first = xr_.end) \
        for (uint32_t i = xr_.first; i < xr_.end; i += xr_.stride)
// the same with whole blocks per step: jb is the block's first index (the
// same on every lane); a lane's index jb + threadIdx.x is in range below
// xb_.end
#define XCD_STRIDE_BLOCKS(jb, n) \
    for (XcdRange xb_ = xcd_range(n); xb_.first - threadIdx.x < xb_.end; xb_.first = xb_.end + threadIdx.x) \
        for (uint32_t jb = xb_.first - threadIdx.x; jb < xb_.end; jb += xb_.stride)

__device__ inline uint32_t find_event(const uint32_t *__restrict__ off, uint32_t n_ev, uint32_t i)
{
    uint32_t lo = 0, hi = n_ev;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// dense index j (< total) of a list split into block regions to its slot:
// the region s with soff[s] <= j < soff[s + 1], s < nsub
__device__ inline uint32_t pair_slot(const uint32_t *s_off, uint32_t j, uint32_t subcap, uint32_t nsub)
{
    uint32_t lo = 0, hi = nsub;
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_off[mid] <= j) lo = mid;
        else hi = mid;
    }
    return lo * subcap + (j - s_off[lo]);
}

// The entries of a list split into block regions (nsub regions of subcap
// slots; soff[r + 1] - soff[r] entries filled in region r, from
// k_sub_offsets): a block per region, its threads over the region's slots,
// so no entry searches for its region.  For lists whose regions are even
// (the seed-pair lists: every walk block took several tiles); the others
// keep the dense grid-stride order with pair_slot, which balances uneven
// regions.
#define REGION_ENTRIES(i, soff, subcap, nsub)                                              \
    for (uint32_t rg_ = blockIdx.x; rg_ < (nsub); rg_ += gridDim.x)                        \
        for (uint32_t q_ = threadIdx.x, cnt_ = (soff)[rg_ + 1] - (soff)[rg_]; q_ < cnt_;   \
             q_ += blockDim.x)                                                             \
            for (uint32_t i = rg_ * (subcap) + q_, once_ = 1; once_; once_ = 0)

// One increment of cnt[key] per active lane with one atomic per distinct
// key of the wave: the lanes sharing a key are ranked by lane order behind
// the first of them, whose single add covers them all (every lane of the
// wave calls it).  Returns the lane's slot among the key's increments.
__device__ inline uint32_t wave_grouped_inc(uint32_t *cnt, uint32_t key, bool active)
{
    const uint32_t lane = threadIdx.x & 63u;
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long todo = __ballot(active);
    uint32_t leader = lane, rank = 0, count = 0;
    while (todo != 0ull) {
        const uint32_t l = (uint32_t)__ffsll(todo) - 1u;
        const uint32_t lk = __shfl(key, l);
        const unsigned long long peers = __ballot(active && key == lk) & todo;
        if ((peers >> lane) & 1ull) {
            leader = l;
            rank = (uint32_t)__popcll(peers & below);
        }
        if (lane == l) count = (uint32_t)__popcll(peers);
        todo &= ~peers;
    }
    uint32_t base = 0;
    if (active && leader == lane) base = atomicAdd(&cnt[key], count);
    return __shfl(base, leader) + rank;
}

// lanes s0 .. e0 - 1 of a wave (0 <= s0 <= e0 <= 64)
__device__ inline unsigned long long lane_range(uint32_t s0, uint32_t e0)
{
    const unsigned long long hi = e0 >= 64u ? ~0ull : (1ull << e0) - 1ull;
    return hi & ~((1ull << s0) - 1ull);
}

// orders a wave's LDS accesses (all lanes of one wave; no block barrier)
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// inclusive prefix maximum across a wave (values >= 0) with row shifts and
// row broadcasts, no LDS round trip
__device__ inline uint32_t wave_incl_max(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
    return v;
}

// Owner lane of the pooled candidate cb + lane, for steps of 64 pooled
// candidates: each lane whose first candidate falls in [cb, cb + 64) marks
// that slot in its wave's 64-entry LDS row; a prefix maximum in registers
// spreads the marks over the following candidates; carry keeps the owner of
// the last candidate of the step before (0 before the first step).
__device__ inline uint32_t pooled_owner(uint32_t *mark, uint32_t lane, uint32_t n_own, uint32_t off, uint32_t cb,
                                        uint32_t &carry)
{
    mark[lane] = 0u;
    wave_lds_sync();
    if (n_own != 0u && off >= cb && off < cb + 64u) mark[off - cb] = lane + 1u;
    wave_lds_sync();
    const uint32_t m = wave_incl_max(max(mark[lane], carry));
    carry = (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
    return m - 1u;
}

__global__ void k_zero_u32(uint32_t *__restrict__ p, const uint32_t *n_ptr, uint32_t cap, uint32_t extra)
{
    const uint32_t n = min(*n_ptr, cap) + extra;
    GRID_STRIDE(i, n) p[i] = 0u;
}

__global__ void k_zero_u8(uint8_t *__restrict__ p, const uint32_t *n_ptr, uint32_t cap)
{
    const uint32_t n = min(*n_ptr, cap);
    GRID_STRIDE(i, n) p[i] = 0u;
}

// derive the per-batch unit counts; clear error flags and statistics
__global__ void k_setup(Totals *t, uint32_t *__restrict__ ev_err, uint32_t cap_ev, uint32_t n_mod, uint32_t n_surf,
                        uint32_t nphi, uint32_t nkb)
{
    for (uint32_t e = threadIdx.x; e < min(t->n_ev, cap_ev); e += blockDim.x) ev_err[e] = 0u;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        t->n_bins = t->n_ev * 2u * n_mod;
        t->n_md_units = t->n_ev * n_mod;
        t->n_rows = t->n_ev * n_surf * nphi;
        t->n_bk = t->n_rows * (3u * nkb + 1u);
        t->err = 0;
        // region needs: written by the stages that append to regions (the
        // small-batch segment stage does not)
        t->n_mds = 0;
        t->n_lss = 0;
        t->n_t3s = 0;
        t->n_t5s = 0;
        t->n_ptc3 = 0;
        t->n_ptc5 = 0;
        for (int i = 0; i < 6; i++) t->cand[i] = 0ull;
    }
}

// ------------------------------------------------------ a1: hit ingest ---

// Hit histogram per event in LDS: a block takes one event and a slice of
// its (module, sensor) bins, counts the event's hits that fall in the slice
// with LDS atomics (the returned value is the hit's slot in its bin) and
// writes the slice's counts out, so no global atomic is needed.  Bad hits
// are reported by the slice-0 block only, for the batch and for their event.
constexpr uint32_t kHistBlock = 1024;

// Input contract of a hit (x, y, z, r = sqrt(x^2 + y^2)) on sensor sn: on
// that sensor (barrel radius or disk plane z within the stated tolerance) and
// inside its module's extent widened by the stated resolutions (coarse
// coordinate, azimuth).  a: the module's accepted extent (azimuth centre,
// half-width, coarse lo, hi); sp: its sensor positions, tolerance, kind.
__device__ inline bool hit_inside(const float4 a, const float4 sp, uint32_t sn, float x, float y, float z, float r)
{
    const bool barrel = sp.w == 0.0f;
    const float across = barrel ? r : z;
    const float coarse = barrel ? z : r;
    if (!(fabsf(across - (sn ? sp.y : sp.x)) <= sp.z)) return false;
    if (!(coarse >= a.z && coarse <= a.w)) return false;
    float d = fabsf(atan2f(y, x) - a.x);
    if (d > kPiF) d = 2.0f * kPiF - d;
    return d <= a.y;
}

__global__ __launch_bounds__(kHistBlock) void k_hit_hist(const Batch b, Totals *t, uint32_t n_mod, uint32_t slice)
{
    extern __shared__ uint32_t s_cnt[];
    const uint32_t n_ev = t->n_ev, n = min(t->n_hits, b.cap_hits);
    const uint32_t bins_ev = 2u * n_mod;
    const uint32_t n_sl = (bins_ev + slice - 1u) / slice;
    for (uint32_t w = blockIdx.x; w < n_ev * n_sl; w += gridDim.x) {
        const uint32_t e = w / n_sl, sl = w - e * n_sl;
        const uint32_t b0 = sl * slice, nb = min(slice, bins_ev - b0);
        for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) s_cnt[i] = 0u;
        __syncthreads();
        const uint32_t h1 = min(b.ev_hit_off[e + 1], n);
        for (uint32_t h = b.ev_hit_off[e] + threadIdx.x; h < h1; h += blockDim.x) {
            const uint32_t m = b.in_mod[h], sn = b.in_sen[h];
            const float x = b.in_x[h], y = b.in_y[h], z = b.in_z[h];
            uint32_t bad = 0;
            if (m >= n_mod || sn > 1u) bad |= kErrBadModule;
            if (!isfinite(x) || !isfinite(y) || !isfinite(z)) bad |= kErrNonFinite;
            if (bad) {
                if (sl == 0u) {
                    atomicOr(&t->err, bad);
                    atomicOr(&b.ev_err[e], bad);
                    b.hbin[h] = kInvalid;
                }
                continue;
            }
            const uint32_t local = 2u * m + sn;
            if (local < b0 || local >= b0 + nb) continue;
            b.hbin[h] = e * bins_ev + local;
            b.hrank[h] = atomicAdd(&s_cnt[local - b0], 1u);
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) b.bin_cnt[e * bins_ev + b0 + i] = s_cnt[i];
        __syncthreads();
    }
}

// four consecutive hits per thread in the scatter: their loads, then their
// offset gathers, are in flight together
constexpr uint32_t kHitsPerThread = 4;

// each hit's record to its bin (coalesced reads, one 16-byte write per hit;
// four hits per thread)
__global__ void k_hit_scatter(const Batch b, const Totals *t)
{
    const uint32_t n = min(t->n_hits, b.cap_hits);
    const uint32_t nq = (n + kHitsPerThread - 1) / kHitsPerThread;
    XCD_STRIDE(qd, nq) {
        const uint32_t h0 = qd * kHitsPerThread;
        uint32_t bin[kHitsPerThread], rank[kHitsPerThread], dst[kHitsPerThread];
        float4 v[kHitsPerThread];
#pragma unroll
        for (uint32_t k = 0; k < kHitsPerThread; k++) {
            const uint32_t h = min(h0 + k, n - 1u);
            bin[k] = h0 + k < n ? b.hbin[h] : kInvalid;
            rank[k] = b.hrank[h];
            v[k] = make_float4(b.in_x[h], b.in_y[h], b.in_z[h], __uint_as_float(h));
        }
#pragma unroll
        for (uint32_t k = 0; k < kHitsPerThread; k++) dst[k] = bin[k] != kInvalid ? b.bin_off[bin[k]] + rank[k] : 0u;
#pragma unroll
        for (uint32_t k = 0; k < kHitsPerThread; k++)
            if (bin[k] != kInvalid) b.hrec[dst[k]] = v[k];
    }
}

// per sorted position: the hit there takes its place in input order within
// its (event, module, sensor) bin -- the scatter used atomic slots -- as the
// number of the bin's hits with a smaller input index, and is written to the
// sorted SoA with r = sqrt(x^2 + y^2).  Each hit is checked against the input
// contract (its module's extent); a hit outside fails its event (its lists
// are not used).
__global__ void k_hit_gather(const Batch b, Totals *t, const float4 *__restrict__ ext, uint32_t n_mod)
{
    const uint32_t n = t->n_sorted;
    XCD_STRIDE(i, n) {
        const float4 v = b.hrec[i];
        const uint32_t h = __float_as_uint(v.w);
        const uint32_t bin = b.hbin[h];
        const uint32_t beg = b.bin_off[bin], end = b.bin_off[bin + 1];
        uint32_t pos = beg;
        for (uint32_t j = beg; j < end; j++) pos += __float_as_uint(b.hrec[j].w) < h ? 1u : 0u;
        const uint32_t e = bin / (2u * n_mod);
        const uint32_t local = bin - e * 2u * n_mod, m = local >> 1, sn = local & 1u;
        const float r = sqrtf(v.x * v.x + v.y * v.y);
        if (!hit_inside(ext[2 * m], ext[2 * m + 1], sn, v.x, v.y, v.z, r)) {
            atomicOr(&t->err, kErrOutside);
            atomicOr(&b.ev_err[e], kErrOutside);
        }
        b.hpos[pos] = make_float4(v.x, v.y, v.z, r);
        b.hin[pos] = h - b.ev_hit_off[e];
        b.hbin_s[pos] = bin;
    }
}

// ------------------------------------------------------ a2: mini-doublets ---

__device__ inline bool md_cut(const float4 mc, bool barrel, float L,
                              float xi, float yi, float zi, float ri,
                              float xj, float yj, float zj, float rj, float &beta)
{
    float dx = xj - xi, dy = yj - yi;
    float c = xi * dy - yi * dx;
    float d = xi * xj + yi * yj;
    float rr = ri * rj;
    if (!(d > 0.0f)) return false;
    if (!(fabsf(c) <= mc.x * rr)) return false;
    if (barrel) {
        if (!(fabsf(zj - zi) * ri <= mc.y * (fabsf(zi) + L) + mc.z * ri)) return false;
    } else {
        if (!(fabsf(rj - ri) <= mc.w)) return false;
    }
    beta = c / rr;
    return true;
}

// MD: the 64 sorted hits of a wave (one per lane; lower-sensor hits own the
// upper-sensor hits of their module as candidates) pool their candidates and
// the lanes take them 64 at a time.  Survivors go to the block's region of
// an unordered MD list as (lower hit, place in its list, upper hit, beta);
// k_md_place writes the MD records in canonical order once the per-hit
// counts are scanned.
__global__ __launch_bounds__(256) void k_md(const Batch b, Totals *t, const DevGeom g, const Consts c,
                                            uint32_t nsub, int stats)
{
    __shared__ uint32_t s_mark[4][64];   // pooled-candidate owner marks, one row per wave
    __shared__ uint32_t s_n;             // appends to this block's region
    const uint32_t n = t->n_sorted;
    const uint32_t n_mod = c.n_mod;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    const uint32_t cap = b.cap_mds / nsub;
    uint4 *out = b.mds + (size_t)blockIdx.x * cap;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    uint64_t cand = 0;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        uint32_t up0 = 0, cnt = 0, m = 0;
        float4 hi = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i < n) {
            const uint32_t bin = b.hbin_s[i];
            if (!(bin & 1u)) {
                up0 = b.bin_off[bin + 1];
                const uint32_t up1 = b.bin_off[bin + 2];
                cnt = up1 > up0 ? up1 - up0 : 0u;
                if (cnt) {
                    m = (bin >> 1) % n_mod;
                    hi = b.hpos[i];
                }
            }
        }
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t off = incl - cnt;
        const uint32_t total = wave_last(incl);
        uint32_t run = 0;
        uint32_t carry = 0;
        for (uint32_t cb = 0; cb < total; cb += 64u) {
            const uint32_t ci = cb + lane;
            const uint32_t o = pooled_owner(s_mark[wv], lane, cnt, off, cb, carry);
            const uint32_t o_up0 = __shfl(up0, o), o_off = __shfl(off, o), o_run = __shfl(run, o);
            const uint32_t o_i = __shfl(i, o), o_m = __shfl(m, o);
            const float hx = __shfl(hi.x, o), hy = __shfl(hi.y, o), hz = __shfl(hi.z, o), hw = __shfl(hi.w, o);
            bool pass = false;
            uint32_t j = 0;
            float beta = 0.f;
            if (ci < total) {
                j = o_up0 + (ci - o_off);
                const float4 mc = g.mdc[o_m];
                const bool barrel = g.mod_kind[o_m] == LST_BARREL;
                const float4 hj = b.hpos[j];
                cand++;
                pass = md_cut(mc, barrel, c.L, hx, hy, hz, hw, hj.x, hj.y, hj.z, hj.w, beta);
            }
            const unsigned long long mk = __ballot(pass);
            const uint32_t np = (uint32_t)__popcll(mk);
            uint32_t at = 0;
            if (np != 0u && lane == 0u) at = atomicAdd(&s_n, np);
            at = __shfl(at, 0);
            if (pass) {
                const uint32_t slot = at + (uint32_t)__popcll(mk & below);
                const uint32_t s0 = o_off > cb ? o_off - cb : 0u;
                if (slot < cap)
                    out[slot] = make_uint4(o_i, o_run + (uint32_t)__popcll(mk & below & ~((1ull << s0) - 1ull)), j,
                                           __float_as_uint(beta));
            }
            if (cnt != 0u && off < cb + 64u && off + cnt > cb) {
                const uint32_t s0 = off > cb ? off - cb : 0u;
                const uint32_t e0 = min(off + cnt - cb, 64u);
                run += (uint32_t)__popcll(mk & lane_range(s0, e0));
            }
        }
        if (i < n) b.md_cnt[i] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) b.mds_sub[blockIdx.x] = s_n;
    if (stats) atomicAdd(&t->cand[0], (unsigned long long)cand);
}

// Latency variant for small batches: one thread per sorted hit, a count
// pass and (after the scan) a fill pass that writes the MDs in place; two
// launches fewer than the pooled walk and its placement.
template <bool kFill>
__global__ __launch_bounds__(256) void k_md_direct(const Batch b, Totals *t, const DevGeom g, const Consts c,
                                                   int stats)
{
    const uint32_t n = t->n_sorted;
    const uint32_t n_mod = c.n_mod;
    uint64_t cand = 0;
    GRID_STRIDE(i, n) {
        const uint32_t bin = b.hbin_s[i];
        uint32_t k = kFill ? b.md_hoff[i] : 0u;
        if (!(bin & 1u)) {
            const uint32_t up0 = b.bin_off[bin + 1], up1 = b.bin_off[bin + 2];
            if (up0 < up1) {
                const uint32_t u = bin >> 1;
                const uint32_t m = u % n_mod;
                const float4 mc = g.mdc[m];
                const bool barrel = g.mod_kind[m] == LST_BARREL;
                const float4 hi = b.hpos[i];
                for (uint32_t j = up0; j < up1; j++) {
                    float beta;
                    const float4 hj = b.hpos[j];
                    if (!kFill) cand++;
                    if (!md_cut(mc, barrel, c.L, hi.x, hi.y, hi.z, hi.w, hj.x, hj.y, hj.z, hj.w, beta))
                        continue;
                    if (kFill && k < b.cap_md) {
                        b.md_pos[k] = make_float4(hi.x, hi.y, hi.z, barrel ? hi.w : -hi.w);
                        b.md_beta[k] = beta;
                        b.md_u[k] = u | (barrel ? 0u : kDiskBit);
                        b.md_hlo[k] = b.hin[i];
                        b.md_hup[k] = b.hin[j];
                    }
                    k++;
                }
            }
        }
        if (!kFill) b.md_cnt[i] = k;
    }
    if (!kFill && stats) atomicAdd(&t->cand[0], (unsigned long long)cand);
}

// MDs from the block regions to their canonical slots, with the anchor
// (the lower hit; the sign of r marks a disk), beta, unit and input hits
__global__ __launch_bounds__(256) void k_md_place(const Batch b, const Totals *t, const DevGeom g, const Consts c,
                                                  uint32_t nsub)
{
    __shared__ uint32_t s_off[kSubLists + 1];
    for (uint32_t i = threadIdx.x; i <= nsub; i += blockDim.x) s_off[i] = b.mds_soff[i];
    __syncthreads();
    const uint32_t n = s_off[nsub];
    const uint32_t subcap = b.cap_mds / nsub;
    XCD_STRIDE(jj, n) {
        const uint4 r = b.mds[pair_slot(s_off, jj, subcap, nsub)];
        const uint32_t k = b.md_hoff[r.x] + r.y;
        if (k < b.cap_md) {
            const uint32_t u = b.hbin_s[r.x] >> 1;
            const bool barrel = g.mod_kind[u % c.n_mod] == LST_BARREL;
            const float4 hi = b.hpos[r.x];
            b.md_pos[k] = make_float4(hi.x, hi.y, hi.z, barrel ? hi.w : -hi.w);
            b.md_beta[k] = __uint_as_float(r.w);
            b.md_u[k] = u | (barrel ? 0u : kDiskBit);
            b.md_hlo[k] = b.hin[r.x];
            b.md_hup[k] = b.hin[r.z];
        }
    }
    // the per-module MD offsets (as k_md_units writes them)
    const uint32_t nu = t->n_md_units;
    GRID_STRIDE(u, nu + 1) b.md_off[u] = b.md_hoff[b.bin_off[2u * u]];
}

// MD range of every (event, module) unit: the MDs of its lower-sensor hits
__global__ void k_md_units(const Batch b, const Totals *t)
{
    const uint32_t nu = t->n_md_units;
    // bin_off has 2 nu + 1 entries and its values index md_hoff (n_sorted + 1)
    GRID_STRIDE(u, nu + 1) b.md_off[u] = b.md_hoff[b.bin_off[2u * u]];
}

// ------------------------------------------------------ a3: line segments ---

// Whether an outer module can hold a segment's outer anchor for an inner
// anchor at azimuth pha: the arc distance from pha to the module's azimuth
// extent (centre, half-width with margin) is within the class's reach.  The
// azimuth cut needs |sin(dphi)| <= S with cos(dphi) > 0, i.e. |dphi| <= asin S,
// so a module out of reach holds no partner and its MDs are not visited; the
// reach carries margins beyond the rounding of this test.
__device__ inline bool in_reach(float pha, const float2 mp, float reach)
{
    float d = fabsf(pha - mp.x);
    if (d > kPiF) d = 2.0f * kPiF - d;
    return d <= mp.y + reach;
}

// Modules [k0, k1) of a segment-walk run (destinations first + k, k below
// its length) that can hold a partner of an inner anchor at azimuth pha: the
// indices k with |delta * inv_pitch - k| <= window (in module indices),
// delta the anchor's azimuth relative to the run's first module; a run of
// one module takes |delta| <= window (radians).  The window covers every
// module the per-module reach test accepts (it holds the largest
// half-width, the reach, the centres' deviation from the pitch and room for
// this arithmetic), and a run spans less than half a turn with its window,
// so no wrap-around beyond delta's is needed.  k1 == k0: none.
__device__ inline uint2 run_range(const uint4 r, float win, float pha)
{
    const float len = (float)(r.y >> 24);
    float d = pha - __uint_as_float(r.z);
    if (d > kPiF) d -= 2.0f * kPiF;
    else if (d < -kPiF) d += 2.0f * kPiF;
    float k0, k1;
    if (r.y >> 24 == 1u) {
        k0 = 0.0f;
        k1 = fabsf(d) <= win ? 1.0f : 0.0f;
    } else {
        const float tc = d * __uint_as_float(r.w);
        k0 = fminf(fmaxf(ceilf(tc - win), 0.0f), len);
        k1 = fmaxf(fminf(floorf(tc + win) + 1.0f, len), k0);
    }
    return make_uint2((uint32_t)k0, (uint32_t)k1);
}

__device__ inline bool ls_cut(const LsK &k, const Consts &c, bool bend,
                              float xa, float ya, float za, float ra, float beta_a,
                              float xb, float yb, float zb, float rb)
{
    const uint32_t type = __float_as_uint(k.b.w);
    float dx = xb - xa, dy = yb - ya;
    float cr = xa * dy - ya * dx;
    float d = xa * xb + ya * yb;
    float rr = ra * rb;
    if (!(d > 0.0f)) return false;
    if (!(fabsf(cr) <= k.a.x * rr)) return false;
    if (type == 0u) {
        const float rho[2] = {k.a.y, k.a.z};
        const float vv[2] = {-c.L, c.L};
        const float zp[2] = {za - c.ec, za + c.ec};
        float lo = rho[0] * (zp[0] - vv[0]) + vv[0];
        float hi = lo;
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int j = 0; j < 2; j++)
#pragma unroll
                for (int l = 0; l < 2; l++) {
                    if (i == 0 && j == 0 && l == 0) continue;
                    float w = rho[i] * (zp[l] - vv[j]) + vv[j];
                    lo = fminf(lo, w);
                    hi = fmaxf(hi, w);
                }
        float mid = 0.5f * (lo + hi), half = 0.5f * (hi - lo) + c.ec;
        if (!(fabsf(zb - mid) <= half)) return false;
        if (bend) {
            float sab = cr / rr;
            float p1 = k.a.w * beta_a, p2 = k.b.x * beta_a;
            float blo = fminf(p1, p2) - k.b.y, bhi = fmaxf(p1, p2) + k.b.y;
            float bmid = 0.5f * (blo + bhi), bhalf = 0.5f * (bhi - blo);
            if (!(fabsf(sab - bmid) <= bhalf)) return false;
        }
        return true;
    }
    if (type == 1u) {
        float lo = k.a.y * (ra - c.ec) - c.ec;
        float hi = k.a.z * (ra + c.ec) + c.ec;
        float mid = 0.5f * (lo + hi), half = 0.5f * (hi - lo);
        return fabsf(rb - mid) <= half;
    }
    float zap = k.a.z * za;
    float dhi = (zap + c.ec) + c.L;
    if (!(dhi > 0.0f)) return false;
    float lo = (k.a.y * (k.a.w / dhi)) * ra - c.ec;
    float dlo = (zap - c.ec) - c.L;
    if (dlo > 0.0f) {
        float hi = (k.b.x / dlo) * ra + c.ec;
        float mid = 0.5f * (lo + hi), half = 0.5f * (hi - lo);
        return fabsf(rb - mid) <= half;
    }
    return lo <= rb;
}

// Large batches: the 64 inner MDs of a wave (one per lane) step through
// their modules' segment-walk runs (edges to consecutive destination modules
// of one class, evenly spaced in azimuth) in groups of 6 together.  For each
// run a lane computes which of its modules are within azimuth reach of its
// anchor (an index range, from the run's record alone) and loads that range's
// MDs (two MD offsets: consecutive modules hold consecutive MDs), storing the
// ranges in LDS; a group thus costs two round trips (the run records, then
// the MD offsets) whatever the number of edges in it.  The wave pools the
// candidates (every MD of every run of the group, lane by lane in (run,
// outer MD) order) and the lanes take them 64 at a time, so the cut
// arithmetic runs on full waves however the degrees and MD counts are
// spread.  A candidate finds its owner lane from a mark each owner leaves in
// LDS at its first candidate of the step, spread to the following
// candidates by a prefix maximum in registers (row shifts and broadcasts, no
// chain of lane shuffles); its run in the owner's group comes from LDS and
// the owner's anchor by lane shuffles.  Survivors go to the block's region of
// an unordered segment list with their place in the owner's list (its
// earlier survivors plus those before it in the same 64); runs follow the
// edges' order by destination module, so that place is the canonical one.
// A step takes two rounds, both rounds' loads issued before either cut.
// kEdgeGroup runs per group; at least kMinWaves waves per SIMD (1: the
// compiler's register choice).  Instantiated for the groups and occupancies
// the tuner may pick (lst_params.ls_group, ls_waves).
template <int kEdgeGroup, int kMinWaves>
__global__ __launch_bounds__(256, kMinWaves) void k_ls(const Batch b, Totals *t, const DevGeom g, const Consts c,
                                                       uint32_t nsub, int stats)
{
    constexpr uint32_t kF = 3 * kEdgeGroup;          // per lane and run of the group: first outer MD, running count, class
    __shared__ uint32_t s_grp[4][kF][64];
    __shared__ uint32_t s_mark[4][128];               // owner lane + 1 at each owner's first candidate of a step
    __shared__ uint32_t s_n;                          // appends to this block's region
    const uint32_t n = min(t->n_md, b.cap_md);
    const uint32_t n_mod = c.n_mod;
    const bool bend = (c.flags & LST_FLAG_BEND) != 0u;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    const uint32_t cap = b.cap_lss / nsub;
    uint32_t *sa = b.lss_a + (size_t)blockIdx.x * cap;
    uint32_t *sb = b.lss_b + (size_t)blockIdx.x * cap;
    uint32_t *sj = b.lss_j + (size_t)blockIdx.x * cap;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    uint64_t cand = 0;
    // every lane of a wave runs the same number of iterations and steps
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t a = base + threadIdx.x;
        uint32_t e0 = 0, e1 = 0, ubase = 0;
        float xa = 0.f, ya = 0.f, za = 0.f, ra = 0.f, ba = 0.f, pha = 0.f;
        if (a < n) {
            const uint32_t u = b.md_u[a] & kUnitMask;
            const uint32_t m = u % n_mod;
            ubase = u - m;
            e0 = g.run_begin[m];
            e1 = g.run_begin[m + 1];
            const float4 pa = b.md_pos[a];
            xa = pa.x;
            ya = pa.y;
            za = pa.z;
            ra = fabsf(pa.w);
            ba = b.md_beta[a];
            pha = atan2f(ya, xa);
        }
        uint32_t run = 0;                             // segments of this lane's MD so far
        for (uint32_t eb = e0;; eb += kEdgeGroup) {
            if (__ballot(eb < e1) == 0ull) break;
            // this lane's group: MD ranges of up to kEdgeGroup runs, to LDS.
            // The loads of all the group's run records go out together (runs
            // past the lane's last load a valid run and are dropped after),
            // then the MD offsets of every run's range in reach together.
            uint4 rr[kEdgeGroup];
            float rw[kEdgeGroup];
#pragma unroll
            for (int j = 0; j < kEdgeGroup; j++) {
                const uint32_t r = min(eb + j, e1 > e0 ? e1 - 1u : 0u);
                rr[j] = g.run[r];
                rw[j] = g.run_win[r];
            }
            uint32_t lo[kEdgeGroup], hi[kEdgeGroup];
#pragma unroll
            for (int j = 0; j < kEdgeGroup; j++) {
                const uint2 kr = run_range(rr[j], rw[j], pha);
                lo[j] = b.md_off[ubase + rr[j].x + kr.x];
                hi[j] = b.md_off[ubase + rr[j].x + kr.y];
            }
            uint32_t T = 0;
#pragma unroll
            for (int j = 0; j < kEdgeGroup; j++) {
                uint32_t bq = 0, eq = 0;
                if (eb + j < e1) {
                    bq = min(lo[j], b.cap_md);
                    eq = max(min(hi[j], b.cap_md), bq);
                }
                T += eq - bq;
                s_grp[wv][j][lane] = bq;
                s_grp[wv][kEdgeGroup + j][lane] = T;  // cum[j + 1]
                s_grp[wv][2 * kEdgeGroup + j][lane] = rr[j].y & 0xFFFFFFu;
            }
            wave_lds_sync();
            const uint32_t incl = wave_incl_scan(T);
            const uint32_t off = incl - T;
            const uint32_t total = wave_last(incl);
            // two pooled rounds per step: the indices and loads of both are
            // issued before either cut, so that twice the loads are in flight
            uint32_t carry = 0;                       // owner + 1 of the last candidate so far
            for (uint32_t cb = 0; cb < total; cb += 128u) {
                uint32_t o[2], q[2];
                float4 pq[2];
                LsK kc[2];
                // owners by a prefix maximum over marks at their first
                // candidates, instead of a search over the lanes' offsets
                s_mark[wv][lane] = 0u;
                s_mark[wv][64u + lane] = 0u;
                wave_lds_sync();
                if (T != 0u && off >= cb && off < cb + 128u) s_mark[wv][off - cb] = lane + 1u;
                wave_lds_sync();
                uint32_t mk2[2] = {s_mark[wv][lane], s_mark[wv][64u + lane]};
#pragma unroll
                for (int r = 0; r < 2; r++) {
                    const uint32_t ci = cb + 64u * r + lane;
                    const uint32_t m = wave_incl_max(max(mk2[r], carry));
                    carry = (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
                    const uint32_t ow = m - 1u;
                    // run j of the owner's group: the last with cum[j] <= tt
                    // (lanes past the total read valid LDS and load entry 0)
                    const uint32_t tt = ci - __shfl(off, ow);
                    uint32_t j = 0, cj = 0;
#pragma unroll
                    for (int k = 0; k < kEdgeGroup - 1; k++) {
                        const uint32_t cum = s_grp[wv][kEdgeGroup + k][ow];
                        if (cum <= tt) {
                            j = k + 1;
                            cj = cum;
                        }
                    }
                    q[r] = ci < total ? s_grp[wv][j][ow] + (tt - cj) : 0u;
                    kc[r] = g.cls[s_grp[wv][2 * kEdgeGroup + j][ow]];
                    pq[r] = b.md_pos[q[r]];
                    o[r] = ow;
                }
                bool pass[2];
#pragma unroll
                for (int r = 0; r < 2; r++) {
                    const uint32_t ci = cb + 64u * r + lane;
                    const float oxa = __shfl(xa, o[r]), oya = __shfl(ya, o[r]), oza = __shfl(za, o[r]);
                    const float ora = __shfl(ra, o[r]), oba = __shfl(ba, o[r]);
                    pass[r] = false;
                    if (ci < total) {
                        cand++;
                        pass[r] = ls_cut(kc[r], c, bend, oxa, oya, oza, ora, oba, pq[r].x, pq[r].y, pq[r].z,
                                         fabsf(pq[r].w));
                    }
                }
#pragma unroll
                for (int r = 0; r < 2; r++) {
                    const uint32_t c0 = cb + 64u * r;
                    if (c0 >= total) break;                   // the same on every lane
                    const uint32_t o_off = __shfl(off, o[r]), o_run = __shfl(run, o[r]);
                    const unsigned long long mk = __ballot(pass[r]);
                    const uint32_t np = (uint32_t)__popcll(mk);
                    uint32_t at = 0;
                    if (np != 0u && lane == 0u) at = atomicAdd(&s_n, np);
                    at = __shfl(at, 0);
                    if (pass[r]) {
                        const uint32_t slot = at + (uint32_t)__popcll(mk & below);
                        const uint32_t s0 = o_off > c0 ? o_off - c0 : 0u;
                        if (slot < cap) {
                            sa[slot] = base + wv * 64u + o[r];
                            sb[slot] = q[r];
                            sj[slot] = o_run + (uint32_t)__popcll(mk & below & ~((1ull << s0) - 1ull));
                        }
                    }
                    if (T != 0u && off < c0 + 64u && off + T > c0) {
                        const uint32_t s0 = off > c0 ? off - c0 : 0u;
                        const uint32_t e0c = min(off + T - c0, 64u);
                        run += (uint32_t)__popcll(mk & lane_range(s0, e0c));
                    }
                }
            }
            wave_lds_sync();
        }
        if (a < n) b.ls_cnt[a] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) b.lss_sub[blockIdx.x] = s_n;
    if (stats) atomicAdd(&t->cand[1], (unsigned long long)cand);
}

// segments from the sub-lists to their canonical slots
__global__ __launch_bounds__(256) void k_ls_place(const Batch b, uint32_t nsub)
{
    __shared__ uint32_t s_off[kSubLists + 1];
    for (uint32_t i = threadIdx.x; i <= nsub; i += blockDim.x) s_off[i] = b.lss_soff[i];
    __syncthreads();
    const uint32_t n = s_off[nsub];
    const uint32_t subcap = b.cap_lss / nsub;
    XCD_STRIDE(j, n) {
        const uint32_t i = pair_slot(s_off, j, subcap, nsub);
        const uint32_t a = b.lss_a[i];
        const uint32_t k = b.ls_off[a] + b.lss_j[i];
        if (k < b.cap_ls) {
            b.ls_a[k] = a;
            b.ls_b[k] = b.lss_b[i];
        }
    }
}

// Latency variant for small batches (a few events): a wave takes two
// consecutive MDs; for each, 32 lanes take
// one edge of the MD's module each (chunks of 32 for larger degrees) and test
// the MDs of the edge's destination module.  Half-wave prefix sums give each
// lane its place, so segments come out ordered by (inner MD, edge, outer MD),
// which is (inner MD, outer MD) because edges are sorted by destination.
constexpr uint32_t kLsLanes = 32;
constexpr uint32_t kLsWaveMaxMd = 1u << 17;   // MD capacity up to which the latency variant runs

// inclusive prefix sum within each half (32 lanes) of a wave: the row
// shifts of wave_incl_scan, then only the broadcast of rows 0 / 2 into
// rows 1 / 3
__device__ inline uint32_t half_incl_scan(uint32_t v)
{
    static_assert(kLsLanes == 32, "half-wave scan");
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
    return v;
}

template <bool kFill>
__global__ __launch_bounds__(256) void k_ls_wave(const Batch b, Totals *t, const DevGeom g, const Consts c,
                                            int stats)
{
    const uint32_t n = min(t->n_md, b.cap_md);
    const uint32_t n_mod = c.n_mod;
    const bool bend = (c.flags & LST_FLAG_BEND) != 0u;
    const uint32_t half = (threadIdx.x >> 5) & 1u, w = threadIdx.x & (kLsLanes - 1);
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    uint64_t cand = 0;
    for (uint32_t a0 = 2 * wave; a0 < n; a0 += 2 * n_waves) {
        const uint32_t a = a0 + half;
        if (a >= n) continue;
        const uint32_t u = b.md_u[a] & kUnitMask;
        const uint32_t m = u % n_mod;
        const uint32_t base = u - m;
        const float4 pa = b.md_pos[a];
        const float xa = pa.x, ya = pa.y, za = pa.z, ra = fabsf(pa.w), ba = b.md_beta[a];
        const float pha = atan2f(ya, xa);
        const uint32_t e0 = g.edge_begin[m], e1 = g.edge_begin[m + 1];
        uint32_t carry = kFill ? b.ls_off[a] : 0u;
        if (kFill) {
            const uint32_t cnt_a = b.ls_off[a + 1] - carry;
            if (cnt_a <= kKeepLs) {
                if (w < cnt_a && carry + w < b.cap_ls) {
                    b.ls_a[carry + w] = a;
                    b.ls_b[carry + w] = b.ls_keep[(size_t)a * kKeepLs + w];
                }
                continue;
            }
        }
        for (uint32_t eb = e0; eb < e1; eb += kLsLanes) {
            const uint32_t e = eb + w;
            uint32_t bb = 0, be = 0;
            LsK kc;
            if (e < e1) {
                const uint2 ed = g.edge[e];
                bb = min(b.md_off[base + ed.x], b.cap_md);
                be = min(b.md_off[base + ed.x + 1], b.cap_md);
                if (bb < be) {
                    kc = g.cls[ed.y];
                    if (!in_reach(pha, g.mod_phi[ed.x], kc.b.z)) be = bb;   // out of azimuth reach
                }
            }
            // pass mask of this lane's candidates (up to 32; beyond, re-test)
            uint32_t cnt = 0, mask = 0;
            for (uint32_t q = bb; q < be; q++) {
                const float4 pq = b.md_pos[q];
                if (ls_cut(kc, c, bend, xa, ya, za, ra, ba, pq.x, pq.y, pq.z, fabsf(pq.w))) {
                    if (q - bb < 32u) mask |= 1u << (q - bb);
                    cnt++;
                }
            }
            if (!kFill) cand += be - bb;
            const uint32_t incl = half_incl_scan(cnt);
            const uint32_t tot = __shfl(incl, kLsLanes - 1, kLsLanes);
            if (!kFill && carry + incl - cnt < kKeepLs) {
                // record this lane's survivors among the MD's first kKeepLs
                uint32_t k = carry + incl - cnt;
                for (uint32_t q = bb; q < be && k < kKeepLs; q++) {
                    bool pass;
                    if (q - bb < 32u) {
                        pass = (mask >> (q - bb)) & 1u;
                    } else {
                        const float4 pq = b.md_pos[q];
                        pass = ls_cut(kc, c, bend, xa, ya, za, ra, ba, pq.x, pq.y, pq.z, fabsf(pq.w));
                    }
                    if (pass) b.ls_keep[(size_t)a * kKeepLs + k++] = q;
                }
            }
            if (kFill) {
                uint32_t k = carry + incl - cnt;
                for (uint32_t q = bb; q < be; q++) {
                    bool pass;
                    if (q - bb < 32u) {
                        pass = (mask >> (q - bb)) & 1u;
                    } else {
                        const float4 pq = b.md_pos[q];
                        pass = ls_cut(kc, c, bend, xa, ya, za, ra, ba, pq.x, pq.y, pq.z, fabsf(pq.w));
                    }
                    if (!pass) continue;
                    if (k < b.cap_ls) {
                        b.ls_a[k] = a;
                        b.ls_b[k] = q;
                    }
                    k++;
                }
            }
            carry += tot;
        }
        if (!kFill && w == 0) b.ls_cnt[a] = carry;
    }
    if (!kFill && stats) atomicAdd(&t->cand[1], (unsigned long long)cand);
}

// ------------------------------------------------------------ a4: T3 ----

struct Anchor {
    float x, y, z, r;
    bool disk;
};


__device__ inline uint32_t phi_bin(float x, float y, uint32_t nphi)
{
    float ph = atan2f(y, x);
    int bi = (int)((ph + kPiF) * ((float)nphi / (2.0f * kPiF)));
    bi = bi < 0 ? 0 : (bi >= (int)nphi ? (int)nphi - 1 : bi);
    return (uint32_t)bi;
}

__device__ inline uint32_t kappa_bin(float k, const Consts &c)
{
    float t = (k + c.kspan) * ((float)c.nkb / (2.0f * c.kspan));
    if (!(t > 0.0f)) return 0u;
    if (t >= (float)c.nkb) return c.nkb - 1u;
    return (uint32_t)t;
}

// Seed-lookup bucket of a T3 or T5, taken where the object is placed in its
// canonical slot: the row (event, surface of the inner anchor's module,
// azimuth bin of the inner anchor), then within the row the resolution class
// and curvature bin (wide objects, or a NaN resolution, in the row's last
// bucket).
__device__ inline uint32_t bucket_row(const Batch &b, const DevGeom &g, const Consts &c, uint32_t a, float x,
                                      float y)
{
    const uint32_t u = b.md_u[a] & kUnitMask;
    const uint32_t e = u / c.n_mod, m = u - e * c.n_mod;
    return ((e * c.n_surf + g.mod_surf[m]) * c.nphi + phi_bin(x, y, c.nphi)) * (3u * c.nkb + 1u);
}

__device__ inline uint32_t bucket_in_row(float k, float sk, const Consts &c)
{
    uint32_t kb = 3u * c.nkb;
    if (sk <= c.sk_cls[0]) kb = kappa_bin(k, c);
    else if (sk <= c.sk_cls[1]) kb = c.nkb + kappa_bin(k, c);
    else if (sk <= c.sk_cls[2]) kb = 2u * c.nkb + kappa_bin(k, c);
    return kb;
}

__device__ inline Anchor anchor_of(const float4 p)
{
    Anchor A;
    A.x = p.x;
    A.y = p.y;
    A.z = p.z;
    A.r = fabsf(p.w);
    A.disk = p.w < 0.0f;
    return A;
}

__device__ inline Anchor load_anchor(const Batch &b, uint32_t i)
{
    Anchor A;
    const float4 p = b.md_pos[i];
    A.x = p.x;
    A.y = p.y;
    A.z = p.z;
    A.r = fabsf(p.w);
    A.disk = p.w < 0.0f;
    return A;
}

// the transverse chord between two anchors
__device__ inline float chord(const Anchor &A, const Anchor &B)
{
    float dx = B.x - A.x, dy = B.y - A.y;
    return sqrtf(dx * dx + dy * dy);
}

// curvature of the circle through three transverse points (positive for a
// clockwise turn) and its resolution, given the chords d1 = A-B and d2 = B-C
// (the walks take the chord their owner fixes once per owner)
__device__ inline void kappa3(const Consts &c, const Anchor &A, const Anchor &B, const Anchor &C,
                              float d1, float d2, float &kap, float &sk)
{
    float dx1 = B.x - A.x, dy1 = B.y - A.y;
    float dx2 = C.x - B.x, dy2 = C.y - B.y;
    float dx3 = C.x - A.x, dy3 = C.y - A.y;
    float cr = dx1 * dy2 - dy1 * dx2;
    float d3 = sqrtf(dx3 * dx3 + dy3 * dy3);
    kap = (-2.0f * cr) / ((d1 * d2) * d3);
    float hC = fminf(1.0f, C.r * c.khalf);
    float sdisk = c.srp + c.sc * hC;
    float sA = A.disk ? sdisk : c.srp;
    float sB = B.disk ? sdisk : c.srp;
    float sC = C.disk ? sdisk : c.srp;
    sk = (2.0f * sqrtf((sA * sA + sB * sB) + sC * sC)) / (d1 * d2);
}

// straight line in (arc length, z) through three anchors, up to resolution
// and the arc-vs-chord bias
__device__ inline bool rz3(const Consts &c, const Anchor &A, const Anchor &B, const Anchor &C,
                           float d1, float d2)
{
    float E = (B.z - A.z) * d2 - (C.z - B.z) * d1;
    float szA = A.disk ? 0.0f : c.sc, szB = B.disk ? 0.0f : c.sc, szC = C.disk ? 0.0f : c.sc;
    float stA = A.disk ? c.sc : c.srp, stB = B.disk ? c.sc : c.srp, stC = C.disk ? c.sc : c.srp;
    float res = (((szA * d2 + szB * (d1 + d2)) + szC * d1) + fabsf(B.z - A.z) * (stB + stC)) +
                fabsf(C.z - B.z) * (stA + stB);
    // the bias term is finite and not negative when d1 + d2 > 0, and adding
    // it cannot lower the rounded bound: a candidate inside the bound without
    // it passes, and the division is only needed for the others
    if (d1 + d2 > 0.0f && fabsf(E) <= c.ns * res) return true;
    float bias = ((c.Kb * (fabsf(C.z - A.z) / (d1 + d2))) * (d1 * d2)) * fabsf(d1 * d1 - d2 * d2);
    return fabsf(E) <= c.ns * res + bias;
}

// T3: the 64 inner LSs of a wave (one per lane) pool their candidates --
// the LSs that start at each one's outer MD (their range from the LS
// offsets, their outer anchors through their outer MDs) -- and the lanes
// take the pooled candidates 64 at a time, so
// the cut arithmetic runs on full waves however the candidates are spread.
// A candidate finds its owner lane by a binary search over the lanes'
// first-candidate offsets and takes the owner's anchors by lane shuffles.
// Survivors go to the block's region of an unordered T3 list with their
// place in the owner's list (the owner's earlier survivors plus those before
// it in the same 64), so k_t3_place can put them in canonical order.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_t3(const Batch b, Totals *t, const Consts c, uint32_t nsub, int stats)
{
    __shared__ uint32_t s_mark[4][64];   // pooled-candidate owner marks, one row per wave
    __shared__ uint32_t s_n;             // appends to this block's region
    const uint32_t n = min(t->n_ls, b.cap_ls);
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    const uint32_t cap = b.cap_t3s / nsub;
    const size_t sb0 = (size_t)blockIdx.x * cap;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    uint64_t cand = 0;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t l1 = base + threadIdx.x;
        uint32_t ia = 0, q0 = 0, cnt = 0;
        float4 pa = make_float4(0.f, 0.f, 0.f, 0.f), pb = pa;
        float dab = 0.f;                                 // the chord A-B, fixed by the owner
        if (l1 < n) {
            ia = b.ls_a[l1];
            const uint32_t q = b.ls_b[l1];
            // the segments that start at the outer MD
            q0 = min(b.ls_off[q], b.cap_ls);
            const uint32_t q1 = min(b.ls_off[q + 1], b.cap_ls);
            cnt = q1 > q0 ? q1 - q0 : 0u;
            if (cnt) {
                pb = b.md_pos[q];
                pa = b.md_pos[ia];
                dab = chord(anchor_of(pa), anchor_of(pb));
            }
        }
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t off = incl - cnt;                 // this lane's first pooled candidate
        const uint32_t total = wave_last(incl);
        uint32_t run = 0;                                // survivors of this lane's LS so far
        uint32_t carry = 0;
        for (uint32_t cb = 0; cb < total; cb += 64u) {
            const uint32_t ci = cb + lane;
            // owner: the last lane o with off_o <= ci (it has ci - off_o < cnt_o)
            const uint32_t o = pooled_owner(s_mark[wv], lane, cnt, off, cb, carry);
            const uint32_t o_q0 = __shfl(q0, o), o_off = __shfl(off, o), o_ia = __shfl(ia, o);
            const uint32_t o_l1 = __shfl(l1, o), o_run = __shfl(run, o);
            const float4 oa = make_float4(__shfl(pa.x, o), __shfl(pa.y, o), __shfl(pa.z, o), __shfl(pa.w, o));
            const float4 ob = make_float4(__shfl(pb.x, o), __shfl(pb.y, o), __shfl(pb.z, o), __shfl(pb.w, o));
            const float d1 = __shfl(dab, o);
            bool pass = false;
            uint32_t l2 = 0, ic = 0;
            float kap = 0.f, sk = 0.f;
            if (ci < total) {
                l2 = o_q0 + (ci - o_off);
                ic = b.ls_b[l2];
                const Anchor A = anchor_of(oa), B = anchor_of(ob), C = anchor_of(b.md_pos[ic]);
                cand++;
                // the rz cut first (it needs the chords A-B and B-C and rejects
                // most candidates), then the curvature cut
                const float d2 = chord(B, C);
                if (rz3(c, A, B, C, d1, d2)) {
                    kappa3(c, A, B, C, d1, d2, kap, sk);
                    pass = fabsf(kap) <= c.kmaxf + c.ns * sk;
                }
            }
            const unsigned long long m = __ballot(pass);
            const uint32_t np = (uint32_t)__popcll(m);
            uint32_t at = 0;
            if (np != 0u && lane == 0u) at = atomicAdd(&s_n, np);
            at = __shfl(at, 0);
            if (pass) {
                const uint32_t slot = at + (uint32_t)__popcll(m & below);
                const uint32_t s0 = o_off > cb ? o_off - cb : 0u;
                const uint32_t jj = o_run + (uint32_t)__popcll(m & below & ~((1ull << s0) - 1ull));
                if (slot < cap) {
                    b.t3s_l1[sb0 + slot] = o_l1;
                    b.t3s_l2[sb0 + slot] = l2;
                    b.t3s_j[sb0 + slot] = jj;
                    b.t3s_ac[sb0 + slot] = make_uint2(o_ia, ic);
                    b.t3s_ks[sb0 + slot] = make_float2(kap, sk);
                }
            }
            // each lane counts the survivors among its own candidates in this 64
            if (cnt != 0u && off < cb + 64u && off + cnt > cb) {
                const uint32_t s0 = off > cb ? off - cb : 0u;
                const uint32_t e0 = min(off + cnt - cb, 64u);
                run += (uint32_t)__popcll(m & lane_range(s0, e0));
            }
        }
        if (l1 < n) b.t3_cnt[l1] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) b.t3s_sub[blockIdx.x] = s_n;
    if (stats) atomicAdd(&t->cand[2], (unsigned long long)cand);
}

// T3s from the sub-lists to their canonical slots
__global__ __launch_bounds__(256) void k_t3_place(const Batch b, const DevGeom g, const Consts c, uint32_t nsub)
{
    __shared__ uint32_t s_off[kSubLists + 1];
    for (uint32_t i = threadIdx.x; i <= nsub; i += blockDim.x) s_off[i] = b.t3s_soff[i];
    __syncthreads();
    const uint32_t n = s_off[nsub];
    const uint32_t subcap = b.cap_t3s / nsub;
    // whole waves per step (the bucket slots are drawn per wave)
    XCD_STRIDE_BLOCKS(jb, n) {
        const uint32_t j = jb + threadIdx.x;
        bool in = false;
        uint32_t k = 0, bk = 0;
        if (j < xb_.end) {
            const uint32_t i = pair_slot(s_off, j, subcap, nsub);
            const uint32_t l1 = b.t3s_l1[i];
            k = b.t3_off[l1] + b.t3s_j[i];
            if (k < b.cap_t3) {
                in = true;
                const uint2 ac = b.t3s_ac[i];
                const float2 ks = b.t3s_ks[i];
                b.t3_l1[k] = l1;
                b.t3_l2[k] = b.t3s_l2[i];
                b.t3_ac[k] = ac;
                b.t3_ks[k] = ks;
                // the object's seed-lookup bucket
                const float4 pa = b.md_pos[ac.x];
                bk = bucket_row(b, g, c, ac.x, pa.x, pa.y) + bucket_in_row(ks.x, ks.y, c);
            }
        }
        const uint32_t slot = wave_grouped_inc(b.bk3_cnt, bk, in);
        if (in) {
            b.bk3_id[k] = bk;
            b.bk3_rank[k] = slot;
        }
    }
}

// ------------------------------------------------------------ a5: T5 ----

// T5: the 64 inner T3s of a wave (one per lane) pool their candidates --
// the T3s whose inner MD is each one's outer MD (through the LS and T3
// offsets) -- and the lanes take the pooled candidates 64 at a time, as in
// the T3 walk.  The stored-curvature test runs first (it needs no new
// arithmetic).  Survivors go to the block's region of an unordered T5 list
// with their place in the owner's list; k_t5_place puts them in order.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_t5(const Batch b, Totals *t, const Consts c, uint32_t nsub, int stats)
{
    __shared__ uint32_t s_mark[4][64];   // pooled-candidate owner marks, one row per wave
    __shared__ uint32_t s_n;             // appends to this block's region
    const uint32_t n = min(t->n_t3, b.cap_t3);
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    const uint32_t cap = b.cap_t5s / nsub;
    const size_t sb0 = (size_t)blockIdx.x * cap;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    uint64_t cand = 0;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t u = base + threadIdx.x;
        uint32_t w0 = 0, cnt = 0;
        float4 pa = make_float4(0.f, 0.f, 0.f, 0.f), pc = pa;
        float2 ks1 = make_float2(0.f, 0.f);
        if (u < n) {
            const uint2 ac = b.t3_ac[u];
            // T3s whose inner MD is ac.y: those built from segments starting at ac.y
            w0 = min(b.t3_off[min(b.ls_off[ac.y], b.cap_ls)], b.cap_t3);
            const uint32_t w1 = min(b.t3_off[min(b.ls_off[ac.y + 1], b.cap_ls)], b.cap_t3);
            cnt = w1 > w0 ? w1 - w0 : 0u;
            if (cnt) {
                pa = b.md_pos[ac.x];
                pc = b.md_pos[ac.y];
                ks1 = b.t3_ks[u];
            }
        }
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t off = incl - cnt;
        const uint32_t total = wave_last(incl);
        uint32_t run = 0;
        uint32_t carry = 0;
        for (uint32_t cb = 0; cb < total; cb += 64u) {
            const uint32_t ci = cb + lane;
            const uint32_t o = pooled_owner(s_mark[wv], lane, cnt, off, cb, carry);
            const uint32_t o_w0 = __shfl(w0, o), o_off = __shfl(off, o), o_run = __shfl(run, o);
            const uint32_t o_u = __shfl(u, o);
            const float4 oa = make_float4(__shfl(pa.x, o), __shfl(pa.y, o), __shfl(pa.z, o), __shfl(pa.w, o));
            const float4 oc = make_float4(__shfl(pc.x, o), __shfl(pc.y, o), __shfl(pc.z, o), __shfl(pc.w, o));
            const float k1 = __shfl(ks1.x, o), sk1 = __shfl(ks1.y, o);
            bool pass = false;
            uint32_t w = 0;
            float k3 = 0.f, sk3 = 0.f;
            if (ci < total) {
                w = o_w0 + (ci - o_off);
                const float2 ks2 = b.t3_ks[w];
                const float k2 = ks2.x, sk2 = ks2.y;
                cand++;
                // the pairwise test of the two stored curvatures needs no new arithmetic
                if (fabsf(k1 - k2) <= c.ns * (sk1 + sk2)) {
                    const Anchor A = anchor_of(oa), C = anchor_of(oc), E = load_anchor(b, b.t3_ac[w].y);
                    const float d1 = chord(A, C), d2 = chord(C, E);
                    kappa3(c, A, C, E, d1, d2, k3, sk3);
                    pass = fabsf(k1 - k3) <= c.ns * (sk1 + sk3) && fabsf(k2 - k3) <= c.ns * (sk2 + sk3) &&
                           rz3(c, A, C, E, d1, d2);
                }
            }
            const unsigned long long mk = __ballot(pass);
            const uint32_t np = (uint32_t)__popcll(mk);
            uint32_t at = 0;
            if (np != 0u && lane == 0u) at = atomicAdd(&s_n, np);
            at = __shfl(at, 0);
            if (pass) {
                const uint32_t slot = at + (uint32_t)__popcll(mk & below);
                const uint32_t s0 = o_off > cb ? o_off - cb : 0u;
                if (slot < cap) {
                    b.t5s_u[sb0 + slot] = o_u;
                    b.t5s_w[sb0 + slot] = w;
                    b.t5s_j[sb0 + slot] = o_run + (uint32_t)__popcll(mk & below & ~((1ull << s0) - 1ull));
                    b.t5s_ks[sb0 + slot] = make_float2(k3, sk3);
                }
            }
            if (cnt != 0u && off < cb + 64u && off + cnt > cb) {
                const uint32_t s0 = off > cb ? off - cb : 0u;
                const uint32_t e0 = min(off + cnt - cb, 64u);
                run += (uint32_t)__popcll(mk & lane_range(s0, e0));
            }
        }
        if (u < n) b.t5_cnt[u] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) b.t5s_sub[blockIdx.x] = s_n;
    if (stats) atomicAdd(&t->cand[3], (unsigned long long)cand);
}

// T5s from the block regions to their canonical slots
__global__ __launch_bounds__(256) void k_t5_place(const Batch b, const DevGeom g, const Consts c, uint32_t nsub)
{
    __shared__ uint32_t s_off[kSubLists + 1];
    for (uint32_t i = threadIdx.x; i <= nsub; i += blockDim.x) s_off[i] = b.t5s_soff[i];
    __syncthreads();
    const uint32_t n = s_off[nsub];
    const uint32_t subcap = b.cap_t5s / nsub;
    // whole waves per step (the bucket slots are drawn per wave)
    XCD_STRIDE_BLOCKS(jb, n) {
        const uint32_t j = jb + threadIdx.x;
        bool in = false;
        uint32_t k = 0, bk = 0;
        if (j < xb_.end) {
            const uint32_t i = pair_slot(s_off, j, subcap, nsub);
            const uint32_t u = b.t5s_u[i];
            k = b.t5_off[u] + b.t5s_j[i];
            if (k < b.cap_t5) {
                in = true;
                const float2 ks = b.t5s_ks[i];
                b.t5_u[k] = u;
                b.t5_w[k] = b.t5s_w[i];
                b.t5_ks[k] = ks;
                // the object's seed-lookup bucket
                const uint32_t a = b.t3_ac[u].x;
                const float4 pa = b.md_pos[a];
                bk = bucket_row(b, g, c, a, pa.x, pa.y) + bucket_in_row(ks.x, ks.y, c);
            }
        }
        const uint32_t slot = wave_grouped_inc(b.bk5_cnt, bk, in);
        if (in) {
            b.bk5_id[k] = bk;
            b.bk5_rank[k] = slot;
        }
    }
}

// --------------------------------------------- a6: seed lookup buckets ----
// T3s (resp. T5s) are bucketed by (event, surface of the inner anchor,
// azimuth bin of the inner anchor, curvature bin).  Buckets of one (event,
// surface, azimuth bin) row are contiguous in curvature order, so a pixel
// seed reads one contiguous item range per row it can reach: the rows its
// helix band crosses, restricted to the curvature bins its curvature cut can
// accept (bounded with the row's largest object resolution).


__device__ inline int kappa_bin_d(double k, const Consts &c)
{
    double t = (k + (double)c.kspan) * ((double)c.nkb / (2.0 * (double)c.kspan));
    if (!(t > 0.0)) return 0;
    if (t >= (double)c.nkb) return (int)c.nkb - 1;
    return (int)t;
}

// kind 0: T3 objects, 1: T5 objects
template <int kKind>
__global__ void k_bucket_scatter(const Batch b, const Totals *t)
{
    const uint32_t n = kKind == 0 ? min(t->n_t3, b.cap_t3) : min(t->n_t5, b.cap_t5);
    const uint32_t *off = kKind == 0 ? b.bk3_off : b.bk5_off;
    const uint32_t *id = kKind == 0 ? b.bk3_id : b.bk5_id;
    const uint32_t *rank = kKind == 0 ? b.bk3_rank : b.bk5_rank;
    float4 *bks = kKind == 0 ? b.bk3_ks : b.bk5_ks;
    const float2 *ks = kKind == 0 ? b.t3_ks : b.t5_ks;
    XCD_STRIDE(i, n) {
        const uint32_t pos = off[id[i]] + rank[i];
        const uint32_t a = kKind == 0 ? b.t3_ac[i].x : b.t3_ac[b.t5_u[i]].x;
        const float4 pa = b.md_pos[a];
        const float2 k = ks[i];
        bks[pos] = make_float4(k.x, k.y, atan2f(pa.y, pa.x), __uint_as_float(i));
    }
}

// ------------------------------------------------- a7: pT3 / pT5 --------

struct Seed {
    double kp, skp, phi0, cot, z0, s11, s22, s44;
    double cphi, sphi;       // cos and sin of phi0
};

__device__ inline Seed load_seed(const Batch &b, const Consts &c, uint32_t p)
{
    Seed s;
    const float *par = b.in_par + 5 * (size_t)p;
    const float *cov = b.in_cov + 15 * (size_t)p;
    s.kp = (double)par[0] * c.kB;
    s.skp = c.kB * sqrt((double)cov[0]);
    s.phi0 = par[1];
    s.cot = par[2];
    s.z0 = par[4];
    s.s11 = sqrt((double)cov[5]);
    s.s22 = sqrt((double)cov[9]);
    s.s44 = sqrt((double)cov[14]);
    sincos(s.phi0, &s.sphi, &s.cphi);
    return s;
}

// seeds: the event of each, the finite check of its parameters, and its
// derived binary64 quantities (load_seed), stored once for the roads and the
// seed cuts of every pair
__global__ void k_pls_prep(const Batch b, Totals *t, const Consts c)
{
    const uint32_t n = min(t->n_pls, b.cap_pls);
    const uint32_t n_ev = t->n_ev;
    GRID_STRIDE(p, n) {
        const uint32_t e = find_event(b.ev_pls_off, n_ev, p);
        b.pls_ev[p] = e;
        bool ok = true;
        for (int k = 0; k < 5; k++) ok = ok && isfinite(b.in_par[5 * p + k]);
        for (int k = 0; k < 15; k++) ok = ok && isfinite(b.in_cov[15 * p + k]);
        if (!ok) {
            atomicOr(&t->err, kErrNonFinite);
            atomicOr(&b.ev_err[e], kErrNonFinite);
        }
        const Seed s = load_seed(b, c, p);
        double2 *r = reinterpret_cast<double2 *>(b.pls_seed) + 5 * (size_t)p;
        r[0] = make_double2(s.kp, s.skp);
        r[1] = make_double2(s.phi0, s.cot);
        r[2] = make_double2(s.z0, s.s11);
        r[3] = make_double2(s.s22, s.s44);
        r[4] = make_double2(s.cphi, s.sphi);
    }
}

__device__ inline Seed seed_of(const Batch &b, uint32_t p)
{
    const double2 *r = reinterpret_cast<const double2 *>(b.pls_seed) + 5 * (size_t)p;
    const double2 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4];
    Seed s;
    s.kp = r0.x;
    s.skp = r0.y;
    s.phi0 = r1.x;
    s.cot = r1.y;
    s.z0 = r2.x;
    s.s11 = r2.y;
    s.s22 = r3.x;
    s.s44 = r3.y;
    s.cphi = r4.x;
    s.sphi = r4.y;
    return s;
}

// binary64 seed-object compatibility: curvature, then azimuth and z (barrel)
// or r (disk) of the helix at the object's inner and outer anchors.  The
// helix direction at radius r is phi0 - asin(u), u = r kappa / 2; its unit
// vector follows from cos/sin of phi0 and u, and the azimuth test
// |dphi| <= W (W in [0, pi)) is taken as cos(dphi) >= cos(W), i.e. on the
// dot product of that unit vector with the anchor.
__device__ inline bool p_cut(const Consts &c, const Seed &s, float kobj, float skobj,
                             const Anchor &in, const Anchor &out)
{
    const double ns = c.n_sigma;
    if (!(fabs(s.kp - (double)kobj) <= ns * (s.skp + (double)skobj))) return false;
#pragma unroll 1
    for (int i = 0; i < 2; i++) {
        const Anchor a = i == 0 ? in : out;
        const double x = a.x, y = a.y, z = a.z;
        const double r = sqrt(x * x + y * y);
        const double u = r * s.kp / 2.0;
        if (!(fabs(u) < 1.0)) return false;
        const double cb = sqrt(1.0 - u * u);
        const double dx = s.cphi * cb + s.sphi * u, dy = s.sphi * cb - s.cphi * u;
        const double dot = dx * x + dy * y;
        const double sr = a.disk ? c.sig_c : 0.0;
        const double W = ns * (s.s11 + (r * s.skp + sr * fabs(s.kp)) / (2.0 * cb) + c.sig_rphi / r);
        if (!(W >= 0.0)) return false;
        if (W < kPiD && !(dot >= r * cos(W))) return false;
        if (!a.disk) {
            const double sa = (u == 0.0) ? r : r * asin(u) / u;
            const double zp = s.z0 + s.cot * sa;
            if (!(fabs(z - zp) <= ns * (s.s44 + sa * s.s22 + c.sig_c))) return false;
        } else {
            if (s.cot == 0.0) return false;
            const double sa = (z - s.z0) / s.cot;
            if (!(sa > 0.0)) return false;
            const double w = fabs(s.kp) * sa / 2.0;
            if (!(w < kPiD / 2)) return false;
            const double rp = (w == 0.0) ? sa : sa * sin(w) / w;
            if (!(fabs(r - rp) <= ns * ((s.s44 + sa * s.s22) / fabs(s.cot) + c.sig_c))) return false;
        }
    }
    return true;
}

// Azimuth bins of surface sf that can hold the inner anchor of an object
// linked to seed s; returns false when the helix band misses the surface.
// Conservative bounds of the seed cuts over the surface's anchor radii.
__device__ inline bool seed_road(const Consts &c, const Seed &s, const Surface &sf,
                                 int &b0, int &b1, double &plo, double &pwidth)
{
    const double ns = c.n_sigma;
    const double ak = fabs(s.kp);
    double ra, rb;
    if (sf.kind == LST_BARREL) {
        ra = sf.r1;
        rb = sf.r2;
        if (ak > 0.0 && ra * ak / 2.0 >= 1.0) return false;
        if (ak > 0.0) rb = fmin(rb, 2.0 / ak);
        double ua = ra * s.kp / 2.0, ub = rb * s.kp / 2.0;
        double sa = (ua == 0.0) ? ra : ra * asin(fmax(-1.0, fmin(1.0, ua))) / ua;
        double sb = (ub == 0.0) ? rb : rb * asin(fmax(-1.0, fmin(1.0, ub))) / ub;
        double za = s.z0 + s.cot * sa, zb = s.z0 + s.cot * sb;
        double wz = ns * (s.s44 + sb * s.s22 + c.sig_c) + 1e-3;
        if (fmax(za, zb) + wz < sf.z1 || fmin(za, zb) - wz > sf.z2) return false;
    } else {
        if (s.cot == 0.0) return false;
        double sa = ((double)sf.z1 - s.z0) / s.cot;
        if (!(sa > 0.0)) return false;
        double w = ak * sa / 2.0;
        if (!(w < kPiD / 2)) return false;
        double rp = (w == 0.0) ? sa : sa * sin(w) / w;
        double wr = ns * ((s.s44 + sa * s.s22) / fabs(s.cot) + c.sig_c) + 0.01 / fabs(s.cot) + 0.01;
        ra = fmax((double)sf.r1, rp - wr);
        rb = fmin((double)sf.r2, rp + wr);
        if (ak > 0.0) rb = fmin(rb, 2.0 / ak);
        if (!(ra <= rb)) return false;
    }
    double ua = ra * s.kp / 2.0, ub = rb * s.kp / 2.0;
    if (!(fabs(ua) < 1.0)) return false;
    // azimuth of the seed reduced to [0, 2 pi) so that the bins stay bounded
    double phi0 = fmod(s.phi0, 2.0 * kPiD);
    if (phi0 < 0.0) phi0 += 2.0 * kPiD;
    double pa = phi0 - asin(ua);
    double pb = fabs(ub) >= 1.0 ? phi0 - (ub > 0 ? kPiD / 2 : -kPiD / 2) : phi0 - asin(ub);
    double lo = fmin(pa, pb), hi = fmax(pa, pb);
    double um = fmin(fabs(ub), 1.0);
    double sr = sf.kind == LST_BARREL ? 0.0 : c.sig_c;
    double den = 2.0 * sqrt(fmax(1.0 - um * um, 0.0));
    double W = den > 1e-6 ? ns * (s.s11 + (rb * s.skp + sr * ak) / den + c.sig_rphi / ra) : 10.0;
    double pad = W + 1e-3;
    lo -= pad;
    hi += pad;
    if (!(hi - lo < 2.0 * kPiD) || !(lo > -3.0 * kPiD) || !(hi < 4.0 * kPiD)) {
        b0 = 0;
        b1 = (int)c.nphi - 1;
        plo = 0.0;
        pwidth = 4.0 * kPiD;     // every azimuth
        return true;
    }
    plo = fmod(lo, 2.0 * kPiD);
    if (plo < 0.0) plo += 2.0 * kPiD;
    pwidth = hi - lo;
    // lo, hi lie within [-3 pi, 4 pi] here
    const double scale = (double)c.nphi / (2.0 * kPiD);
    b0 = (int)floor((lo + kPiD) * scale);
    b1 = (int)floor((hi + kPiD) * scale);
    if (b1 - b0 >= (int)c.nphi) b1 = b0 + (int)c.nphi - 1;
    return true;
}

// Road of every (seed, surface) unit: the azimuth bins and curvature bins
// of the buckets that can hold objects linked to the seed (binary64, once
// per unit; shared by the T3 and the T5 lookup).
__global__ __launch_bounds__(256) void k_road(const Batch b, const Totals *t, const DevGeom g, const Consts c)
{
    const uint32_t n = min(t->n_pls, b.cap_pls) * c.n_surf;
    GRID_STRIDE(unit, n) {
        const uint32_t p = unit / c.n_surf, sfi = unit - p * c.n_surf;
        const Surface sf = g.surf[sfi];
        uint4 r = make_uint4(0u, 0u, 0u, 0u);
        float2 rp = make_float2(0.0f, 0.0f);
        int b0 = 0, b1 = -1;
        double plo = 0.0, pwidth = 0.0;
        if (sf.kind <= 1u) {
            const Seed s = seed_of(b, p);
            if (seed_road(c, s, sf, b0, b1, plo, pwidth)) {
                rp = make_float2((float)plo, (float)pwidth);
                // objects of resolution class i: curvature within the seed's
                // window widened by the class's largest resolution
                uint32_t kr[3];
                for (int i = 0; i < 3; i++) {
                    const double wide = c.n_sigma * (s.skp + (double)c.sk_cls[i]) + 1e-6;
                    const int k0 = kappa_bin_d(s.kp - wide, c), k1 = kappa_bin_d(s.kp + wide, c);
                    kr[i] = (uint32_t)k0 | ((uint32_t)k1 << 8);
                }
                const int first = ((b0 % (int)c.nphi) + (int)c.nphi) % (int)c.nphi;
                r.x = (uint32_t)first | ((uint32_t)(b1 - b0 + 1) << 16);
                r.y = kr[0] | (kr[1] << 16);
                r.z = kr[2] | 0x80000000u;
            }
        }
        b.road[unit] = r;
        b.road_phi[unit] = rp;
    }
}

// Candidates: the 64 (seed, surface) units of a wave (one per lane) step
// through the azimuth bins of their roads together, two bins a step: a lane
// loads the offsets of the four ranges of each of its next two bins (the
// curvature range of each resolution class, and the wide objects; all
// sixteen loads in flight together) and stores them in LDS; the wave
// pools the entries of all lanes' ranges and the lanes take them 64 at a
// time, so loads and tests run on full waves however the bucket sizes are
// spread.  An entry finds its owner lane by a binary search over the lanes'
// first-entry offsets, its range in the owner's LDS slot, and the owner's
// azimuth window and curvature by lane shuffles.  Entries inside the road's
// azimuth window (padded, conservative) that pass the exact binary64
// curvature test are appended as (seed, object) pairs to the block's region
// of an unordered pair list; the other seed cuts run in k_pt_eval, one
// thread per pair.
template <int kKind>
__global__ __launch_bounds__(256) void k_ptc(const Batch b, Totals *t, const Consts c, uint32_t nsub, int stats)
{
    // per lane: the starts of the eight ranges of its two bins, then the
    // cumulative sizes c1..c7
    __shared__ uint32_t s_rng[4][15][64];
    __shared__ uint32_t s_mark[4][64];                // pooled-candidate owner marks, one row per wave
    __shared__ uint32_t s_n;                          // appends to this block's region
    const uint32_t n = min(t->n_pls, b.cap_pls) * c.n_surf;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    const uint32_t *bk_off = kKind == 0 ? b.bk3_off : b.bk5_off;
    const float4 *bks = kKind == 0 ? b.bk3_ks : b.bk5_ks;
    const uint32_t cap = (kKind == 0 ? b.cap_ptc3 : b.cap_ptc5) / nsub;
    uint32_t *out_p = (kKind == 0 ? b.ptc3_p : b.ptc5_p) + (size_t)blockIdx.x * cap;
    uint32_t *out_o = (kKind == 0 ? b.ptc3_o : b.ptc5_o) + (size_t)blockIdx.x * cap;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const uint32_t per_row = 3u * c.nkb + 1u;
    const float two_pi = 2.0f * kPiF;
    uint64_t cand = 0;
    // every lane of a wave runs the same number of iterations and steps
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t unit = base + threadIdx.x;
        const uint32_t p = unit / c.n_surf;
        const uint4 r = unit < n ? b.road[unit] : make_uint4(0u, 0u, 0u, 0u);
        const bool road = (r.z & 0x80000000u) != 0u;
        uint32_t row0 = 0, first = 0, nbins = 0;
        double kp = 0.0, skp = 0.0;
        float2 rp = make_float2(0.f, 0.f);
        if (road) {
            const uint32_t sfi = unit - p * c.n_surf;
            kp = (double)b.in_par[5 * (size_t)p] * c.kB;
            skp = c.kB * sqrt((double)b.in_cov[15 * (size_t)p]);
            row0 = (b.pls_ev[p] * c.n_surf + sfi) * c.nphi;
            first = r.x & 0xFFFFu;
            nbins = r.x >> 16;
            rp = b.road_phi[unit];
        }
        const uint32_t kr0 = r.y & 0xFFFFu, kr1 = r.y >> 16, kr2 = r.z & 0xFFFFu;
        for (uint32_t j = 0;; j += 2u) {
            if (__ballot(j < nbins) == 0ull) break;
            // this lane's next two bins: the offsets of their eight ranges,
            // all loads in flight together
            uint32_t T = 0;
            {
                uint32_t lo[8], hi[8];
#pragma unroll
                for (uint32_t h = 0; h < 2u; h++) {
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        lo[4 * h + k] = 0u;
                        hi[4 * h + k] = 0u;
                    }
                    if (j + h < nbins) {
                        uint32_t bin = first + j + h;
                        if (bin >= c.nphi) bin -= c.nphi;
                        const uint32_t rb = (row0 + bin) * per_row;
                        lo[4 * h] = bk_off[rb + (kr0 & 0xFFu)];
                        hi[4 * h] = bk_off[rb + (kr0 >> 8) + 1u];
                        lo[4 * h + 1] = bk_off[rb + c.nkb + (kr1 & 0xFFu)];
                        hi[4 * h + 1] = bk_off[rb + c.nkb + (kr1 >> 8) + 1u];
                        lo[4 * h + 2] = bk_off[rb + 2u * c.nkb + (kr2 & 0xFFu)];
                        hi[4 * h + 2] = bk_off[rb + 2u * c.nkb + (kr2 >> 8) + 1u];
                        lo[4 * h + 3] = bk_off[rb + 3u * c.nkb];
                        hi[4 * h + 3] = bk_off[rb + per_row];
                    }
                }
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    s_rng[wv][k][lane] = lo[k];
                    T += hi[k] > lo[k] ? hi[k] - lo[k] : 0u;
                    if (k < 7) s_rng[wv][8 + k][lane] = T;
                }
            }
            wave_lds_sync();
            const uint32_t incl = wave_incl_scan(T);
            const uint32_t off = incl - T;
            const uint32_t total = wave_last(incl);
            uint32_t carry = 0;
            for (uint32_t cb = 0; cb < total; cb += 64u) {
                const uint32_t ci = cb + lane;
                const uint32_t o = pooled_owner(s_mark[wv], lane, T, off, cb, carry);
                const uint32_t o_off = __shfl(off, o), o_p = __shfl(p, o);
                const double o_kp = __shfl(kp, o), o_skp = __shfl(skp, o);
                const float o_plo = __shfl(rp.x, o), o_pw = __shfl(rp.y, o);
                bool pass = false;
                uint32_t obj = 0;
                if (ci < total) {
                    // range k of the owner's two bins: the last with cum[k] <= tt
                    const uint32_t tt = ci - o_off;
                    uint32_t k = 0, ck = 0;
#pragma unroll
                    for (int q = 0; q < 7; q++) {
                        const uint32_t cum = s_rng[wv][8 + q][o];
                        if (cum <= tt) {
                            k = q + 1;
                            ck = cum;
                        }
                    }
                    const uint32_t i = s_rng[wv][k][o] + (tt - ck);
                    const float4 q = bks[i];
                    cand++;
                    float dphi = q.z - o_plo;
                    dphi -= two_pi * floorf(dphi / two_pi);
                    pass = dphi <= o_pw && fabs(o_kp - (double)q.x) <= c.n_sigma * (o_skp + (double)q.y);
                    obj = __float_as_uint(q.w);
                }
                const unsigned long long mk = __ballot(pass);
                const uint32_t np = (uint32_t)__popcll(mk);
                uint32_t at = 0;
                if (np != 0u && lane == 0u) at = atomicAdd(&s_n, np);
                at = __shfl(at, 0);
                if (pass) {
                    const uint32_t slot = at + (uint32_t)__popcll(mk & below);
                    if (slot < cap) {
                        out_p[slot] = o_p;
                        out_o[slot] = obj;
                    }
                }
            }
            wave_lds_sync();
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) (kKind == 0 ? b.ptc3_sub : b.ptc5_sub)[blockIdx.x] = s_n;
    if (stats) atomicAdd(&t->cand[4 + kKind], (unsigned long long)cand);
}

// Region sizes (nsub <= kSubLists, one block of 256 threads, each summing a
// run of consecutive regions) to dense offsets soff[0..nsub].  need receives
// the total or, when a region overflowed, the list capacity that holds it
// (the host then grows the list and runs the batch again).
__device__ inline void sub_offsets_block(const uint32_t *__restrict__ sub, uint32_t *__restrict__ soff,
                                         uint32_t cap_total, uint32_t nsub, uint32_t *need)
{
    __shared__ uint32_t s_max;
    const uint32_t cap = cap_total / nsub;
    const uint32_t per = (nsub + 255u) / 256u;
    const uint32_t i0 = min(threadIdx.x * per, nsub), i1 = min(i0 + per, nsub);
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    uint32_t sum = 0, vmax = 0;
    for (uint32_t i = i0; i < i1; i++) {
        const uint32_t v = sub[i];
        vmax = max(vmax, v);
        sum += min(v, cap);
    }
    if (vmax > cap) atomicMax(&s_max, vmax);
    uint32_t tot;
    uint32_t ex = block_excl_scan(sum, tot);
    for (uint32_t i = i0; i < i1; i++) {
        soff[i] = ex;
        ex += min(sub[i], cap);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        soff[nsub] = tot;
        *need = s_max > cap ? (uint32_t)min(0xFFFFFFF0ull, (unsigned long long)s_max * nsub) : tot;
    }
}

__global__ __launch_bounds__(256) void k_sub_offsets(const uint32_t *__restrict__ sub,
                                                     uint32_t *__restrict__ soff, uint32_t cap_total,
                                                     uint32_t nsub, uint32_t *need)
{
    sub_offsets_block(sub, soff, cap_total, nsub, need);
}

// The first pass of a scan (blocks 0 .. gridDim.x - 2) and, in the last
// block, the region offsets of a walk's sub-lists: both read only what the
// walk wrote, so one launch does both (one kernel boundary fewer per stage).
__global__ __launch_bounds__(kScanBlock) void k_scan_up_sub(const uint32_t *__restrict__ in,
                                                            const uint32_t *n_ptr, uint32_t cap,
                                                            uint32_t *__restrict__ part,
                                                            const uint32_t *__restrict__ sub,
                                                            uint32_t *__restrict__ soff, uint32_t cap_total,
                                                            uint32_t nsub, uint32_t *need)
{
    if (blockIdx.x == gridDim.x - 1u)
        sub_offsets_block(sub, soff, cap_total, nsub, need);
    else
        scan_up_block(in, n_ptr, cap, part, gridDim.x - 1u, blockIdx.x);
}

// full seed cuts, one thread per pair; an accepted pair draws its rank
// among the accepted pairs of its seed
template <int kKind>
__global__ __launch_bounds__(256) void k_pt_eval(const Batch b, const Consts c, uint32_t nsub)
{
    const uint32_t *soff = kKind == 0 ? b.ptc3_soff : b.ptc5_soff;
    const uint32_t subcap = (kKind == 0 ? b.cap_ptc3 : b.cap_ptc5) / nsub;
    const uint32_t *cp = kKind == 0 ? b.ptc3_p : b.ptc5_p;
    const uint32_t *co = kKind == 0 ? b.ptc3_o : b.ptc5_o;
    uint32_t *rank = kKind == 0 ? b.ptc3_rank : b.ptc5_rank;
    uint32_t *pcnt = kKind == 0 ? b.pt3_cnt : b.pt5_cnt;
    REGION_ENTRIES(i, soff, subcap, nsub) {
        const uint32_t p = cp[i], o = co[i];
        uint32_t ia, io;
        float2 ks;
        if (kKind == 0) {
            const uint2 ac = b.t3_ac[o];
            ia = ac.x;
            io = ac.y;
            ks = b.t3_ks[o];
        } else {
            ia = b.t3_ac[b.t5_u[o]].x;
            io = b.t3_ac[b.t5_w[o]].y;
            ks = b.t5_ks[o];
        }
        const Seed s = seed_of(b, p);
        const bool pass = p_cut(c, s, ks.x, ks.y, load_anchor(b, ia), load_anchor(b, io));
        rank[i] = pass ? atomicAdd(&pcnt[p], 1u) : kInvalid;
    }
}

// accepted pairs to their seed's slots (in rank order)
template <int kKind>
__global__ __launch_bounds__(256) void k_pt_place(const Batch b, uint32_t nsub)
{
    const uint32_t *soff = kKind == 0 ? b.ptc3_soff : b.ptc5_soff;
    const uint32_t subcap = (kKind == 0 ? b.cap_ptc3 : b.cap_ptc5) / nsub;
    const uint32_t *cp = kKind == 0 ? b.ptc3_p : b.ptc5_p;
    const uint32_t *co = kKind == 0 ? b.ptc3_o : b.ptc5_o;
    const uint32_t *rank = kKind == 0 ? b.ptc3_rank : b.ptc5_rank;
    const uint32_t *poff = kKind == 0 ? b.pt3_off : b.pt5_off;
    uint32_t *tp = kKind == 0 ? b.pt3_tp : b.pt5_tp;
    uint32_t *to = kKind == 0 ? b.pt3_to : b.pt5_to;
    const uint32_t cap = kKind == 0 ? b.cap_pt3 : b.cap_pt5;
    REGION_ENTRIES(i, soff, subcap, nsub) {
        const uint32_t r = rank[i];
        if (r == kInvalid) continue;
        const uint32_t p = cp[i];
        const uint32_t k = poff[p] + r;
        if (k < cap) {
            tp[k] = p;
            to[k] = co[i];
        }
    }
}

// first pT index of seed p (seeds p <= n_pls)
template <int kKind>
__device__ inline uint32_t pt_first(const Batch &b, uint32_t p)
{
    return kKind == 0 ? min(b.pt3_off[p], b.cap_pt3) : min(b.pt5_off[p], b.cap_pt5);
}

// canonical order within each seed: every element counts the elements of
// its seed with a smaller object index (ties, which a seed's pairs do not
// have, by position) and moves to that rank
template <int kKind>
__global__ void k_pt_order(const Batch b, const Totals *t)
{
    const uint32_t n = kKind == 0 ? min(t->n_pt3, b.cap_pt3) : min(t->n_pt5, b.cap_pt5);
    const uint32_t *tp = kKind == 0 ? b.pt3_tp : b.pt5_tp;
    const uint32_t *to = kKind == 0 ? b.pt3_to : b.pt5_to;
    uint32_t *out_p = kKind == 0 ? b.pt3_p : b.pt5_p;
    uint32_t *out_o = kKind == 0 ? b.pt3_o : b.pt5_o;
    GRID_STRIDE(j, n) {
        const uint32_t p = tp[j], o = to[j];
        const uint32_t a = pt_first<kKind>(b, p), e = min(pt_first<kKind>(b, p + 1), n);
        uint32_t r = 0;
        for (uint32_t i = a; i < e; i++) {
            const uint32_t w = to[i];
            r += (w < o || (w == o && i < j)) ? 1u : 0u;
        }
        out_p[a + r] = p;
        out_o[a + r] = o;
        // the track-candidate flags: seeds and T5s used by a pT5, seeds used by a pT3
        if (kKind == 1) {
            b.pls_used5[p] = 1u;
            b.t5_used[o] = 1u;
        } else {
            b.pls_used3[p] = 1u;
        }
    }
}

// ------------------------------------------------ a8: track candidates ----

// keep flags over [pT3 | T5 | pLS]: pT3 whose seed has no pT5, T5 in no pT5,
// seeds in neither (every pT5 is a track candidate)
__global__ void k_tc_keep(const Batch b, Totals *t)
{
    const uint32_t n3 = min(t->n_pt3, b.cap_pt3), n5 = min(t->n_t5, b.cap_t5), np = min(t->n_pls, b.cap_pls);
    const uint32_t n = n3 + n5 + np;
    if (blockIdx.x == 0 && threadIdx.x == 0) t->n_tcu = n;
    GRID_STRIDE(i, n) {
        uint32_t keep;
        if (i < n3) keep = b.pls_used5[b.pt3_p[i]] ? 0u : 1u;
        else if (i < n3 + n5) keep = b.t5_used[i - n3] ? 0u : 1u;
        else {
            uint32_t p = i - n3 - n5;
            keep = (b.pls_used5[p] | b.pls_used3[p]) ? 0u : 1u;
        }
        b.tc_cnt[i] = keep;
    }
}

__global__ void k_tc_write(const Batch b, const Totals *t)
{
    const uint32_t n = t->n_tcu;
    const uint32_t n3 = min(t->n_pt3, b.cap_pt3), n5 = min(t->n_t5, b.cap_t5);
    GRID_STRIDE(i, n) {
        if (!b.tc_cnt[i]) continue;
        uint32_t k = b.tc_off[i];
        if (k >= b.cap_tc) continue;
        uint32_t type, idx;
        if (i < n3) { type = LST_TC_PT3; idx = i; }
        else if (i < n3 + n5) { type = LST_TC_T5; idx = i - n3; }
        else { type = LST_TC_PLS; idx = i - n3 - n5; }
        b.tc_type[k] = type;
        b.tc_idx[k] = idx;
    }
}

// ------------------------------------------- track-candidate cleaning ---
//
// Candidates with outer-tracker MDs are compared pairwise through the MDs
// they share: candidate i (i < n_pT5: pT5 i; otherwise the kept entry
// i - n_pT5 of [pT3 | T5 | pLS]) is removed when another candidate that
// ranks higher shares more than half of the smaller of the two MD sets.
// Rank: type (pT5, pT3, T5), then the curvature disagreement q (binary64:
// seed against object for pT5 / pT3, inner against outer T3 for a T5), then
// the index in the candidate's own list.  Seed-only candidates are kept.

__device__ inline uint32_t tcc_type(const Batch &b, uint32_t n5, uint32_t i)
{
    return i < n5 ? LST_TC_PT5 : b.tc_type[i - n5];
}

__device__ inline uint32_t tcc_index(const Batch &b, uint32_t n5, uint32_t i)
{
    return i < n5 ? i : b.tc_idx[i - n5];
}

// MD set and rank quality of every candidate; each MD counts its candidates
// (the returned slot is the candidate's place in that MD's list)
__global__ void k_tcc_prep(const Batch b, const Totals *t)
{
    const uint32_t n5 = min(t->n_pt5, b.cap_pt5);
    const uint32_t n = n5 + min(t->n_tc, b.cap_tc);
    GRID_STRIDE(i, n) {
        const uint32_t typ = tcc_type(b, n5, i), idx = tcc_index(b, n5, i);
        uint32_t nm = 0;
        uint32_t m[5] = {0u, 0u, 0u, 0u, 0u};
        double q = 0.0;
        if (typ != LST_TC_PLS) {
            uint32_t u, w = 0u, obj = 0u, seed = 0u;
            if (typ == LST_TC_PT5) {
                seed = b.pt5_p[idx];
                obj = b.pt5_o[idx];
                u = b.t5_u[obj];
                w = b.t5_w[obj];
            } else if (typ == LST_TC_PT3) {
                seed = b.pt3_p[idx];
                u = b.pt3_o[idx];
            } else {
                u = b.t5_u[idx];
                w = b.t5_w[idx];
            }
            m[0] = b.t3_ac[u].x;
            m[1] = b.ls_b[b.t3_l1[u]];
            m[2] = b.t3_ac[u].y;
            nm = 3u;
            if (typ != LST_TC_PT3) {
                m[3] = b.ls_b[b.t3_l1[w]];
                m[4] = b.t3_ac[w].y;
                nm = 5u;
            }
            if (typ == LST_TC_T5) {
                const float2 ki = b.t3_ks[u], ko = b.t3_ks[w];
                q = fabs((double)ki.x - (double)ko.x) / ((double)ki.y + (double)ko.y);
            } else {
                const double2 sk = reinterpret_cast<const double2 *>(b.pls_seed)[5 * (size_t)seed];
                const float2 ko = typ == LST_TC_PT5 ? b.t5_ks[obj] : b.t3_ks[u];
                q = fabs(sk.x - (double)ko.x) / (sk.y + (double)ko.y);
            }
        }
        b.tcc_nm[i] = nm;
        b.tcc_q[i] = q;
        for (uint32_t k = 0; k < 5u; k++) {
            b.tcc_md[5 * (size_t)i + k] = m[k];
            if (k < nm) b.tcc_rank[5 * (size_t)i + k] = atomicAdd(&b.md_tcc_cnt[m[k]], 1u);
        }
    }
}

__global__ void k_tcc_fill(const Batch b, const Totals *t)
{
    const uint32_t n5 = min(t->n_pt5, b.cap_pt5);
    const uint32_t n = n5 + min(t->n_tc, b.cap_tc);
    GRID_STRIDE(i, n) {
        const uint32_t nm = b.tcc_nm[i];
        for (uint32_t k = 0; k < nm; k++)
            b.md_tcc[b.md_tcc_off[b.tcc_md[5 * (size_t)i + k]] + b.tcc_rank[5 * (size_t)i + k]] = i;
    }
}

// Duplicate decision: a candidate is dropped when one that ranks higher
// shares more than half of the smaller of the two MD sets.  kTccLanes lanes
// take one candidate and split the concatenated candidate lists of its MDs
// between them: a well-measured track leaves tens of candidates on each of
// its MDs, and one lane per candidate left the chip a wave or two per SIMD
// each walking those lists one dependent load after the other.  The group
// stops once any of its lanes has found a reason to drop.
constexpr uint32_t kTccLanes = 16;

__global__ void k_tcc_decide(const Batch b, const Totals *t)
{
    const uint32_t n5 = min(t->n_pt5, b.cap_pt5);
    const uint32_t n = n5 + min(t->n_tc, b.cap_tc);
    const uint32_t lane = threadIdx.x % kTccLanes;
    const uint32_t gbase = (threadIdx.x & 63u) & ~(kTccLanes - 1u);
    const uint64_t gmask = ((1ull << kTccLanes) - 1ull) << gbase;
    const uint32_t groups = gridDim.x * (blockDim.x / kTccLanes);
    for (uint32_t i = (blockIdx.x * blockDim.x + threadIdx.x) / kTccLanes; i < n; i += groups) {
        const uint32_t nm = b.tcc_nm[i];   // the same in every lane of the group
        bool drop = false;
        if (nm) {
            uint32_t m[5], beg[5], pre[5];
            uint32_t total = 0;
#pragma unroll
            for (uint32_t k = 0; k < 5u; k++) {
                m[k] = k < nm ? b.tcc_md[5 * (size_t)i + k] : 0xFFFFFFFFu;
                beg[k] = k < nm ? b.md_tcc_off[m[k]] : 0u;
                const uint32_t deg = k < nm ? b.md_tcc_off[m[k] + 1] - beg[k] : 0u;
                pre[k] = total;
                total += deg;
            }
            const uint32_t ti = tcc_type(b, n5, i), xi = tcc_index(b, n5, i);
            const double qi = b.tcc_q[i];
            for (uint32_t base = 0; base < total; base += kTccLanes) {
                const uint32_t p = base + lane;
                if (p < total && !drop) {
                    uint32_t s = beg[0] + p;
#pragma unroll
                    for (uint32_t k = 1; k < 5u; k++)
                        if (k < nm && p >= pre[k]) s = beg[k] + (p - pre[k]);
                    const uint32_t j = b.md_tcc[s];
                    if (j != i) {
                        const uint32_t tj = tcc_type(b, n5, j);
                        const double qj = b.tcc_q[j];
                        const bool better =
                            tj < ti || (tj == ti && (qj < qi || (qj == qi && tcc_index(b, n5, j) < xi)));
                        if (better) {
                            const uint32_t nj = b.tcc_nm[j];
                            uint32_t shared = 0;
                            for (uint32_t y = 0; y < nj; y++) {
                                const uint32_t mj = b.tcc_md[5 * (size_t)j + y];
#pragma unroll
                                for (uint32_t x = 0; x < 5u; x++) shared += mj == m[x] ? 1u : 0u;
                            }
                            drop = 2u * shared > min(nm, nj);
                        }
                    }
                }
                if (__ballot(drop) & gmask) break;
            }
        }
        const bool any = (__ballot(drop) & gmask) != 0;
        if (lane == 0) b.tcc_keep[i] = any ? 0u : 1u;
    }
}

// per-event first index of every list (row n_ev holds the totals)
__global__ void k_event_table(const Batch b, const Totals *t, const Consts c)
{
    const uint32_t n_mod = c.n_mod;
    const uint32_t n_ev = t->n_ev;
    const uint32_t n3 = min(t->n_pt3, b.cap_pt3), n5 = min(t->n_t5, b.cap_t5);
    GRID_STRIDE(e, n_ev + 1) {
        uint32_t *row = b.ev_tab + (size_t)e * kEvTabCols;
        uint32_t hit = b.ev_hit_off[e], pls = b.ev_pls_off[e];
        uint32_t md = min(b.md_off[e * n_mod], b.cap_md);
        uint32_t ls = min(b.ls_off[md], b.cap_ls);
        uint32_t t3 = min(b.t3_off[ls], b.cap_t3);
        uint32_t t5 = min(b.t5_off[t3], b.cap_t5);
        uint32_t p3 = pt_first<0>(b, pls);
        uint32_t p5 = pt_first<1>(b, pls);
        row[0] = hit;
        row[1] = pls;
        row[2] = md;
        row[3] = ls;
        row[4] = t3;
        row[5] = t5;
        row[6] = p3;
        row[7] = p5;
        row[8] = b.tc_off[min(p3, n3)];
        row[9] = b.tc_off[n3 + min(t5, n5)];
        row[10] = b.tc_off[n3 + n5 + pls];
        row[11] = e < n_ev ? b.ev_err[e] : 0u;   // input errors of the event
    }
}

// ----------------------------------------------------------- launchers ----

void Launcher::scan(const uint32_t *in, uint32_t *out, const uint32_t *n_ptr, uint32_t cap,
                    uint32_t *total, const char *name)
{
    // blocks for the capacity (the count itself is known on the device only)
    const uint32_t nb = (uint32_t)std::max<uint64_t>(
        1u, std::min<uint64_t>(kScanGrid, ((uint64_t)cap + kScanTile - 1) / kScanTile));
    uint32_t *pt = (side && cur == side) ? part_side : part;
    launch(name, k_scan_up, dim3(nb), dim3(kScanBlock), in, n_ptr, cap, pt);
    launch(name, k_scan_down, dim3(nb), dim3(kScanBlock), in, n_ptr, cap, (const uint32_t *)pt, out, total);
}

void Launcher::scan_sub(const uint32_t *in, uint32_t *out, const uint32_t *n_ptr, uint32_t cap, uint32_t *total,
                        const char *name, const uint32_t *sub, uint32_t *soff, uint32_t cap_total, uint32_t nsub,
                        uint32_t *need)
{
    const uint32_t nb = (uint32_t)std::max<uint64_t>(
        1u, std::min<uint64_t>(kScanGrid, ((uint64_t)cap + kScanTile - 1) / kScanTile));
    uint32_t *pt = (side && cur == side) ? part_side : part;
    launch(name, k_scan_up_sub, dim3(nb + 1), dim3(kScanBlock), in, n_ptr, cap, pt, sub, soff, cap_total, nsub,
           need);
    launch(name, k_scan_down, dim3(nb), dim3(kScanBlock), in, n_ptr, cap, (const uint32_t *)pt, out, total);
}

static inline dim3 grid_for(uint64_t units) { return dim3(walk_blocks(units)); }

using LsWalk = void (*)(const Batch, Totals *, const DevGeom, const Consts, uint32_t, int);

// the instantiation of the segment walk for an edge-group size (4, 6, 8) and
// a minimum of waves per SIMD (0: the compiler's choice, 6, 8)
static LsWalk ls_walk_kernel(uint32_t group, uint32_t waves)
{
    switch (group * 16u + waves) {
    case 4 * 16 + 6: return k_ls<4, 6>;
    case 4 * 16 + 8: return k_ls<4, 8>;
    case 4 * 16: return k_ls<4, 1>;
    case 8 * 16 + 6: return k_ls<8, 6>;
    case 8 * 16 + 8: return k_ls<8, 8>;
    case 8 * 16: return k_ls<8, 1>;
    case 6 * 16 + 6: return k_ls<6, 6>;
    case 6 * 16 + 8: return k_ls<6, 8>;
    default: return k_ls<6, 1>;
    }
}

static const char *const kStageRange[LST_N_STAGES] = {"lst stage: ingest",     "lst stage: mini-doublets",
                                                      "lst stage: line segments", "lst stage: T3",
                                                      "lst stage: T5",          "lst stage: seed lookup",
                                                      "lst stage: pT3/pT5",     "lst stage: track candidates"};

void Launcher::set_stage(int st)
{
    stage = st;
    if (range_open) roctxRangePop();
    range_open = st >= 0 && st < LST_N_STAGES;
    if (range_open) roctxRangePushA(kStageRange[st]);
}

void Launcher::end_stages()
{
    if (range_open) roctxRangePop();
    range_open = false;
}

void enqueue_chain(Launcher &L, const Batch &b, Totals *t, const DevGeom &g, const Consts &c, int stats)
{
    const dim3 blk(256);
    const uint32_t n_mod = c.n_mod;
    const uint32_t cap_rows = b.cap_ev * c.n_surf * c.nphi;
    const uint32_t cap_bk = cap_rows * (3 * c.nkb + 1);
    const uint64_t cap_pu = (uint64_t)b.cap_pls * c.n_surf;
    const dim3 gwalk = grid_for(cap_pu);
    const uint32_t nsub = gwalk.x;
    // Two streams: the seed checks and roads, then (after T3) T5, its
    // buckets and pT5, run on the side stream alongside the main chain; the
    // track-candidate selection waits for both.
    L.on_side(false);
    L.set_stage(LST_STAGE_INGEST);
    launch_setup(L, b, t, c);
    L.fork(0);
    // Side: the seed quantities and roads, and the counters of later stages
    // that need clearing; main: a1, hit ingest and sort by (event, module,
    // sensor).  Enqueued in turn, the main stream's first (the enqueueing
    // costs of the branches after the T3 placement, below, hold here too).
    const uint32_t n_sl = (2u * n_mod + g.hist_slice - 1u) / g.hist_slice;
    const dim3 gh((unsigned)std::min<uint64_t>((uint64_t)b.cap_ev * n_sl, kMaxGrid));
    const std::function<void()> ingest_ops[] = {
        [&] {
            L.launch_lds("hit_hist", k_hit_hist, gh, dim3(kHistBlock), g.hist_slice * 4u, b, t, n_mod,
                         g.hist_slice);
        },
        [&] { L.scan(b.bin_cnt, b.bin_off, &t->n_bins, b.cap_ev * 2u * n_mod, &t->n_sorted, "scan_hits"); },
        [&] { L.launch("hit_scatter", k_hit_scatter, grid_for(b.cap_hits), blk, b, (const Totals *)t); },
        [&] { L.launch("hit_gather", k_hit_gather, grid_for(b.cap_hits), blk, b, t, g.mod_ext, n_mod); },
    };
    const std::function<void()> seed_ops[] = {
        [&] { L.launch("pls_prep", k_pls_prep, grid_for(b.cap_pls), blk, b, t, c); },
        [&] { L.launch("road", k_road, grid_for(cap_pu), blk, b, (const Totals *)t, g, c); },
        [&] {
            L.launch("zero", k_zero_u32, grid_for((uint64_t)cap_bk + 1), blk, b.bk3_cnt, &t->n_bk, cap_bk, 1u);
            L.launch("zero", k_zero_u32, grid_for((uint64_t)cap_bk + 1), blk, b.bk5_cnt, &t->n_bk, cap_bk, 1u);
        },
        [&] {
            L.launch("zero", k_zero_u32, grid_for((uint64_t)b.cap_pls + 1), blk, b.pt3_cnt, &t->n_pls, b.cap_pls, 1u);
            L.launch("zero", k_zero_u32, grid_for((uint64_t)b.cap_pls + 1), blk, b.pt5_cnt, &t->n_pls, b.cap_pls, 1u);
            L.launch("zero8", k_zero_u8, grid_for(b.cap_pls), blk, b.pls_used5, &t->n_pls, b.cap_pls);
            L.launch("zero8", k_zero_u8, grid_for(b.cap_pls), blk, b.pls_used3, &t->n_pls, b.cap_pls);
        },
    };
    for (size_t k = 0; k < 4; k++) {
        L.on_side(false);
        L.set_stage(LST_STAGE_INGEST);
        ingest_ops[k]();
        L.on_side(true);
        L.set_stage(LST_STAGE_SEED_LOOKUP);
        seed_ops[k]();
    }
    L.mark(0);                           // the main stream waits for this only before its seed-lookup stage
    L.on_side(false);
    // a2: mini-doublets
    L.set_stage(LST_STAGE_MD);
    // small batches: count and fill in place for latency; large ones: pooled walk
    const dim3 gmd = grid_for(b.cap_hits);
    if (b.cap_md <= kLsWaveMaxMd) {
        L.launch("md_count", k_md_direct<false>, gmd, blk, b, t, g, c, stats);
        L.scan(b.md_cnt, b.md_hoff, &t->n_sorted, b.cap_hits, &t->n_md, "scan_md");
        L.launch("md_fill", k_md_direct<true>, gmd, blk, b, t, g, c, 0);
        L.launch("md_units", k_md_units, grid_for((uint64_t)b.cap_ev * n_mod + 1), blk, b, (const Totals *)t);
    } else {
        const uint32_t nsub_md = gmd.x;
        L.launch("md_walk", k_md, gmd, blk, b, t, g, c, nsub_md, stats);
        L.scan_sub(b.md_cnt, b.md_hoff, &t->n_sorted, b.cap_hits, &t->n_md, "scan_md", b.mds_sub, b.mds_soff,
                   b.cap_mds, nsub_md, &t->n_mds);
        L.launch("md_place", k_md_place, grid_for(std::max<uint64_t>(b.cap_md, (uint64_t)b.cap_ev * n_mod + 1)), blk,
                 b, (const Totals *)t, g, c, nsub_md);
    }
    // a3: line segments over the connection map
    L.set_stage(LST_STAGE_LS);
    // small batches: 32 lanes per MD for latency; large ones: pooled walk
    if (b.cap_md <= kLsWaveMaxMd) {
        L.launch("ls_count", k_ls_wave<false>, grid_for(32ull * b.cap_md), blk, b, t, g, c, stats);
        L.scan(b.ls_cnt, b.ls_off, &t->n_md, b.cap_md, &t->n_ls, "scan_ls");
        L.launch("ls_fill", k_ls_wave<true>, grid_for(32ull * b.cap_md), blk, b, t, g, c, 0);
    } else {
        const dim3 gls = grid_for(b.cap_md);
        const uint32_t nsub_ls = gls.x;
        L.launch("ls_walk", ls_walk_kernel(c.ls_group, c.ls_waves), gls, blk, b, t, g, c, nsub_ls, stats);
        L.scan_sub(b.ls_cnt, b.ls_off, &t->n_md, b.cap_md, &t->n_ls, "scan_ls", b.lss_sub, b.lss_soff, b.cap_lss,
                   nsub_ls, &t->n_lss);
        L.launch("ls_place", k_ls_place, grid_for(b.cap_ls), blk, b, nsub_ls);
    }
    // a4: T3
    L.set_stage(LST_STAGE_T3);
    const dim3 gt3 = grid_for(b.cap_ls);
    const uint32_t nsub_t3 = gt3.x;
    L.launch("t3_walk", k_t3, gt3, blk, b, t, c, nsub_t3, stats);
    L.scan_sub(b.t3_cnt, b.t3_off, &t->n_ls, b.cap_ls, &t->n_t3, "scan_t3", b.t3s_sub, b.t3s_soff, b.cap_t3s,
               nsub_t3, &t->n_t3s);
    L.wait(0);                           // the placement counts into the cleared T3 buckets
    L.launch("t3_place", k_t3_place, grid_for(b.cap_t3), blk, b, g, c, nsub_t3);

    // Two branches after the T3 placement: on the side stream a5 T5, its
    // seed-lookup buckets (a6) and pT5 (a7); on the main stream the T3
    // buckets (a6) and pT3 (a7), the longer of the two.  Every launch costs
    // the host a few microseconds to enqueue (also when a captured graph is
    // replayed, node after node), so the two branches' launches are enqueued
    // in turn, the main branch's first: enqueued one branch after the other,
    // the second started only once the first branch's dozen launches were
    // queued, 50-75 us after the placement.
    L.fork(1);
    struct Op {
        int stage;
        std::function<void()> run;
    };
    const Op side_ops[] = {
        {LST_STAGE_T5, [&] { L.launch("t5_walk", k_t5, grid_for(b.cap_t3), blk, b, t, c, grid_for(b.cap_t3).x, stats); }},
        {LST_STAGE_T5,
         [&] {
             L.scan_sub(b.t5_cnt, b.t5_off, &t->n_t3, b.cap_t3, &t->n_t5, "scan_t5", b.t5s_sub, b.t5s_soff,
                        b.cap_t5s, grid_for(b.cap_t3).x, &t->n_t5s);
         }},
        {LST_STAGE_T5,
         [&] { L.launch("t5_place", k_t5_place, grid_for(b.cap_t5), blk, b, g, c, grid_for(b.cap_t3).x); }},
        {LST_STAGE_SEED_LOOKUP, [&] { L.scan(b.bk5_cnt, b.bk5_off, &t->n_bk, cap_bk, &t->n_bk5, "scan_bucket"); }},
        {LST_STAGE_SEED_LOOKUP,
         [&] { L.launch("bucket_scatter", k_bucket_scatter<1>, grid_for(b.cap_t5), blk, b, (const Totals *)t); }},
        {LST_STAGE_SEED_LOOKUP, [&] { L.launch("pt5c_walk", k_ptc<1>, gwalk, blk, b, t, c, nsub, stats); }},
        {LST_STAGE_PT,
         [&] {
             L.launch("sub_offsets", k_sub_offsets, dim3(1), blk, b.ptc5_sub, b.ptc5_soff, b.cap_ptc5, nsub,
                      &t->n_ptc5);
         }},
        {LST_STAGE_PT, [&] { L.launch("pt5_eval", k_pt_eval<1>, dim3(nsub), blk, b, c, nsub); }},
        {LST_STAGE_PT, [&] { L.scan(b.pt5_cnt, b.pt5_off, &t->n_pls, b.cap_pls, &t->n_pt5, "scan_pt"); }},
        {LST_STAGE_PT, [&] { L.launch("pt_place", k_pt_place<1>, dim3(nsub), blk, b, nsub); }},
        {LST_STAGE_PT, [&] { L.launch("zero8", k_zero_u8, grid_for(b.cap_t5), blk, b.t5_used, &t->n_t5, b.cap_t5); }},
        {LST_STAGE_PT,
         [&] { L.launch("pt_order", k_pt_order<1>, grid_for(b.cap_pt5), blk, b, (const Totals *)t); }},
    };
    const Op main_ops[] = {
        {LST_STAGE_SEED_LOOKUP, [&] { L.scan(b.bk3_cnt, b.bk3_off, &t->n_bk, cap_bk, &t->n_bk3, "scan_bucket"); }},
        {LST_STAGE_SEED_LOOKUP,
         [&] { L.launch("bucket_scatter", k_bucket_scatter<0>, grid_for(b.cap_t3), blk, b, (const Totals *)t); }},
        {LST_STAGE_SEED_LOOKUP, [&] { L.launch("pt3c_walk", k_ptc<0>, gwalk, blk, b, t, c, nsub, stats); }},
        {LST_STAGE_PT,
         [&] {
             L.launch("sub_offsets", k_sub_offsets, dim3(1), blk, b.ptc3_sub, b.ptc3_soff, b.cap_ptc3, nsub,
                      &t->n_ptc3);
         }},
        {LST_STAGE_PT, [&] { L.launch("pt3_eval", k_pt_eval<0>, dim3(nsub), blk, b, c, nsub); }},
        {LST_STAGE_PT, [&] { L.scan(b.pt3_cnt, b.pt3_off, &t->n_pls, b.cap_pls, &t->n_pt3, "scan_pt"); }},
        {LST_STAGE_PT, [&] { L.launch("pt_place", k_pt_place<0>, dim3(nsub), blk, b, nsub); }},
        {LST_STAGE_PT,
         [&] { L.launch("pt_order", k_pt_order<0>, grid_for(b.cap_pt3), blk, b, (const Totals *)t); }},
    };
    const size_t n_side = sizeof(side_ops) / sizeof(side_ops[0]), n_main = sizeof(main_ops) / sizeof(main_ops[0]);
    for (size_t k = 0; k < std::max(n_side, n_main); k++) {
        if (k < n_main) {
            L.on_side(false);
            L.set_stage(main_ops[k].stage);
            main_ops[k].run();
        }
        if (k < n_side) {
            L.on_side(true);
            L.set_stage(side_ops[k].stage);
            side_ops[k].run();
        }
    }
    L.on_side(false);

    // a8: track candidates, once both branches are done
    L.mark(1);
    L.wait(1);
    L.set_stage(LST_STAGE_TC);
    L.launch("tc_keep", k_tc_keep, grid_for((uint64_t)b.cap_pt3 + b.cap_t5 + b.cap_pls), blk, b, t);
    L.scan(b.tc_cnt, b.tc_off, &t->n_tcu, b.cap_pt3 + b.cap_t5 + b.cap_pls, &t->n_tc, "scan_tc");
    L.launch("tc_write", k_tc_write, grid_for((uint64_t)b.cap_pt3 + b.cap_t5 + b.cap_pls), blk, b,
             (const Totals *)t);
    if (c.flags & LST_FLAG_TC_CLEAN) {
        const uint64_t cap_tcc = (uint64_t)b.cap_pt5 + b.cap_tc;
        L.launch("zero", k_zero_u32, grid_for((uint64_t)b.cap_md + 1), blk, b.md_tcc_cnt, &t->n_md, b.cap_md, 1u);
        L.launch("tcc_prep", k_tcc_prep, grid_for(cap_tcc), blk, b, (const Totals *)t);
        L.scan(b.md_tcc_cnt, b.md_tcc_off, &t->n_md, b.cap_md, &t->n_tccm, "scan_tcc");
        L.launch("tcc_fill", k_tcc_fill, grid_for(cap_tcc), blk, b, (const Totals *)t);
        L.launch("tcc_decide", k_tcc_decide, grid_for(cap_tcc * kTccLanes), blk, b, (const Totals *)t);
    }
    L.launch("event_table", k_event_table, grid_for(b.cap_ev + 1), blk, b, (const Totals *)t, c);
    L.end_stages();
}

__global__ void k_event_init(Totals *t, uint32_t *__restrict__ hit_off, uint32_t *__restrict__ pls_off,
                             uint32_t n_hits, uint32_t n_pls)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        t->n_ev = 1u;
        t->n_hits = n_hits;
        t->n_pls = n_pls;
        hit_off[0] = 0u;
        hit_off[1] = n_hits;
        pls_off[0] = 0u;
        pls_off[1] = n_pls;
    }
}

// The lists of a one-event batch as flat pairs: MD (lower, upper input hit),
// LS (inner, outer MD), T3 (inner, outer LS), T5 (inner, outer T3), pT3 /
// pT5 (seed, object), TC (type, index): every pT5, then the kept pT3s, T5s
// and seeds in the order of the keep flags.
__global__ void k_event_out(const Batch b, const Totals *t, const EventOut o)
{
    const uint32_t nmd = t->n_md, nls = t->n_ls, nt3 = t->n_t3, nt5 = t->n_t5;
    const uint32_t np3 = t->n_pt3, np5 = t->n_pt5, ntc = t->n_tc;
    const uint64_t n = (uint64_t)nmd + nls + nt3 + nt5 + np3 + np5 + np5 + ntc;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t k = i;
        uint32_t *dst;
        uint32_t a, c;
        if (k < nmd) { dst = o.md; a = b.md_hlo[k]; c = b.md_hup[k]; }
        else if ((k -= nmd) < nls) { dst = o.ls; a = b.ls_a[k]; c = b.ls_b[k]; }
        else if ((k -= nls) < nt3) {
            dst = o.t3; a = b.t3_l1[k]; c = b.t3_l2[k];
            if (o.t3_kappa) o.t3_kappa[k] = b.t3_ks[k].x;
        }
        else if ((k -= nt3) < nt5) { dst = o.t5; a = b.t5_u[k]; c = b.t5_w[k]; }
        else if ((k -= nt5) < np3) { dst = o.pt3; a = b.pt3_p[k]; c = b.pt3_o[k]; }
        else if ((k -= np3) < np5) { dst = o.pt5; a = b.pt5_p[k]; c = b.pt5_o[k]; }
        else if ((k -= np5) < np5) { dst = o.tc; a = LST_TC_PT5; c = (uint32_t)k; }
        else { k -= np5; dst = o.tc + 2u * np5; a = b.tc_type[k]; c = b.tc_idx[k]; }
        dst[2 * k] = a;
        dst[2 * k + 1] = c;
    }
}

// Served events arrive as one block per event in host order
// [x | y | z | module | sensor | seed parameters | seed covariance], each
// part starting at a multiple of 16 bytes (served_block_bytes); the blocks
// are copied to the device as they are and unpacked here into the batch's
// arrays.
__device__ inline uint32_t pad16(uint32_t v) { return (v + 15u) & ~15u; }

__global__ void k_unpack(const Batch b, const Totals *t, const char *__restrict__ raw,
                         const unsigned long long *__restrict__ raw_off)
{
    const uint32_t n_ev = t->n_ev, nh = min(t->n_hits, b.cap_hits), np = min(t->n_pls, b.cap_pls);
    GRID_STRIDE(h, nh) {
        const uint32_t e = find_event(b.ev_hit_off, n_ev, h);
        const uint32_t i = h - b.ev_hit_off[e], n = b.ev_hit_off[e + 1] - b.ev_hit_off[e];
        const char *blk = raw + raw_off[e];
        const uint32_t s4 = pad16(4u * n);
        b.in_x[h] = reinterpret_cast<const float *>(blk)[i];
        b.in_y[h] = reinterpret_cast<const float *>(blk + s4)[i];
        b.in_z[h] = reinterpret_cast<const float *>(blk + 2u * s4)[i];
        b.in_mod[h] = reinterpret_cast<const uint32_t *>(blk + 3u * s4)[i];
        b.in_sen[h] = reinterpret_cast<const uint8_t *>(blk + 4u * s4)[i];
    }
    GRID_STRIDE(p, np) {
        const uint32_t e = find_event(b.ev_pls_off, n_ev, p);
        const uint32_t j = p - b.ev_pls_off[e], m = b.ev_pls_off[e + 1] - b.ev_pls_off[e];
        const uint32_t n = b.ev_hit_off[e + 1] - b.ev_hit_off[e];
        const char *par = raw + raw_off[e] + 4u * pad16(4u * n) + pad16(n);
        const float *pp = reinterpret_cast<const float *>(par) + 5u * j;
        const float *pc = reinterpret_cast<const float *>(par + pad16(20u * m)) + 15u * j;
        for (uint32_t w = 0; w < 5u; w++) b.in_par[5u * (size_t)p + w] = pp[w];
        for (uint32_t w = 0; w < 15u; w++) b.in_cov[15u * (size_t)p + w] = pc[w];
        b.in_nhit[p] = reinterpret_cast<const uint8_t *>(par + pad16(20u * m) + pad16(60u * m))[j];
    }
}

// Output image of a batch, in 32-bit words: the event table ((n_ev + 1) rows),
// then per event the number of kept candidates of the duplicate cleaning,
// then per event the number of exported seeds, then each event's lists in
// the layout of lst_event_out with event-local indices: MD, LS, T3, T5, pT3,
// pT5 pairs, the track-candidate pairs (every pT5, then the kept pT3, T5 and
// seed entries), the T3 curvatures, with the cleaning the candidates it
// keeps, and the exported seeds.  The host copies a batch's outputs
// in one transfer and hands each event pointers into it.
__device__ inline uint64_t image_words_before(const uint32_t *r, bool clean)
{
    // r holds the first index of every list of an event: the words of the
    // images of all events before it, up to those of event 0 (the last term:
    // room for the exported seeds, one word per seed-only candidate)
    const uint64_t pairs = (uint64_t)r[2] + r[3] + r[4] + r[5] + r[6] + 2ull * r[7] + r[8] + r[9] + r[10];
    return 2ull * pairs + r[4] + (clean ? 2ull * ((uint64_t)r[7] + r[8] + r[9] + r[10]) : 0ull) + r[10];
}

struct EventImage {
    uint32_t *md, *ls, *t3, *t5, *pt3, *pt5, *tc, *kappa, *tcc, *seeds;
    uint32_t cp5, c3, c5;   // pT5s, and track candidates from pT3s and from T5s
};

__device__ inline EventImage event_image(uint32_t *img, uint64_t head, const uint32_t *tab, uint32_t e, bool clean)
{
    const uint32_t *r0 = tab + (size_t)e * kEvTabCols, *r1 = r0 + kEvTabCols;
    EventImage m;
    const uint32_t cmd = r1[2] - r0[2], cls = r1[3] - r0[3], ct3 = r1[4] - r0[4], ct5 = r1[5] - r0[5];
    const uint32_t cp3 = r1[6] - r0[6];
    m.cp5 = r1[7] - r0[7];
    m.c3 = r1[8] - r0[8];
    m.c5 = r1[9] - r0[9];
    const uint32_t ctc = m.cp5 + m.c3 + m.c5 + (r1[10] - r0[10]);
    m.md = img + head + (image_words_before(r0, clean) - image_words_before(tab, clean));
    m.ls = m.md + 2u * cmd;
    m.t3 = m.ls + 2u * cls;
    m.t5 = m.t3 + 2u * ct3;
    m.pt3 = m.t5 + 2u * ct5;
    m.pt5 = m.pt3 + 2u * cp3;
    m.tc = m.pt5 + 2u * m.cp5;
    m.kappa = m.tc + 2u * ctc;
    m.tcc = m.kappa + ct3;
    m.seeds = m.tcc + (clean ? 2u * ctc : 0u);
    return m;
}

// The blocks of row y take event y and stride over its entries, list by
// list (consecutive threads, consecutive entries); row 0 also copies the
// event table.  Nothing is written at or past cap words.
__global__ void k_pack(const Batch b, const Totals *t, uint32_t *__restrict__ img, uint64_t head, uint64_t cap,
                       uint32_t clean)
{
    const uint32_t n_ev = t->n_ev;
    const uint32_t e = blockIdx.y;
    if (e >= n_ev) return;
    const uint32_t *tab = b.ev_tab;
    const uint32_t stride = gridDim.x * blockDim.x, first = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0u) {
        const uint32_t n_tab = (n_ev + 1u) * kEvTabCols;
        for (uint32_t q = first; q < n_tab; q += stride)
            if (q < cap) img[q] = tab[q];
    }
    const uint32_t *r0 = tab + (size_t)e * kEvTabCols, *r1 = r0 + kEvTabCols;
    const EventImage m = event_image(img, head, tab, e, clean != 0u);
    const uint32_t md0 = r0[2], ls0 = r0[3], t30 = r0[4], t50 = r0[5], p30 = r0[6], p50 = r0[7], pls0 = r0[1];
    const uint32_t cmd = r1[2] - md0, cls = r1[3] - ls0, ct3 = r1[4] - t30, ct5 = r1[5] - t50;
    const uint32_t cp3 = r1[6] - p30, cp = r1[10] - r0[10];
    // entry q of the event: [md | ls | t3 | t5 | pt3 | pt5 | pT5 candidates |
    // candidates from pT3s, T5s, seeds | curvatures]
    const uint32_t b1 = cmd, b2 = b1 + cls, b3 = b2 + ct3, b4 = b3 + ct5, b5 = b4 + cp3, b6 = b5 + m.cp5;
    const uint32_t b7 = b6 + m.cp5, b8 = b7 + m.c3, b9 = b8 + m.c5, b10 = b9 + cp, b11 = b10 + ct3;
    for (uint32_t q = first; q < b11; q += stride) {
        uint32_t *d;
        uint32_t x, y;
        if (q < b1) {
            const uint32_t k = md0 + q;
            d = m.md + 2u * q; x = b.md_hlo[k]; y = b.md_hup[k];
        } else if (q < b2) {
            const uint32_t i = q - b1, k = ls0 + i;
            d = m.ls + 2u * i; x = b.ls_a[k] - md0; y = b.ls_b[k] - md0;
        } else if (q < b3) {
            const uint32_t i = q - b2, k = t30 + i;
            d = m.t3 + 2u * i; x = b.t3_l1[k] - ls0; y = b.t3_l2[k] - ls0;
        } else if (q < b4) {
            const uint32_t i = q - b3, k = t50 + i;
            d = m.t5 + 2u * i; x = b.t5_u[k] - t30; y = b.t5_w[k] - t30;
        } else if (q < b5) {
            const uint32_t i = q - b4, k = p30 + i;
            d = m.pt3 + 2u * i; x = b.pt3_p[k] - pls0; y = b.pt3_o[k] - t30;
        } else if (q < b6) {
            const uint32_t i = q - b5, k = p50 + i;
            d = m.pt5 + 2u * i; x = b.pt5_p[k] - pls0; y = b.pt5_o[k] - t50;
        } else if (q < b7) {
            const uint32_t i = q - b6;
            d = m.tc + 2u * i; x = LST_TC_PT5; y = i;
        } else if (q < b10) {
            // index relative to the event's first object of the candidate's kind
            const uint32_t i = q - b7;
            uint32_t k, base;
            if (q < b8) { k = r0[8] + i; base = p30; }
            else if (q < b9) { k = r0[9] + (q - b8); base = t50; }
            else { k = r0[10] + (q - b9); base = pls0; }
            d = m.tc + 2u * (m.cp5 + i); x = b.tc_type[k]; y = b.tc_idx[k] - base;
        } else {
            const uint32_t i = q - b10;
            d = m.kappa + i;
            if ((uint64_t)(d - img) < cap) *d = __float_as_uint(b.t3_ks[t30 + i].x);
            continue;
        }
        if ((uint64_t)(d - img) + 1u < cap) {
            d[0] = x;
            d[1] = y;
        }
    }
}

// Duplicate cleaning: the kept candidates of each event, in the order of its
// track-candidate list, and their number (one block per event).
__global__ void __launch_bounds__(256) k_pack_tcc(const Batch b, const Totals *t, uint32_t *__restrict__ img,
                                                  uint64_t head, uint64_t cap)
{
    __shared__ uint32_t s_cnt[4];
    const uint32_t n_ev = t->n_ev;
    const uint32_t e = blockIdx.x;
    if (e >= n_ev) return;
    const uint32_t *tab = b.ev_tab;
    const uint32_t *r0 = tab + (size_t)e * kEvTabCols, *r1 = r0 + kEvTabCols;
    const uint32_t np5 = tab[(size_t)n_ev * kEvTabCols + 7];
    const EventImage m = event_image(img, head, tab, e, true);
    const uint32_t ctc = m.cp5 + m.c3 + m.c5 + (r1[10] - r0[10]);
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint32_t kept = 0;
    for (uint32_t j0 = 0; j0 < ctc; j0 += 256u) {
        const uint32_t j = j0 + threadIdx.x;
        bool keep = false;
        uint32_t x = 0, y = 0;
        if (j < ctc) {
            if (j < m.cp5) {
                keep = b.tcc_keep[r0[7] + j] != 0;
                x = LST_TC_PT5;
                y = j;
            } else {
                uint32_t r = j - m.cp5, col = 8u;
                if (r >= m.c3) { r -= m.c3; col = 9u; }
                if (col == 9u && r >= m.c5) { r -= m.c5; col = 10u; }
                const uint32_t k = r0[col] + r;
                const uint32_t base = col == 8u ? r0[6] : col == 9u ? r0[5] : r0[1];
                keep = b.tcc_keep[np5 + k] != 0;
                x = b.tc_type[k];
                y = b.tc_idx[k] - base;
            }
        }
        const unsigned long long bal = __ballot(keep);
        if (lane == 0) s_cnt[wv] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = kept;
        for (uint32_t w = 0; w < wv; w++) before += s_cnt[w];
        before += (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (keep) {
            uint32_t *d = m.tcc + 2u * before;
            if ((uint64_t)(d - img) + 1u < cap) {
                d[0] = x;
                d[1] = y;
            }
        }
        kept += s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        __syncthreads();
    }
    const uint64_t at = (uint64_t)(n_ev + 1) * kEvTabCols + e;
    if (threadIdx.x == 0 && at < cap) img[at] = kept;
}

// Seed export: the seed-only candidates of each event (in increasing seed
// order) with at least 4 pixel hits, or with 3 as well when triplets are
// exported, compacted per event (one block per event), and their number.
__global__ void __launch_bounds__(256) k_pack_seeds(const Batch b, const Totals *t, uint32_t *__restrict__ img,
                                                    uint64_t head, uint64_t cap, uint32_t clean, uint32_t triplets)
{
    __shared__ uint32_t s_cnt[4];
    const uint32_t n_ev = t->n_ev;
    const uint32_t e = blockIdx.x;
    if (e >= n_ev) return;
    const uint32_t *tab = b.ev_tab;
    const uint32_t *r0 = tab + (size_t)e * kEvTabCols, *r1 = r0 + kEvTabCols;
    const EventImage m = event_image(img, head, tab, e, clean != 0u);
    const uint32_t cp = r1[10] - r0[10];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint32_t kept = 0;
    for (uint32_t j0 = 0; j0 < cp; j0 += 256u) {
        const uint32_t j = j0 + threadIdx.x;
        bool keep = false;
        uint32_t seed = 0;
        if (j < cp) {
            const uint32_t g = b.tc_idx[r0[10] + j];   // the seed's index in the batch
            const uint32_t nh = b.in_nhit[g];
            keep = nh >= 4u || (triplets != 0u && nh == 3u);
            seed = g - r0[1];
        }
        const unsigned long long bal = __ballot(keep);
        if (lane == 0) s_cnt[wv] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = kept;
        for (uint32_t w = 0; w < wv; w++) before += s_cnt[w];
        before += (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (keep) {
            uint32_t *d = m.seeds + before;
            if ((uint64_t)(d - img) < cap) *d = seed;
        }
        kept += s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        __syncthreads();
    }
    const uint64_t at = (uint64_t)(n_ev + 1) * kEvTabCols + n_ev + e;
    if (threadIdx.x == 0 && at < cap) img[at] = kept;
}

void launch_pack(Launcher &L, const Batch &b, const Totals *t, uint32_t *img, uint32_t n_ev, uint64_t head,
                 uint64_t cap, bool clean, bool triplets, uint64_t n_items)
{
    // the image goes over the host link (≈ 55 GB/s), which 256 blocks keep
    // busy; the rest of the device stays free for the other slot's chain
    (void)n_items;
    const uint32_t bx = std::max<uint32_t>(1u, 256u / std::max<uint32_t>(n_ev, 1u));
    if (n_ev) L.launch("pack", k_pack, dim3(bx, n_ev), dim3(256), b, t, img, head, cap, clean ? 1u : 0u);
    if (clean && n_ev) L.launch("pack_tcc", k_pack_tcc, dim3(n_ev), dim3(256), b, t, img, head, cap);
    if (n_ev)
        L.launch("pack_seeds", k_pack_seeds, dim3(n_ev), dim3(256), b, t, img, head, cap, clean ? 1u : 0u,
                 triplets ? 1u : 0u);
}

void launch_unpack(Launcher &L, const Batch &b, const Totals *t, const char *raw, const unsigned long long *raw_off)
{
    L.launch("unpack", k_unpack, grid_for(b.cap_hits), dim3(256), b, t, raw, raw_off);
}

void launch_event_init(Launcher &L, const Batch &b, Totals *t, uint32_t n_hits, uint32_t n_pls)
{
    L.launch("event_init", k_event_init, dim3(1), dim3(64), t, b.ev_hit_off, b.ev_pls_off, n_hits, n_pls);
}

void launch_event_out(Launcher &L, const Batch &b, const Totals *t, const EventOut &o, uint64_t n_items)
{
    L.launch("event_out", k_event_out, grid_for(n_items), dim3(256), b, t, o);
}

void launch_setup(Launcher &L, const Batch &b, Totals *t, const Consts &c)
{
    L.launch("setup", k_setup, dim3(1), dim3(256), t, b.ev_err, b.cap_ev, c.n_mod, c.n_surf, c.nphi, c.nkb);
}

}  // namespace lst
