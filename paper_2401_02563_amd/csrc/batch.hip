// Batched earliest arrival, vertex-major: one wavefront lane per query.
//
// Queries are taken in groups of 64, the wavefront width of gfx950.  For a
// group, the arrival of query q at vertex v lives at arr[v][q], so the 64
// arrivals of one vertex are one contiguous 256-byte row.  A frontier entry
// is a vertex together with the 64-bit mask of the queries for which it must
// be expanded.  One wavefront expands one entry: lane q claims the part of
// the vertex's time-sorted adjacency that query q may newly use (binary
// search on the departure times from its own arrival, atomicMin on its own
// claim word, as in the single-query kernel), then the wavefront reads the
// union of the claimed ranges once, 64 edges at a time, and every lane
// checks each edge against its own range and window.  Relaxing one edge for
// all 64 queries is one coalesced row read and, where it improves, coalesced
// atomicMin updates.  The lanes that improved an edge's head are OR-ed into
// that head's next-round mask; the lane whose OR found the mask empty
// enqueues the head, which also makes every head appear once per round.
// Unions of at least `split` edges are cut into chunks that a second kernel
// spreads over all wavefronts, with the per-lane ranges kept in a side table.
//
// Compared with one query per thread (query-major), the edge stream is read
// once per group instead of once per query and the arrival reads coalesce,
// which is where batching pays (the paper runs its 100 sources one after the
// other, §6.1).
//
// The sweep form (batch_layout 3, sweep.h) reads every edge of a group's
// windows once in departure order instead of following frontiers; it pays
// where the group's windows overlap and the graph is large.

#include "internal.h"
#include "stage.h"
#include "sweep.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace kairos {

namespace {

constexpr int BTB = 256;   // threads per block (4 wavefronts)
constexpr int BU = 8;      // edges in flight per lane

struct BArgs {
    const uint32_t *off;
    const uint32_t *tt;
    const uint2 *da;
    uint32_t n;
    const uint2 *qw;                 // [groups*64] {t_alpha, t_omega}
    uint32_t *arr;                   // [groups*n*64]
    uint32_t *done;                  // [groups*n*64]
    unsigned long long *mask_cur;    // [groups*n]
    unsigned long long *mask_next;   // [groups*n]
    const uint32_t *cur;             // frontier items g*n+u
    uint32_t *next;
    uint32_t *cnt;                   // counters (same rotation as the single-query path)
    uint4 *chunks;                   // {item, range slot, start, len}
    uint32_t chunk_cap;
    uint2 *ranges;                   // [slot*64 + lane] {lo, end}
    uint32_t range_cap;
    unsigned long long *stats;
    uint32_t round;
    uint32_t split;
    uint32_t chunk;
    uint32_t max_t;                  // largest departure time in the graph
    uint32_t dedupe;                 // one atomic per run of lanes into the same slot
    uint32_t n_live;                 // vertices from this id on have no out-edges: never enqueued
};

enum : int { BCNT_RANGE = 10 };  // [10..12] rotating range-table sizes

__device__ __forceinline__ uint32_t lb_u32(const uint32_t *__restrict__ a, uint32_t lo, uint32_t hi, uint32_t key)
{
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t x)
{
    for (int o = 32; o > 0; o >>= 1) x = min(x, (uint32_t)__shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x)
{
    for (int o = 32; o > 0; o >>= 1) x = max(x, (uint32_t)__shfl_xor(x, o));
    return x;
}

constexpr int SCAP = 512;  // staged frontier entries per wavefront
using BStage = Stage<SCAP>;

// Relax edges [c0, c0 + cnt) of group g for every lane whose claimed range
// [lo, end) holds them.  All loads of BU edges are issued before use.
__device__ __forceinline__ void relax_span(const BArgs &A, uint32_t g, uint32_t c0, uint32_t total_end,
                                           bool has, uint32_t lo, uint32_t end, uint32_t tw, BStage &S,
                                           unsigned long long &n_relax)
{
    const uint32_t lane = threadIdx.x & 63;
    const size_t gbase = (size_t)g * A.n;
    for (uint32_t b0 = c0; b0 < total_end; b0 += 64) {
        const uint32_t e_l = b0 + lane;
        const uint2 dv = A.da[e_l < total_end ? e_l : b0];
        const uint32_t cnt = min(64u, total_end - b0);
        for (uint32_t k0 = 0; k0 < cnt; k0 += BU) {
            uint32_t vk[BU], ak[BU], cur[BU];
            bool ok[BU];
#pragma unroll
            for (int j = 0; j < BU; ++j) {
                const uint32_t k = k0 + j;
                vk[j] = __shfl(dv.x, k & 63);
                ak[j] = __shfl(dv.y, k & 63);
                const uint32_t ek = b0 + k;
                ok[j] = k < cnt && has && ek >= lo && ek < end && ak[j] <= tw;
                cur[j] = A.arr[ok[j] ? (gbase + vk[j]) * 64 + lane : 0];
            }
            // all BU atomic minima of this lane are in flight together
            uint32_t old[BU];
#pragma unroll
            for (int j = 0; j < BU; ++j) {
                ok[j] = ok[j] && ak[j] < cur[j];
                if (ok[j]) old[j] = atomicMin(&A.arr[(gbase + vk[j]) * 64 + lane], ak[j]);
            }
            unsigned long long mymask = 0;
            uint32_t myv = 0;
#pragma unroll
            for (int j = 0; j < BU; ++j) {
                const bool succ = ok[j] && ak[j] < old[j];
                n_relax += succ ? 1ull : 0ull;
                const unsigned long long b = __ballot(succ);
                if (lane == (uint32_t)j) {
                    mymask = b;
                    myv = vk[j];
                }
            }
            // lanes 0..BU-1 publish the improved heads in parallel
            bool first = false;
            // a head without out-edges never joins the frontier
            if (mymask && myv < A.n_live) {
                const unsigned long long old = atomicOr(&A.mask_next[gbase + myv], mymask);
                first = old == 0ull;
            }
            const unsigned long long fb[1] = {__ballot(first)};
            const uint32_t head[1] = {(uint32_t)(gbase + myv)};
            stage_append(S, fb, head);
        }
    }
}

__global__ __launch_bounds__(BTB) void bpush_kernel(BArgs A)
{
    __shared__ uint32_t s_stage[BTB / 64][SCAP];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wid = threadIdx.x >> 6;
    const uint32_t r3 = A.round % 3u;
    const uint32_t F = A.cnt[CNT_FRONT + r3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.cnt[CNT_FRONT + (A.round + 2u) % 3u] = 0u;
        A.cnt[CNT_CHUNK + (A.round + 1u) % 3u] = 0u;
        A.cnt[BCNT_RANGE + (A.round + 1u) % 3u] = 0u;
    }
    BStage S{s_stage[wid], 0u, A.next, &A.cnt[CNT_FRONT + (A.round + 1u) % 3u]};
    uint32_t *chunk_cnt = &A.cnt[CNT_CHUNK + r3];
    uint32_t *range_cnt = &A.cnt[BCNT_RANGE + r3];
    unsigned long long n_edges = 0, n_relax = 0, n_items = 0;
    const uint32_t waves = gridDim.x * (BTB / 64);
    for (uint32_t i = blockIdx.x * (BTB / 64) + wid; i < F; i += waves) {
        const uint32_t item = A.cur[i];
        const uint32_t g = item / A.n;
        const uint32_t u = item - g * A.n;
        const unsigned long long M = A.mask_cur[item];
        if (lane == 0) A.mask_cur[item] = 0ull;  // reused as a next-round mask
        const bool active = (M >> lane) & 1ull;
        const uint2 w = A.qw[(size_t)g * 64 + lane];
        const uint32_t b = A.off[u], e = A.off[u + 1];
        uint32_t lo = 0, end = 0;
        if (active) {
            n_items += 1;
            // one wavefront per entry per round, rounds are separate launches:
            // plain reads and writes of the lane's own arrival and claim word
            const size_t slot = (size_t)item * 64 + lane;
            const uint32_t r = A.arr[slot];
            const uint32_t old = A.done[slot];
            lo = lb_u32(A.tt, b, old == INF ? e : min(old, e), r);
            end = old == INF ? (w.y > A.max_t ? e : lb_u32(A.tt, lo, e, w.y)) : old;
            if (end < lo) end = lo;
            if (lo < end) A.done[slot] = lo;
        }
        const bool has = active && lo < end;
        if (!__ballot(has)) continue;
        uint32_t umin = wave_min(has ? lo : INF);
        const uint32_t umax = wave_max(has ? end : 0u);
        n_edges += umax - umin;
        if (umax - umin >= A.split) {
            uint32_t rs = 0;
            if (lane == 0) rs = atomicAdd(range_cnt, 1u);
            rs = __shfl(rs, 0);
            if (rs < A.range_cap) {
                A.ranges[(size_t)rs * 64 + lane] = has ? make_uint2(lo, end) : make_uint2(0u, 0u);
                const uint32_t L = umax - umin;
                const uint32_t nch = (L + A.chunk - 1) / A.chunk;
                uint32_t cb = 0;
                if (lane == 0) cb = atomicAdd(chunk_cnt, nch);
                cb = __shfl(cb, 0);
                const uint32_t fit = cb >= A.chunk_cap ? 0u : min(nch, A.chunk_cap - cb);
                for (uint32_t k = lane; k < fit; k += 64)
                    A.chunks[cb + k] = make_uint4(item, rs, umin + k * A.chunk, min(A.chunk, L - k * A.chunk));
                const uint32_t covered = (uint32_t)min((uint64_t)L, (uint64_t)fit * A.chunk);
                umin += covered;
                n_edges -= covered;  // the chunk kernel counts what it reads
            }
        }
        if (umin < umax) relax_span(A, g, umin, umax, has, lo, end, w.y, S, n_relax);
    }
    stage_flush_block<SCAP, BTB / 64>(S);
    unsigned long long v[3] = {n_relax, n_items, lane == 0 ? n_edges : 0ull};  // n_edges is per wavefront
    const int slot[3] = {ST_RELAX, ST_ITEMS, ST_EDGES};
    block_stats<BTB / 64>(A.stats, v, slot);
}

__global__ __launch_bounds__(BTB) void bchunk_kernel(BArgs A)
{
    __shared__ uint32_t s_stage[BTB / 64][SCAP];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wid = threadIdx.x >> 6;
    const uint32_t r3 = A.round % 3u;
    const uint32_t C = min(A.cnt[CNT_CHUNK + r3], A.chunk_cap);
    BStage S{s_stage[wid], 0u, A.next, &A.cnt[CNT_FRONT + (A.round + 1u) % 3u]};
    unsigned long long n_edges = 0, n_relax = 0;
    const uint32_t waves = gridDim.x * (BTB / 64);
    for (uint32_t c = blockIdx.x * (BTB / 64) + wid; c < C; c += waves) {
        const uint4 ch = A.chunks[c];
        const uint32_t g = ch.x / A.n;
        const uint2 rg = A.ranges[(size_t)ch.y * 64 + lane];
        const uint2 w = A.qw[(size_t)g * 64 + lane];
        n_edges += ch.w;
        relax_span(A, g, ch.z, ch.z + ch.w, rg.x < rg.y, rg.x, rg.y, w.y, S, n_relax);
    }
    stage_flush_block<SCAP, BTB / 64>(S);
    unsigned long long v[2] = {n_relax, lane == 0 ? n_edges : 0ull};  // n_edges is per wavefront
    const int slot[2] = {ST_RELAX, ST_CHUNK_EDGES};
    block_stats<BTB / 64>(A.stats, v, slot);
}

// ---------------------------------------------------------------------------
// Lane-dense variant of the same batch (batch_layout 2).  The frontier and
// the arrival rows are those of the vertex-major kernel, but an entry's mask
// is expanded into (vertex, query) pairs that are dealt to threads densely,
// so a pair with one active query costs one thread, not a wavefront.  Each
// thread claims its pair's range as the single-query kernel does; claims
// shorter than `split` are relaxed by the block through a prefix sum over
// claim lengths, longer ones go to the chunk kernel below.  Pairs of one
// vertex sit in neighbouring threads, so their edge records and arrival rows
// are fetched together.
constexpr int HU = 4;  // edges in flight per lane

struct HGroup {
    uint32_t v[HU], a[HU], row[HU], bit[HU], tw[HU];
    bool ok[HU];
};

__device__ __forceinline__ uint32_t nth_set_bit(unsigned long long m, uint32_t j)
{
    for (uint32_t i = 0; i < j; ++i) m &= m - 1ull;
    return (uint32_t)__builtin_ctzll(m);
}

// Relax HU edges per lane: arrival-row reads, atomic minima and head-mask ORs
// are each issued together.  Heads whose mask was empty go to the next
// frontier through the wavefront's staging buffer.
// Stage 1 of hrelax: the window test and the heads' arrival reads
// (unconditional loads from valid addresses, so nothing forces a wait
// between the HU requests).
__device__ __forceinline__ void hrelax_load(const BArgs &A, HGroup &H, size_t (&idx)[HU], uint32_t (&cur)[HU])
{
#pragma unroll
    for (int k = 0; k < HU; ++k) {
        H.ok[k] = H.ok[k] && H.a[k] <= H.tw[k];
        idx[k] = ((size_t)H.row[k] + H.v[k]) * 64 + H.bit[k];
        cur[k] = A.arr[H.ok[k] ? idx[k] : 0];
    }
}

// Stage 2: run dedupe, atomic minima, head-mask ORs and staging
// (predicated atomics without default values).
__device__ __forceinline__ void hrelax_apply(const BArgs &A, HGroup &H, const size_t (&idx)[HU],
                                             const uint32_t (&cur)[HU], BStage &S, unsigned long long &n_relax)
{
    uint32_t old[HU];
#pragma unroll
    for (int k = 0; k < HU; ++k) {
        H.ok[k] = H.ok[k] && H.a[k] < cur[k];
        if (A.dedupe) dedupe_runs(H.ok[k], H.a[k], (uint64_t)idx[k]);  // one atomic per run of equal slots
    }
#pragma unroll
    for (int k = 0; k < HU; ++k)
        if (H.ok[k]) old[k] = atomicMin(&A.arr[idx[k]], H.a[k]);
    unsigned long long om[HU];
#pragma unroll
    for (int k = 0; k < HU; ++k) {
        H.ok[k] = H.ok[k] && H.a[k] < old[k];
        n_relax += H.ok[k] ? 1ull : 0ull;
        // a head without out-edges never joins the frontier
        if (H.ok[k] && H.v[k] < A.n_live) om[k] = atomicOr(&A.mask_next[(size_t)H.row[k] + H.v[k]], 1ull << H.bit[k]);
    }
    unsigned long long bal[HU];
    uint32_t head[HU];
#pragma unroll
    for (int k = 0; k < HU; ++k) {
        bal[k] = __ballot(H.ok[k] && H.v[k] < A.n_live && om[k] == 0ull);
        head[k] = H.row[k] + H.v[k];
    }
    stage_append(S, bal, head);
}

__device__ __forceinline__ void hrelax(const BArgs &A, HGroup &H, BStage &S, unsigned long long &n_relax)
{
    size_t idx[HU];
    uint32_t cur[HU];
    hrelax_load(A, H, idx, cur);
    hrelax_apply(A, H, idx, cur, S, n_relax);
}

// Expansion of one round's F frontier entries by the whole grid (every
// block calls this; it contains block barriers).  Heads found go to S.
__device__ __forceinline__ void hpush_phase(const BArgs &A, uint32_t F, BStage &S, unsigned long long &n_edges,
                                            unsigned long long &n_relax, unsigned long long &n_items)
{
    __shared__ uint32_t s_ent[BTB];
    __shared__ unsigned long long s_mask[BTB];
    __shared__ uint32_t s_pp[BTB + 1];
    __shared__ uint32_t s_lo[BTB], s_row[BTB], s_bit[BTB], s_tw[BTB];
    __shared__ uint32_t s_pref[BTB + 1];
    __shared__ uint32_t s_wsum[BTB / 64];
    __shared__ uint32_t s_csum[BTB / 64];
    __shared__ uint32_t s_cb;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const uint32_t r3 = A.round % 3u;
    if (blockIdx.x == 0 && tid == 0) {
        A.cnt[CNT_FRONT + (A.round + 2u) % 3u] = 0u;
        A.cnt[CNT_CHUNK + (A.round + 1u) % 3u] = 0u;
    }
    uint32_t *chunk_cnt = &A.cnt[CNT_CHUNK + r3];

    for (uint32_t base = blockIdx.x * BTB; base < F; base += gridDim.x * BTB) {
        // entries of this block and their query counts
        const uint32_t i = base + tid;
        uint32_t ent = 0, c = 0;
        unsigned long long M = 0;
        if (i < F) {
            ent = A.cur[i];
            M = A.mask_cur[ent];
            A.mask_cur[ent] = 0ull;  // one expander per entry per round; reused next round
            c = __popcll(M);
        }
        uint32_t x = c;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_wsum[w] = x;
        s_ent[tid] = ent;
        s_mask[tid] = M;
        __syncthreads();
        uint32_t woff = 0, P = 0;
        for (int w2 = 0; w2 < BTB / 64; ++w2) {
            if (w2 < w) woff += s_wsum[w2];
            P += s_wsum[w2];
        }
        s_pp[tid] = woff + x - c;
        if (tid == 0) s_pp[BTB] = P;
        __syncthreads();
        for (uint32_t p0 = 0; p0 < P; p0 += BTB) {
            // one (vertex, query) pair per thread: claim its newly usable range
            const uint32_t p = p0 + tid;
            uint32_t lo = 0, len = 0, row = 0, bit = 0, tw = 0, e_ = 0, nch = 0;
            if (p < P) {
                int lk = 0, hk = BTB;
                while (hk - lk > 1) {
                    const int mid = (lk + hk) >> 1;
                    if (s_pp[mid] <= p)
                        lk = mid;
                    else
                        hk = mid;
                }
                e_ = s_ent[lk];
                bit = nth_set_bit(s_mask[lk], p - s_pp[lk]);
                const uint32_t g = e_ / A.n;
                const uint32_t u = e_ - g * A.n;
                row = g * A.n;
                tw = A.qw[(size_t)g * 64 + bit].y;
                const size_t slot = (size_t)e_ * 64 + bit;
                const uint32_t r = A.arr[slot];
                const uint32_t b = A.off[u], e = A.off[u + 1];
                const uint32_t old = A.done[slot];
                lo = lb_u32(A.tt, b, old == INF ? e : min(old, e), r);
                uint32_t end = old == INF ? (tw > A.max_t ? e : lb_u32(A.tt, lo, e, tw)) : old;
                ++n_items;
                if (lo < end) {
                    len = end - lo;
                    A.done[slot] = lo;
                }
                if (len >= A.split) nch = (len + A.chunk - 1) / A.chunk;
            }
            // prefix sums over the block: short claim lengths (each below
            // `split`) and chunk counts (one chunk-list reservation per pass)
            const uint32_t sl = nch ? 0u : len;
            uint32_t y2 = sl, c2 = nch;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t2 = __shfl_up(y2, o);
                const uint32_t t3 = __shfl_up(c2, o);
                if (lane >= o) {
                    y2 += t2;
                    c2 += t3;
                }
            }
            __syncthreads();
            if (lane == 63) {
                s_wsum[w] = y2;
                s_csum[w] = c2;
            }
            s_lo[tid] = lo;
            s_row[tid] = row;
            s_bit[tid] = bit;
            s_tw[tid] = tw;
            __syncthreads();
            uint32_t wo = 0, total = 0, co = 0, ctotal = 0;
            for (int w2 = 0; w2 < BTB / 64; ++w2) {
                if (w2 < w) {
                    wo += s_wsum[w2];
                    co += s_csum[w2];
                }
                total += s_wsum[w2];
                ctotal += s_csum[w2];
            }
            s_pref[tid] = wo + y2 - sl;
            if (tid == 0) {
                s_pref[BTB] = total;
                if (ctotal) s_cb = atomicAdd(chunk_cnt, ctotal);
            }
            __syncthreads();
            uint32_t ser_lo = 0, ser_len = 0;
            if (nch) {
                const uint32_t cb = s_cb + co + c2 - nch;
                const uint32_t fit = cb >= A.chunk_cap ? 0u : min(nch, A.chunk_cap - cb);
                for (uint32_t k = 0; k < fit; ++k)
                    A.chunks[cb + k] = make_uint4(e_, bit, lo + k * A.chunk, min(A.chunk, len - k * A.chunk));
                const uint32_t covered = (uint32_t)min((uint64_t)len, (uint64_t)fit * A.chunk);
                // chunk list full: this lane walks the rest by itself
                ser_lo = lo + covered;
                ser_len = len - covered;
            }
            if (tid == 0) n_edges += total;
            for (uint32_t j0 = 0; j0 < total; j0 += BTB * HU) {
                HGroup H;
#pragma unroll
                for (int k = 0; k < HU; ++k) {
                    const uint32_t j = j0 + k * BTB + tid;
                    H.ok[k] = j < total;
                    int lk = 0, hk = BTB;
                    while (hk - lk > 1) {
                        const int mid = (lk + hk) >> 1;
                        if (s_pref[mid] <= j)
                            lk = mid;
                        else
                            hk = mid;
                    }
                    const uint2 dv = A.da[H.ok[k] ? s_lo[lk] + (j - s_pref[lk]) : 0u];
                    H.v[k] = dv.x;
                    H.a[k] = dv.y;
                    H.row[k] = s_row[lk];
                    H.bit[k] = s_bit[lk];
                    H.tw[k] = s_tw[lk];
                }
                hrelax(A, H, S, n_relax);
            }
            n_edges += ser_len;
            uint32_t ser_done = 0;
            while (__ballot(ser_done < ser_len)) {
                HGroup H;
#pragma unroll
                for (int k = 0; k < HU; ++k) {
                    H.ok[k] = ser_done < ser_len;
                    const uint2 dv = A.da[H.ok[k] ? ser_lo + ser_done : 0u];
                    if (H.ok[k]) ++ser_done;
                    H.v[k] = dv.x;
                    H.a[k] = dv.y;
                    H.row[k] = row;
                    H.bit[k] = bit;
                    H.tw[k] = tw;
                }
                hrelax(A, H, S, n_relax);
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(BTB) void hpush_kernel(BArgs A)
{
    __shared__ uint32_t s_stage[BTB / 64][SCAP];
    BStage S{s_stage[threadIdx.x >> 6], 0u, A.next, &A.cnt[CNT_FRONT + (A.round + 1u) % 3u]};
    unsigned long long n_edges = 0, n_relax = 0, n_items = 0;
    hpush_phase(A, A.cnt[CNT_FRONT + A.round % 3u], S, n_edges, n_relax, n_items);
    stage_flush_block<SCAP, BTB / 64>(S);
    unsigned long long v[3] = {n_relax, n_items, n_edges};
    const int slot[3] = {ST_RELAX, ST_ITEMS, ST_EDGES};
    block_stats<BTB / 64>(A.stats, v, slot);
}

// Chunks of the lane-dense variant: {entry, query bit, start, len}; one
// wavefront per chunk, HU edges per lane in flight, every lane active.
// The chunks of round A.round, one wavefront per chunk, grid-stride.
__device__ __forceinline__ void hchunk_phase(const BArgs &A, BStage &S, unsigned long long &n_edges,
                                             unsigned long long &n_relax)
{
    const uint32_t r3 = A.round % 3u;
    const uint32_t C = min(A.cnt[CNT_CHUNK + r3], A.chunk_cap);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (BTB / 64);
    for (uint32_t c = blockIdx.x * (BTB / 64) + (threadIdx.x >> 6); c < C; c += waves) {
        const uint4 ch = A.chunks[c];
        const uint32_t g = ch.x / A.n;
        const uint32_t tw = A.qw[(size_t)g * 64 + ch.y].y;
        if (lane == 0) n_edges += ch.w;
        // a chunk is one (query, vertex) pair's: the next group's records
        // are requested while this group's arrival reads are in flight
        uint2 r[HU];
#pragma unroll
        for (int k = 0; k < HU; ++k) {
            const uint32_t off = k * 64 + lane;
            r[k] = A.da[ch.z + (off < ch.w ? off : 0u)];
        }
        for (uint32_t k0 = 0; k0 < ch.w; k0 += 64 * HU) {
            HGroup H;
#pragma unroll
            for (int k = 0; k < HU; ++k) {
                H.ok[k] = k0 + k * 64 + lane < ch.w;
                H.v[k] = r[k].x;
                H.a[k] = r[k].y;
                H.row[k] = g * A.n;
                H.bit[k] = ch.y;
                H.tw[k] = tw;
            }
            size_t idx[HU];
            uint32_t cur[HU];
            hrelax_load(A, H, idx, cur);
            // after all arrival reads, unconditional (past the end: the
            // chunk's first record), so the waits for those reads do not
            // cover these
            __builtin_amdgcn_sched_barrier(0);
            const uint32_t k1 = k0 + 64 * HU;
#pragma unroll
            for (int k = 0; k < HU; ++k) {
                const uint32_t off = k1 + k * 64 + lane;
                r[k] = A.da[ch.z + (off < ch.w ? off : 0u)];
            }
            hrelax_apply(A, H, idx, cur, S, n_relax);
        }
    }
}

__global__ __launch_bounds__(BTB) void hchunk_kernel(BArgs A)
{
    __shared__ uint32_t s_stage[BTB / 64][SCAP];
    BStage S{s_stage[threadIdx.x >> 6], 0u, A.next, &A.cnt[CNT_FRONT + (A.round + 1u) % 3u]};
    unsigned long long n_edges = 0, n_relax = 0;
    hchunk_phase(A, S, n_edges, n_relax);
    stage_flush_block<SCAP, BTB / 64>(S);
    unsigned long long v[2] = {n_relax, n_edges};
    const int slot[2] = {ST_RELAX, ST_CHUNK_EDGES};
    block_stats<BTB / 64>(A.stats, v, slot);
}

// All rounds of a lane-dense batch in one cooperative launch: push phase,
// grid barrier, chunk phase, grid barrier, then every block reads the next
// frontier size from the same word and stops together when it is zero (or
// after max_rounds, or when a barrier wait gave up; the host reports both as
// errors).  Queues and masks alternate by round parity as in the per-round
// launches.
enum : int { BCNT_ROUNDS = 13, BCNT_CAPPED = 14 };

__global__ __launch_bounds__(BTB) void hpersist_kernel(BArgs A, uint32_t *q0, uint32_t *q1, unsigned long long *m0,
                                                       unsigned long long *m1, uint32_t *bar, uint32_t max_rounds,
                                                       uint32_t spin_limit)
{
    __shared__ uint32_t s_stage[BTB / 64][SCAP];
    __shared__ uint32_t s_F;
    unsigned long long n_edges = 0, n_relax = 0, n_items = 0, n_cedges = 0, n_crelax = 0;
    uint32_t r = A.round;
    for (;;) {
        // the abort word is sampled into the same LDS word: either every
        // block sees it raised before this round, or every block reaches the
        // next barrier, whose waits then all end
        if (threadIdx.x == 0)
            s_F = grid_aborted(bar) ? 0u
                                    : __hip_atomic_load(&A.cnt[CNT_FRONT + r % 3u], __ATOMIC_ACQUIRE,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t F = s_F;
        __syncthreads();
        if (F == 0 || r - A.round >= max_rounds) break;
        BArgs B = A;
        B.round = r;
        B.cur = (r & 1u) ? q1 : q0;
        B.next = (r & 1u) ? q0 : q1;
        B.mask_cur = (r & 1u) ? m1 : m0;
        B.mask_next = (r & 1u) ? m0 : m1;
        BStage S{s_stage[threadIdx.x >> 6], 0u, B.next, &A.cnt[CNT_FRONT + (r + 1u) % 3u]};
        hpush_phase(B, F, S, n_edges, n_relax, n_items);
        stage_flush_block<SCAP, BTB / 64>(S);
        grid_barrier(bar, spin_limit);
        hchunk_phase(B, S, n_cedges, n_crelax);
        stage_flush_block<SCAP, BTB / 64>(S);
        grid_barrier(bar, spin_limit);
        ++r;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.cnt[BCNT_ROUNDS] = r - A.round;
        A.cnt[BCNT_CAPPED] = (r - A.round >= max_rounds || grid_aborted(bar)) ? 1u : 0u;
    }
    unsigned long long v[5] = {n_relax + n_crelax, n_items, n_edges, n_cedges, 0ull};
    const int slot[5] = {ST_RELAX, ST_ITEMS, ST_EDGES, ST_CHUNK_EDGES, ST_ATTEMPTS};
    block_stats<BTB / 64>(A.stats, v, slot);
}

// Group start: every query's source gets its t_alpha and its mask bit; the
// lane that finds the source's mask empty enqueues it.
__global__ void binit_kernel(BArgs A, const uint4 *__restrict__ hq, uint32_t q)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < q; i += gridDim.x * blockDim.x) {
        const uint4 p = hq[i];  // {src, ta, tw, _}
        const uint32_t g = i / 64, lane = i % 64;
        const size_t item = (size_t)g * A.n + p.x;
        ((uint2 *)A.qw)[i] = make_uint2(p.y, p.z);
        A.arr[item * 64 + lane] = p.y;
        const unsigned long long old = atomicOr(&A.mask_cur[item], 1ull << lane);
        if (old == 0ull) {
            const uint32_t pos = atomicAdd(&A.cnt[CNT_FRONT + A.round % 3u], 1u);
            A.next[pos] = (uint32_t)item;  // `next` names the first round's queue here
        }
    }
}

// out[(g*64+q)*n + v] = arr[(g*n+perm[v])*64 + q] (caller id v) through a
// 64x64 LDS tile: 64 gathered 256-byte rows in, 64 coalesced columns out.
__global__ __launch_bounds__(256) void btranspose_kernel(const uint32_t *__restrict__ arr, uint32_t *__restrict__ out,
                                                         const uint32_t *__restrict__ perm, uint32_t n,
                                                         uint32_t q_total, uint32_t groups)
{
    __shared__ uint32_t tile[64][65];
    const uint32_t tiles_v = (n + 63) / 64;
    for (uint64_t t = blockIdx.x; t < (uint64_t)tiles_v * groups; t += gridDim.x) {
        const uint32_t g = (uint32_t)(t / tiles_v);
        const uint32_t v0 = (uint32_t)(t % tiles_v) * 64;
        for (int k = threadIdx.x; k < 64 * 64; k += 256) {
            const uint32_t vv = k / 64, qq = k % 64;
            if (v0 + vv < n) tile[vv][qq] = arr[((size_t)g * n + perm[v0 + vv]) * 64 + qq];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < 64 * 64; k += 256) {
            const uint32_t qq = k / 64, vv = k % 64;
            const uint32_t qg = g * 64 + qq;
            if (qg < q_total && v0 + vv < n) out[(size_t)qg * n + v0 + vv] = tile[vv][qq];
        }
        __syncthreads();
    }
}

__global__ void bfill_kernel(uint32_t *p, uint64_t count, uint32_t value)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

int gridc(uint64_t work, int per_block, int cap)
{
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (uint64_t)cap) g = cap;
    return (int)g;
}

}  // namespace

// Device state of one vertex-major batch (kept by the graph between calls).
struct VBatch {
    uint32_t groups = 0, n = 0;
    uint32_t *arr = nullptr, *done = nullptr, *queue[2] = {nullptr, nullptr}, *cnt = nullptr;
    unsigned long long *mask[2] = {nullptr, nullptr};
    uint2 *qw = nullptr;
    uint4 *chunks = nullptr;
    uint2 *ranges = nullptr;
    uint64_t chunk_cap = 0, range_cap = 0;
    unsigned long long *stats = nullptr;
    uint32_t *bar = nullptr;  // grid barrier words of the persistent launch
    uint32_t *h_pin = nullptr;
    uint4 *h_q = nullptr;  // groups * 64: pinned staging of query parameters
    hipStream_t stream = nullptr;
    bool own_stream = false;
};

void vbatch_destroy(VBatch *b)
{
    if (!b) return;
    if (b->stream) hipStreamSynchronize(b->stream);
    dev_free(b->arr);
    dev_free(b->done);
    dev_free(b->queue[0]);
    dev_free(b->queue[1]);
    dev_free(b->cnt);
    dev_free(b->mask[0]);
    dev_free(b->mask[1]);
    dev_free(b->qw);
    dev_free(b->chunks);
    dev_free(b->ranges);
    dev_free(b->stats);
    dev_free(b->bar);
    if (b->h_pin) hipHostFree(b->h_pin);
    if (b->h_q) hipHostFree(b->h_q);
    if (b->own_stream && b->stream) hipStreamDestroy(b->stream);
    delete b;
}

static int vbatch_alloc(kairos_graph *g, uint32_t groups, VBatch **out)
{
    VBatch *b = new VBatch();
    b->groups = groups;
    b->n = g->n;
    const size_t gn = (size_t)groups * g->n;
    b->arr = (uint32_t *)dev_alloc(gn * 64 * 4, nullptr);
    b->done = (uint32_t *)dev_alloc(gn * 64 * 4, nullptr);
    b->queue[0] = (uint32_t *)dev_alloc(gn * 4 + 256, nullptr);
    b->queue[1] = (uint32_t *)dev_alloc(gn * 4 + 256, nullptr);
    b->cnt = (uint32_t *)dev_alloc(64 * 4, nullptr);
    b->mask[0] = (unsigned long long *)dev_alloc(gn * 8, nullptr);
    b->mask[1] = (unsigned long long *)dev_alloc(gn * 8, nullptr);
    b->qw = (uint2 *)dev_alloc((size_t)groups * 64 * sizeof(uint2), nullptr);
    // chunks of one round: the lane-dense layout can split per query
    const uint64_t per_g = (g->tuning.batch_layout == 2 ? 64 : 1) *
                           (g->m / std::max<uint32_t>(g->tuning.chunk, 64) +
                            g->m / std::max<uint32_t>(g->tuning.split, 64) + 1);
    b->chunk_cap = std::min<uint64_t>((uint64_t)groups * per_g, 1ull << 26);
    // the sweep form's fix-up chunks of one pass: at most a slab's edges in
    // chunks of SW_C plus one partial chunk per listed vertex
    if (g->tuning.batch_layout == 3)
        b->chunk_cap = std::max<uint64_t>(b->chunk_cap, std::min<uint64_t>(SWEEP_SLAB / SW_C + g->n + 64, 1ull << 26));
    b->range_cap = std::min<uint64_t>((uint64_t)groups * (g->m / std::max<uint32_t>(g->tuning.split, 64) + 1),
                                      1ull << 22);
    if (const char *cap = std::getenv("KAIROS_TEST_CHUNK_CAP")) {
        b->chunk_cap = std::strtoull(cap, nullptr, 10);
        b->range_cap = std::min<uint64_t>(b->range_cap, b->chunk_cap);
    }
    b->chunks = (uint4 *)dev_alloc(std::max<uint64_t>(b->chunk_cap, 1) * sizeof(uint4), nullptr);
    b->ranges = (uint2 *)dev_alloc(std::max<uint64_t>(b->range_cap, 1) * 64 * sizeof(uint2), nullptr);
    b->stats = (unsigned long long *)dev_alloc(ST_TOTAL_WORDS * 8, nullptr);
    b->bar = (uint32_t *)dev_alloc(BAR_WORDS * 4, nullptr);
    bool ok = b->arr && b->done && b->queue[0] && b->queue[1] && b->cnt && b->mask[0] && b->mask[1] && b->qw &&
              b->chunks && b->ranges && b->stats && b->bar;
    if (ok && hipHostMalloc((void **)&b->h_pin, 256, hipHostMallocDefault) != hipSuccess) {
        b->h_pin = nullptr;
        ok = false;
    }
    if (ok && hipHostMalloc((void **)&b->h_q, (size_t)groups * 64 * sizeof(uint4), hipHostMallocDefault) !=
                  hipSuccess) {
        b->h_q = nullptr;
        ok = false;
    }
    if (ok) {
        if (g->stream) {
            b->stream = g->stream;
        } else if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess) {
            b->own_stream = true;
        } else {
            ok = false;
        }
    }
    if (ok)
        ok = hipMemsetAsync(b->stats, 0, ST_TOTAL_WORDS * 8, b->stream) == hipSuccess &&
             hipMemsetAsync(b->mask[0], 0, gn * 8, b->stream) == hipSuccess &&
             hipMemsetAsync(b->mask[1], 0, gn * 8, b->stream) == hipSuccess &&
             hipStreamSynchronize(b->stream) == hipSuccess;
    if (!ok) {
        vbatch_destroy(b);
        return KAIROS_ERR_NOMEM;
    }
    *out = b;
    return KAIROS_OK;
}

static int bfill(hipStream_t st, uint32_t *p, uint64_t count, uint32_t v)
{
    hipLaunchKernelGGL(bfill_kernel, dim3(gridc(count, 256 * 8, 16384)), dim3(256), 0, st, p, count, v);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

// Runs every round of a lane-dense batch whose first frontier is in place in
// one cooperative launch.  Returns KAIROS_ERR_BUSY when the runtime refuses
// the launch (nothing ran; state unchanged).
static int run_persistent(kairos_graph *g, VBatch *b, BArgs A, hipStream_t st)
{
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, hpersist_kernel, BTB, 0) != hipSuccess || occ < 1) {
        (void)hipGetLastError();
        return KAIROS_ERR_BUSY;
    }
    const int grid = g->num_cus * std::min(occ, 4);
    constexpr uint32_t kMaxRounds = 1u << 22;  // far beyond any batch; a stop for the loop, reported as an error
    KAIROS_HIP(hipMemsetAsync(b->bar, 0, BAR_WORDS * 4, st));
    A.round = 0;
    uint32_t *q0 = b->queue[0], *q1 = b->queue[1];
    unsigned long long *m0 = b->mask[0], *m1 = b->mask[1];
    uint32_t *bar = b->bar;
    uint32_t max_rounds = kMaxRounds;
    uint32_t spin_limit = 1u << 24;  // about 4 s of polling: far beyond one phase
    void *args[] = {&A, &q0, &q1, &m0, &m1, &bar, &max_rounds, &spin_limit};
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    const hipError_t e = hipLaunchCooperativeKernel((const void *)hpersist_kernel, dim3(grid), dim3(BTB), args, 0, st);
    prof_end(g, st, KAIROS_K_PUSH, ev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return KAIROS_ERR_BUSY;
    }
    KAIROS_HIP(hipMemcpyAsync(b->h_pin, b->cnt, 64, hipMemcpyDeviceToHost, st));
    KAIROS_HIP(hipStreamSynchronize(st));
    if (b->h_pin[BCNT_CAPPED]) return KAIROS_ERR_DEVICE;
    if (g->prof.on) {
        std::lock_guard<std::mutex> lk(g->prof.mu);
        g->prof.rounds += b->h_pin[BCNT_ROUNDS];
    }
    return KAIROS_OK;
}

// q queries (q <= 64 * groups of b); out is query-major [q][n].
int run_vbatch(kairos_graph *g, VBatch *b, uint32_t q, const uint32_t *src, const uint32_t *ta,
               const uint32_t *tw, uint32_t *out)
{
    hipStream_t st = b->stream;
    const uint32_t groups = (q + 63) / 64;
    const size_t gn = (size_t)groups * g->n;
    int rc;
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    if ((rc = bfill(st, b->arr, gn * 64, INF))) return rc;
    if ((rc = bfill(st, b->done, gn * 64, INF))) return rc;
    KAIROS_HIP(hipMemsetAsync(b->cnt, 0, 64 * 4, st));
    prof_end(g, st, KAIROS_K_INIT, ev);
    // masks are left all-zero by every completed run (each processed entry
    // clears its word); a failed run destroys this state instead

    // query parameters go through the batch state's pinned staging array
    // (groups * 64 entries, allocated with the state; the init kernel reads
    // it before the synchronisation below)
    if (q > (size_t)b->groups * 64) return KAIROS_ERR_INVALID;
    uint4 *staging = b->h_q;
    for (uint32_t i = 0; i < q; ++i) staging[i] = make_uint4(g->h_perm[src[i]], ta[i], tw[i], 0);

    BArgs A{};
    A.off = g->off_out;
    A.tt = g->t_out;
    A.da = g->da_out;
    A.n = g->n;
    A.qw = b->qw;
    A.arr = b->arr;
    A.done = b->done;
    A.cnt = b->cnt;
    A.chunks = b->chunks;
    A.chunk_cap = (uint32_t)std::min<uint64_t>(b->chunk_cap, 0xFFFFFFF0u);
    A.ranges = b->ranges;
    A.range_cap = (uint32_t)b->range_cap;
    A.stats = g->prof.on ? b->stats : nullptr;
    A.split = std::max<uint32_t>(g->tuning.split, 16);
    A.chunk = std::max<uint32_t>(g->tuning.chunk, 16);
    A.max_t = g->max_t;
    A.dedupe = g->tuning.run_dedupe;
    A.n_live = g->n_live;
    A.round = 0;
    A.mask_cur = b->mask[0];
    A.mask_next = b->mask[1];
    A.next = b->queue[0];
    prof_begin(g, st, &ev);
    hipLaunchKernelGGL(binit_kernel, dim3(gridc(q, 256, 64)), dim3(256), 0, st, A, staging, q);
    prof_end(g, st, KAIROS_K_INIT, ev);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return KAIROS_ERR_DEVICE;
    KAIROS_HIP(hipMemcpyAsync(b->h_pin, b->cnt, 64, hipMemcpyDeviceToHost, st));
    KAIROS_HIP(hipStreamSynchronize(st));
    uint32_t F = b->h_pin[CNT_FRONT];
    const int wave_cap = std::max(1, g->num_cus * 8);
    const bool dense = g->tuning.batch_layout == 2;
    uint32_t r = 0;
    if (dense && g->tuning.batch_persistent && F > 0) {
        int prc = run_persistent(g, b, A, st);
        if (prc == KAIROS_OK) F = 0;  // every round ran on the device
        else if (prc != KAIROS_ERR_BUSY) return prc;
        // KAIROS_ERR_BUSY: the launch was refused (no room for every block);
        // run the same rounds with one launch per phase instead
    }
    while (F > 0) {
        A.round = r;
        A.cur = b->queue[0];
        A.next = b->queue[1];
        A.mask_cur = b->mask[r & 1];
        A.mask_next = b->mask[(r + 1) & 1];
        prof_begin(g, st, &ev);
        if (dense)
            hipLaunchKernelGGL(hpush_kernel, dim3(gridc(F, BTB, wave_cap / 4)), dim3(BTB), 0, st, A);
        else
            hipLaunchKernelGGL(bpush_kernel, dim3(gridc(F, BTB / 64, wave_cap)), dim3(BTB), 0, st, A);
        prof_end(g, st, KAIROS_K_PUSH, ev);
        prof_begin(g, st, &ev);
        if (dense)
            hipLaunchKernelGGL(hchunk_kernel, dim3(std::max(1, g->num_cus * 8)), dim3(BTB), 0, st, A);
        else
            hipLaunchKernelGGL(bchunk_kernel, dim3(std::max(1, g->num_cus * 8)), dim3(BTB), 0, st, A);
        prof_end(g, st, KAIROS_K_CHUNK, ev);
        KAIROS_HIP(hipGetLastError());
        ++r;
        std::swap(b->queue[0], b->queue[1]);
        KAIROS_HIP(hipMemcpyAsync(b->h_pin, b->cnt, 64, hipMemcpyDeviceToHost, st));
        KAIROS_HIP(hipStreamSynchronize(st));
        F = b->h_pin[CNT_FRONT + r % 3u];
        if (g->prof.on) {
            std::lock_guard<std::mutex> lk(g->prof.mu);
            g->prof.rounds += 1;
        }
    }
    prof_begin(g, st, &ev);
    hipLaunchKernelGGL(btranspose_kernel, dim3(gridc((uint64_t)((g->n + 63) / 64) * groups, 1, 16384)), dim3(256), 0,
                       st, b->arr, out, g->perm, g->n, q, groups);
    prof_end(g, st, KAIROS_K_INIT, ev);
    KAIROS_HIP(hipGetLastError());
    KAIROS_HIP(hipStreamSynchronize(st));
    if (g->prof.on) {
        std::vector<unsigned long long> raw((size_t)ST_SHARDS * ST_WORDS);
        unsigned long long h[ST_WORDS];
        KAIROS_HIP(hipMemcpy(raw.data(), b->stats, raw.size() * 8, hipMemcpyDeviceToHost));
        KAIROS_HIP(hipMemset(b->stats, 0, raw.size() * 8));
        stats_sum_shards(raw.data(), h);
        prof_add_stats(g, h);
    }
    return KAIROS_OK;
}

// The graph's departure-ordered edge records, built on first use.
static int ensure_time_order(kairos_graph *g, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g->ts_mu);
    if (g->tsorted || g->m == 0) return KAIROS_OK;
    uint4 *ts = nullptr;
    int rc = build_time_order(g, st, &ts);
    if (rc == KAIROS_OK) g->tsorted = ts;
    return rc;
}

// One group of the sweep form in one cooperative launch.  KAIROS_ERR_BUSY:
// the launch was refused, or the group needs the lane-dense rounds (a
// fix-up list overflowed or a slab would not settle); its rows are then
// rewritten by the caller's fallback.
static int sweep_group(kairos_graph *g, VBatch *b, uint32_t gi, uint32_t q0, uint32_t nq, hipStream_t st)
{
    const size_t n = g->n;
    uint32_t *arr = b->arr + (size_t)gi * n * 64;
    // the group's claim area (64 n words) holds the stamps (n words) and,
    // 8-byte aligned after them, the per-vertex pass notes (2 n words)
    uint32_t *stamp = b->done + (size_t)gi * n * 64;
    unsigned long long *low = (unsigned long long *)(stamp + (n + 1) / 2 * 2);
    int rc;
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    if ((rc = bfill(st, arr, n * 64, INF))) return rc;
    if ((rc = bfill(st, stamp, n, 0u))) return rc;
    if ((rc = bfill(st, (uint32_t *)low, 2 * n, 0xFFFFFFFFu))) return rc;
    hipLaunchKernelGGL(sweep_init_kernel, dim3(1), dim3(64), 0, st, b->qw + (size_t)gi * 64, arr, b->h_q, q0, nq);
    KAIROS_HIP(hipMemsetAsync(b->cnt, 0, 64 * 4, st));
    KAIROS_HIP(hipMemsetAsync(b->bar, 0, BAR_WORDS * 4, st));
    prof_end(g, st, KAIROS_K_INIT, ev);
    KAIROS_HIP(hipGetLastError());
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, sweep_kernel, SW_TB, 0) != hipSuccess || occ < 1) {
        (void)hipGetLastError();
        return KAIROS_ERR_BUSY;
    }
    SwArgs S{};
    S.E = g->tsorted;
    S.m = g->m;
    S.off = g->off_out;
    S.tt = g->t_out;
    S.da = g->da_out;
    S.arr = arr;
    S.qw = b->qw + (size_t)gi * 64;
    S.stamp = stamp;
    S.low = low;
    S.list0 = b->queue[0];
    S.list1 = b->queue[1];
    S.chunks = b->chunks;
    S.chunk_cap = (uint32_t)std::min<uint64_t>(b->chunk_cap, 0xFFFFFFF0u);
    S.cnt = b->cnt;
    S.bar = b->bar;
    S.spin_limit = 1u << 24;  // about 4 s of polling: far beyond one phase
    // slabs of about n / 4 records (2^14 .. 2^22, never more than n: a pass
    // lists up to one head per record and a list holds n).  Larger slabs
    // mean fewer pass-0 phases but longer chains inside a slab, i.e. more
    // fix-up passes, each a few dependent memory round trips and two grid
    // barriers; on the scale-24 graph (64 queries) n / 16, n / 8, n / 4 and
    // n / 2 took 239, 207, 199 and 217 ms.
    S.slab = std::min<uint32_t>(SWEEP_SLAB, std::max<uint32_t>(std::min<uint32_t>(1u << 14, g->n), g->n / 4));
    S.max_passes = 1u << 12;
    S.list_cap = (uint32_t)std::min<uint64_t>((uint64_t)b->groups * n + 64, 0xFFFFFFF0u);
    const int grid = g->num_cus * std::min(occ, 4);
    void *args[] = {&S};
    prof_begin(g, st, &ev);
    const hipError_t e = hipLaunchCooperativeKernel((const void *)sweep_kernel, dim3(grid), dim3(SW_TB), args, 0, st);
    prof_end(g, st, KAIROS_K_PUSH, ev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return KAIROS_ERR_BUSY;
    }
    KAIROS_HIP(hipMemcpyAsync(b->h_pin, b->cnt, 64, hipMemcpyDeviceToHost, st));
    KAIROS_HIP(hipStreamSynchronize(st));
    if (b->h_pin[SWC_ABORT]) return KAIROS_ERR_DEVICE;
    if (g->prof.on) {
        std::lock_guard<std::mutex> lk(g->prof.mu);
        g->prof.rounds += b->h_pin[SWC_PASSES];
        g->prof.sw_slabs += b->h_pin[SWC_SLABS];
        g->prof.sw_passes += b->h_pin[SWC_PASSES];
        g->prof.sw_fix += b->h_pin[SWC_FIXEDGES];
    }
    return b->h_pin[SWC_OVER] ? KAIROS_ERR_BUSY : KAIROS_OK;
}

int run_vbatch_sweep(kairos_graph *g, VBatch *b, uint32_t q, const uint32_t *src, const uint32_t *ta,
                     const uint32_t *tw, uint32_t *out)
{
    hipStream_t st = b->stream;
    if (q > (size_t)b->groups * 64) return KAIROS_ERR_INVALID;
    int rc = ensure_time_order(g, st);
    if (rc) return rc;
    const uint32_t groups = (q + 63) / 64;
    uint4 *staging = b->h_q;
    for (uint32_t i = 0; i < q; ++i) staging[i] = make_uint4(g->h_perm[src[i]], ta[i], tw[i], 0);
    for (uint32_t gi = 0; gi < groups; ++gi) {
        rc = sweep_group(g, b, gi, gi * 64, std::min<uint32_t>(64, q - gi * 64), st);
        // a group the sweep could not settle, or a refused launch: the
        // lane-dense rounds answer the whole batch (they rewrite every row)
        if (rc == KAIROS_ERR_BUSY) {
            if (g->prof.on) {
                std::lock_guard<std::mutex> lk(g->prof.mu);
                g->prof.sw_fallbacks += 1;
            }
            return run_vbatch(g, b, q, src, ta, tw, out);
        }
        if (rc) return rc;
    }
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    hipLaunchKernelGGL(btranspose_kernel, dim3(gridc((uint64_t)((g->n + 63) / 64) * groups, 1, 16384)), dim3(256), 0,
                       st, b->arr, out, g->perm, g->n, q, groups);
    prof_end(g, st, KAIROS_K_INIT, ev);
    KAIROS_HIP(hipGetLastError());
    KAIROS_HIP(hipStreamSynchronize(st));
    return KAIROS_OK;
}

int vbatch_acquire(kairos_graph *g, uint32_t groups, VBatch **out)
{
    {
        std::lock_guard<std::mutex> lk(g->pool_mu);
        for (size_t i = 0; i < g->vbatches.size(); ++i)
            if (g->vbatches[i]->groups >= groups) {
                *out = g->vbatches[i];
                g->vbatches.erase(g->vbatches.begin() + i);
                return KAIROS_OK;
            }
        for (VBatch *b : g->vbatches) vbatch_destroy(b);
        g->vbatches.clear();
    }
    return vbatch_alloc(g, groups, out);
}

void vbatch_release(kairos_graph *g, VBatch *b)
{
    std::lock_guard<std::mutex> lk(g->pool_mu);
    g->vbatches.push_back(b);
}

}  // namespace kairos
