// Sweep form of a batched earliest-arrival group (batch_layout 3).
//
// The group's 64 queries share one pass over the graph's edges in departure
// order, as the one-pass scan of §7's temporal-paths reference takes them
// for one query: a wavefront holds a few edges at a time and lane q relaxes
// each for query q against the arrival rows of its tail and head (64 words
// of 4 bytes each, so a row is two cache lines read by one instruction).
// Edge records are read once for the whole group instead of once per query.
//
// The edges of the group's range [lo, hi) (departures in [min t_alpha,
// max t_omega)) are cut into slabs of `slab` consecutive records, taken in
// order.  An edge arrives after it departs (lambda >= 1), so no edge of a
// later slab can enable an edge of an earlier one, and a slab relaxed to a
// fixpoint stays final.  Inside a slab every edge is relaxed at once (pass
// 0), which can miss an edge whose tail is lowered by another edge of the
// same slab.  Every vertex lowered in a pass is listed, with a note of the
// least arrival the pass wrote into its row, and the next pass re-relaxes,
// through the out-index, each listed vertex's out-edges that depart from
// that arrival to the slab's last departure, for all lanes (a vertex listed
// twice is expanded once); passes repeat until one lowers nothing.  Edges
// departing at the slab's last time may belong to the next slab: relaxing
// them early with a real arrival is harmless.
//
// One cooperative launch runs all slabs and passes of a group, with grid
// barriers between phases; every block reads the same counters after a
// barrier, so all take the same branches.  A fix-up chunk list that would
// overflow, or a slab that needs more than `max_passes` passes, raises a
// flag and the host answers the group with the lane-dense rounds instead.
#pragma once

#include "stage.h"

namespace kairos {

constexpr int SW_TB = 256;    // threads per block
constexpr uint32_t SWEEP_SLAB = 1u << 22;  // most records per slab
constexpr int SW_E = 8;       // edges a wavefront holds at once in pass 0
constexpr uint32_t SW_C = 32; // out-edges per fix-up chunk

// counters (words of the group's counter array)
constexpr int SWC_LIST = 0;    // [2] lengths of the two changed-vertex lists
constexpr int SWC_CHUNK = 2;   // [2] fix-up chunk counts, by pass parity
constexpr int SWC_OVER = 4;    // 1: chunk list overflow or pass limit (the host falls back)
constexpr int SWC_PASSES = 5;  // passes run (all slabs)
constexpr int SWC_FIXEDGES = 6;// out-edges relaxed by fix-up passes (low 32 bits, profiling)
constexpr int SWC_SLABS = 7;   // slabs run
constexpr int SWC_ABORT = 8;   // 1: a barrier wait gave up

struct SwArgs {
    const uint4 *E;          // every edge {tail, head, t, a} in departure order
    uint64_t m;
    const uint32_t *off;     // out-index offsets
    const uint32_t *tt;      // out-edge departures
    const uint2 *da;         // out-edge {head, arrival}
    uint32_t *arr;           // [v][64] arrivals of the group's queries
    const uint2 *qw;         // [64] {t_alpha, t_omega}; lanes without a query {INF, 0}
    uint32_t *stamp;         // [n] id of the last expansion that took the vertex (0: none)
    unsigned long long *low; // [n] (~pass id << 32 | least arrival written to the row in that pass)
    uint32_t *list0, *list1; // changed vertices, n entries each
    uint4 *chunks;           // fix-up chunks {vertex, first out-edge, count, _}
    uint32_t chunk_cap;
    uint32_t *cnt;
    uint32_t *bar;
    uint32_t spin_limit;
    uint32_t slab;
    uint32_t max_passes;
    uint32_t list_cap;       // entries each list holds; a longer list is an overflow
};

// [lo, hi): the records departing in [min t_alpha, max t_omega) of the
// group (an edge departing at t_omega or later arrives after it).
__device__ __forceinline__ void sweep_range(const SwArgs &S, uint64_t &lo, uint64_t &hi)
{
    uint32_t ta = INF, tw = 0;
    for (int i = 0; i < 64; ++i) {
        const uint2 w = S.qw[i];
        if (w.x <= w.y) {
            ta = min(ta, w.x);
            tw = max(tw, w.y);
        }
    }
    uint64_t l = 0, h = S.m;
    while (l < h) {
        const uint64_t mid = (l + h) >> 1;
        if (S.E[mid].z < ta)
            l = mid + 1;
        else
            h = mid;
    }
    lo = l;
    h = S.m;
    while (l < h) {
        const uint64_t mid = (l + h) >> 1;
        if (S.E[mid].z < tw)
            l = mid + 1;
        else
            h = mid;
    }
    hi = ta <= tw ? l : lo;
}

// Records the least arrival that pass `pid` wrote into v's row: pass ids
// only grow, so keying the word by the complement of the id makes one
// atomic minimum keep the newest pass and, within it, the least arrival.
__device__ __forceinline__ void sweep_note_low(unsigned long long *low, uint32_t v, uint32_t pid, uint32_t a)
{
    atomicMin(&low[v], ((unsigned long long)(0xFFFFFFFFu - pid) << 32) | a);
}

// Lane q relaxes edge (u -> v, t, a) for its query given the tail's arrival
// and the head's arrival as read; true if the edge beat what was read.  The
// atomic minimum returns nothing (nothing waits on it): an edge that beat
// the read but lost to a concurrent lower value only lists its head once
// more, which costs a fix-up its work and never a result.
__device__ __forceinline__ bool sweep_relax(uint32_t *arr, uint2 w, uint32_t lane, uint32_t v, uint32_t t, uint32_t a,
                                            uint32_t tail_arr, uint32_t head_arr)
{
    const bool ok = t >= w.x && a <= w.y && tail_arr <= t && a < head_arr;
    if (ok) (void)__hip_atomic_fetch_min(&arr[(size_t)v * 64 + lane], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return ok;
}

// Pass 0 of a slab: records [s0, s1), SW_E per wavefront task; the next
// task's records are requested before this task's rows are used.  Every
// lowered head is appended (lane k for edge k); repeats are dropped when
// the list is expanded.
__device__ __forceinline__ void sweep_pass0(const SwArgs &S, uint64_t s0, uint64_t s1, uint32_t pid, uint2 w,
                                            Stage<512> &St)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t step = (uint64_t)gridDim.x * (SW_TB / 64) * SW_E;
    uint64_t e0 = s0 + ((uint64_t)blockIdx.x * (SW_TB / 64) + (threadIdx.x >> 6)) * SW_E;
    uint4 r[SW_E];
#pragma unroll
    for (int k = 0; k < SW_E; ++k) r[k] = S.E[e0 + k < s1 ? e0 + k : s0];
    for (; e0 < s1; e0 += step) {
        uint32_t ta[SW_E], ha[SW_E];
#pragma unroll
        for (int k = 0; k < SW_E; ++k) {
            ta[k] = S.arr[(size_t)r[k].x * 64 + lane];
            ha[k] = S.arr[(size_t)r[k].y * 64 + lane];
        }
        // the next task's records: issued after the rows (the in-order load
        // counter then lets the rows be used while these are in flight)
        __builtin_amdgcn_sched_barrier(0);
        uint4 nx[SW_E];
        const uint64_t e1 = e0 + step;
#pragma unroll
        for (int k = 0; k < SW_E; ++k) nx[k] = S.E[e1 + k < s1 ? e1 + k : s0];
        uint32_t mine = 0;
        bool mine_low = false;
#pragma unroll
        for (int k = 0; k < SW_E; ++k) {
            const bool live = e0 + k < s1;
            const bool low = live && sweep_relax(S.arr, w, lane, r[k].y, r[k].z, r[k].w, ta[k], ha[k]);
            const bool any = __ballot(low) != 0ull;
            if (any && lane == (uint32_t)k) sweep_note_low(S.low, r[k].y, pid, r[k].w);
            if (lane == (uint32_t)k) {
                mine = r[k].y;
                mine_low = any;
            }
        }
        unsigned long long bal[1];
        uint32_t item[1];
        bal[0] = __ballot(lane < (uint32_t)SW_E && mine_low);
        item[0] = mine;
        stage_append(St, bal, item);
#pragma unroll
        for (int k = 0; k < SW_E; ++k) r[k] = nx[k];
    }
}

// Fix-up expansion: lane per listed vertex; chunks of its out-edges that
// depart in [max(a, t_lo), t_hi], a the least arrival the listing pass
// wrote into the vertex's row (earlier departures cannot use any arrival
// that pass wrote, and arrivals written before it were expanded already).
// A vertex listed more than once is expanded once: the stamp names the
// last expansion that took it (a plain read and write; two lanes racing on
// one vertex only expand it twice, which repeats work and changes no
// result).
__device__ __forceinline__ void sweep_expand(const SwArgs &S, const uint32_t *list, uint32_t L, uint32_t t_lo,
                                             uint32_t t_hi, uint32_t pid, uint32_t listed_by, uint32_t *chunk_cnt)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (SW_TB / 64);
    const uint32_t wave = blockIdx.x * (SW_TB / 64) + (threadIdx.x >> 6);
    for (uint32_t i0 = wave * 64; i0 < L; i0 += waves * 64) {
        const uint32_t i = i0 + lane;
        uint32_t v = 0, b = 0, len = 0;
        if (i < L) {
            v = list[i];
            if (S.stamp[v] != pid) {
                S.stamp[v] = pid;
                const uint32_t o0 = S.off[v], o1 = S.off[v + 1];
                const unsigned long long lw = S.low[v];
                // the listing pass's note (always there for a listed vertex;
                // a stale one would only widen the range)
                const uint32_t least = (uint32_t)(lw >> 32) == 0xFFFFFFFFu - listed_by ? (uint32_t)lw : t_lo;
                const uint32_t from = max(least, t_lo);
                // first departure >= from and first departure > t_hi, side by side
                uint32_t l1 = o0, h1 = o1, l2 = o0, h2 = o1;
                while (l1 < h1 || l2 < h2) {
                    const uint32_t m1 = l1 + ((h1 - l1) >> 1), m2 = l2 + ((h2 - l2) >> 1);
                    const bool s1 = l1 < h1, s2 = l2 < h2;
                    const uint32_t x1 = S.tt[s1 ? m1 : o0], x2 = S.tt[s2 ? m2 : o0];
                    if (s1) {
                        if (x1 < from)
                            l1 = m1 + 1;
                        else
                            h1 = m1;
                    }
                    if (s2) {
                        if (x2 <= t_hi)
                            l2 = m2 + 1;
                        else
                            h2 = m2;
                    }
                }
                b = l1;
                len = from <= t_hi && l2 > l1 ? l2 - l1 : 0u;
            }
        }
        const uint32_t nch = (len + SW_C - 1) / SW_C;
        // wave prefix sum of the chunk counts, one reservation per wave
        uint32_t x = nch;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= (uint32_t)o) x += y;
        }
        const uint32_t total = __shfl(x, 63);
        uint32_t base = 0;
        if (lane == 63 && total) base = atomicAdd(chunk_cnt, total);
        base = __shfl(base, 63) + x - nch;
        for (uint32_t k = 0; k < nch; ++k) {
            const uint32_t c = base + k;
            if (c < S.chunk_cap) S.chunks[c] = make_uint4(v, b + k * SW_C, min(SW_C, len - k * SW_C), 0u);
        }
        if (base + nch > S.chunk_cap && nch) S.cnt[SWC_OVER] = 1u;
    }
}

// Fix-up relaxation: wavefront per chunk of at most SW_C out-edges, lane
// per query.  Lane j < SW_C reads record j; every lane then reads the head
// rows of all SW_C records at once, so a chunk costs about two round trips.
__device__ __forceinline__ void sweep_fix(const SwArgs &S, uint32_t C, uint32_t pid, uint2 w, Stage<512> &St,
                                          uint32_t &fix_edges)
{
    static_assert(SW_C <= 64, "a chunk's records are read one per lane");
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (SW_TB / 64);
    for (uint32_t c = blockIdx.x * (SW_TB / 64) + (threadIdx.x >> 6); c < C; c += waves) {
        const uint4 ch = S.chunks[c];
        const uint32_t tail_arr = S.arr[(size_t)ch.x * 64 + lane];
        const uint32_t f = ch.y + (lane < ch.z ? lane : 0u);
        const uint2 dv = S.da[f];
        const uint32_t tv = S.tt[f];
        fix_edges += ch.z;
        uint32_t v[SW_C], ha[SW_C];
#pragma unroll
        for (int j = 0; j < (int)SW_C; ++j) {
            v[j] = __builtin_amdgcn_readlane(dv.x, j);
            ha[j] = S.arr[(size_t)v[j] * 64 + lane];
        }
        uint32_t mine = 0;
        bool mine_low = false;
#pragma unroll
        for (int j = 0; j < (int)SW_C; ++j) {
            const bool live = (uint32_t)j < ch.z;
            const uint32_t t = __builtin_amdgcn_readlane(tv, j), a = __builtin_amdgcn_readlane(dv.y, j);
            const bool low = live && sweep_relax(S.arr, w, lane, v[j], t, a, tail_arr, ha[j]);
            const bool any = __ballot(low) != 0ull;
            if (any && lane == (uint32_t)j) sweep_note_low(S.low, v[j], pid, a);
            if (lane == (uint32_t)j) {
                mine = v[j];
                mine_low = any;
            }
        }
        unsigned long long bal[1];
        uint32_t item[1];
        bal[0] = __ballot(lane < SW_C && mine_low);
        item[0] = mine;
        stage_append(St, bal, item);
    }
}

// Grid barrier, then every block learns whether a barrier wait gave up (the
// word is sticky, so a block released by it sees it): block-uniform.
__device__ __forceinline__ bool sweep_sync(const SwArgs &S, uint32_t *s_word)
{
    grid_barrier(S.bar, S.spin_limit);
    if (threadIdx.x == 0) s_word[1] = grid_aborted(S.bar) ? 1u : 0u;
    __syncthreads();
    const bool ab = s_word[1] != 0u;
    __syncthreads();
    return ab;
}

// A counter every block reads after a barrier (block-uniform).
__device__ __forceinline__ uint32_t sweep_read(uint32_t *w, uint32_t *s_word)
{
    if (threadIdx.x == 0) s_word[0] = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t v = s_word[0];
    __syncthreads();
    return v;
}

// Counter discipline (all counters start at zero):
//  * list counter `cur` is appended to by one phase and read by every block
//    after the next barrier; the phase after that read (a fix-up's
//    relaxation) clears it, so both list counters are zero whenever a slab
//    settles;
//  * a settled slab's next pass 0 appends to the other list, never to the
//    counter that slower blocks may still be reading;
//  * chunk counters alternate with the fix-up iteration count, which runs on
//    across slabs; an expansion clears the one the following expansion
//    will use.
__global__ __launch_bounds__(SW_TB) void sweep_kernel(SwArgs S)
{
    __shared__ uint32_t s_stage[SW_TB / 64][512];
    __shared__ uint32_t s_word[2];
    const uint32_t lane = threadIdx.x & 63;
    const uint2 w = S.qw[lane];
    uint64_t lo, hi;
    sweep_range(S, lo, hi);
    uint32_t pid = 0, cur = 0, passes = 0, fix_edges = 0, slabs = 0, fi = 0;
    bool stop = false;
    for (uint64_t s0 = lo; s0 < hi && !stop; s0 += S.slab) {
        const uint64_t s1 = min(hi, s0 + (uint64_t)S.slab);
        const uint32_t t_lo = S.E[s0].z, t_hi = S.E[s1 - 1].z;
        ++slabs;
        ++passes;
        uint32_t listed_by = ++pid;
        {
            Stage<512> St{s_stage[threadIdx.x >> 6], 0u, cur ? S.list1 : S.list0, &S.cnt[SWC_LIST + cur],
                          S.list_cap};
            sweep_pass0(S, s0, s1, listed_by, w, St);
            stage_flush_block<512, SW_TB / 64>(St);
        }
        if (sweep_sync(S, s_word)) break;
        for (uint32_t f = 0;; ++f, ++fi) {
            const uint32_t L = sweep_read(&S.cnt[SWC_LIST + cur], s_word);
            if (L == 0) {
                cur ^= 1u;  // both list counters are zero; read this one no more
                break;
            }
            if (f + 1 >= S.max_passes || L > S.list_cap) {
                // a slab that will not settle: the host answers the group
                // another way
                if (blockIdx.x == 0 && threadIdx.x == 0) S.cnt[SWC_OVER] = 1u;
                stop = true;
                break;
            }
            if (blockIdx.x == 0 && threadIdx.x == 0) S.cnt[SWC_CHUNK + ((fi + 1) & 1u)] = 0u;
            const uint32_t xid = ++pid;
            sweep_expand(S, cur ? S.list1 : S.list0, L, t_lo, t_hi, xid, listed_by, &S.cnt[SWC_CHUNK + (fi & 1u)]);
            if (sweep_sync(S, s_word)) {
                stop = true;
                break;
            }
            const uint32_t C = min(sweep_read(&S.cnt[SWC_CHUNK + (fi & 1u)], s_word), S.chunk_cap);
            ++passes;
            if (blockIdx.x == 0 && threadIdx.x == 0) S.cnt[SWC_LIST + cur] = 0u;
            {
                Stage<512> St{s_stage[threadIdx.x >> 6], 0u, cur ? S.list0 : S.list1, &S.cnt[SWC_LIST + (cur ^ 1u)],
                              S.list_cap};
                listed_by = ++pid;
                sweep_fix(S, C, listed_by, w, St, fix_edges);
                stage_flush_block<512, SW_TB / 64>(St);
            }
            if (sweep_sync(S, s_word)) {
                stop = true;
                break;
            }
            cur ^= 1u;
        }
    }
    if (lane == 0 && fix_edges) atomicAdd(&S.cnt[SWC_FIXEDGES], fix_edges);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S.cnt[SWC_PASSES] = passes;
        S.cnt[SWC_SLABS] = slabs;
        S.cnt[SWC_ABORT] = grid_aborted(S.bar) ? 1u : 0u;
    }
}

// Lanes of the group's queries: {t_alpha, t_omega} and the source's word;
// lanes without a query get a window no edge fits.
__global__ void sweep_init_kernel(uint2 *qw, uint32_t *arr, const uint4 *__restrict__ hq, uint32_t q0, uint32_t nq)
{
    const uint32_t lane = threadIdx.x;
    if (lane >= 64) return;
    if (lane < nq) {
        const uint4 p = hq[q0 + lane];  // {src, t_alpha, t_omega, _}
        qw[lane] = make_uint2(p.y, p.z);
        arr[(size_t)p.x * 64 + lane] = p.y;
    } else {
        qw[lane] = make_uint2(INF, 0u);
    }
}

}  // namespace kairos
