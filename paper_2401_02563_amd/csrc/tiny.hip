// Earliest arrival of one query on a small graph, in one workgroup whose
// LDS holds the whole query state.
//
// On a graph of a few thousand vertices a query is a chain of short
// label-correcting rounds (Alg. 2's frontier loop) over a few hundred
// vertices each; the general one-workgroup kernel spends each round on
// dependent round trips to memory for the arrival words, claim words and
// atomic minima.  Here those live in LDS: per vertex its arrival, its claim
// (the lowest out-edge already claimed, as in the general kernels) and the
// round that last put it in the frontier, 12 bytes, so graphs of up to
// TINY_N vertices fit.  The index (offsets, departures, edge records) is
// read from global memory, where a graph this size stays in L2.  Rounds
// are the general kernels' rounds: claims of the newly usable part of each
// frontier vertex's time-sorted adjacency by binary search, a block prefix
// sum over the claim lengths, each edge relaxed by one thread (LDS atomic
// minimum), improved heads with out-edges appended once per round.  The
// result is the fixpoint of the same relaxation, so it equals the general
// path's bit for bit.
#include "internal.h"

#include <vector>

namespace kairos {

namespace {

constexpr int TY = 1024;              // threads of the workgroup
constexpr int TY_UNR = 4;             // edges per thread per pass of the relaxation loop

__device__ __forceinline__ uint32_t ty_lower_bound(const uint32_t *__restrict__ a, uint32_t lo, uint32_t hi,
                                                   uint32_t key)
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

// q0, q1: n entries each (global; a vertex enters a round's queue once).
// stats (or null): the work counters' first shard.
__global__ __launch_bounds__(TY) void tiny_ea_kernel(const uint32_t *__restrict__ off, const uint32_t *__restrict__ tt,
                                                     const uint2 *__restrict__ da, uint32_t n, uint32_t n_live,
                                                     uint32_t max_t, uint32_t src, uint32_t ta, uint32_t tw,
                                                     uint32_t strict, const uint32_t *__restrict__ perm,
                                                     uint32_t *__restrict__ out, uint32_t *q0, uint32_t *q1,
                                                     unsigned long long *stats)
{
    __shared__ uint32_t s_arr[TINY_N];
    __shared__ uint32_t s_done[TINY_N];
    __shared__ uint32_t s_mark[TINY_N];
    __shared__ uint32_t s_pref[TY + 1];
    __shared__ uint32_t s_lo[TY];
    __shared__ uint32_t s_wsum[TY / 64];
    __shared__ uint32_t s_next;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63, w = tid >> 6;
    for (uint32_t v = tid; v < n; v += TY) {
        s_arr[v] = INF;
        s_done[v] = INF;
        s_mark[v] = 0u;
    }
    __syncthreads();
    if (tid == 0) {
        s_arr[src] = ta;
        q0[0] = src;
    }
    uint32_t F = 1, rounds = 0, items = 0, edges = 0, relax = 0, tries = 0;
    uint32_t *cur = q0, *nxt = q1;
    __syncthreads();
    for (uint32_t r = 1; F > 0; ++r) {
        ++rounds;
        if (tid == 0) s_next = 0u;
        __syncthreads();
        for (uint32_t base = 0; base < F; base += TY) {
            const uint32_t i = base + tid;
            uint32_t lo = 0, len = 0;
            if (i < F) {
                ++items;
                const uint32_t u = cur[i];
                const uint32_t ru = s_arr[u];
                // "Strictly succeeds": departures from ru + 1, except the
                // source's own edges
                const uint32_t key = ru + (strict && u != src ? 1u : 0u);
                const uint32_t b = off[u], e = off[u + 1];
                const uint32_t old = s_done[u];
                lo = ty_lower_bound(tt, b, old == INF ? e : min(old, e), key);
                uint32_t end = old;
                if (old == INF) end = tw > max_t ? e : ty_lower_bound(tt, lo, e, tw);
                if (lo < end) {
                    len = end - lo;
                    s_done[u] = lo;
                }
            }
            // block prefix sum of the claim lengths
            uint32_t x = len;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o);
                if (lane >= (uint32_t)o) x += y;
            }
            if (lane == 63) s_wsum[w] = x;
            s_lo[tid] = lo;
            __syncthreads();
            uint32_t woff = 0, total = 0;
            for (int w2 = 0; w2 < TY / 64; ++w2) {
                if ((uint32_t)w2 < w) woff += s_wsum[w2];
                total += s_wsum[w2];
            }
            s_pref[tid] = woff + x - len;
            if (tid == 0) s_pref[TY] = total;
            __syncthreads();
            edges += tid == 0 ? total : 0u;
            for (uint32_t j0 = 0; j0 < total; j0 += TY * TY_UNR) {
                uint32_t v[TY_UNR], a[TY_UNR];
                bool ok[TY_UNR];
#pragma unroll
                for (int k = 0; k < TY_UNR; ++k) {
                    const uint32_t j = j0 + k * TY + tid;
                    ok[k] = j < total;
                    // owner: the last item whose prefix is <= j
                    int lo_k = 0, hi_k = TY;
                    while (hi_k - lo_k > 1) {
                        const int mid = (lo_k + hi_k) >> 1;
                        if (s_pref[mid] <= j)
                            lo_k = mid;
                        else
                            hi_k = mid;
                    }
                    const uint2 dv = da[ok[k] ? s_lo[lo_k] + (j - s_pref[lo_k]) : 0u];
                    v[k] = dv.x;
                    a[k] = dv.y;
                }
#pragma unroll
                for (int k = 0; k < TY_UNR; ++k) {
                    if (ok[k] && a[k] <= tw && a[k] < s_arr[v[k]]) {
                        ++tries;
                        if (a[k] < atomicMin(&s_arr[v[k]], a[k])) {
                            ++relax;
                            // first improvement of this round: the head joins
                            // the next frontier (a head without out-edges has
                            // nothing to expand)
                            if (v[k] < n_live && atomicExch(&s_mark[v[k]], r) != r)
                                nxt[atomicAdd(&s_next, 1u)] = v[k];
                        }
                    }
                }
            }
            __syncthreads();
        }
        F = s_next;
        uint32_t *t = cur;
        cur = nxt;
        nxt = t;
        __syncthreads();
    }
    for (uint32_t c = tid; c < n; c += TY) out[c] = s_arr[perm[c]];
    if (stats) {
        // frontier entries, edges, atomic attempts and improvements summed
        // over each wavefront, one addition per wavefront; rounds once
        uint32_t c[4] = {items, edges, tries, relax};
        const int slot[4] = {ST_TAIL_ITEMS, ST_TAIL_EDGES, ST_ATTEMPTS, ST_RELAX};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            for (int o = 32; o > 0; o >>= 1) c[k] += __shfl_xor(c[k], o);
            if (lane == 0 && c[k]) atomicAdd(&stats[slot[k]], (unsigned long long)c[k]);
        }
        if (tid == 0) atomicAdd(&stats[ST_ROUNDS], (unsigned long long)rounds);
    }
}

}  // namespace

bool tiny_eligible(const kairos_graph *g)
{
    return g->n <= TINY_N && g->tuning.tail_limit > 0;
}

int run_tiny_earliest_arrival(kairos_graph *g, Slot *s, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out,
                              bool strict)
{
    if (!tiny_eligible(g)) return KAIROS_ERR_INVALID;
    hipStream_t st = s->stream;
    const uint32_t isrc = g->h_perm[src];
    // profiling: the slot's work counters (all shards zero between calls)
    const bool prof = g->prof.on && !s->fixed;
    unsigned long long *stats = prof ? s->stats : nullptr;
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    hipLaunchKernelGGL(tiny_ea_kernel, dim3(1), dim3(TY), 0, st, g->off_out, g->t_out, g->da_out, g->n, g->n_live,
                       g->max_t, isrc, ta, tw, strict ? 1u : 0u, g->perm, out, s->queue[0], s->queue[1], stats);
    prof_end(g, st, KAIROS_K_TAIL, ev);
    KAIROS_HIP(hipGetLastError());
    if (prof) {
        std::vector<unsigned long long> raw((size_t)ST_SHARDS * ST_WORDS);
        unsigned long long h[ST_WORDS];
        KAIROS_HIP(hipMemcpyAsync(raw.data(), s->stats, raw.size() * 8, hipMemcpyDeviceToHost, st));
        KAIROS_HIP(hipStreamSynchronize(st));
        KAIROS_HIP(hipMemsetAsync(s->stats, 0, raw.size() * 8, st));
        stats_sum_shards(raw.data(), h);
        prof_add_stats(g, h);
        std::lock_guard<std::mutex> lk(g->prof.mu);
        g->prof.rounds += h[ST_ROUNDS];
    }
    return KAIROS_OK;
}

}  // namespace kairos
