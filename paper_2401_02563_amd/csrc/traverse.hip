// Frontier traversal over the time-sorted temporal CSR: earliest arrival
// (Alg. 2), and latest departure / fastest by a sweep over departure times.
//
// Differences from the paper's Alg. 2, and why:
//  * A vertex re-enters the frontier whenever its arrival improves (the
//    visit-once flag of Alg. 2 can keep a late arrival found in an early
//    round).  The source starts at t_alpha; edges are usable iff
//    t >= t_alpha and a <= t_omega; succession is non-strict (t >= arrival).
//  * TemporalEdgeMap's per-vertex choice between a T-CSR scan and an interval
//    index (§4.4, §5) becomes two binary searches into the vertex's
//    time-sorted adjacency: the first edge departing at or after the vertex's
//    arrival, and the first departing at or after t_omega (any such edge
//    arrives after t_omega).  Only the edges in between are read.
//  * done[u] remembers the lowest adjacency position already claimed for u.
//    When u comes back with an earlier arrival only the newly usable prefix
//    [lo, done[u]) is read: whether an edge relaxes its head does not depend
//    on the tail's arrival once it is usable, so every out-edge is read at
//    most once per query.  Claims are made with atomicMin, so concurrent
//    claims never overlap.
//  * Each (query, vertex) owns one 64-bit word: its arrival in the high half
//    and the stamp of the round that last lowered it in the low half.
//    writeMin is one device-scope 64-bit atomicMin of (arrival, round stamp):
//    it lowers the arrival and, in the same operation, tells whether this
//    round already lowered it (then the vertex is already in the next
//    frontier).  Stamps grow from round to round, so an equal arrival never
//    replaces a newer stamp.  Arrivals only decrease, so a stale plain read
//    of the arrival can only cause a redundant atomic, never a missed update.
//  * New frontier entries are collected per wave in LDS and reserved in the
//    global frontier with one atomicAdd per flush, since same-address atomics
//    are serialised at the memory side.
//  * Work is balanced inside a block by a prefix sum over the claimed range
//    lengths; ranges of at least `split` edges are cut into chunks of `chunk`
//    edges that a second kernel spreads over the whole GPU.

#include "internal.h"
#include "scan.h"
#include "stage.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace kairos {

namespace {

constexpr int TB = 256;  // threads per traversal block

struct TravArgs {
    const uint32_t *off;     // out-index offsets
    const uint32_t *tt;      // out-edge departure
    const uint2 *da;         // out-edge {head, arrival}
    const uint32_t *off_in;  // in-index offsets
    const uint32_t *a_in;    // in-edge arrival
    const uint2 *st_in;      // in-edge {tail, departure}
    const uint4 *qp;         // per query {src, t_alpha, t_omega, sweep departure}
    uint32_t n;
    unsigned long long *av;  // per (query, vertex): arrival << 32 | round stamp
    uint32_t *done;
    uint32_t *fa;
    uint32_t *l1;
    const uint32_t *cur;
    uint32_t *next;
    uint32_t *cnt;
    uint4 *chunks;
    uint32_t chunk_cap;
    unsigned long long *stats;
    uint32_t round;
    uint32_t stamp_val;
    uint32_t split;
    uint32_t chunk;
    uint32_t nq;             // queries (dense pull covers nq*n vertices)
    uint32_t track_volume;   // accumulate out-degree of enqueued vertices
    uint32_t *qflag;         // per query: round+1 when it enqueued something (or null)
    uint32_t max_t;          // largest departure time in the graph
    const uint32_t *steps;   // sweep departure times, descending (single query)
    uint32_t nsteps;
    uint32_t dense;          // 1: walk all vertices, members have stamp == front_stamp
    uint32_t front_stamp;    // stamp value that marked the current frontier
    uint8_t *filt;           // packed arrival codes, filt_stride(n) bytes per query (null: none)
    uint2 *fpar;             // per query: arrival-code parameters {base, shift | bits << 8}
    uint32_t fbits;          // code width given to queries started by this launch (0: off)
    uint32_t fstride;        // bytes per query region of filt
    uint32_t max_a;          // largest arrival time in the graph
    // level-synchronous rounds (temporal BFS): the tails of round r expand
    // from their arrivals at the start of r, snap[i] for frontier entry i,
    // and a vertex first reached in round r gets hop[v] = r + 1
    uint32_t *snap;
    uint32_t *hop;
    uint32_t strict;         // succession of queries started by this launch (1: "Strictly succeeds")
    uint32_t dedupe;         // one atomic per run of lanes into the same slot
    uint32_t n_live;         // vertices from this id on have no out-edges: never enqueued
    uint32_t max_deg;        // largest out-degree
    uint32_t min_per;        // least frontier entries per block and pass of the push phase
};

// Per-query parameter word fpar.y: code shift (bits 0-7), code width (bits
// 8-15), strict succession (bit 16).
__device__ __forceinline__ uint32_t fp_bits(uint32_t fp) { return (fp >> 8) & 0xFFu; }
__device__ __forceinline__ uint32_t fp_strict(uint32_t fp) { return (fp >> 16) & 1u; }

// Key of the binary search for the first usable out-edge of tail u reached
// at r: "Succeeds" allows departures at r, "Strictly succeeds" from r + 1.
// The source's own edges need only t >= its start under either predicate
// (the first edge of a path has no predecessor).  r <= TMAX, so r + 1 does
// not wrap.
__device__ __forceinline__ uint32_t departure_key(uint32_t r, uint32_t fp, uint32_t u, uint32_t src)
{
    return r + (fp_strict(fp) && u != src ? 1u : 0u);
}

__device__ __forceinline__ uint32_t arrival_of(const unsigned long long *av, size_t i)
{
    return ((const uint32_t *)av)[2 * i + 1];
}
__device__ __forceinline__ uint32_t stamp_of(const unsigned long long *av, size_t i)
{
    return ((const uint32_t *)av)[2 * i];
}
__device__ __forceinline__ unsigned long long av_word(uint32_t arrival, uint32_t stamp)
{
    return ((unsigned long long)arrival << 32) | stamp;
}

// Arrival codes.  For a query with window [t_alpha, t_omega] and code width
// B (2, 4 or 8 bits, L = 2^B - 1), code c < L of a vertex promises
// arr <= t_alpha + (c + 1) * 2^shift, and c = L promises nothing; shift is
// the smallest with 2^B * 2^shift >= min(t_omega, max arrival) - t_alpha, so
// the L finite codes split the reachable range into 2^B equal parts.  An
// edge arriving at or after the promised bound cannot improve its head and is
// dropped without reading the arrival word.  Codes only decrease, and a code
// is only ever stored from a real arrival of the vertex or copied from an
// earlier read of the same byte, so every code read, however stale, is a
// valid promise.
__device__ __forceinline__ uint2 filter_params(uint32_t ta, uint32_t tw, uint32_t max_a, uint32_t bits)
{
    if (bits == 0) return make_uint2(0u, 0u);
    const uint32_t hi = min(tw, max_a);
    const uint64_t range = hi > ta ? (uint64_t)(hi - ta) : 1ull;
    uint32_t sh = 0;
    while (((1ull << bits) << sh) < range) ++sh;
    return make_uint2(ta, sh | (bits << 8));
}

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *__restrict__ a, uint32_t lo,
                                                    uint32_t hi, uint32_t key)
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

// Edges are relaxed UNR at a time per lane: all loads of the group are
// issued before any result is used, so each lane keeps several independent
// memory requests in flight (the edge record, then the head's arrival).
constexpr int UNR = 4;

struct EdgeGroup {
    uint32_t v[UNR], a[UNR], q[UNR], tw[UNR], sd[UNR], cur[UNR];
    uint32_t fb[UNR], fp[UNR];  // the query's arrival-code parameters
    bool ok[UNR];
};

// Relax a group of UNR edges per lane.  The arrival reads, the atomic
// minima and the stamp exchanges of the group are each issued together (they
// are independent), so a lane waits for one round trip per stage instead of
// one per edge.  On return bal[k] holds the lanes whose edge k put its head
// into the next frontier (first improvement of the round) and item[k] that
// entry; the caller appends them to its output.
template <bool SWEEP>
__device__ __forceinline__ void relax_group(const TravArgs &A, EdgeGroup &G, unsigned long long (&bal)[UNR],
                                            uint32_t (&item)[UNR], uint32_t *vol_cnt, unsigned long long &nrelax)
{
    // Loads are unconditional from a valid address (a masked-off lane reads
    // word 0), and results of predicated atomics get no default value: a
    // conditional load or atomic whose register is also written on the other
    // path must complete before that write, which would serialise the group.
    size_t sv[UNR];
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
        G.ok[k] = G.ok[k] && G.a[k] <= G.tw[k];
        sv[k] = (size_t)G.q[k] * A.n + G.v[k];
    }
    size_t fbyte[UNR];
    uint32_t fsh[UNR];
    if (A.filt) {
        // the head's arrival code (see filter_params); at 2 bits per vertex
        // the codes of 2^24 vertices take 4 MB and stay in L2, where the
        // arrival words themselves (64 MB) do not
        uint32_t f[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const uint32_t bits = fp_bits(G.fp[k]);
            const uint64_t bit = (uint64_t)G.q[k] * A.fstride * 8u + (uint64_t)G.v[k] * bits;
            fbyte[k] = (size_t)(bit >> 3);
            fsh[k] = (uint32_t)(bit & 7u);
            f[k] = A.filt[G.ok[k] ? fbyte[k] : 0];
        }
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const uint32_t L = (1u << fp_bits(G.fp[k])) - 1u;  // 0 when the query has no codes
            const uint32_t c = (f[k] >> fsh[k]) & L;
            // the bound can exceed 32 bits (c + 1 <= 255, shift <= 31)
            const uint64_t bound = (uint64_t)G.fb[k] + ((uint64_t)(c + 1u) << (G.fp[k] & 31u));
            G.ok[k] = G.ok[k] && (c == L || (uint64_t)G.a[k] < bound);
        }
    }
#pragma unroll
    for (int k = 0; k < UNR; ++k) G.cur[k] = arrival_of(A.av, G.ok[k] ? sv[k] : 0);
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
        G.ok[k] = G.ok[k] && G.a[k] < G.cur[k];
        if (A.dedupe) dedupe_runs(G.ok[k], G.a[k], (uint64_t)sv[k]);
    }
    unsigned long long old[UNR];
#pragma unroll
    for (int k = 0; k < UNR; ++k)
        if (G.ok[k]) old[k] = atomicMin(&A.av[sv[k]], av_word(G.a[k], A.stamp_val));
    uint32_t st[UNR];
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
        nrelax += G.ok[k] ? (1ull << 32) : 0ull;  // high half: atomic attempts
        G.ok[k] = G.ok[k] && G.a[k] < (uint32_t)(old[k] >> 32);
        nrelax += G.ok[k] ? 1ull : 0ull;
        if (G.ok[k]) st[k] = (uint32_t)old[k];  // stamp of the round that last lowered it
        // the one atomic that finds the vertex unreached sets its level
        if (A.hop && G.ok[k] && (uint32_t)(old[k] >> 32) == INF) A.hop[sv[k]] = A.round + 1u;
    }
    if (A.filt) {
        // plain byte read-modify-write: a racing store may put back an older
        // (looser) code of this or a neighbouring vertex, which stays valid
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const uint32_t bits = fp_bits(G.fp[k]);
            if (G.ok[k] && bits) {
                const uint32_t L = (1u << bits) - 1u, sh = G.fp[k] & 31u;
                const uint64_t d = G.a[k] > G.fb[k] ? (uint64_t)(G.a[k] - G.fb[k]) : 0ull;
                const uint32_t c = d ? (uint32_t)(((d + (1ull << sh) - 1ull) >> sh) - 1ull) : 0u;
                if (c < L) {
                    const uint32_t cur = A.filt[fbyte[k]];
                    if (c < ((cur >> fsh[k]) & L))
                        A.filt[fbyte[k]] = (uint8_t)((cur & ~(L << fsh[k])) | (c << fsh[k]));
                }
            }
        }
    }
    if (SWEEP) {
#pragma unroll
        for (int k = 0; k < UNR; ++k)
            if (G.ok[k] && G.sd[k] != INF) {
                atomicMin(&A.fa[sv[k]], G.a[k] - G.sd[k]);
                atomicMax(&A.l1[sv[k]], G.sd[k] + 1u);
            }
    }
    uint32_t vol = 0;
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
        // a head without out-edges has nothing to expand: its arrival is
        // final for this round's purpose, so it stays out of the frontier
        const bool push = G.ok[k] && st[k] != A.stamp_val && G.v[k] < A.n_live;
        bal[k] = __ballot(push);
        item[k] = (uint32_t)sv[k];
        if (push) {
            if (A.qflag) A.qflag[G.q[k]] = A.round + 1u;
            if (A.track_volume) vol += A.off[G.v[k] + 1] - A.off[G.v[k]];
        }
    }
    if (A.track_volume) {
        for (int o = 32; o > 0; o >>= 1) vol += __shfl_xor(vol, o);
        if ((threadIdx.x & 63) == 0 && vol) atomicAdd(vol_cnt, vol);
    }
}

// One query's view for relax_group_u: its rows and parameters, all
// wave-uniform.
struct QueryRow {
    unsigned long long *av;  // arrival words of the query
    uint32_t *fa, *l1;       // sweep rows (SWEEP only)
    uint32_t *hop;           // level row (temporal BFS) or null
    uint32_t q, qbase;       // query index; its entries are qbase + v
    uint32_t tw, sd;
};

__device__ __forceinline__ QueryRow query_row(const TravArgs &A, uint32_t q, bool sweep)
{
    const uint4 p = A.qp[q];
    const size_t base = (size_t)q * A.n;
    QueryRow Q;
    Q.av = A.av + base;
    Q.fa = sweep ? A.fa + base : nullptr;
    Q.l1 = sweep ? A.l1 + base : nullptr;
    Q.hop = A.hop ? A.hop + base : nullptr;
    Q.q = q;
    Q.qbase = (uint32_t)base;
    Q.tw = p.z;
    Q.sd = p.w;
    return Q;
}

// relax_group for a wavefront whose lanes all relax edges of one query and
// no arrival codes: the query's values are scalars, slots are head ids into
// its own rows, and runs of equal heads are found on 32-bit keys.  Same
// steps and results as relax_group.
// Stage 1: the window test and the heads' arrival reads.
__device__ __forceinline__ void relax_load_u(const QueryRow &Q, const uint32_t (&v)[UNR], const uint32_t (&a)[UNR],
                                             bool (&ok)[UNR], uint32_t (&cur)[UNR])
{
#pragma unroll
    for (int k = 0; k < UNR; ++k) ok[k] = ok[k] && a[k] <= Q.tw;
#pragma unroll
    for (int k = 0; k < UNR; ++k) cur[k] = arrival_of(Q.av, ok[k] ? v[k] : 0u);
}

// Stage 2: everything after the arrival reads.
template <bool SWEEP>
__device__ __forceinline__ void relax_apply_u(const TravArgs &A, const QueryRow &Q, const uint32_t (&v)[UNR],
                                              uint32_t (&a)[UNR], bool (&ok)[UNR], const uint32_t (&cur)[UNR],
                                              unsigned long long (&bal)[UNR], uint32_t (&item)[UNR],
                                              uint32_t *vol_cnt, unsigned long long &nrelax)
{
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
        ok[k] = ok[k] && a[k] < cur[k];
        if (A.dedupe) dedupe_runs32(ok[k], a[k], v[k]);
    }
    unsigned long long old[UNR];
#pragma unroll
    for (int k = 0; k < UNR; ++k)
        if (ok[k]) old[k] = atomicMin(&Q.av[v[k]], av_word(a[k], A.stamp_val));
    uint32_t st[UNR];
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
        nrelax += ok[k] ? (1ull << 32) : 0ull;
        ok[k] = ok[k] && a[k] < (uint32_t)(old[k] >> 32);
        nrelax += ok[k] ? 1ull : 0ull;
        if (ok[k]) st[k] = (uint32_t)old[k];
        if (Q.hop && ok[k] && (uint32_t)(old[k] >> 32) == INF) Q.hop[v[k]] = A.round + 1u;
    }
    if (SWEEP && Q.sd != INF) {
#pragma unroll
        for (int k = 0; k < UNR; ++k)
            if (ok[k]) {
                atomicMin(&Q.fa[v[k]], a[k] - Q.sd);
                atomicMax(&Q.l1[v[k]], Q.sd + 1u);
            }
    }
    uint32_t vol = 0;
    bool any = false;
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
        const bool push = ok[k] && st[k] != A.stamp_val && v[k] < A.n_live;
        bal[k] = __ballot(push);
        item[k] = Q.qbase + v[k];
        any = any || push;
        if (push && A.track_volume) vol += A.off[v[k] + 1] - A.off[v[k]];
    }
    if (A.qflag && any) A.qflag[Q.q] = A.round + 1u;
    if (A.track_volume) {
        for (int o = 32; o > 0; o >>= 1) vol += __shfl_xor(vol, o);
        if ((threadIdx.x & 63) == 0 && vol) atomicAdd(vol_cnt, vol);
    }
}

template <bool SWEEP>
__device__ __forceinline__ void relax_group_u(const TravArgs &A, const QueryRow &Q, const uint32_t (&v)[UNR],
                                              uint32_t (&a)[UNR], bool (&ok)[UNR], unsigned long long (&bal)[UNR],
                                              uint32_t (&item)[UNR], uint32_t *vol_cnt, unsigned long long &nrelax)
{
    uint32_t cur[UNR];
    relax_load_u(Q, v, a, ok, cur);
    relax_apply_u<SWEEP>(A, Q, v, a, ok, cur, bal, item, vol_cnt, nrelax);
}

// Appends the group's entries to a frontier whose length lives in LDS (the
// one-workgroup kernel): one LDS atomic per wavefront.
__device__ __forceinline__ void lds_append(uint32_t *next, uint32_t *s_cnt, const unsigned long long (&bal)[UNR],
                                           const uint32_t (&item)[UNR])
{
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < UNR; ++k) total += __popcll(bal[k]);
    if (total == 0) return;
    const uint32_t lane = threadIdx.x & 63;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(s_cnt, total);
    base = __shfl(base, 0);
    const uint64_t lt = lanes_below();
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
        if ((bal[k] >> lane) & 1ull) next[base + __popcll(bal[k] & lt)] = item[k];
        base += __popcll(bal[k]);
    }
}

constexpr int SCAP = 512;  // staged frontier entries per wavefront
using TStage = Stage<SCAP>;

// Push round, part 1: one thread per frontier item claims the newly usable
// part of its adjacency; short claims are relaxed by the block with a
// prefix-sum load balance, claims of at least `split` edges are cut into
// chunks for part 2 (one chunk-list reservation per block and pass).
template <bool SWEEP, int B, bool UQ>
__device__ __forceinline__ void push_phase(const TravArgs &A, uint32_t F, TStage &S, unsigned long long &n_edges,
                                           unsigned long long &n_relax, unsigned long long &n_items)
{
    // UQ: one query and no arrival codes; every entry is a vertex of query
    // 0 and edges go through relax_group_u
    QueryRow Q0;
    if (UQ) Q0 = query_row(A, 0u, SWEEP);
    __shared__ uint32_t s_pref[B + 1];
    __shared__ uint32_t s_lo[B];
    __shared__ uint32_t s_q[B];
    __shared__ uint32_t s_tw[B];
    __shared__ uint32_t s_sd[B];
    __shared__ uint2 s_fp[B];
    __shared__ uint32_t s_wsum[B / 64];
    __shared__ uint32_t s_csum[B / 64];
    __shared__ uint32_t s_cb;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const uint32_t r3 = A.round % 3u;
    if (blockIdx.x == 0 && tid == 0) {
        A.cnt[CNT_FRONT + (A.round + 2u) % 3u] = 0u;
        A.cnt[CNT_PULLVOL + (A.round + 2u) % 3u] = 0u;
        A.cnt[CNT_CHUNK + (A.round + 1u) % 3u] = 0u;
    }
    uint32_t *vol_cnt = &A.cnt[CNT_PULLVOL + (A.round + 1u) % 3u];
    uint32_t *chunk_cnt = &A.cnt[CNT_CHUNK + r3];

    // sparse rounds walk the frontier queue; dense rounds walk every vertex
    // in id order and expand the members (stamped by the previous round), so
    // offsets, claim words and adjacency ranges are read in address order
    const uint32_t span = A.dense ? A.n : F;
    // entries per block and pass: B, or fewer when the frontier would not
    // fill the grid and adjacencies are long, so that a small frontier is
    // spread over more blocks and each block relaxes fewer edges (a block
    // relaxes its entries' short claims itself: 256 entries with 100-edge
    // claims keep one block busy for a hundred edge groups while others
    // idle).  Never below A.min_per, about B * 32 / average out-degree:
    // with short adjacencies every extra block only adds its fixed cost.
    const uint32_t per = max(min((uint32_t)B, A.min_per), min((uint32_t)B, (span + gridDim.x - 1u) / gridDim.x));
    for (uint32_t base = blockIdx.x * per; base < span; base += gridDim.x * per) {
        const uint32_t i = base + tid;
        uint32_t lo = 0, len = 0, q = 0, tw = 0, sd = 0, nch = 0;
        uint2 fpq = make_uint2(0u, 0u);
        if (tid < per && i < span && (!A.dense || stamp_of(A.av, i) == A.front_stamp)) {
            ++n_items;
            const uint32_t item = A.dense ? i : A.cur[i];
            q = UQ ? 0u : item / A.n;
            const uint32_t u = item - q * A.n;
            const uint4 p = A.qp[q];
            fpq = A.fpar[q];
            tw = p.z;
            sd = p.w;
            const size_t su = (size_t)q * A.n + u;
            // Each (query, vertex) is expanded by one thread per round (round
            // stamps), and rounds are separate launches, so the tail's
            // arrival and its claim word need no atomics here.
            const uint32_t r = A.snap ? A.snap[i] : arrival_of(A.av, su);
            const uint32_t b = A.off[u], e = A.off[u + 1];
            const uint32_t old = A.done[su];
            lo = lower_bound_u32(A.tt, b, old == INF ? e : min(old, e), departure_key(r, fpq.y, u, p.x));
            uint32_t end = old;
            if (old == INF) end = tw > A.max_t ? e : lower_bound_u32(A.tt, lo, e, tw);
            if (lo < end) {
                len = end - lo;
                A.done[su] = lo;
            }
            if (len >= A.split) nch = (len + A.chunk - 1) / A.chunk;
        }
        // exclusive prefix sums over the block of the short claim lengths
        // (so the block total stays below B * split) and of the chunk counts
        const uint32_t sl = nch ? 0u : len;
        uint32_t x = sl, c = nch;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            const uint32_t z = __shfl_up(c, o);
            if (lane >= o) {
                x += y;
                c += z;
            }
        }
        if (lane == 63) {
            s_wsum[w] = x;
            s_csum[w] = c;
        }
        s_lo[tid] = lo;
        if (!UQ) {
            s_q[tid] = q;
            s_tw[tid] = tw;
            s_sd[tid] = sd;
            s_fp[tid] = fpq;
        }
        __syncthreads();
        uint32_t woff = 0, total = 0, coff = 0, ctotal = 0;
        for (int w2 = 0; w2 < B / 64; ++w2) {
            if (w2 < w) {
                woff += s_wsum[w2];
                coff += s_csum[w2];
            }
            total += s_wsum[w2];
            ctotal += s_csum[w2];
        }
        s_pref[tid] = woff + x - sl;
        if (tid == 0) {
            s_pref[B] = total;
            if (ctotal) s_cb = atomicAdd(chunk_cnt, ctotal);
        }
        __syncthreads();
        uint32_t ser_lo = 0, ser_len = 0;
        if (nch) {
            const uint32_t cb = s_cb + coff + c - nch;
            const uint32_t fit = cb >= A.chunk_cap ? 0u : min(nch, A.chunk_cap - cb);
            for (uint32_t k = 0; k < fit; ++k)
                A.chunks[cb + k] = make_uint4(q, lo + k * A.chunk, min(A.chunk, len - k * A.chunk), 0u);
            const uint32_t covered = (uint32_t)min((uint64_t)len, (uint64_t)fit * A.chunk);
            // chunk list full (not expected with the list sized from the
            // tuning): this lane walks the rest by itself
            ser_lo = lo + covered;
            ser_len = len - covered;
        }
        if (tid == 0) n_edges += total;
        if (UQ) {
            for (uint32_t j0 = 0; j0 < total; j0 += B * UNR) {
                uint32_t v[UNR], a[UNR];
                bool ok[UNR];
#pragma unroll
                for (int k = 0; k < UNR; ++k) {
                    const uint32_t j = j0 + k * B + tid;
                    ok[k] = j < total;
                    int lo_k = 0, hi_k = B;
                    while (hi_k - lo_k > 1) {
                        const int mid = (lo_k + hi_k) >> 1;
                        if (s_pref[mid] <= j)
                            lo_k = mid;
                        else
                            hi_k = mid;
                    }
                    const uint2 dv = A.da[ok[k] ? s_lo[lo_k] + (j - s_pref[lo_k]) : 0u];
                    v[k] = dv.x;
                    a[k] = dv.y;
                }
                unsigned long long bal[UNR];
                uint32_t item[UNR];
                relax_group_u<SWEEP>(A, Q0, v, a, ok, bal, item, vol_cnt, n_relax);
                stage_append(S, bal, item);
            }
            n_edges += ser_len;
            uint32_t ser_done = 0;
            while (__ballot(ser_done < ser_len)) {
                uint32_t v[UNR], a[UNR];
                bool ok[UNR];
#pragma unroll
                for (int k = 0; k < UNR; ++k) {
                    ok[k] = ser_done < ser_len;
                    const uint2 dv = A.da[ok[k] ? ser_lo + ser_done : 0u];
                    if (ok[k]) ++ser_done;
                    v[k] = dv.x;
                    a[k] = dv.y;
                }
                unsigned long long bal[UNR];
                uint32_t item[UNR];
                relax_group_u<SWEEP>(A, Q0, v, a, ok, bal, item, vol_cnt, n_relax);
                stage_append(S, bal, item);
            }
            __syncthreads();
            continue;
        }
        for (uint32_t j0 = 0; j0 < total; j0 += B * UNR) {
            EdgeGroup G;
#pragma unroll
            for (int k = 0; k < UNR; ++k) {
                const uint32_t j = j0 + k * B + tid;
                G.ok[k] = j < total;
                // owner: the last item whose prefix is <= j
                int lo_k = 0, hi_k = B;
                while (hi_k - lo_k > 1) {
                    const int mid = (lo_k + hi_k) >> 1;
                    if (s_pref[mid] <= j)
                        lo_k = mid;
                    else
                        hi_k = mid;
                }
                const uint32_t e = G.ok[k] ? s_lo[lo_k] + (j - s_pref[lo_k]) : 0u;
                const uint2 dv = A.da[e];
                G.v[k] = dv.x;
                G.a[k] = dv.y;
                G.q[k] = s_q[lo_k];
                G.tw[k] = s_tw[lo_k];
                G.sd[k] = s_sd[lo_k];
                const uint2 f = s_fp[lo_k];
                G.fb[k] = f.x;
                G.fp[k] = f.y;
            }
            unsigned long long bal[UNR];
            uint32_t item[UNR];
            relax_group<SWEEP>(A, G, bal, item, vol_cnt, n_relax);
            stage_append(S, bal, item);
        }
        // per-lane walk of an overflowed claim, wave-uniform trip count
        n_edges += ser_len;
        uint32_t ser_done = 0;
        while (__ballot(ser_done < ser_len)) {
            EdgeGroup G;
#pragma unroll
            for (int k = 0; k < UNR; ++k) {
                G.ok[k] = ser_done < ser_len;
                const uint2 dv = A.da[G.ok[k] ? ser_lo + ser_done : 0u];
                if (G.ok[k]) ++ser_done;
                G.v[k] = dv.x;
                G.a[k] = dv.y;
                G.q[k] = q;
                G.tw[k] = tw;
                G.sd[k] = sd;
                G.fb[k] = fpq.x;
                G.fp[k] = fpq.y;
            }
            unsigned long long bal[UNR];
            uint32_t item[UNR];
            relax_group<SWEEP>(A, G, bal, item, vol_cnt, n_relax);
            stage_append(S, bal, item);
        }
        __syncthreads();
    }
}

template <bool SWEEP, int B, bool UQ>
__global__ __launch_bounds__(B) void push_kernel(TravArgs A)
{
    __shared__ uint32_t s_stage[B / 64][SCAP];
    TStage S{s_stage[threadIdx.x >> 6], 0u, A.next, &A.cnt[CNT_FRONT + (A.round + 1u) % 3u]};
    unsigned long long n_edges = 0, n_relax = 0, n_items = 0;
    push_phase<SWEEP, B, UQ>(A, A.cnt[CNT_FRONT + A.round % 3u], S, n_edges, n_relax, n_items);
    stage_flush_block<SCAP, B / 64>(S);
    unsigned long long v[4] = {n_relax & 0xFFFFFFFFull, n_relax >> 32, n_items, n_edges};
    const int slot[4] = {ST_RELAX, ST_ATTEMPTS, ST_ITEMS, ST_EDGES};
    block_stats<B / 64>(A.stats, v, slot);
}

// Push round, part 2: every wave takes whole chunks (grid-stride over the
// chunk list) and relaxes their edges UNR per lane at a time.
template <bool SWEEP, int B, bool UQ>
__device__ __forceinline__ void chunk_phase(const TravArgs &A, TStage &S, unsigned long long &n_edges,
                                            unsigned long long &n_relax)
{
    const uint32_t r3 = A.round % 3u;
    const uint32_t C = min(A.cnt[CNT_CHUNK + r3], A.chunk_cap);
    uint32_t *vol_cnt = &A.cnt[CNT_PULLVOL + (A.round + 1u) % 3u];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (B / 64);
    for (uint32_t c = blockIdx.x * (B / 64) + (threadIdx.x >> 6); c < C; c += waves) {
        if (UQ) {
            // the chunk's query, start and length are the same for the
            // whole wavefront: scalars
            const uint4 chv = A.chunks[c];
            const uint32_t cq = __builtin_amdgcn_readfirstlane(chv.x);
            const uint32_t c0 = __builtin_amdgcn_readfirstlane(chv.y);
            const uint32_t cz = __builtin_amdgcn_readfirstlane(chv.z);
            const QueryRow Q = query_row(A, cq, SWEEP);
            const uint2 *rec = A.da + c0;
            if (lane == 0) n_edges += cz;
            // the next group's records are requested while this group's
            // arrival reads are in flight
            uint2 r[UNR];
#pragma unroll
            for (int k = 0; k < UNR; ++k) {
                const uint32_t off = k * 64 + lane;
                r[k] = rec[off < cz ? off : 0u];
            }
            for (uint32_t k0 = 0; k0 < cz; k0 += 64 * UNR) {
                uint32_t v[UNR], a[UNR], cur[UNR];
                bool ok[UNR];
#pragma unroll
                for (int k = 0; k < UNR; ++k) {
                    ok[k] = k0 + k * 64 + lane < cz;
                    v[k] = r[k].x;
                    a[k] = r[k].y;
                }
                relax_load_u(Q, v, a, ok, cur);
                // issued after all arrival reads (the scheduler may not mix
                // them in: the in-order load counter would then make the
                // arrival waits cover these too), and unconditional (past
                // the end: the chunk's first record) for the same reason
                __builtin_amdgcn_sched_barrier(0);
                const uint32_t k1 = k0 + 64 * UNR;
#pragma unroll
                for (int k = 0; k < UNR; ++k) {
                    const uint32_t off = k1 + k * 64 + lane;
                    r[k] = rec[off < cz ? off : 0u];
                }
                unsigned long long bal[UNR];
                uint32_t item[UNR];
                relax_apply_u<SWEEP>(A, Q, v, a, ok, cur, bal, item, vol_cnt, n_relax);
                stage_append(S, bal, item);
            }
            continue;
        }
        const uint4 ch = A.chunks[c];
        const uint4 p = A.qp[ch.x];
        const uint2 fpq = A.fpar[ch.x];
        if (lane == 0) n_edges += ch.z;
        for (uint32_t k0 = 0; k0 < ch.z; k0 += 64 * UNR) {
            EdgeGroup G;
#pragma unroll
            for (int k = 0; k < UNR; ++k) {
                const uint32_t off = k0 + k * 64 + lane;
                G.ok[k] = off < ch.z;
                const uint2 dv = A.da[G.ok[k] ? ch.y + off : 0u];
                G.v[k] = dv.x;
                G.a[k] = dv.y;
                G.q[k] = ch.x;
                G.tw[k] = p.z;
                G.sd[k] = p.w;
                G.fb[k] = fpq.x;
                G.fp[k] = fpq.y;
            }
            unsigned long long bal[UNR];
            uint32_t item[UNR];
            relax_group<SWEEP>(A, G, bal, item, vol_cnt, n_relax);
            stage_append(S, bal, item);
        }
    }
}

template <bool SWEEP, int B, bool UQ>
__global__ __launch_bounds__(B) void chunk_kernel(TravArgs A)
{
    __shared__ uint32_t s_stage[B / 64][SCAP];
    TStage S{s_stage[threadIdx.x >> 6], 0u, A.next, &A.cnt[CNT_FRONT + (A.round + 1u) % 3u]};
    unsigned long long n_edges = 0, n_relax = 0;
    chunk_phase<SWEEP, B, UQ>(A, S, n_edges, n_relax);
    stage_flush_block<SCAP, B / 64>(S);
    unsigned long long v[3] = {n_relax & 0xFFFFFFFFull, n_relax >> 32, n_edges};
    const int slot[3] = {ST_RELAX, ST_ATTEMPTS, ST_CHUNK_EDGES};
    block_stats<B / 64>(A.stats, v, slot);
}

// Rounds of one query set in a single cooperative launch: push phase, grid
// barrier, chunk phase, grid barrier, until the frontier holds at most
// `stop_below` entries (small frontiers go to the one-workgroup kernel) or
// `max_rounds` rounds ran.  Every block reads the frontier size from the same
// word after a barrier, so all leave together.  On exit the round, the queue
// holding the frontier and the number of rounds run are left in cnt as the
// one-workgroup kernel leaves them; CNT_ABORT is raised if a barrier wait gave
// up (the launch then ends early and the host reports an error).  Round
// stamps are stamp_val, stamp_val + 1, ... (the host keeps them clear of
// wrap-around).
template <bool SWEEP>
__global__ __launch_bounds__(TB) void persist_kernel(TravArgs A, uint32_t which0, uint32_t *q0, uint32_t *q1,
                                                     uint32_t stop_below, uint32_t max_rounds, uint32_t dense_div,
                                                     uint32_t *bar, uint32_t spin_limit)
{
    __shared__ uint32_t s_stage[TB / 64][SCAP];
    __shared__ uint32_t s_F;
    unsigned long long n_edges = 0, n_relax = 0, n_items = 0, n_cedges = 0;
    const uint32_t r0 = A.round;
    uint32_t r = r0;
    for (;;) {
        if (threadIdx.x == 0)
            s_F = grid_aborted(bar) ? 0u
                                    : __hip_atomic_load(&A.cnt[CNT_FRONT + r % 3u], __ATOMIC_ACQUIRE,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t F = s_F;
        __syncthreads();
        if (F <= stop_below || r - r0 >= max_rounds) break;
        const uint32_t odd = (which0 ^ (r - r0)) & 1u;
        TravArgs B = A;
        B.round = r;
        B.stamp_val = A.stamp_val + (r - r0);
        B.front_stamp = B.stamp_val - 1u;
        B.cur = odd ? q1 : q0;
        B.next = odd ? q0 : q1;
        B.dense = (A.nq == 1 && dense_div && (uint64_t)F * dense_div >= A.n) ? 1u : 0u;
        TStage S{s_stage[threadIdx.x >> 6], 0u, B.next, &A.cnt[CNT_FRONT + (r + 1u) % 3u]};
        push_phase<SWEEP, TB, false>(B, F, S, n_edges, n_relax, n_items);
        stage_flush_block<SCAP, TB / 64>(S);
        grid_barrier(bar, spin_limit);
        chunk_phase<SWEEP, TB, false>(B, S, n_cedges, n_relax);
        stage_flush_block<SCAP, TB / 64>(S);
        grid_barrier(bar, spin_limit);
        ++r;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.cnt[CNT_TAIL_ROUND] = r;
        A.cnt[CNT_TAIL_WHICH] = (which0 ^ (r - r0)) & 1u;
        A.cnt[CNT_TAIL_ROUNDS] = r - r0;
        A.cnt[CNT_ABORT] = grid_aborted(bar) ? 1u : 0u;
    }
    unsigned long long v[5] = {n_relax & 0xFFFFFFFFull, n_relax >> 32, n_items, n_edges, n_cedges};
    const int slot[5] = {ST_RELAX, ST_ATTEMPTS, ST_ITEMS, ST_EDGES, ST_CHUNK_EDGES};
    block_stats<TB / 64>(A.stats, v, slot);
}

// Small-frontier rounds in one workgroup.  While the frontier holds at most
// `limit` entries, one 1024-thread workgroup runs round after round with a
// workgroup barrier in between, keeping the frontier count in LDS; it stops
// when the frontier is empty, outgrows the limit, or after `max_rounds`, and
// leaves the round number, the queue holding the frontier and its size for
// the host.  One workgroup never waits on another, so nothing here depends
// on which workgroups are resident.  The tail's arrival is read with an
// agent-scope atomic load: within one launch a cached copy may predate the
// improvement that put the vertex in the frontier.
constexpr int TT = 1024;

template <bool SWEEP>
__global__ __launch_bounds__(TT) void tail_kernel(TravArgs A, uint32_t which0, uint32_t limit,
                                                  uint32_t vol_limit, uint32_t max_rounds, uint32_t *q0,
                                                  uint32_t *q1)
{
    __shared__ uint32_t s_pref[TT + 1];
    __shared__ uint32_t s_lo[TT];
    __shared__ uint32_t s_q[TT];
    __shared__ uint32_t s_tw[TT];
    __shared__ uint32_t s_sd[TT];
    __shared__ uint2 s_fp[TT];
    __shared__ uint32_t s_wsum[TT / 64];
    __shared__ uint32_t s_next;
    __shared__ uint32_t s_F;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    __shared__ uint32_t s_step, s_sdep;
    uint32_t r = A.round;
    uint32_t which = which0;
    if (tid == 0) {
        s_F = A.cnt[CNT_FRONT + r % 3u];
        s_step = A.cnt[CNT_STEP];
        s_sdep = A.qp[0].w;
    }
    __syncthreads();
    unsigned long long n_edges = 0, n_relax = 0, n_items = 0;
    uint32_t rounds = 0;
    uint32_t dummy_vol = 0;
    for (;;) {
        if (SWEEP && s_F == 0 && s_step < A.nsteps && rounds < max_rounds) {
            // next departure time of the sweep: the source leaves at s
            if (tid == 0) {
                const uint32_t sd = A.steps[s_step];
                const uint32_t src = A.qp[0].x;
                ((uint4 *)A.qp)[0].w = sd;
                // no relaxation runs now; the stamp marks the coming round's frontier
                A.av[src] = av_word(min(arrival_of(A.av, src), sd), A.stamp_val + rounds - 1u);
                (which ? q1 : q0)[0] = src;
                s_sdep = sd;
                s_step += 1;
                s_F = 1;
                A.cnt[CNT_FRONT + r % 3u] = 1u;
            }
            __syncthreads();
        }
        const uint32_t F = s_F;
        if (F == 0 || F > limit || rounds >= max_rounds) break;
        if ((uint64_t)F * A.max_deg > vol_limit) {
            // out-degree volume of the frontier bounds this round's edge work;
            // beyond vol_limit the multi-block kernels are faster (no need to
            // count when F entries of the largest out-degree stay within it)
            uint32_t vol = 0;
            const uint32_t *cq = which ? q1 : q0;
            for (uint32_t i = tid; i < F; i += TT) {
                const uint32_t u = cq[i] % A.n;
                vol += A.off[u + 1] - A.off[u];
            }
            for (int o = 32; o > 0; o >>= 1) vol += __shfl_xor(vol, o);
            if (lane == 0) s_wsum[w] = vol;
            __syncthreads();
            uint32_t tot = 0;
            for (int w2 = 0; w2 < TT / 64; ++w2) tot += s_wsum[w2];
            __syncthreads();
            if (tot > vol_limit) break;
        }
        TravArgs B = A;
        B.cur = which ? q1 : q0;
        B.next = which ? q0 : q1;
        B.round = r;
        B.stamp_val = A.stamp_val + rounds;
        B.track_volume = 0;
        if (A.snap) {
            // level-synchronous rounds: arrivals of the frontier before any
            // relaxation of this round
            for (uint32_t i = tid; i < F; i += TT)
                A.snap[i] = __hip_atomic_load((const uint32_t *)A.av + 2 * (size_t)B.cur[i] + 1, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tid == 0) s_next = 0;
        __syncthreads();
        for (uint32_t base = 0; base < F; base += TT) {
            const uint32_t i = base + tid;
            uint32_t lo = 0, len = 0, q = 0, tw = 0, sd = 0;
            uint2 fpq = make_uint2(0u, 0u);
            if (i < F) {
                ++n_items;
                const uint32_t item = B.cur[i];
                q = item / A.n;
                const uint32_t u = item - q * A.n;
                const uint4 p = A.qp[q];
                fpq = A.fpar[q];
                tw = p.z;
                sd = SWEEP ? s_sdep : p.w;
                const size_t su = (size_t)q * A.n + u;
                const uint32_t ru = A.snap ? A.snap[i]
                                           : __hip_atomic_load((const uint32_t *)A.av + 2 * su + 1, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t b = A.off[u], e = A.off[u + 1];
                const uint32_t old = A.done[su];
                lo = lower_bound_u32(A.tt, b, old == INF ? e : min(old, e), departure_key(ru, fpq.y, u, p.x));
                uint32_t end = old;
                if (old == INF) end = tw > A.max_t ? e : lower_bound_u32(A.tt, lo, e, tw);
                if (lo < end) {
                    len = end - lo;
                    A.done[su] = lo;
                }
            }
            uint32_t x = len;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane == 63) s_wsum[w] = x;
            s_lo[tid] = lo;
            s_q[tid] = q;
            s_tw[tid] = tw;
            s_sd[tid] = sd;
            s_fp[tid] = fpq;
            __syncthreads();
            uint32_t woff = 0, total = 0;
            for (int w2 = 0; w2 < TT / 64; ++w2) {
                if (w2 < w) woff += s_wsum[w2];
                total += s_wsum[w2];
            }
            s_pref[tid] = woff + x - len;
            if (tid == 0) s_pref[TT] = total;
            __syncthreads();
            if (tid == 0) n_edges += total;
            for (uint32_t j0 = 0; j0 < total; j0 += TT * UNR) {
                EdgeGroup G;
#pragma unroll
                for (int k = 0; k < UNR; ++k) {
                    const uint32_t j = j0 + k * TT + tid;
                    G.ok[k] = j < total;
                    int lo_k = 0, hi_k = TT;
                    while (hi_k - lo_k > 1) {
                        const int mid = (lo_k + hi_k) >> 1;
                        if (s_pref[mid] <= j)
                            lo_k = mid;
                        else
                            hi_k = mid;
                    }
                    const uint32_t e = G.ok[k] ? s_lo[lo_k] + (j - s_pref[lo_k]) : 0u;
                    const uint2 dv = A.da[e];
                    G.v[k] = dv.x;
                    G.a[k] = dv.y;
                    G.q[k] = s_q[lo_k];
                    G.tw[k] = s_tw[lo_k];
                    G.sd[k] = s_sd[lo_k];
                    const uint2 f = s_fp[lo_k];
                    G.fb[k] = f.x;
                    G.fp[k] = f.y;
                }
                unsigned long long bal[UNR];
                uint32_t item[UNR];
                relax_group<SWEEP>(B, G, bal, item, &dummy_vol, n_relax);
                lds_append(B.next, &s_next, bal, item);
            }
            __syncthreads();
        }
        ++r;
        ++rounds;
        which ^= 1u;
        if (tid == 0) {
            s_F = s_next;
            A.cnt[CNT_FRONT + r % 3u] = s_next;
        }
        __syncthreads();
    }
    if (tid == 0) {
        A.cnt[CNT_TAIL_ROUND] = r;
        A.cnt[CNT_TAIL_WHICH] = which;
        A.cnt[CNT_TAIL_ROUNDS] = rounds;
        A.cnt[CNT_STEP] = s_step;
        // the multi-block kernels of round r expect these zeroed
        A.cnt[CNT_CHUNK + r % 3u] = 0u;
        A.cnt[CNT_FRONT + (r + 1u) % 3u] = 0u;
        A.cnt[CNT_PULLVOL + (r + 1u) % 3u] = 0u;
    }
    unsigned long long v[4] = {n_relax & 0xFFFFFFFFull, n_relax >> 32, n_items, n_edges};
    const int slot[4] = {ST_RELAX, ST_ATTEMPTS, ST_TAIL_ITEMS, ST_TAIL_EDGES};
    block_stats<TT / 64>(A.stats, v, slot);
}

// Dense pull round: every vertex v of every query looks at its in-edges in
// ascending arrival (only those arriving before its current value and within
// the window); the first whose tail has arrived by its departure is the new
// minimum.  One writer per vertex, no atomics.
template <bool SWEEP>
__global__ __launch_bounds__(TB) void pull_kernel(TravArgs A)
{
    __shared__ uint32_t s_stage[TB / 64][SCAP];
    TStage S{s_stage[threadIdx.x >> 6], 0u, A.next, &A.cnt[CNT_FRONT + (A.round + 1u) % 3u]};
    uint32_t *vol_cnt = &A.cnt[CNT_PULLVOL + (A.round + 1u) % 3u];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.cnt[CNT_FRONT + (A.round + 2u) % 3u] = 0u;
        A.cnt[CNT_PULLVOL + (A.round + 2u) % 3u] = 0u;
        A.cnt[CNT_CHUNK + (A.round + 1u) % 3u] = 0u;
        A.cnt[CNT_CHUNK + A.round % 3u] = 0u;
    }
    unsigned long long n_edges = 0, n_verts = 0, n_relax = 0;
    const uint64_t total = (uint64_t)A.nq * A.n;
    const uint64_t stride = (uint64_t)gridDim.x * TB;
    const uint64_t rounds = (total + stride - 1) / stride;
    for (uint64_t it = 0; it < rounds; ++it) {
        const uint64_t idx = it * stride + (uint64_t)blockIdx.x * TB + threadIdx.x;
        bool push = false;
        uint32_t item = 0, v = 0;
        if (idx < total) {
            const uint32_t q = (uint32_t)(idx / A.n);
            v = (uint32_t)(idx - (uint64_t)q * A.n);
            const uint4 p = A.qp[q];
            const uint32_t strict = fp_strict(A.fpar[q].y);
            if (v != p.x) {
                ++n_verts;
                const size_t sv = (size_t)q * A.n + v;
                const uint32_t rv = arrival_of(A.av, sv);
                const uint32_t lim = min(rv, p.z + 1u);
                const uint32_t b = A.off_in[v], e = A.off_in[v + 1];
                const uint32_t ub = lower_bound_u32(A.a_in, b, e, lim);
                for (uint32_t k = b; k < ub; ++k) {
                    ++n_edges;
                    const uint2 st = A.st_in[k];
                    const uint32_t ru = arrival_of(A.av, (size_t)q * A.n + st.x);
                    if (st.y >= p.y && (strict && st.x != p.x ? ru < st.y : ru <= st.y)) {
                        const uint32_t a = A.a_in[k];
                        // single writer; the stamp gives frontier membership for dense rounds
                        A.av[sv] = av_word(a, A.stamp_val);
                        ++n_relax;
                        if (SWEEP && p.w != INF) {
                            A.fa[sv] = min(A.fa[sv], a - p.w);
                            A.l1[sv] = max(A.l1[sv], p.w + 1u);
                        }
                        push = true;
                        item = (uint32_t)sv;
                        break;
                    }
                }
            }
        }
        if (A.track_volume) {
            uint32_t vol = push ? A.off[v + 1] - A.off[v] : 0u;
            for (int o = 32; o > 0; o >>= 1) vol += __shfl_xor(vol, o);
            if ((threadIdx.x & 63) == 0 && vol) atomicAdd(vol_cnt, vol);
        }
        const unsigned long long bal[1] = {__ballot(push)};
        const uint32_t items[1] = {item};
        stage_append(S, bal, items);
    }
    stage_flush_block<SCAP, TB / 64>(S);
    unsigned long long vals[3] = {n_edges, n_verts, n_relax};
    const int slot[3] = {ST_PULL_EDGES, ST_PULL_VERTS, ST_RELAX};
    block_stats<TB / 64>(A.stats, vals, slot);
}

// Start the next departure step of a sweep from the host side of the loop
// (the one-workgroup kernel does the same by itself).
__global__ void step_kernel(TravArgs A, uint32_t *queue)
{
    const uint32_t idx = A.cnt[CNT_STEP];
    const uint32_t sd = A.steps[idx];
    const uint32_t src = A.qp[0].x;
    ((uint4 *)A.qp)[0].w = sd;
    A.av[src] = av_word(min(arrival_of(A.av, src), sd), A.front_stamp);
    queue[0] = src;
    A.cnt[CNT_FRONT + A.round % 3u] = 1u;
    A.cnt[CNT_STEP] = idx + 1u;
}

// Query start: parameters, source arrival, first frontier, counters.
__global__ void init_queries_kernel(TravArgs A, const uint4 *__restrict__ host_qp, uint32_t nq,
                                    uint32_t src_arrival_from_w)
{
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        const uint4 p = host_qp[q];
        ((uint4 *)A.qp)[q] = p;
        uint2 fp = filter_params(p.y, p.z, A.max_a, A.fbits);
        fp.y |= A.strict << 16;
        A.fpar[q] = fp;
        const size_t ss = (size_t)q * A.n + p.x;
        // the stamp lets a dense first round find the source
        A.av[ss] = av_word(src_arrival_from_w ? p.w : p.y, A.front_stamp);
        A.next[q] = (uint32_t)ss;  // `next` names the buffer read by the first round here
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.cnt[CNT_FRONT + A.round % 3u] = nq;
        A.cnt[CNT_FRONT + (A.round + 1u) % 3u] = 0u;
        A.cnt[CNT_CHUNK + A.round % 3u] = 0u;
        A.cnt[CNT_PULLVOL + A.round % 3u] = 0u;
        A.cnt[CNT_PULLVOL + (A.round + 1u) % 3u] = 0u;
        A.cnt[CNT_STEP] = src_arrival_from_w ? 1u : 0u;  // a sweep starts at its first step
    }
}

// Results back in caller ids: out[v] for caller vertex v from internal slot
// perm[v].  kind 0 copies arrivals, 1 turns latest departure + 1 into latest
// departure, 2 copies fastest durations, 3 copies hop counts (kept in the
// fastest array); the source gets its convention.
__global__ void finalize_sweep_kernel(uint32_t *out, const unsigned long long *__restrict__ av,
                                      const uint32_t *__restrict__ l1,
                                      const uint32_t *__restrict__ fa, const uint32_t *__restrict__ perm, uint32_t n,
                                      int kind, uint32_t src, uint32_t tw)
{
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t x = perm[v];
        uint32_t r;
        if (kind == 0)
            r = arrival_of(av, x);
        else if (v == src)
            r = kind == 1 ? tw : 0u;  // hops of the source: 0
        else if (kind == 1)
            r = l1[x] ? l1[x] - 1u : INF;
        else
            r = fa[x];
        out[v] = r;
    }
}

// Level-synchronous rounds: the frontier's arrivals before the round starts.
__global__ void snapshot_kernel(TravArgs A)
{
    const uint32_t F = A.cnt[CNT_FRONT + A.round % 3u];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < F; i += gridDim.x * blockDim.x)
        A.snap[i] = arrival_of(A.av, A.cur[i]);
}

// Last edge of an earliest-arrival path into every vertex, from finished
// arrivals.  The in-edges of x arriving exactly at its arrival are one block
// of the in-index (ordered by arrival, then departure), found by binary
// search; scanning it from the latest departure down, the first edge whose
// tail had arrived by its departure fixes the departure, and among the edges
// leaving at that time the smallest caller tail id is taken.  Results are in
// caller ids; INF for the source and unreached vertices.
__global__ void predecessor_kernel(const unsigned long long *__restrict__ av, const uint32_t *__restrict__ off_in,
                                   const uint32_t *__restrict__ a_in, const uint2 *__restrict__ st_in,
                                   const uint32_t *__restrict__ inv, uint32_t n, uint32_t src, uint32_t ta,
                                   uint32_t *pred_tail, uint32_t *pred_dep)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
        const uint32_t a = arrival_of(av, x);
        uint32_t bt = INF, bc = INF;
        if (a != INF && x != src) {
            const uint32_t b = off_in[x], e = off_in[x + 1];
            const uint32_t lo = lower_bound_u32(a_in, b, e, a);
            const uint32_t hi = lower_bound_u32(a_in, lo, e, a + 1u);  // a <= TMAX: no wrap
            for (uint32_t k = hi; k > lo; --k) {
                const uint2 st = st_in[k - 1];
                if (bt != INF && st.y < bt) break;
                if (st.y >= ta && arrival_of(av, st.x) <= st.y) {
                    const uint32_t cu = inv[st.x];
                    if (bt == INF) {
                        bt = st.y;
                        bc = cu;
                    } else {
                        bc = min(bc, cu);
                    }
                }
            }
        }
        const uint32_t c = inv[x];
        pred_tail[c] = bc;
        pred_dep[c] = bt;
    }
}

// Grouped latest-departure / fastest sweep: every slot but `from` takes slot
// `from`'s arrivals (with their stamps) and claims, the warm start of the
// next group of departure times.
__global__ void warm_slots_kernel(unsigned long long *av, uint32_t *done, uint32_t n, uint32_t nslots, uint32_t from)
{
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const unsigned long long w = av[(size_t)from * n + v];
        const uint32_t d = done[(size_t)from * n + v];
        for (uint32_t j = 0; j < nslots; ++j) {
            if (j == from) continue;
            av[(size_t)j * n + v] = w;
            done[(size_t)j * n + v] = d;
        }
    }
}

// After a group: slot j holds the earliest arrivals for the source leaving
// at dep[j], so F[v] = min(F[v], EA_j[v] - dep[j]) and, where v is reached,
// L1[v] = max(L1[v], dep[j] + 1) (latest departure + 1, 0 = none).
__global__ void sweep_reduce_kernel(const unsigned long long *__restrict__ av, const uint32_t *__restrict__ dep,
                                    uint32_t n, uint32_t nslots, uint32_t *fa, uint32_t *l1)
{
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        uint32_t f = fa[v], l = l1[v];
        for (uint32_t j = 0; j < nslots; ++j) {
            const uint32_t a = arrival_of(av, (size_t)j * n + v);
            if (a != INF) {
                f = min(f, a - dep[j]);
                l = max(l, dep[j] + 1u);
            }
        }
        fa[v] = f;
        l1[v] = l;
    }
}

// Time-reversed edge list from the in-index: in-edge e of head x, (u, x, t,
// a), becomes (x, u, TMAX - a, a - t), all in caller ids.  The head is the
// last x with off_in[x] <= e.
__global__ void reverse_edges_kernel(const uint32_t *__restrict__ off_in, const uint32_t *__restrict__ a_in,
                                     const uint2 *__restrict__ st_in, const uint32_t *__restrict__ inv, uint32_t n,
                                     uint64_t m, uint32_t *src, uint32_t *dst, uint32_t *t, uint32_t *lam)
{
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = n;
        while (lo < hi) {
            const uint32_t mid = lo + ((hi - lo + 1) >> 1);
            if (off_in[mid] <= e)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint2 st = st_in[e];
        const uint32_t a = a_in[e];
        src[e] = inv[lo];
        dst[e] = inv[st.x];
        t[e] = TMAX - a;
        lam[e] = a - st.y;
    }
}

// Arrivals on the time-reversed graph back to departure times.
__global__ void flip_times_kernel(uint32_t *out, uint32_t n)
{
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (out[v] != INF) out[v] = TMAX - out[v];
}

__global__ void count_traversed_kernel(const uint32_t *__restrict__ a_in, const uint2 *__restrict__ st_in,
                                       uint64_t m, const uint32_t *__restrict__ ea, const uint32_t *__restrict__ inv,
                                       uint32_t ta, uint32_t tw, unsigned long long *out)
{
    __shared__ unsigned long long s_c[4];
    unsigned long long c = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint2 st = st_in[e];
        const uint32_t r = ea[inv[st.x]];  // ea is in caller ids
        if (r != INF && st.y >= max(r, ta) && a_in[e] <= tw) ++c;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
    __syncthreads();
    // one partial sum per shard, out[blockIdx % ST_SHARDS] (256 threads)
    if (threadIdx.x == 0) {
        const unsigned long long t = s_c[0] + s_c[1] + s_c[2] + s_c[3];
        if (t) atomicAdd(&out[blockIdx.x % ST_SHARDS], t);
    }
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t count, uint32_t value)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

int grid_cap(uint64_t work, int per_block, int cap)
{
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (uint64_t)cap) g = cap;
    return (int)g;
}

#include "binned.h"

int fill(hipStream_t st, uint32_t *p, uint64_t count, uint32_t value)
{
    if (!count) return KAIROS_OK;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_cap(count, 256 * 4, 8192)), dim3(256), 0, st, p,
                       count, value);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

__global__ void fill_u64_kernel(unsigned long long *p, uint64_t count, unsigned long long value)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void clear_stamps_kernel(unsigned long long *p, uint64_t count)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] &= 0xFFFFFFFF00000000ull;
}

// Every arrival unreached (INF), every stamp 0 (older than any round).
int fill_arrivals(hipStream_t st, unsigned long long *av, uint64_t count)
{
    if (!count) return KAIROS_OK;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_cap(count, 256 * 4, 8192)), dim3(256), 0, st, av, count,
                       (unsigned long long)INF << 32);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

// Stamps back to 0 with the arrivals kept (the stamp counter wrapped).
int clear_stamps(hipStream_t st, unsigned long long *av, uint64_t count)
{
    if (!count) return KAIROS_OK;
    hipLaunchKernelGGL(clear_stamps_kernel, dim3(grid_cap(count, 256 * 4, 8192)), dim3(256), 0, st, av, count);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

// Arrival codes of `nq` query regions: every bit set (no bound yet).  Done
// whether or not codes are switched on, so switching them on between queries
// never exposes codes of an earlier query.
int fill_filter(kairos_graph *g, hipStream_t st, uint8_t *filt, uint64_t nq)
{
    return fill(st, (uint32_t *)filt, nq * filt_stride(g->n) / 4, 0xFFFFFFFFu);
}

// About 32 edges per thread of a 256-thread block: 256 entries on the
// scale-20/24 R-MAT graphs (32 out-edges per vertex), 34 on the bursty graph
// (240).  Measured on the bursty graph (first 16 queries) 3.03 -> 2.88 ms
// when small frontiers spread; spreading on the R-MAT graphs cost 2-7%.
uint32_t min_entries_per_block(const kairos_graph *g)
{
    const uint64_t avg = std::max<uint64_t>(1, g->m / std::max<uint32_t>(g->n_live, 1));
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(256, 256 * 32 / avg));
}

TravArgs make_args(kairos_graph *g, Slot *s, uint32_t nq)
{
    TravArgs A{};
    A.off = g->off_out;
    A.tt = g->t_out;
    A.da = g->da_out;
    A.off_in = g->off_in;
    A.a_in = g->a_in;
    A.st_in = g->st_in;
    A.n_live = g->n_live;
    A.max_deg = g->max_out_degree;
    A.min_per = min_entries_per_block(g);
    A.qp = s->qp;
    A.n = g->n;
    A.av = s->av;
    A.done = s->done;
    A.fa = s->fa;
    A.l1 = s->l1;
    A.cnt = s->cnt;
    A.chunks = s->chunks;
    A.chunk_cap = (uint32_t)std::min<uint64_t>(s->chunk_cap, 0xFFFFFFF0u);
    A.stats = g->prof.on && !s->fixed ? s->stats : nullptr;
    A.split = std::max<uint32_t>(g->tuning.split, 1);
    A.chunk = std::max<uint32_t>(g->tuning.chunk, 1);
    A.nq = nq;
    A.track_volume = g->tuning.pull_alpha ? 1u : 0u;
    A.max_t = g->max_t;
    // skipping the codes is always valid: a query started with codes on
    // finds them again, possibly looser, when they are switched back on
    A.filt = g->tuning.arrival_filter ? s->filt : nullptr;
    A.fpar = s->fpar;
    A.fbits = g->tuning.arrival_filter;
    A.fstride = (uint32_t)filt_stride(g->n);
    A.max_a = g->max_a;
    A.dedupe = g->tuning.run_dedupe;
    return A;
}

uint32_t next_stamp(Slot *s, int *rc)
{
    if (s->stamp_next >= 0xFFFFF000u) {
        *rc = clear_stamps(s->stream, s->av, (uint64_t)s->qcap * s->n);
        s->stamp_next = 2;
    }
    return s->stamp_next++;
}

// Rounds with more than `stop` frontier entries in one cooperative launch
// (persist_kernel).  Updates the round, the queue holding the frontier and
// its size from what the kernel left.  KAIROS_ERR_BUSY: the runtime refused
// the launch and nothing ran.
template <bool SWEEP>
int run_persistent(kairos_graph *g, Slot *s, TravArgs A, uint32_t *r, int *which, uint32_t *F, uint32_t stop)
{
    hipStream_t st = s->stream;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, persist_kernel<SWEEP>, TB, 0) != hipSuccess || occ < 1) {
        (void)hipGetLastError();
        return KAIROS_ERR_BUSY;
    }
    constexpr uint32_t kMaxRounds = 1u << 16;  // per launch; the host launches again if needed
    if (s->stamp_next >= 0xFFFFF000u - kMaxRounds) {
        int rc = clear_stamps(st, s->av, (uint64_t)s->qcap * s->n);
        if (rc) return rc;
        s->stamp_next = 2;
    }
    KAIROS_HIP(hipMemsetAsync(s->bar, 0, BAR_WORDS * 4, st));
    A.round = *r;
    A.stamp_val = s->stamp_next;
    uint32_t which0 = (uint32_t)*which, max_rounds = kMaxRounds, dense_div = g->tuning.dense_frontier;
    uint32_t spin_limit = 1u << 24;  // about 4 s of polling: far beyond one phase
    uint32_t *q0 = s->queue[0], *q1 = s->queue[1], *bar = s->bar;
    void *args[] = {&A, &which0, &q0, &q1, &stop, &max_rounds, &dense_div, &bar, &spin_limit};
    const int grid = g->num_cus * std::min(occ, 4);
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    const hipError_t e = hipLaunchCooperativeKernel((const void *)persist_kernel<SWEEP>, dim3(grid), dim3(TB), args, 0, st);
    prof_end(g, st, KAIROS_K_PUSH, ev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return KAIROS_ERR_BUSY;
    }
    KAIROS_HIP(hipMemcpyAsync(s->h_pin, s->cnt, CNT_WORDS * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    KAIROS_HIP(hipStreamSynchronize(st));
    if (s->h_pin[CNT_ABORT]) return KAIROS_ERR_DEVICE;
    const uint32_t rounds = s->h_pin[CNT_TAIL_ROUNDS];
    *r = s->h_pin[CNT_TAIL_ROUND];
    *which = (int)s->h_pin[CNT_TAIL_WHICH];
    *F = s->h_pin[CNT_FRONT + *r % 3u];
    s->stamp_next += rounds;
    if (g->prof.on) {
        std::lock_guard<std::mutex> lk(g->prof.mu);
        g->prof.rounds += rounds;
    }
    return KAIROS_OK;
}

// Runs frontier rounds until the frontier is empty.  The first round's
// frontier (nq items) is already in s->queue[0] and the counters set for
// round `r0`.
template <bool SWEEP>
int run_rounds(kairos_graph *g, Slot *s, TravArgs A, uint32_t first_front, uint32_t *round_io)
{
    hipStream_t st = s->stream;
    const kairos_tuning &tu = g->tuning;
    const int spec_grid = std::max(1, g->num_cus * 8);
    const int chunk_grid = std::max(1, g->num_cus * 4);
    const uint32_t R = std::max<uint32_t>(1, tu.rounds_per_sync);
    uint32_t r = *round_io;
    uint32_t F = first_front;
    uint64_t vol = 0;
    bool pulling = false;
    int which = 0;  // queue holding the current frontier
    const uint64_t total_v = (uint64_t)A.nq * g->n;
    int rc = KAIROS_OK;
    uint32_t step = (SWEEP && A.steps) ? 1u : 0u;  // host mirror of CNT_STEP
    // level-synchronous rounds take a snapshot between rounds, so they run
    // one push and one chunk launch per round (no pull, no dense walk, no
    // rounds inside one cooperative launch)
    const bool levels = A.snap != nullptr;
    bool persist = tu.single_persistent != 0 && !levels;
    const uint32_t stop = tu.tail_limit;  // persistent launches leave small frontiers to the tail kernel
    for (;;) {
        if (F == 0) {
            if (!SWEEP || !A.steps || step >= A.nsteps) break;
            A.round = r;
            A.front_stamp = s->stamp_next - 1u;
            hipLaunchKernelGGL(step_kernel, dim3(1), dim3(1), 0, st, A, s->queue[which]);
            KAIROS_HIP(hipGetLastError());
            F = 1;
            ++step;
        }
        if (tu.tail_limit && F <= tu.tail_limit && !pulling) {
            constexpr uint32_t kMaxTail = 4096;
            if (s->stamp_next >= 0xFFFFF000u - kMaxTail) {
                if ((rc = clear_stamps(st, s->av, (uint64_t)s->qcap * s->n))) return rc;
                s->stamp_next = 2;
            }
            A.round = r;
            A.stamp_val = s->stamp_next;
            hipEvent_t ev;
            prof_begin(g, st, &ev);
            hipLaunchKernelGGL(tail_kernel<SWEEP>, dim3(1), dim3(TT), 0, st, A, (uint32_t)which, tu.tail_limit,
                               tu.tail_limit * 32u, kMaxTail, s->queue[0], s->queue[1]);
            prof_end(g, st, KAIROS_K_TAIL, ev);
            KAIROS_HIP(hipGetLastError());
            KAIROS_HIP(hipMemcpyAsync(s->h_pin, s->cnt, CNT_WORDS * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            KAIROS_HIP(hipStreamSynchronize(st));
            const uint32_t done_rounds = s->h_pin[CNT_TAIL_ROUNDS];
            r = s->h_pin[CNT_TAIL_ROUND];
            which = (int)s->h_pin[CNT_TAIL_WHICH];
            s->stamp_next += done_rounds;
            F = s->h_pin[CNT_FRONT + r % 3u];
            step = s->h_pin[CNT_STEP];
            if (g->prof.on) {
                std::lock_guard<std::mutex> lk(g->prof.mu);
                g->prof.rounds += done_rounds;
            }
            if (F == 0) continue;
            if (done_rounds > 0 && F <= tu.tail_limit) continue;  // stopped at max_rounds
            vol = 0;
        }
        if (persist && !tu.pull_alpha && F > stop) {
            int prc = run_persistent<SWEEP>(g, s, A, &r, &which, &F, stop);
            if (prc == KAIROS_OK) continue;
            if (prc != KAIROS_ERR_BUSY) return prc;
            persist = false;  // launch refused: per-round launches from here on
        }
        // a large round of a single earliest-arrival query: destination-
        // binned, then back to the host for the next decision
        if (!SWEEP && !levels && !pulling && A.nq == 1 && !A.filt && !s->fixed && !tu.pull_alpha && tu.binned &&
            F >= tu.binned && binned_supported(g)) {
            if ((rc = binned_alloc(g, s))) return rc;
            A.round = r;
            A.stamp_val = next_stamp(s, &rc);
            if (rc) return rc;
            A.cur = s->queue[which];
            A.next = s->queue[which ^ 1];
            A.dense = 0;
            if ((rc = binned_round(g, s, A, F))) return rc;
            ++r;
            which ^= 1;
            KAIROS_HIP(hipMemcpyAsync(s->h_pin, s->cnt, CNT_WORDS * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            KAIROS_HIP(hipStreamSynchronize(st));
            F = s->h_pin[CNT_FRONT + r % 3u];
            if (g->prof.on) {
                std::lock_guard<std::mutex> lk(g->prof.mu);
                g->prof.rounds += 1;
            }
            if (which == 1 && F > 0) {
                std::swap(s->queue[0], s->queue[1]);
                which = 0;
            }
            continue;
        }
        for (uint32_t k = 0; k < R; ++k) {
            A.round = r;
            A.stamp_val = next_stamp(s, &rc);
            if (rc) return rc;
            A.cur = s->queue[which];
            A.next = s->queue[which ^ 1];
            hipEvent_t ev;
            if (k == 0 && tu.pull_alpha && !levels) {
                // direction choice from the last read-back
                if (!pulling && vol > (uint64_t)g->m * A.nq / tu.pull_alpha) pulling = true;
                else if (pulling && (uint64_t)F * std::max<uint32_t>(tu.pull_beta, 1) < total_v) pulling = false;
            }
            if (pulling && k == 0) {
                prof_begin(g, st, &ev);
                hipLaunchKernelGGL(pull_kernel<SWEEP>, dim3(grid_cap(total_v, TB * 4, g->num_cus * 16)),
                                   dim3(TB), 0, st, A);
                prof_end(g, st, KAIROS_K_PULL, ev);
            } else {
                // dense walk when the frontier is a large share of the vertices
                A.dense = (A.nq == 1 && tu.dense_frontier && k == 0 && !levels &&
                           (uint64_t)F * tu.dense_frontier >= g->n) ? 1u : 0u;
                A.front_stamp = A.stamp_val - 1u;
                // workgroup size from the tuning: 512 threads take half as
                // many blocks for the same number of threads
                const bool wide = tu.block == 512;
                const int bs = wide ? 512 : TB;
                const int sg = wide ? std::max(1, spec_grid / 2) : spec_grid;
                const int cg = wide ? std::max(1, chunk_grid / 2) : chunk_grid;
                // one query without arrival codes: the push kernel relaxes
                // through the query-uniform path, whose lighter register use
                // would let twice the blocks share a CU; half the grid keeps
                // the number in flight where the general kernel has it (more
                // of them only contend for the same memory)
                const bool up = A.nq == 1 && A.filt == nullptr;
                const int sgp = up ? std::max(1, sg / 2) : sg;
                const int pg = A.dense ? grid_cap(g->n, bs, sgp) : (k == 0 ? grid_cap(F, bs, sgp) : sgp);
                if (levels)
                    hipLaunchKernelGGL(snapshot_kernel, dim3(k == 0 ? grid_cap(F, 256, spec_grid) : chunk_grid),
                                       dim3(256), 0, st, A);
                prof_begin(g, st, &ev);
                if (wide && up)
                    hipLaunchKernelGGL((push_kernel<SWEEP, 512, true>), dim3(pg), dim3(512), 0, st, A);
                else if (wide)
                    hipLaunchKernelGGL((push_kernel<SWEEP, 512, false>), dim3(pg), dim3(512), 0, st, A);
                else if (up)
                    hipLaunchKernelGGL((push_kernel<SWEEP, TB, true>), dim3(pg), dim3(TB), 0, st, A);
                else
                    hipLaunchKernelGGL((push_kernel<SWEEP, TB, false>), dim3(pg), dim3(TB), 0, st, A);
                prof_end(g, st, KAIROS_K_PUSH, ev);
                prof_begin(g, st, &ev);
                // without arrival codes the chunk kernel takes the
                // query-uniform relaxation (one query per chunk)
                const bool uq = A.filt == nullptr;
                if (wide && uq)
                    hipLaunchKernelGGL((chunk_kernel<SWEEP, 512, true>), dim3(cg), dim3(512), 0, st, A);
                else if (wide)
                    hipLaunchKernelGGL((chunk_kernel<SWEEP, 512, false>), dim3(cg), dim3(512), 0, st, A);
                else if (uq)
                    hipLaunchKernelGGL((chunk_kernel<SWEEP, TB, true>), dim3(cg), dim3(TB), 0, st, A);
                else
                    hipLaunchKernelGGL((chunk_kernel<SWEEP, TB, false>), dim3(cg), dim3(TB), 0, st, A);
                prof_end(g, st, KAIROS_K_CHUNK, ev);
            }
            KAIROS_HIP(hipGetLastError());
            ++r;
            which ^= 1;
            if (pulling) break;  // decide again after every pull round
        }
        KAIROS_HIP(hipMemcpyAsync(s->h_pin, s->cnt, CNT_WORDS * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        KAIROS_HIP(hipStreamSynchronize(st));
        F = s->h_pin[CNT_FRONT + r % 3u];
        vol = s->h_pin[CNT_PULLVOL + r % 3u];
        if (g->prof.on) {
            std::lock_guard<std::mutex> lk(g->prof.mu);
            g->prof.rounds += 1;
        }
        if (which == 1 && F > 0) {
            // keep the invariant "current frontier in queue[0]" cheap: swap pointers
            std::swap(s->queue[0], s->queue[1]);
            which = 0;
        }
    }
    *round_io = r;
    return KAIROS_OK;
}

int slot_alloc(kairos_graph *g, uint32_t qcap, Slot **out)
{
    Slot *s = new Slot();
    s->qcap = qcap;
    s->n = g->n;
    const size_t qn = (size_t)qcap * g->n;
    uint64_t *acct = &s->bytes;
    s->done = (uint32_t *)dev_alloc(qn * 4, acct);
    s->queue[0] = (uint32_t *)dev_alloc(std::max<size_t>(qn, qcap) * 4, acct);
    s->queue[1] = (uint32_t *)dev_alloc(std::max<size_t>(qn, qcap) * 4, acct);
    const uint64_t per_q = g->m / std::max<uint32_t>(g->tuning.chunk, 64) +
                           g->m / std::max<uint32_t>(g->tuning.split, 64) + 1;
    // bound on one round's chunks; beyond 2^26 entries (1 GiB) the push
    // kernel walks the excess itself
    s->chunk_cap = std::min<uint64_t>((uint64_t)qcap * per_q, 1ull << 26);
    // test hook: a tiny list exercises the overflow walk
    if (const char *cap = std::getenv("KAIROS_TEST_CHUNK_CAP")) s->chunk_cap = std::strtoull(cap, nullptr, 10);
    s->chunks = (uint4 *)dev_alloc(s->chunk_cap * sizeof(uint4), acct);
    s->qp = (uint4 *)dev_alloc((size_t)qcap * sizeof(uint4), acct);
    s->cnt = (uint32_t *)dev_alloc(CNT_WORDS * 4, acct);
    s->bar = (uint32_t *)dev_alloc(BAR_WORDS * 4, acct);
    s->stats = (unsigned long long *)dev_alloc(ST_TOTAL_WORDS * 8, acct);
    s->av = (unsigned long long *)dev_alloc(qn * 8, acct);
    s->filt = (uint8_t *)dev_alloc((size_t)qcap * filt_stride(g->n), acct);
    s->fpar = (uint2 *)dev_alloc((size_t)qcap * sizeof(uint2), acct);
    if (qcap == 1) {
        s->fa = (uint32_t *)dev_alloc((size_t)g->n * 4, acct);
        s->l1 = (uint32_t *)dev_alloc((size_t)g->n * 4, acct);
        s->steps = (uint32_t *)dev_alloc((size_t)std::max<uint32_t>(g->max_out_degree, 1) * 4, acct);
    }
    bool ok = s->done && s->av && s->queue[0] && s->queue[1] && s->chunks && s->qp && s->cnt && s->bar &&
              s->stats && s->filt && s->fpar && (qcap != 1 || (s->fa && s->l1 && s->steps));
    if (ok && hipHostMalloc((void **)&s->h_pin, 1024, hipHostMallocDefault) != hipSuccess) {
        s->h_pin = nullptr;
        ok = false;
    }
    if (ok && qcap > 8 && hipHostMalloc((void **)&s->h_q, (size_t)qcap * sizeof(uint4), hipHostMallocDefault) !=
                              hipSuccess) {
        s->h_q = nullptr;
        ok = false;
    }
    if (ok) {
        if (g->stream) {
            s->stream = g->stream;
        } else if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess) {
            s->own_stream = true;
        } else {
            ok = false;
        }
    }
    if (ok) {
        ok = hipMemsetAsync(s->av, 0, qn * 8, s->stream) == hipSuccess &&
             hipMemsetAsync(s->cnt, 0, CNT_WORDS * 4, s->stream) == hipSuccess &&
             hipMemsetAsync(s->stats, 0, ST_TOTAL_WORDS * 8, s->stream) == hipSuccess &&
             hipStreamSynchronize(s->stream) == hipSuccess;
    }
    if (!ok) {
        slot_destroy(s);
        return KAIROS_ERR_NOMEM;
    }
    *out = s;
    return KAIROS_OK;
}

}  // namespace

uint64_t slot_layout(const kairos_graph *g, uint64_t chunk_cap, unsigned char *base, uint64_t bytes,
                     uint32_t *host_words, Slot *s)
{
    const uint64_t n = g->n;
    uint64_t off = 0;
    auto take = [&](uint64_t b) {
        const uint64_t at = off;
        off += (b + 255) / 256 * 256;
        return at;
    };
    const uint64_t o_av = take(n * 8), o_done = take(n * 4), o_q0 = take(n * 4), o_q1 = take(n * 4);
    const uint64_t o_filt = take(filt_stride(g->n)), o_fpar = take(sizeof(uint2)), o_qp = take(sizeof(uint4));
    const uint64_t o_stage = take(sizeof(uint4)), o_cnt = take(CNT_WORDS * 4), o_bar = take(BAR_WORDS * 4);
    const uint64_t o_stats = take(ST_TOTAL_WORDS * 8), o_chunks = take(chunk_cap * sizeof(uint4));
    if (off > bytes || !s) return off;
    *s = Slot{};
    s->qcap = 1;
    s->n = g->n;
    s->av = (unsigned long long *)(base + o_av);
    s->done = (uint32_t *)(base + o_done);
    s->queue[0] = (uint32_t *)(base + o_q0);
    s->queue[1] = (uint32_t *)(base + o_q1);
    s->filt = base + o_filt;
    s->fpar = (uint2 *)(base + o_fpar);
    s->qp = (uint4 *)(base + o_qp);
    s->d_stage = (uint4 *)(base + o_stage);
    s->cnt = (uint32_t *)(base + o_cnt);
    s->bar = (uint32_t *)(base + o_bar);
    s->stats = (unsigned long long *)(base + o_stats);
    s->chunks = (uint4 *)(base + o_chunks);
    s->chunk_cap = chunk_cap;
    s->h_pin = host_words;
    s->fixed = true;
    s->stream = g->stream;  // the caller's stream, or the null stream
    return off;
}

namespace {

int read_stats(kairos_graph *g, Slot *s)
{
    if (!g->prof.on || s->fixed) return KAIROS_OK;
    std::vector<unsigned long long> raw((size_t)ST_SHARDS * ST_WORDS);
    unsigned long long h[ST_WORDS];
    KAIROS_HIP(hipMemcpyAsync(raw.data(), s->stats, raw.size() * 8, hipMemcpyDeviceToHost, s->stream));
    KAIROS_HIP(hipStreamSynchronize(s->stream));
    KAIROS_HIP(hipMemsetAsync(s->stats, 0, raw.size() * 8, s->stream));
    stats_sum_shards(raw.data(), h);
    prof_add_stats(g, h);
    return KAIROS_OK;
}

}  // namespace

// ------------------------------------------------------------ profiling --
// Launches of the allocation-free entry point are never profiled (a
// profiled launch creates events); it clears this flag on its thread.
thread_local bool tl_unprofiled = false;

void set_unprofiled(bool on) { tl_unprofiled = on; }

void prof_begin(kairos_graph *g, hipStream_t st, hipEvent_t *ev0)
{
    *ev0 = nullptr;
    if (!g->prof.on || tl_unprofiled) return;
    std::lock_guard<std::mutex> lk(g->prof.mu);
    hipEvent_t e = nullptr;
    if (!g->prof.free_events.empty()) {
        e = g->prof.free_events.back();
        g->prof.free_events.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return;
    }
    hipEventRecord(e, st);
    *ev0 = e;
}

void prof_end(kairos_graph *g, hipStream_t st, int cls, hipEvent_t ev0)
{
    if (!g->prof.on || !ev0) return;
    std::lock_guard<std::mutex> lk(g->prof.mu);
    hipEvent_t e = nullptr;
    if (!g->prof.free_events.empty()) {
        e = g->prof.free_events.back();
        g->prof.free_events.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        g->prof.free_events.push_back(ev0);
        return;
    }
    hipEventRecord(e, st);
    g->prof.pending.push_back({cls, {ev0, e}});
    g->prof.launches[cls] += 1;
}

void prof_add_stats(kairos_graph *g, const unsigned long long *h)
{
    std::lock_guard<std::mutex> lk(g->prof.mu);
    g->prof.edges += h[ST_EDGES];
    g->prof.chunk_edges += h[ST_CHUNK_EDGES];
    g->prof.attempts += h[ST_ATTEMPTS];
    g->prof.tail_edges += h[ST_TAIL_EDGES];
    g->prof.tail_items += h[ST_TAIL_ITEMS];
    g->prof.items += h[ST_ITEMS];
    g->prof.relax += h[ST_RELAX];
    g->prof.pull_edges += h[ST_PULL_EDGES];
    g->prof.pull_verts += h[ST_PULL_VERTS];
    g->prof.bin_edges += h[ST_BIN_EDGES];
    g->prof.bin_items += h[ST_BIN_ITEMS];
}

// ---------------------------------------------------------------- slots --
void slot_destroy(Slot *s)
{
    if (!s) return;
    if (s->stream) hipStreamSynchronize(s->stream);
    binned_free(s);
    dev_free(s->done);
    dev_free(s->queue[0]);
    dev_free(s->queue[1]);
    dev_free(s->chunks);
    dev_free(s->qp);
    dev_free(s->cnt);
    dev_free(s->stats);
    dev_free(s->av);
    dev_free(s->filt);
    dev_free(s->fpar);
    dev_free(s->bar);
    dev_free(s->fa);
    dev_free(s->l1);
    dev_free(s->steps);
    if (s->h_pin) hipHostFree(s->h_pin);
    if (s->h_q) hipHostFree(s->h_q);
    if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
    delete s;
}

int slot_acquire(kairos_graph *g, uint32_t qcap, bool /*sweep*/, Slot **out)
{
    {
        std::lock_guard<std::mutex> lk(g->pool_mu);
        auto &pool = qcap == 1 ? g->free_slots : g->batch_slots;
        for (size_t i = 0; i < pool.size(); ++i) {
            if (pool[i]->qcap >= qcap) {
                *out = pool[i];
                pool.erase(pool.begin() + i);
                return KAIROS_OK;
            }
        }
        // a batch slot too small: drop the cached ones so memory is reused
        if (qcap != 1) {
            for (Slot *s : pool) slot_destroy(s);
            pool.clear();
        }
    }
    return slot_alloc(g, qcap, out);
}

void slot_release(kairos_graph *g, Slot *s)
{
    std::lock_guard<std::mutex> lk(g->pool_mu);
    (s->qcap == 1 ? g->free_slots : g->batch_slots).push_back(s);
}

// -------------------------------------------------------------- queries --
static int start_queries(kairos_graph *g, Slot *s, const uint4 *hqp, uint32_t nq, bool from_w, TravArgs &A,
                         uint32_t &round, bool strict = false)
{
    hipStream_t st = s->stream;
    A = make_args(g, s, nq);
    A.strict = strict ? 1u : 0u;
    round = 0;
    A.round = 0;
    A.next = s->queue[0];
    A.front_stamp = s->stamp_next - 1u;
    // parameters travel through the pinned mirror (up to 8 queries) or the
    // slot's pinned staging array (qcap entries, allocated with the slot)
    if (nq > s->qcap) return KAIROS_ERR_INVALID;
    uint4 *dq = nullptr;
    if (s->fixed) {
        // ordinary host memory: copy to the device first (the source may
        // be reused as soon as the copy has finished)
        KAIROS_HIP(hipMemcpyAsync(s->d_stage, hqp, nq * sizeof(uint4), hipMemcpyHostToDevice, st));
        KAIROS_HIP(hipStreamSynchronize(st));
        dq = s->d_stage;
    } else if (nq * sizeof(uint4) <= 128) {
        std::memcpy(s->h_pin + 32, hqp, nq * sizeof(uint4));
        dq = (uint4 *)(s->h_pin + 32);
    } else {
        std::memcpy(s->h_q, hqp, nq * sizeof(uint4));
        dq = s->h_q;
    }
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    hipLaunchKernelGGL(init_queries_kernel, dim3(grid_cap(nq, 256, 1024)), dim3(256), 0, st, A, dq, nq,
                       from_w ? 1u : 0u);
    prof_end(g, st, KAIROS_K_INIT, ev);
    hipError_t e1 = hipGetLastError();
    if (!s->fixed && nq * sizeof(uint4) > 128 && e1 == hipSuccess) {
        // the staging array is rewritten by the next start on this slot
        e1 = hipStreamSynchronize(st);
    }
    if (e1 != hipSuccess) {
        note_hip_error(e1, "init_queries_kernel", __FILE__, __LINE__);
        return KAIROS_ERR_DEVICE;
    }
    return KAIROS_OK;
}

int run_earliest_arrival(kairos_graph *g, Slot *s, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out,
                         bool strict)
{
    hipStream_t st = s->stream;
    int rc;
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    if ((rc = fill_arrivals(st, s->av, g->n))) return rc;
    if ((rc = fill(st, s->done, g->n, INF))) return rc;
    if ((rc = fill_filter(g, st, s->filt, 1))) return rc;
    prof_end(g, st, KAIROS_K_INIT, ev);
    const uint4 qp = make_uint4(g->h_perm[src], ta, tw, ta);
    TravArgs A;
    uint32_t round;
    if ((rc = start_queries(g, s, &qp, 1, false, A, round, strict))) return rc;
    if ((rc = run_rounds<false>(g, s, A, 1, &round))) return rc;
    prof_begin(g, st, &ev);
    hipLaunchKernelGGL(finalize_sweep_kernel, dim3(grid_cap(g->n, 256, 4096)), dim3(256), 0, st, out, s->av,
                       s->l1, s->fa, g->perm, g->n, 0, src, tw);
    prof_end(g, st, KAIROS_K_INIT, ev);
    KAIROS_HIP(hipGetLastError());
    return read_stats(g, s);
}

int run_earliest_arrival_path(kairos_graph *g, Slot *s, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out,
                              uint32_t *pred_tail, uint32_t *pred_dep)
{
    int rc = run_earliest_arrival(g, s, src, ta, tw, out, false);
    if (rc) return rc;
    hipEvent_t ev;
    prof_begin(g, s->stream, &ev);
    hipLaunchKernelGGL(predecessor_kernel, dim3(grid_cap(g->n, 256, 4096)), dim3(256), 0, s->stream, s->av,
                       g->off_in, g->a_in, g->st_in, g->inv, g->n, g->h_perm[src], ta, pred_tail, pred_dep);
    prof_end(g, s->stream, KAIROS_K_INIT, ev);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

// Temporal BFS: level-synchronous rounds from the source; the round that
// first reaches a vertex gives its hop count (kept in the slot's fastest
// array; the latest-departure array holds the frontier snapshots).
int run_temporal_bfs(kairos_graph *g, Slot *s, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out, bool strict)
{
    hipStream_t st = s->stream;
    int rc;
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    if ((rc = fill_arrivals(st, s->av, g->n))) return rc;
    if ((rc = fill(st, s->done, g->n, INF))) return rc;
    if ((rc = fill_filter(g, st, s->filt, 1))) return rc;
    if ((rc = fill(st, s->fa, g->n, INF))) return rc;
    prof_end(g, st, KAIROS_K_INIT, ev);
    const uint4 qp = make_uint4(g->h_perm[src], ta, tw, ta);
    TravArgs A;
    uint32_t round;
    if ((rc = start_queries(g, s, &qp, 1, false, A, round, strict))) return rc;
    A.hop = s->fa;
    A.snap = s->l1;
    if ((rc = run_rounds<false>(g, s, A, 1, &round))) return rc;
    prof_begin(g, st, &ev);
    hipLaunchKernelGGL(finalize_sweep_kernel, dim3(grid_cap(g->n, 256, 4096)), dim3(256), 0, st, out, s->av,
                       s->l1, s->fa, g->perm, g->n, 3, src, tw);
    prof_end(g, st, KAIROS_K_INIT, ev);
    KAIROS_HIP(hipGetLastError());
    return read_stats(g, s);
}

int reverse_edge_list(kairos_graph *g, hipStream_t st, uint32_t *src, uint32_t *dst, uint32_t *t, uint32_t *lam)
{
    if (!g->m) return KAIROS_OK;
    hipLaunchKernelGGL(reverse_edges_kernel, dim3(grid_cap(g->m, 256 * 4, 16384)), dim3(256), 0, st, g->off_in,
                       g->a_in, g->st_in, g->inv, g->n, g->m, src, dst, t, lam);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

// A path from u to the target within [ta, tw] read backwards is a path from
// the target to u on the reversed graph within [TMAX - tw, TMAX - ta] (the
// succession predicates carry over: a1 <= t2 becomes a2' <= t1'), and its
// first departure t is TMAX minus its reversed last arrival.  So the latest
// departure is TMAX - (earliest reversed arrival); the target gets tw.
int run_latest_departure_to(kairos_graph *rev, Slot *s, uint32_t target, uint32_t ta, uint32_t tw, uint32_t *out,
                            bool strict)
{
    int rc = run_earliest_arrival(rev, s, target, TMAX - tw, TMAX - ta, out, strict);
    if (rc) return rc;
    hipLaunchKernelGGL(flip_times_kernel, dim3(grid_cap(rev->n, 256, 4096)), dim3(256), 0, s->stream, out, rev->n);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

int run_batch(kairos_graph *g, Slot *s, uint32_t q, const uint32_t *src, const uint32_t *ta,
              const uint32_t *tw, uint32_t *out)
{
    hipStream_t st = s->stream;
    int rc;
    const uint64_t qn = (uint64_t)q * g->n;
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    if ((rc = fill_arrivals(st, s->av, qn))) return rc;
    if ((rc = fill(st, s->done, qn, INF))) return rc;
    if ((rc = fill_filter(g, st, s->filt, q))) return rc;
    prof_end(g, st, KAIROS_K_INIT, ev);
    std::vector<uint4> hq(q);
    for (uint32_t i = 0; i < q; ++i) hq[i] = make_uint4(g->h_perm[src[i]], ta[i], tw[i], ta[i]);
    TravArgs A;
    uint32_t round;
    if ((rc = start_queries(g, s, hq.data(), q, false, A, round))) return rc;
    if ((rc = run_rounds<false>(g, s, A, q, &round))) return rc;
    prof_begin(g, st, &ev);
    for (uint32_t i = 0; i < q; ++i)
        hipLaunchKernelGGL(finalize_sweep_kernel, dim3(grid_cap(g->n, 256, 4096)), dim3(256), 0, st,
                           out + (size_t)i * g->n, s->av + (size_t)i * g->n, s->l1, s->fa, g->perm, g->n, 0,
                           src[i], tw[i]);
    prof_end(g, st, KAIROS_K_INIT, ev);
    KAIROS_HIP(hipGetLastError());
    return read_stats(g, s);
}

// Grouped sweep (tuning sweep_group = G > 1): the departure times S
// (descending) are taken G at a time, each group as G queries answered
// together, query j with the source leaving at its own time s_j.  Every
// query of a group starts from the arrivals and claims of the previous
// group's last query (the earliest arrivals for a later departure bound
// those for s_j from above, and its claims record edges already relaxed
// for them), so each ends with the earliest arrivals EA_j for leaving at
// s_j.  F and LD then follow from their cross-route definitions,
// F[v] = min_j (EA_j[v] - s_j) and LD[v] = max{s_j : EA_j[v] finite}
// (`sweep_reduce_kernel`).  Queries of one group also explore paths that
// leave at later times of the same group; that is redundant work, not an
// error.  fa / l1 / steps live in the single-query slot s.
int run_sweep_groups(kairos_graph *g, Slot *s, uint32_t src, uint32_t ta, uint32_t tw,
                     const std::vector<uint32_t> &S, uint32_t G, bool strict)
{
    Slot *b = nullptr;
    int rc = slot_acquire(g, G, false, &b);
    if (rc) return rc;
    const hipStream_t st = b->stream;
    hipEvent_t ev;
    // s's fills and step upload precede this stream's work
    if (b->stream != s->stream) {
        if (hipStreamSynchronize(s->stream) != hipSuccess) rc = KAIROS_ERR_DEVICE;
    }
    uint32_t last = INF;  // slot holding the previous group's last query
    for (size_t g0 = 0; g0 < S.size() && rc == KAIROS_OK; g0 += G) {
        const uint32_t q = (uint32_t)std::min<size_t>(G, S.size() - g0);
        prof_begin(g, st, &ev);
        if (last == INF) {
            if ((rc = fill_arrivals(st, b->av, (uint64_t)q * g->n))) break;
            if ((rc = fill(st, b->done, (uint64_t)q * g->n, INF))) break;
        } else {
            // slots [0, q) take slot `last`'s state (`last` itself, if it is
            // one of them, keeps it)
            hipLaunchKernelGGL(warm_slots_kernel, dim3(grid_cap(g->n, 256, 4096)), dim3(256), 0, st, b->av, b->done,
                               g->n, q, last);
            if (hipGetLastError() != hipSuccess) { rc = KAIROS_ERR_DEVICE; break; }
        }
        if ((rc = fill_filter(g, st, b->filt, q))) break;
        prof_end(g, st, KAIROS_K_INIT, ev);
        std::vector<uint4> hq(q);
        for (uint32_t j = 0; j < q; ++j) hq[j] = make_uint4(src, ta, tw, S[g0 + j]);
        TravArgs A;
        uint32_t r = 0;
        if ((rc = start_queries(g, b, hq.data(), q, true, A, r, strict))) break;
        if ((rc = run_rounds<false>(g, b, A, q, &r))) break;
        prof_begin(g, st, &ev);
        hipLaunchKernelGGL(sweep_reduce_kernel, dim3(grid_cap(g->n, 256, 4096)), dim3(256), 0, st, b->av,
                           s->steps + g0, g->n, q, s->fa, s->l1);
        prof_end(g, st, KAIROS_K_INIT, ev);
        if (hipGetLastError() != hipSuccess) { rc = KAIROS_ERR_DEVICE; break; }
        last = q - 1;
    }
    if (rc == KAIROS_OK && hipStreamSynchronize(st) != hipSuccess) rc = KAIROS_ERR_DEVICE;
    if (rc == KAIROS_OK && (rc = read_stats(g, b)) == KAIROS_OK) {
        slot_release(g, b);
    } else {
        hipStreamSynchronize(st);
        slot_destroy(b);
    }
    return rc;
}

// Latest departure / fastest (kind 1 / 2).  The departure times S of the
// source's usable out-edges are taken in descending order; for each s the
// source is set to s and push rounds run to a fixpoint, warm-started from
// the previous s (arrivals for a later start bound those for an earlier
// one from above).  Every arrival that improves during step s belongs to a
// path leaving the source exactly at s (all later departures were already
// at their fixpoint), so each improvement updates
//   F[v] = min(F[v], a - s)   and   L1[v] = max(L1[v], s + 1),
// the latter giving LD[v] = L1[v] - 1, with 0 meaning unreachable.
int run_sweep(kairos_graph *g, Slot *s, int kind, uint32_t src_caller, uint32_t ta, uint32_t tw, uint32_t *out,
              bool strict)
{
    hipStream_t st = s->stream;
    int rc;
    const uint32_t src = g->h_perm[src_caller];
    uint32_t hoff[2];
    KAIROS_HIP(hipMemcpyAsync(s->h_pin, g->off_out + src, 8, hipMemcpyDeviceToHost, st));
    KAIROS_HIP(hipStreamSynchronize(st));
    hoff[0] = s->h_pin[0];
    hoff[1] = s->h_pin[1];
    const uint32_t deg = hoff[1] - hoff[0];
    std::vector<uint32_t> ht(deg);
    std::vector<uint2> hda(deg);
    if (deg) {
        KAIROS_HIP(hipMemcpy(ht.data(), g->t_out + hoff[0], deg * 4ull, hipMemcpyDeviceToHost));
        KAIROS_HIP(hipMemcpy(hda.data(), g->da_out + hoff[0], deg * 8ull, hipMemcpyDeviceToHost));
    }
    std::vector<uint32_t> S;
    for (uint32_t i = 0; i < deg; ++i)
        if (ht[i] >= ta && hda[i].y <= tw) S.push_back(ht[i]);
    std::sort(S.begin(), S.end());
    S.erase(std::unique(S.begin(), S.end()), S.end());
    std::reverse(S.begin(), S.end());

    uint32_t *l1 = s->l1;
    uint32_t *fa = s->fa;
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    if ((rc = fill_arrivals(st, s->av, g->n))) return rc;
    if ((rc = fill(st, s->done, g->n, INF))) return rc;
    if ((rc = fill_filter(g, st, s->filt, 1))) return rc;
    if ((rc = fill(st, fa, g->n, INF))) return rc;
    if ((rc = fill(st, l1, g->n, 0u))) return rc;
    prof_end(g, st, KAIROS_K_INIT, ev);
    const uint32_t G = std::min<uint32_t>(std::max<uint32_t>(g->tuning.sweep_group, 1), (uint32_t)S.size());
    if (G > 1) {
        KAIROS_HIP(hipMemcpy(s->steps, S.data(), S.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        rc = run_sweep_groups(g, s, src, ta, tw, S, G, strict);
        if (rc) return rc;
    } else if (!S.empty()) {
        KAIROS_HIP(hipMemcpy(s->steps, S.data(), S.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        const uint4 qp = make_uint4(src, ta, tw, S[0]);
        TravArgs A;
        uint32_t r = 0;
        if ((rc = start_queries(g, s, &qp, 1, true, A, r, strict))) return rc;
        A.fa = fa;
        A.l1 = l1;
        A.steps = s->steps;
        A.nsteps = (uint32_t)S.size();
        if ((rc = run_rounds<true>(g, s, A, 1, &r))) return rc;
    }
    prof_begin(g, st, &ev);
    hipLaunchKernelGGL(finalize_sweep_kernel, dim3(grid_cap(g->n, 256, 4096)), dim3(256), 0, st, out, s->av,
                       l1, fa, g->perm, g->n, kind, src_caller, tw);
    prof_end(g, st, KAIROS_K_INIT, ev);
    KAIROS_HIP(hipGetLastError());
    KAIROS_HIP(hipStreamSynchronize(st));
    return read_stats(g, s);
}

int count_traversed(kairos_graph *g, uint32_t ta, uint32_t tw, const uint32_t *ea, uint64_t *count)
{
    Slot *s = nullptr;
    int rc = slot_acquire(g, 1, false, &s);
    if (rc) return rc;
    hipStream_t st = s->stream;
    unsigned long long *d = s->stats + (size_t)ST_SHARDS * ST_WORDS;  // ST_SHARDS partial sums
    do {
        if (hipMemsetAsync(d, 0, ST_SHARDS * 8, st) != hipSuccess) { rc = KAIROS_ERR_DEVICE; break; }
        if (g->m)
            hipLaunchKernelGGL(count_traversed_kernel, dim3(grid_cap(g->m, 256 * 8, 16384)), dim3(256), 0,
                               st, g->a_in, g->st_in, g->m, ea, g->inv, ta, tw, d);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(s->h_pin, d, ST_SHARDS * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = KAIROS_ERR_DEVICE;
            break;
        }
        uint64_t v = 0;
        for (int k = 0; k < ST_SHARDS; ++k) {
            uint64_t x;
            std::memcpy(&x, (const char *)s->h_pin + 8 * k, 8);
            v += x;
        }
        *count = v;
    } while (0);
    slot_release(g, s);
    return rc;
}

kairos_tuning default_tuning(const kairos_graph *g)
{
    kairos_tuning t{};
    t.block = 256;
    t.chunk = 256;
    t.split = 128;
    t.pull_alpha = 0;
    t.pull_beta = 24;
    t.rounds_per_sync = 8;  // measured best: queued empty rounds cost less than host checks
    t.batch_persistent = 1;
    t.single_persistent = 0;  // measured slower: barrier fences cost more than the host round trip
    // departure times per group of a latest-departure / fastest sweep.
    // Measured (G = 1, 2, 4, 8, 16): 2^20 vertices, 32 edges per vertex,
    // first 8 queries 9.1, 7.2, 5.5, 4.2, 4.4 ms; 2^24 vertices, 32 per
    // vertex, first 4: 50, 48, 47, 52, 62 ms (each group copies and reduces
    // G arrival arrays of n words); the bursty graph, 240 edges per vertex:
    // 11.2, 14.7, 16.1, 22.5, 38.9 ms (dense adjacencies make the queries of
    // a group repeat each other's exploration)
    t.sweep_group = !g || g->m > 64ull * g->n ? 1u : g->n <= (1u << 21) ? 8u : 4u;
    // lane-dense rows for graphs with real work per round; on small graphs
    // the query-major layout wins, since it hands small frontiers to the
    // one-workgroup kernel (10^5 edges, 16 queries: 0.59 ms against 1.9 ms)
    t.batch_layout = g && g->m >= (1u << 22) ? 2u : 1u;
    t.tail_limit = 4096;
    t.dense_frontier = 0;
    // arrival codes add a dependent read in front of the arrival read: at
    // 2^22 and 2^24 vertices every width measured slower than none (2, 4, 8
    // bits: 5.88, 5.78, 5.75 ms against 5.13 ms per query at 2^24); at 2^20
    // vertices 8-bit codes tie on earliest arrival and lose 7% on latest
    // departure (2.75 against 2.56 ms), at 10^4 vertices 5% on both
    t.arrival_filter = 0;
    // runs of equal heads (bursty pairs): 2.1x on single queries and 2.5x
    // on batches of the 10^9-edge bursty graph; on R-MAT graphs, which have
    // almost none, the extra ballot costs up to 1.4%
    t.run_dedupe = g && g->repeat_heads * 32 > g->m ? 1u : 0u;
    // longer chunks where bursts of one pair's contacts fill long claims:
    // the 10^9-edge bursty graph (first 16 queries) 3.28 -> 3.10 ms with
    // 1024 (2048: 3.20, 4096: 3.40); the R-MAT graphs lose 2% with 1024
    // (scale 24 4.41 -> 4.49 ms, scale 20 0.779 -> 0.796 ms)
    if (t.run_dedupe) t.chunk = 1024;
    t.binned = 0;
    return t;
}


// ------------------------------------------------------ server stepping --
namespace {

__global__ void inject_kernel(TravArgs A, const Inject *__restrict__ list, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const Inject in = list[i];
        ((uint4 *)A.qp)[in.q] = make_uint4(in.src, in.ta, in.tw, in.sdep);
        A.fpar[in.q] = filter_params(in.ta, in.tw, A.max_a, A.fbits);
        if (in.sweep) continue;  // a sweep slot's source starts with its first step
        const size_t ss = (size_t)in.q * A.n + in.src;
        // stamp 0: older than every round's stamp, so the source's first
        // improvement (a sweep step) still enqueues it
        A.av[ss] = av_word(in.sdep == INF ? in.ta : in.sdep, 0u);
        const uint32_t pos = atomicAdd(&A.cnt[CNT_FRONT + A.round % 3u], 1u);
        A.next[pos] = (uint32_t)ss;  // `next` names the queue of the coming round here
    }
}

// Departure times of the sweep slots in `list`, on the device: the distinct
// departure times t >= t_alpha of the source's out-edges that arrive by
// t_omega, ascending, into the slot's row of `steps` (at most the largest
// out-degree).  Edges of equal departure time sit in ascending arrival
// order, so a time qualifies iff the first edge of its group arrives by
// t_omega.  One block of SB threads per slot; the block compacts in order.
constexpr int SB = 256;

__global__ __launch_bounds__(SB) void sweep_steps_kernel(TravArgs A, const uint32_t *__restrict__ list,
                                                          uint32_t *steps, uint32_t cap, uint32_t *step_cnt,
                                                          uint32_t *step_pos)
{
    __shared__ uint32_t s_w[SB / 64];
    __shared__ uint32_t s_base;
    const uint32_t q = list[blockIdx.x];
    const uint4 p = A.qp[q];
    const uint32_t b = A.off[p.x], e = A.off[p.x + 1];
    const uint32_t lo = lower_bound_u32(A.tt, b, e, p.y);
    const uint32_t hi = lower_bound_u32(A.tt, lo, e, p.z);  // departing at t_omega or later arrives after it
    uint32_t *row = steps + (size_t)q * cap;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (uint32_t j0 = lo; j0 < hi; j0 += SB) {
        const uint32_t j = j0 + threadIdx.x;
        bool f = false;
        uint32_t t = 0;
        if (j < hi) {
            t = A.tt[j];
            f = (j == b || A.tt[j - 1] != t) && A.da[j].y <= p.z;
        }
        const unsigned long long bal = __ballot(f);
        if (lane == 0) s_w[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t off = s_base, tot = 0;
        for (int k = 0; k < SB / 64; ++k) {
            if (k < w) off += s_w[k];
            tot += s_w[k];
        }
        if (f) row[off + __popcll(bal & ((1ull << lane) - 1ull))] = t;
        __syncthreads();
        if (threadIdx.x == 0) s_base += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        step_cnt[q] = s_base;
        step_pos[q] = 0u;
    }
}

// Between rounds: a sweep slot that enqueued nothing for the coming round
// (its flag is older than the round) starts its next departure time, latest
// first, warm-started from the arrivals and claims it holds.  One thread
// per slot; `A.next` is the coming round's queue.
__global__ void advance_steps_kernel(TravArgs A, const uint32_t *__restrict__ steps, uint32_t cap,
                                     const uint32_t *__restrict__ step_cnt, uint32_t *step_pos, uint32_t nslots)
{
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nslots; q += gridDim.x * blockDim.x) {
        const uint32_t c = step_cnt[q], k = step_pos[q];
        if (k >= c || A.qflag[q] == A.round) continue;
        const uint32_t sd = steps[(size_t)q * cap + (c - 1u - k)];
        const uint32_t src = A.qp[q].x;
        ((uint4 *)A.qp)[q].w = sd;
        const size_t ss = (size_t)q * A.n + src;
        A.av[ss] = av_word(min(arrival_of(A.av, ss), sd), 0u);
        const uint32_t pos = atomicAdd(&A.cnt[CNT_FRONT + A.round % 3u], 1u);
        A.next[pos] = (uint32_t)ss;
        A.qflag[q] = A.round;
        step_pos[q] = k + 1u;
    }
}

// Grouped sweep in the server: the query's departure times (its lead slot's
// row, latest first) are taken `width` at a time by the consecutive slots
// lead .. lead + width - 1.  Member j of a group starting at step pos0 runs
// the earliest-arrival query leaving the source at its step s (t_alpha = s,
// no sweep accumulators, no arrival codes), warm-started from what the slot
// holds; a member without a step gets t_alpha = INF and no frontier.  The
// lead's own device stepping is switched off.  One thread per member.
__global__ void group_start_kernel(TravArgs A, const GroupStart *__restrict__ list, uint32_t count,
                                   const uint32_t *__restrict__ steps, uint32_t cap, const uint32_t *__restrict__ step_cnt,
                                   uint32_t *step_pos)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count * 64u; i += gridDim.x * blockDim.x) {
        const GroupStart e = list[i >> 6];
        const uint32_t j = i & 63u;
        if (j >= e.width) continue;
        const uint32_t m = e.lead + j, k = e.pos0 + j, c = step_cnt[e.lead];
        if (j == 0) step_pos[e.lead] = INF;
        if (k >= c) {
            ((uint4 *)A.qp)[m] = make_uint4(e.src, INF, e.tw, INF);
            continue;
        }
        const uint32_t sd = steps[(size_t)e.lead * cap + (c - 1u - k)];
        ((uint4 *)A.qp)[m] = make_uint4(e.src, sd, e.tw, INF);
        A.fpar[m] = filter_params(sd, e.tw, A.max_a, 0u);
        const size_t ss = (size_t)m * A.n + e.src;
        A.av[ss] = av_word(min(arrival_of(A.av, ss), sd), 0u);
        const uint32_t pos = atomicAdd(&A.cnt[CNT_FRONT + A.round % 3u], 1u);
        A.next[pos] = (uint32_t)ss;
    }
}

// After a group: member j holds the earliest arrivals for the source leaving
// at its t_alpha, so the lead's F[v] = min(F[v], EA_j[v] - t_alpha_j) and,
// where v is reached, L1[v] = max(L1[v], t_alpha_j + 1).
__global__ void group_reduce_kernel(TravArgs A, uint32_t lead, uint32_t width)
{
    const size_t base = (size_t)lead * A.n;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < A.n; v += gridDim.x * blockDim.x) {
        uint32_t f = A.fa[base + v], l = A.l1[base + v];
        for (uint32_t j = 0; j < width; ++j) {
            const uint32_t d = A.qp[lead + j].y;
            if (d == INF) continue;
            const uint32_t a = arrival_of(A.av, base + (size_t)j * A.n + v);
            if (a != INF) {
                f = min(f, a - d);
                l = max(l, d + 1u);
            }
        }
        A.fa[base + v] = f;
        A.l1[base + v] = l;
    }
}

// Fresh state for the listed slots: arrival, claims and fastest = INF,
// latest departure + 1 = 0, no arrival bound, no sweep steps, no activity
// flag.  Block (x, y): slot list[y], stride over n.
__global__ void init_slots_kernel(TravArgs A, const uint32_t *__restrict__ list, uint8_t *filt, uint32_t *step_cnt,
                                  uint32_t *step_pos)
{
    const size_t base = (size_t)list[blockIdx.y] * A.n;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        step_cnt[list[blockIdx.y]] = 0u;
        step_pos[list[blockIdx.y]] = 0u;
        A.qflag[list[blockIdx.y]] = INF;  // never a round number
    }
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < A.n; v += gridDim.x * blockDim.x) {
        A.av[base + v] = av_word(INF, 0u);
        A.done[base + v] = INF;
        A.fa[base + v] = INF;
        A.l1[base + v] = 0u;
    }
    uint32_t *fw = (uint32_t *)(filt + (size_t)list[blockIdx.y] * A.fstride);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < A.fstride / 4; i += gridDim.x * blockDim.x)
        fw[i] = 0xFFFFFFFFu;
}

TravArgs multi_args(kairos_graph *g, MultiState *ms)
{
    TravArgs A{};
    A.off = g->off_out;
    A.tt = g->t_out;
    A.da = g->da_out;
    A.off_in = g->off_in;
    A.a_in = g->a_in;
    A.st_in = g->st_in;
    A.n_live = g->n_live;
    A.max_deg = g->max_out_degree;
    A.min_per = min_entries_per_block(g);
    A.qp = ms->qp;
    A.n = g->n;
    A.av = ms->av;
    A.done = ms->done;
    A.fa = ms->fa;
    A.l1 = ms->l1;
    A.cnt = ms->cnt;
    A.qflag = ms->cnt + CNT_WORDS;
    A.chunks = ms->chunks;
    A.chunk_cap = (uint32_t)std::min<uint64_t>(ms->chunk_cap, 0xFFFFFFF0u);
    A.stats = g->prof.on ? ms->stats : nullptr;
    A.split = std::max<uint32_t>(g->tuning.split, 1);
    A.chunk = std::max<uint32_t>(g->tuning.chunk, 1);
    A.nq = ms->qcap;
    A.round = ms->round;
    A.cur = ms->queue[0];
    A.next = ms->queue[1];
    A.max_t = g->max_t;
    // skipping the codes is always valid: a query started with codes on
    // finds them again, possibly looser, when they are switched back on
    A.filt = g->tuning.arrival_filter ? ms->filt : nullptr;
    A.fpar = ms->fpar;
    A.fbits = g->tuning.arrival_filter;
    A.fstride = (uint32_t)filt_stride(g->n);
    A.max_a = g->max_a;
    A.dedupe = g->tuning.run_dedupe;
    return A;
}

}  // namespace

int multi_push_round(kairos_graph *g, MultiState *ms)
{
    TravArgs A = multi_args(g, ms);
    if (ms->stamp_next >= 0xFFFFF000u) {
        int rc = clear_stamps(ms->stream, ms->av, (uint64_t)ms->qcap * ms->n);
        if (rc) return rc;
        ms->stamp_next = 2;
    }
    A.stamp_val = ms->stamp_next++;
    hipEvent_t ev;
    prof_begin(g, ms->stream, &ev);
    hipLaunchKernelGGL((push_kernel<true, TB, false>), dim3(std::max(1, g->num_cus * 8)), dim3(TB), 0, ms->stream, A);
    prof_end(g, ms->stream, KAIROS_K_PUSH, ev);
    prof_begin(g, ms->stream, &ev);
    hipLaunchKernelGGL((chunk_kernel<true, TB, false>), dim3(std::max(1, g->num_cus * 4)), dim3(TB), 0, ms->stream, A);
    prof_end(g, ms->stream, KAIROS_K_CHUNK, ev);
    KAIROS_HIP(hipGetLastError());
    ms->round += 1;
    std::swap(ms->queue[0], ms->queue[1]);
    return KAIROS_OK;
}

int multi_inject(kairos_graph *g, MultiState *ms, const Inject *host_pinned, uint32_t count)
{
    if (!count) return KAIROS_OK;
    TravArgs A = multi_args(g, ms);
    A.next = ms->queue[0];
    hipLaunchKernelGGL(inject_kernel, dim3(grid_cap(count, 256, 64)), dim3(256), 0, ms->stream, A,
                       host_pinned, count);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

int multi_init_slots(kairos_graph *g, MultiState *ms, const uint32_t *host_pinned, uint32_t count)
{
    if (!count) return KAIROS_OK;
    TravArgs A = multi_args(g, ms);
    hipLaunchKernelGGL(init_slots_kernel, dim3(grid_cap(g->n, 256 * 4, 256), count), dim3(256), 0,
                       ms->stream, A, host_pinned, ms->filt, ms->step_cnt, ms->step_pos);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

int multi_sweep_steps(kairos_graph *g, MultiState *ms, const uint32_t *host_pinned, uint32_t count)
{
    if (!count) return KAIROS_OK;
    TravArgs A = multi_args(g, ms);
    hipLaunchKernelGGL(sweep_steps_kernel, dim3(count), dim3(SB), 0, ms->stream, A, host_pinned, ms->steps,
                       ms->step_cap, ms->step_cnt, ms->step_pos);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

int multi_group_start(kairos_graph *g, MultiState *ms, const GroupStart *host_pinned, uint32_t count)
{
    if (!count) return KAIROS_OK;
    TravArgs A = multi_args(g, ms);
    A.next = ms->queue[0];
    hipLaunchKernelGGL(group_start_kernel, dim3(grid_cap((uint64_t)count * 64, 256, 64)), dim3(256), 0, ms->stream,
                       A, host_pinned, count, ms->steps, ms->step_cap, ms->step_cnt, ms->step_pos);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

int multi_group_reduce(kairos_graph *g, MultiState *ms, uint32_t lead, uint32_t width)
{
    TravArgs A = multi_args(g, ms);
    hipLaunchKernelGGL(group_reduce_kernel, dim3(grid_cap(g->n, 256, 4096)), dim3(256), 0, ms->stream, A, lead,
                       width);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

int multi_group_warm(kairos_graph *g, MultiState *ms, uint32_t lead, uint32_t width, uint32_t from)
{
    const size_t base = (size_t)lead * g->n;
    hipLaunchKernelGGL(warm_slots_kernel, dim3(grid_cap(g->n, 256, 4096)), dim3(256), 0, ms->stream, ms->av + base,
                       ms->done + base, g->n, width, from);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

int multi_advance(kairos_graph *g, MultiState *ms)
{
    TravArgs A = multi_args(g, ms);
    A.next = ms->queue[0];
    hipLaunchKernelGGL(advance_steps_kernel, dim3(grid_cap(ms->qcap, 256, 64)), dim3(256), 0, ms->stream, A,
                       ms->steps, ms->step_cap, ms->step_cnt, ms->step_pos, ms->qcap);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

int multi_finalize(kairos_graph *g, MultiState *ms, uint32_t q, int kind, uint32_t src, uint32_t tw,
                   uint32_t *out)
{
    const size_t base = (size_t)q * g->n;
    hipLaunchKernelGGL(finalize_sweep_kernel, dim3(grid_cap(g->n, 256, 4096)), dim3(256), 0, ms->stream, out,
                       ms->av + base, ms->l1 + base, ms->fa + base, g->perm, g->n, kind, src, tw);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

}  // namespace kairos
