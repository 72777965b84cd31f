// Shortest duration (Table 4's "S. Duration" row): the least total duration
// (sum of lambda) of a time-respecting path from the source to each vertex
// within the query interval.
//
// Unlike an arrival time, the duration of the best path into a vertex is not
// one label: a path that arrives later with a smaller total can be the one
// worth extending, so the state of a vertex v is a step function
// D_v(t) = least duration of a path reaching v by time t.  It is kept per
// in-edge: the index sorts v's in-edges by arrival, and after a prefix
// minimum pm[k] over that order equals D_v(a_k).  An out-edge f = (v, w, t,
// lambda) has the candidate D_v(t) + lambda, read at the last in-edge of v
// arriving by t (before t under "Strictly succeeds"), and lowers pm at f's
// own position in w's in-list (o2i[f]).  Both positions depend on the graph
// alone: o2i[f] and o2k[f] (the last in-edge of v arriving by t; the strict
// case steps back over in-edges arriving exactly at t) are built once per
// graph.
//
// Label-correcting rounds.  A relaxation that lowers pm at position k of w's
// in-list widens w's dirty range [lo, hi] for the next round and enqueues w
// once.  Expanding v redoes the prefix minimum over [lo, hi]; with C its
// value at hi, the new value at k > hi is min(C, pm[k]), because an expanded
// list is non-increasing and nothing past hi was lowered since.  So the
// values past hi change exactly up to `stop`, the first position past hi
// holding at most C (a binary search), and there they all become C.  D_v
// changed exactly on departures in [a_lo, a_stop), so only v's out-edges
// departing in that interval are relaxed again.  A lane expands one
// vertex; long scans and fills go to its wavefront, and dirty ranges longer
// than SD_BIG to a whole workgroup.  Every
// value is the duration of a real path and values only decrease, so a stale
// read costs work, never a wrong result.  The source's D is 0 from t_alpha on: its usable out-edges are
// relaxed once at the start with their own lambda, and it is never expanded.
// When no vertex is left to expand, every vertex with out-edges has a
// non-increasing list, whose minimum is its last label; the others (never
// expanded) take the minimum over the list.

#include "internal.h"
#include "scan.h"
#include "stage.h"

#include <algorithm>
#include <cstring>

namespace kairos {

struct SDState {
    uint32_t *pm = nullptr;                         // m: per in-edge duration label
    uint32_t *dlo[2] = {nullptr, nullptr};          // n each: dirty range start (INF: clean)
    uint32_t *dhi[2] = {nullptr, nullptr};          // n each: dirty range end (inclusive)
    uint32_t *queue[2] = {nullptr, nullptr};        // n each: frontier vertices
    uint4 *rng = nullptr;                           // n: {v, first out-edge, count, lo}
    uint32_t *big = nullptr;                        // n: frontier indices whose dirty range a workgroup expands
    uint32_t *base = nullptr;                       // n + 1: out-edge counts, then their exclusive scan
    uint32_t *bsum = nullptr;                       // block sums of the scan
    uint32_t *cnt = nullptr;                        // SD_CNT_WORDS counters
    uint32_t *h_pin = nullptr;                      // pinned read-back of cnt
    hipStream_t stream = nullptr;
    bool own_stream = false;
};

namespace {

constexpr int SDT = 256;                  // threads per block
constexpr int SDB = 1024;                 // threads of a workgroup expanding one long dirty range
constexpr int SDB_PER = 8;                // positions per thread per tile of that scan
constexpr uint32_t SD_BIG = 4096;         // dirty ranges longer than this go to a workgroup
constexpr uint32_t SD_LANE = 8;           // dirty ranges a lane scans by itself (longer: its wavefront)
constexpr uint32_t SD_LANE_FILL = 16;     // fills a lane writes by itself (longer: its wavefront)
constexpr int SD_SCAP = 512;              // staged frontier entries per wavefront
constexpr int SD_U = 4;                   // out-edges per lane per pass of the relaxation loop
using SDStage = Stage<SD_SCAP>;
// counters: frontier sizes of the two parities, relax total, long ranges
enum : int { SD_FRONT = 0, SD_TOTAL = 2, SD_BIG_CNT = 3, SD_CNT_WORDS = 4 };

struct SDArgs {
    const uint32_t *off_out, *t_out;
    const uint2 *da_out;
    const uint32_t *off_in, *a_in;
    const uint32_t *o2i, *o2k;
    uint32_t *pm;
    uint32_t n, n_live, max_t, src, ta, tw, strict;
};

__device__ __forceinline__ uint32_t lower_bound_t(const uint32_t *__restrict__ a, uint32_t lo, uint32_t hi,
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

// First position in [lo, hi) whose value exceeds key.
__device__ __forceinline__ uint32_t upper_bound_t(const uint32_t *__restrict__ a, uint32_t lo, uint32_t hi,
                                                  uint32_t key)
{
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// First position in [lo, hi) of a non-increasing run whose value is at most
// key (hi when none).  The answer is usually at or just past lo, so the
// search gallops from lo (steps 1, 2, 4, ...) before bisecting.
__device__ __forceinline__ uint32_t first_at_most(const uint32_t *a, uint32_t lo, uint32_t hi, uint32_t key)
{
    if (lo >= hi || a[lo] <= key) return lo;
    uint32_t b, step = 1;
    for (;;) {  // a[lo] > key; the answer lies in (lo, b]
        if (step >= hi - lo) {
            b = hi;
            break;
        }
        b = lo + step;
        if (a[b] <= key) break;
        lo = b;
        step <<= 1;
    }
    ++lo;
    while (lo < b) {
        const uint32_t mid = lo + ((b - lo) >> 1);
        if (a[mid] <= key)
            b = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// lower_bound_t galloping from lo, for answers expected near lo.
__device__ __forceinline__ uint32_t gallop_lower_bound(const uint32_t *__restrict__ a, uint32_t lo, uint32_t hi,
                                                       uint32_t key)
{
    if (lo >= hi || a[lo] >= key) return lo;
    uint32_t b, step = 1;
    for (;;) {  // a[lo] < key; the answer lies in (lo, b]
        if (step >= hi - lo) {
            b = hi;
            break;
        }
        b = lo + step;
        if (a[b] >= key) break;
        lo = b;
        step <<= 1;
    }
    ++lo;
    while (lo < b) {
        const uint32_t mid = lo + ((b - lo) >> 1);
        if (a[mid] >= key)
            b = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Out-edges of v departing in [a_p, a_stop) ([a_p + 1, a_stop + 1) under
// strict succession) and before t_omega: {first, count}.  Arrivals are at
// most TMAX = 2^32 - 2 (the index rejects larger ones), so a + 1 does not
// wrap.
__device__ __forceinline__ uint2 changed_out_range(const SDArgs &A, uint32_t v, uint32_t p, uint32_t stop,
                                                   uint32_t end)
{
    const uint32_t ob = A.off_out[v], oe = A.off_out[v + 1];
    const uint32_t lo = lower_bound_t(A.t_out, ob, oe, A.a_in[p] + A.strict);
    uint32_t hi_out;
    if (stop < end) {
        const uint32_t khi = min(A.a_in[stop] + A.strict, A.tw);
        hi_out = gallop_lower_bound(A.t_out, lo, oe, khi);
    } else {
        hi_out = A.tw > A.max_t ? oe : gallop_lower_bound(A.t_out, lo, oe, A.tw);
    }
    return make_uint2(lo, hi_out > lo ? hi_out - lo : 0u);
}

__global__ __launch_bounds__(SDT) void sd_fill_kernel(uint32_t *p, uint64_t count, uint32_t value)
{
    for (uint64_t i = (uint64_t)blockIdx.x * SDT + threadIdx.x; i < count; i += (uint64_t)gridDim.x * SDT)
        p[i] = value;
}

// o2i[f] = position in the in-index of out-edge f: copies of one edge
// (equal in tail, head, t and a) sit next to each other in both indexes,
// and the d-th copy in the out-index takes the d-th in the in-index, so
// every in-index position belongs to exactly one out-edge.  o2k[f] =
// position of the last in-edge of f's tail arriving by f's departure (the
// list's start minus one when none).  One wavefront per tail.
__global__ __launch_bounds__(SDT) void o2i_kernel(const uint32_t *__restrict__ off_out,
                                                  const uint32_t *__restrict__ t_out,
                                                  const uint2 *__restrict__ da_out,
                                                  const uint32_t *__restrict__ off_in,
                                                  const uint32_t *__restrict__ a_in,
                                                  const uint2 *__restrict__ st_in, uint32_t n_live,
                                                  uint32_t *__restrict__ o2i, uint32_t *__restrict__ o2k,
                                                  uint32_t *err)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (SDT / 64);
    for (uint32_t u = blockIdx.x * (SDT / 64) + (threadIdx.x >> 6); u < n_live; u += waves) {
        const uint32_t e = off_out[u + 1];
        const uint32_t ib = off_in[u], ie = off_in[u + 1];
        for (uint32_t f = off_out[u] + lane; f < e; f += 64) {
            const uint2 va = da_out[f];
            const uint32_t t = t_out[f];
            o2k[f] = upper_bound_t(a_in, ib, ie, t) - 1u;
            uint32_t lo = off_in[va.x], hi = off_in[va.x + 1];
            // in-list order: (a, t, tail)
            while (lo < hi) {
                const uint32_t mid = lo + ((hi - lo) >> 1);
                const uint32_t am = a_in[mid];
                const uint2 st = st_in[mid];
                const bool less = am < va.y || (am == va.y && (st.y < t || (st.y == t && st.x < u)));
                if (less)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            // copies of this edge before it in the out-index
            uint32_t d = 0;
            while (f - d > off_out[u] && t_out[f - d - 1] == t && da_out[f - d - 1].x == va.x &&
                   da_out[f - d - 1].y == va.y)
                ++d;
            lo += d;
            // the same edge is in the in-index; anything else is an index
            // fault, reported instead of used
            const bool found = lo < off_in[va.x + 1] && a_in[lo] == va.y && st_in[lo].y == t && st_in[lo].x == u;
            if (!found) atomicOr(err, 1u);
            o2i[f] = found ? lo : off_in[va.x];
        }
    }
}

// Widens head w's dirty range to cover pos and reports whether this is the
// range's first entry of the round (then the caller enqueues w).  Within a
// round dlo only falls and dhi only rises, so a plain read that already
// covers pos (even a stale one) makes the atomic unnecessary: the many
// in-edges of a hub lowered in one round would otherwise queue on its two
// words.
__device__ __forceinline__ bool sd_mark(uint32_t *dlo, uint32_t *dhi, uint32_t w, uint32_t pos)
{
    if (pos > __hip_atomic_load(&dhi[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&dhi[w], pos);
    if (pos >= __hip_atomic_load(&dlo[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    return atomicMin(&dlo[w], pos) == INF;
}

// Lowers pm[pos] to `cand` and, on success, marks it as sd_mark does.
// Position pos belongs to one out-edge, which a round relaxes at most once,
// so nothing else writes it meanwhile and a plain store suffices.
__device__ __forceinline__ bool sd_lower(uint32_t *pm, uint32_t pos, uint32_t cand, uint32_t *dlo, uint32_t *dhi,
                                         uint32_t w)
{
    if (cand >= pm[pos]) return false;
    pm[pos] = cand;
    return sd_mark(dlo, dhi, w, pos);
}

// The source's usable out-edges (t >= t_alpha, a <= t_omega), each a path
// of one edge with duration lambda.
__global__ __launch_bounds__(SDT) void sd_seed_kernel(SDArgs A, uint32_t *dlo, uint32_t *dhi, uint32_t *next,
                                                      uint32_t *cnt)
{
    __shared__ uint32_t s_stage[SDT / 64][SD_SCAP];
    SDStage S{s_stage[threadIdx.x >> 6], 0u, next, cnt};
    const uint32_t b = A.off_out[A.src], e = A.off_out[A.src + 1];
    const uint32_t lo = lower_bound_t(A.t_out, b, e, A.ta);
    const uint32_t hi = A.tw > A.max_t ? e : lower_bound_t(A.t_out, lo, e, A.tw);
    for (uint32_t f0 = lo + blockIdx.x * SDT; f0 < hi; f0 += gridDim.x * SDT) {
        const uint32_t f = f0 + threadIdx.x;
        bool push = false;
        uint32_t w = 0;
        if (f < hi) {
            const uint2 va = A.da_out[f];
            w = va.x;
            if (va.y <= A.tw && w != A.src)
                push = sd_lower(A.pm, A.o2i[f], va.y - A.t_out[f], dlo, dhi, w) && w < A.n_live;
        }
        const unsigned long long bal[1] = {__ballot(push)};
        const uint32_t item[1] = {w};
        stage_append<SD_SCAP, 1>(S, bal, item);
    }
    stage_flush_block<SD_SCAP, SDT / 64>(S);
}

// One lane per frontier vertex v: prefix minimum of pm over v's dirty
// range, then the values past it up to `stop` set to the range's last
// minimum, then the range of v's out-edges whose candidate can have changed.
// A lane scans at most SD_LANE and fills at most SD_LANE_FILL positions
// itself; longer scans and fills are taken by the whole wavefront, one
// vertex at a time.  A dirty range longer than SD_BIG is left whole to
// sd_expand_big_kernel: its index goes to `big` and rng[i] carries
// {v, hi, 0, lo}.
__global__ __launch_bounds__(SDT) void sd_expand_kernel(SDArgs A, const uint32_t *__restrict__ cur,
                                                        const uint32_t *F_p, uint32_t *dlo, uint32_t *dhi,
                                                        uint4 *rng, uint32_t *lens, uint32_t *cnt_next,
                                                        uint32_t *big, uint32_t *big_cnt)
{
    const uint32_t F = min(*F_p, A.n);
    if (blockIdx.x == 0 && threadIdx.x == 0) *cnt_next = 0u;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t stride = gridDim.x * SDT;
    for (uint32_t i0 = blockIdx.x * SDT + (threadIdx.x & ~63u); i0 < F; i0 += stride) {
        const uint32_t i = i0 + lane;
        const bool act = i < F;
        // the dirty range, cleaned for the round after next (the
        // relaxations of this round write the other parity)
        uint32_t v = 0, p = 0, hi = 0;
        if (act) {
            v = cur[i];
            p = dlo[v];
            hi = dhi[v];
            dlo[v] = INF;
            dhi[v] = 0u;
        }
        const bool isbig = act && hi - p >= SD_BIG;
        const unsigned long long bb = __ballot(isbig);
        if (bb) {
            uint32_t at = 0;
            if (lane == 0) at = atomicAdd(big_cnt, (uint32_t)__popcll(bb));
            at = __shfl(at, 0);
            if (isbig) {
                rng[i] = make_uint4(v, hi, 0u, p);
                big[at + __popcll(bb & lanes_below())] = i;
            }
        }
        const bool mine = act && !isbig;
        uint32_t end = 0, carry = INF;
        if (mine) {
            end = A.off_in[v + 1];
            if (p > A.off_in[v]) carry = A.pm[p - 1];
        }
        const bool lane_scan = mine && hi - p < SD_LANE;
        if (lane_scan) {
            for (uint32_t k = p; k <= hi; ++k) {
                const uint32_t old = A.pm[k];
                if (old < carry)
                    carry = old;
                else if (old != carry)
                    A.pm[k] = carry;
            }
        }
        for (unsigned long long m = __ballot(mine && !lane_scan); m; m &= m - 1) {
            const int l = __ffsll((long long)m) - 1;
            const uint32_t pl = __shfl(p, l), hl = __shfl(hi, l);
            uint32_t c = __shfl(carry, l);
            for (uint32_t k0 = pl; k0 <= hl; k0 += 64) {
                const uint32_t k = k0 + lane;
                const uint32_t old = k <= hl ? A.pm[k] : INF;
                uint32_t x = old;
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(x, o);
                    if (lane >= (uint32_t)o) x = min(x, y);
                }
                x = min(x, c);
                if (k <= hl && x != old) A.pm[k] = x;
                c = __shfl(x, 63);
            }
            if (lane == (uint32_t)l) carry = c;
        }
        uint32_t stop = 0;
        if (mine) stop = first_at_most(A.pm, hi + 1, end, carry);
        const bool lane_fill = mine && stop - hi - 1 <= SD_LANE_FILL;
        if (lane_fill)
            for (uint32_t k = hi + 1; k < stop; ++k) A.pm[k] = carry;
        for (unsigned long long m = __ballot(mine && !lane_fill); m; m &= m - 1) {
            const int l = __ffsll((long long)m) - 1;
            const uint32_t h1 = __shfl(hi, l) + 1u, sl = __shfl(stop, l), cl = __shfl(carry, l);
            for (uint32_t k = h1 + lane; k < sl; k += 64) A.pm[k] = cl;
        }
        if (mine) {
            const uint2 oc = changed_out_range(A, v, p, stop, end);
            rng[i] = make_uint4(v, oc.x, oc.y, p);
            lens[i] = oc.y;
        }
    }
}

// One workgroup per long dirty range (listed by sd_expand_kernel): the same
// expansion, the prefix minimum taken tile by tile (SDB * SDB_PER positions
// through LDS, a run of SDB_PER per thread, a block scan of the runs' minima).
__global__ __launch_bounds__(SDB) void sd_expand_big_kernel(SDArgs A, const uint32_t *__restrict__ big,
                                                            const uint32_t *__restrict__ big_cnt, uint4 *rng,
                                                            uint32_t *lens)
{
    constexpr uint32_t TILE = SDB * SDB_PER;
    __shared__ uint32_t s_old[TILE];
    __shared__ uint32_t s_new[TILE];
    __shared__ uint32_t s_w[SDB / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t nb = *big_cnt;
    for (uint32_t j = blockIdx.x; j < nb; j += gridDim.x) {
        const uint32_t i = big[j];
        const uint4 r = rng[i];
        const uint32_t v = r.x, hi = r.y, p = r.w;
        const uint32_t end = A.off_in[v + 1];
        uint32_t carry = p > A.off_in[v] ? A.pm[p - 1] : INF;
        for (uint32_t k0 = p; k0 <= hi; k0 += TILE) {
            const uint32_t cnt = min(TILE, hi + 1 - k0);
            for (uint32_t q = tid; q < TILE; q += SDB) s_old[q] = q < cnt ? A.pm[k0 + q] : INF;
            __syncthreads();
            uint32_t run[SDB_PER];
            uint32_t m = INF;
#pragma unroll
            for (int c = 0; c < SDB_PER; ++c) {
                run[c] = s_old[tid * SDB_PER + c];
                m = min(m, run[c]);
            }
            // inclusive min-scan of the runs' minima over the wavefront
            uint32_t x = m;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o);
                if (lane >= (uint32_t)o) x = min(x, y);
            }
            if (lane == 63) s_w[w] = x;
            uint32_t ex = __shfl_up(x, 1);
            if (lane == 0) ex = INF;
            __syncthreads();
            uint32_t pre = carry, tot = carry;
            for (uint32_t w2 = 0; w2 < SDB / 64; ++w2) {
                if (w2 < w) pre = min(pre, s_w[w2]);
                tot = min(tot, s_w[w2]);
            }
            pre = min(pre, ex);
#pragma unroll
            for (int c = 0; c < SDB_PER; ++c) {
                pre = min(pre, run[c]);
                s_new[tid * SDB_PER + c] = pre;
            }
            __syncthreads();
            for (uint32_t q = tid; q < cnt; q += SDB)
                if (s_new[q] != s_old[q]) A.pm[k0 + q] = s_new[q];
            carry = tot;
            __syncthreads();  // the next tile reuses s_old, s_new and s_w
        }
        const uint32_t stop = first_at_most(A.pm, hi + 1, end, carry);
        __syncthreads();  // every wavefront has searched before any fills
        for (uint32_t k = hi + 1 + tid; k < stop; k += SDB) A.pm[k] = carry;
        const uint2 oc = changed_out_range(A, v, p, stop, end);
        if (tid == 0) {
            rng[i] = make_uint4(v, oc.x, oc.y, p);
            lens[i] = oc.y;
        }
    }
}

// One thread per out-edge of the ranges, SD_U of them per lane per pass (a
// wavefront takes 64 * SD_U consecutive edges and issues each step's loads
// for all of them before using any): candidate D_v(t) + lambda into the
// head's in-list position.  The range holding a wavefront's first edge comes
// from one search over the scanned range lengths; each edge's range is then
// found among the next 64 range starts (a search over the lanes), or, past
// them (runs of empty or short ranges), by a search of its own.
__global__ __launch_bounds__(SDT) void sd_relax_kernel(SDArgs A, const uint32_t *__restrict__ F_p,
                                                       const uint32_t *__restrict__ base,
                                                       const uint4 *__restrict__ rng,
                                                       const uint32_t *__restrict__ total_p, uint32_t *dlo,
                                                       uint32_t *dhi, uint32_t *next, uint32_t *cnt,
                                                       uint32_t *big_cnt)
{
    // the long-range list is consumed; the next round's expansion refills it
    if (blockIdx.x == 0 && threadIdx.x == 0) *big_cnt = 0u;
    __shared__ uint32_t s_stage[SDT / 64][SD_SCAP];
    SDStage S{s_stage[threadIdx.x >> 6], 0u, next, cnt};
    const uint32_t F = min(*F_p, A.n);
    const uint32_t total = *total_p;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t stride = (uint64_t)gridDim.x * SDT * SD_U;
    for (uint64_t jw64 = (uint64_t)(blockIdx.x * SDT + (threadIdx.x & ~63u)) * SD_U; jw64 < total; jw64 += stride) {
        const uint32_t jw = (uint32_t)jw64;
        const uint32_t i0 = upper_bound_t(base, 0, F, jw) - 1u;
        const uint32_t nb = i0 + 1 + lane < F ? base[i0 + 1 + lane] : INF;
        const uint32_t y63 = __shfl(nb, 63);
        uint32_t j[SD_U], ri[SD_U];
        bool act[SD_U];
#pragma unroll
        for (int u = 0; u < SD_U; ++u) {
            j[u] = jw + (uint32_t)u * 64u + lane;
            act[u] = jw64 + (uint64_t)u * 64u + lane < total;
            // how many of the 64 starts after i0's are <= j (they ascend)
            uint32_t pos = 0;
            for (uint32_t step = 32; step > 0; step >>= 1) {
                const uint32_t y = __shfl(nb, (int)(pos + step - 1));
                if (y <= j[u]) pos += step;
            }
            if (pos == 63 && y63 <= j[u]) pos = 64;
            ri[u] = i0 + pos;
            if (act[u] && pos == 64) ri[u] = upper_bound_t(base, i0 + 65, F, j[u]) - 1u;
        }
        uint32_t f[SD_U], rb[SD_U];
#pragma unroll
        for (int u = 0; u < SD_U; ++u) {
            f[u] = act[u] ? rng[ri[u]].y : 0u;
            rb[u] = act[u] ? base[ri[u]] : 0u;
        }
        uint2 va[SD_U];
        uint32_t t[SD_U], k[SD_U], oi[SD_U];
#pragma unroll
        for (int u = 0; u < SD_U; ++u) {
            f[u] += j[u] - rb[u];
            va[u] = make_uint2(0u, 0u);
            t[u] = k[u] = oi[u] = 0u;
            if (act[u]) {
                va[u] = A.da_out[f[u]];
                t[u] = A.t_out[f[u]];
                k[u] = A.o2k[f[u]];
                oi[u] = A.o2i[f[u]];
            }
        }
        bool ok[SD_U];
        uint32_t d[SD_U], old[SD_U];
#pragma unroll
        for (int u = 0; u < SD_U; ++u) {
            ok[u] = act[u] && va[u].y <= A.tw && va[u].x != A.src;
            // last in-edge of v arriving by t (before t when strict); the
            // range's departures lie in [a_lo, a_stop) (+1 when strict), so
            // that edge lies in [lo, stop)
            if (ok[u] && A.strict)
                while (A.a_in[k[u]] == t[u]) --k[u];
            d[u] = ok[u] ? A.pm[k[u]] : INF;
            old[u] = ok[u] ? A.pm[oi[u]] : 0u;
        }
        // the label at oi has one writer per round (its edge), so a plain
        // store lowers it
        uint32_t w[SD_U];
        unsigned long long bal[SD_U];
#pragma unroll
        for (int u = 0; u < SD_U; ++u) {
            w[u] = va[u].x;
            bool push = false;
            if (ok[u] && d[u] != INF) {
                const uint32_t cand = d[u] + (va[u].y - t[u]);
                if (cand < old[u]) {
                    A.pm[oi[u]] = cand;
                    push = sd_mark(dlo, dhi, w[u], oi[u]) && w[u] < A.n_live;
                }
            }
            bal[u] = __ballot(push);
        }
        stage_append<SD_SCAP, SD_U>(S, bal, w);
    }
    stage_flush_block<SD_SCAP, SDT / 64>(S);
}

// out[c] for caller vertex c: 0 at the source, else the least label over
// its in-list (INF when none): the last label of an expanded (non-increasing)
// list, i.e. of every vertex with out-edges; a minimum over the list for the
// others, by the lane itself for short lists and by the whole wavefront for
// lists longer than 32.
__global__ __launch_bounds__(SDT) void sd_output_kernel(const uint32_t *__restrict__ off_in,
                                                        const uint32_t *__restrict__ pm,
                                                        const uint32_t *__restrict__ perm, uint32_t n,
                                                        uint32_t n_live, uint32_t src, uint32_t *__restrict__ out)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t stride = gridDim.x * SDT;
    for (uint32_t c0 = blockIdx.x * SDT + (threadIdx.x & ~63u); c0 < n; c0 += stride) {
        const uint32_t c = c0 + lane;
        uint32_t x = INF, b = 0, e = 0;
        bool scan = false;
        if (c < n) {
            const uint32_t v = perm[c];
            b = off_in[v];
            e = off_in[v + 1];
            if (v == src) {
                x = 0u;
            } else if (v < n_live) {
                if (e > b) x = pm[e - 1];
            } else if (e - b <= 32) {
                for (uint32_t k = b; k < e; ++k) x = min(x, pm[k]);
            } else {
                scan = true;
            }
        }
        for (unsigned long long m = __ballot(scan); m; m &= m - 1) {
            const int l = __ffsll((long long)m) - 1;
            const uint32_t bl = __shfl(b, l), el = __shfl(e, l);
            uint32_t y = INF;
            for (uint32_t k = bl + lane; k < el; k += 64) y = min(y, pm[k]);
            for (int o = 32; o > 0; o >>= 1) y = min(y, (uint32_t)__shfl_xor(y, o));
            if (lane == (uint32_t)l) x = y;
        }
        if (c < n) out[c] = x;
    }
}

uint32_t grid_for(uint64_t items, uint32_t per_block, uint32_t cap)
{
    const uint64_t b = (items + per_block - 1) / per_block;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, cap));
}

void sd_state_free(SDState *s)
{
    if (!s) return;
    if (s->stream) hipStreamSynchronize(s->stream);
    dev_free(s->pm);
    for (int k = 0; k < 2; ++k) {
        dev_free(s->dlo[k]);
        dev_free(s->dhi[k]);
        dev_free(s->queue[k]);
    }
    dev_free(s->rng);
    dev_free(s->big);
    dev_free(s->base);
    dev_free(s->bsum);
    dev_free(s->cnt);
    if (s->h_pin) hipHostFree(s->h_pin);
    if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
    delete s;
}

int sd_state_alloc(kairos_graph *g, SDState **out)
{
    SDState *s = new SDState();
    const size_t n = g->n, m = std::max<uint64_t>(g->m, 1);
    bool ok = (s->pm = (uint32_t *)dev_alloc(m * 4, nullptr)) != nullptr;
    for (int k = 0; k < 2; ++k) {
        ok = ok && (s->dlo[k] = (uint32_t *)dev_alloc(n * 4, nullptr)) != nullptr;
        ok = ok && (s->dhi[k] = (uint32_t *)dev_alloc(n * 4, nullptr)) != nullptr;
        ok = ok && (s->queue[k] = (uint32_t *)dev_alloc(n * 4, nullptr)) != nullptr;
    }
    ok = ok && (s->rng = (uint4 *)dev_alloc(n * sizeof(uint4), nullptr)) != nullptr;
    ok = ok && (s->big = (uint32_t *)dev_alloc(n * 4, nullptr)) != nullptr;
    ok = ok && (s->base = (uint32_t *)dev_alloc((n + 1) * 4, nullptr)) != nullptr;
    ok = ok && (s->bsum = (uint32_t *)dev_alloc(scan_scratch_words(n) * 4, nullptr)) != nullptr;
    ok = ok && (s->cnt = (uint32_t *)dev_alloc(SD_CNT_WORDS * 4, nullptr)) != nullptr;
    if (ok && hipHostMalloc((void **)&s->h_pin, SD_CNT_WORDS * 4, hipHostMallocDefault) != hipSuccess) {
        s->h_pin = nullptr;
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
    if (!ok) {
        sd_state_free(s);
        return KAIROS_ERR_NOMEM;
    }
    *out = s;
    return KAIROS_OK;
}

// The out-edge -> in-edge position maps, built once per graph.
int ensure_o2i(kairos_graph *g, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g->sd_mu);
    if (g->o2i) return KAIROS_OK;
    uint32_t *o2i = (uint32_t *)dev_alloc(std::max<uint64_t>(g->m, 1) * 4, nullptr);
    uint32_t *o2k = (uint32_t *)dev_alloc(std::max<uint64_t>(g->m, 1) * 4, nullptr);
    uint32_t *err = (uint32_t *)dev_alloc(4, nullptr);
    if (!o2i || !o2k || !err) {
        dev_free(o2i);
        dev_free(o2k);
        dev_free(err);
        return KAIROS_ERR_NOMEM;
    }
    if (g->m > 0) {
        uint32_t h_err = 0;
        hipLaunchKernelGGL(sd_fill_kernel, dim3(1), dim3(SDT), 0, st, err, (uint64_t)1, 0u);
        hipLaunchKernelGGL(o2i_kernel, dim3(grid_for(g->n_live, SDT / 64, (uint32_t)g->num_cus * 16)), dim3(SDT), 0,
                           st, g->off_out, g->t_out, g->da_out, g->off_in, g->a_in, g->st_in, g->n_live, o2i, o2k,
                           err);
        if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&h_err, err, 4, hipMemcpyDeviceToHost, st) !=
                                                    hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess || h_err != 0) {
            dev_free(o2i);
            dev_free(o2k);
            dev_free(err);
            return KAIROS_ERR_DEVICE;
        }
    }
    dev_free(err);
    g->o2i = o2i;
    g->o2k = o2k;
    g->sd_map_bytes = std::max<uint64_t>(g->m, 1) * 8;
    return KAIROS_OK;
}

int run_sd(kairos_graph *g, SDState *s, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out, bool strict)
{
    hipStream_t st = s->stream;
    const uint32_t n = g->n;
    const uint32_t src_i = g->h_perm[src];
    const uint32_t cap = (uint32_t)g->num_cus * 16;
    SDArgs A{};
    A.off_out = g->off_out;
    A.t_out = g->t_out;
    A.da_out = g->da_out;
    A.off_in = g->off_in;
    A.a_in = g->a_in;
    A.o2i = g->o2i;
    A.o2k = g->o2k;
    A.pm = s->pm;
    A.n = n;
    A.n_live = g->n_live;
    A.max_t = g->max_t;
    A.src = src_i;
    A.ta = ta;
    A.tw = tw;
    A.strict = strict ? 1u : 0u;
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    const uint64_t m = std::max<uint64_t>(g->m, 1);
    hipLaunchKernelGGL(sd_fill_kernel, dim3(grid_for(m, SDT, cap * 4)), dim3(SDT), 0, st, s->pm, m, INF);
    for (int k = 0; k < 2; ++k) {
        hipLaunchKernelGGL(sd_fill_kernel, dim3(grid_for(n, SDT, cap)), dim3(SDT), 0, st, s->dlo[k], (uint64_t)n, INF);
        hipLaunchKernelGGL(sd_fill_kernel, dim3(grid_for(n, SDT, cap)), dim3(SDT), 0, st, s->dhi[k], (uint64_t)n, 0u);
    }
    hipLaunchKernelGGL(sd_fill_kernel, dim3(1), dim3(SDT), 0, st, s->cnt, (uint64_t)SD_CNT_WORDS, 0u);
    prof_end(g, st, KAIROS_K_INIT, ev);
    KAIROS_HIP(hipGetLastError());
    if (g->m > 0 && src_i < g->n_live) {
        const uint32_t deg = g->max_out_degree;
        prof_begin(g, st, &ev);
        hipLaunchKernelGGL(sd_seed_kernel, dim3(grid_for(deg, SDT, cap)), dim3(SDT), 0, st, A, s->dlo[0], s->dhi[0],
                           s->queue[0], s->cnt + SD_FRONT);
        prof_end(g, st, KAIROS_K_PUSH, ev);
        KAIROS_HIP(hipGetLastError());
        KAIROS_HIP(hipMemcpyAsync(s->h_pin, s->cnt, SD_CNT_WORDS * 4, hipMemcpyDeviceToHost, st));
        KAIROS_HIP(hipStreamSynchronize(st));
        uint32_t F = s->h_pin[SD_FRONT];
        uint32_t r = 0;
        uint64_t items = 0, edges = 0;
        const uint32_t big_grid = (uint32_t)g->num_cus * 2;  // two 1024-thread workgroups per CU
        const uint32_t egrid = grid_for(n, SDT, 2 * cap);   // a lane per frontier vertex
        // rounds queued per host check; a round whose frontier is empty
        // ends at once, and so do the queued ones after it (with work
        // counters on, every round is checked, for exact counts)
        const uint32_t R = g->prof.on ? 1u : std::max<uint32_t>(1, g->tuning.rounds_per_sync);
        while (F > 0) {
            if (F > n) return KAIROS_ERR_DEVICE;  // a vertex is enqueued at most once per round
            items += F;
            for (uint32_t k = 0; k < R; ++k, ++r) {
                const uint32_t p = r & 1u, q = p ^ 1u;
                uint32_t *Fp = s->cnt + SD_FRONT + p;
                prof_begin(g, st, &ev);
                hipLaunchKernelGGL(sd_expand_kernel, dim3(egrid), dim3(SDT), 0, st, A, s->queue[p], Fp, s->dlo[p],
                                   s->dhi[p], s->rng, s->base, s->cnt + SD_FRONT + q, s->big, s->cnt + SD_BIG_CNT);
                hipLaunchKernelGGL(sd_expand_big_kernel, dim3(big_grid), dim3(SDB), 0, st, A, s->big,
                                   s->cnt + SD_BIG_CNT, s->rng, s->base);
                exclusive_scan_dev(st, s->base, n, Fp, s->bsum, s->cnt + SD_TOTAL);
                hipLaunchKernelGGL(sd_relax_kernel, dim3(2 * cap), dim3(SDT), 0, st, A, Fp, s->base, s->rng,
                                   s->cnt + SD_TOTAL, s->dlo[q], s->dhi[q], s->queue[q], s->cnt + SD_FRONT + q,
                                   s->cnt + SD_BIG_CNT);
                prof_end(g, st, KAIROS_K_PUSH, ev);
                KAIROS_HIP(hipGetLastError());
            }
            KAIROS_HIP(hipMemcpyAsync(s->h_pin, s->cnt, SD_CNT_WORDS * 4, hipMemcpyDeviceToHost, st));
            KAIROS_HIP(hipStreamSynchronize(st));
            edges += s->h_pin[SD_TOTAL];  // the last queued round's (every round's when R = 1)
            F = s->h_pin[SD_FRONT + (r & 1u)];
        }
        if (g->prof.on) {
            std::lock_guard<std::mutex> lk(g->prof.mu);
            g->prof.rounds += r;
            g->prof.items += items;  // vertices expanded
            g->prof.edges += edges;  // out-edges relaxed
        }
    }
    prof_begin(g, st, &ev);
    hipLaunchKernelGGL(sd_output_kernel, dim3(grid_for(n, SDT, cap * 4)), dim3(SDT), 0, st, g->off_in, s->pm,
                       g->perm, n, g->n_live, src_i, out);
    prof_end(g, st, KAIROS_K_INIT, ev);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

}  // namespace

int run_shortest_duration(kairos_graph *g, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out, bool strict)
{
    SDState *s = nullptr;
    {
        std::lock_guard<std::mutex> lk(g->pool_mu);
        if (!g->sd_states.empty()) {
            s = g->sd_states.back();
            g->sd_states.pop_back();
        }
    }
    int rc = s ? KAIROS_OK : sd_state_alloc(g, &s);
    if (rc) return rc;
    rc = ensure_o2i(g, s->stream);
    if (rc == KAIROS_OK) rc = run_sd(g, s, src, ta, tw, out, strict);
    if (rc == KAIROS_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = KAIROS_ERR_DEVICE;
    if (rc == KAIROS_OK) {
        std::lock_guard<std::mutex> lk(g->pool_mu);
        g->sd_states.push_back(s);
    } else {
        sd_state_free(s);
    }
    return rc;
}

void release_duration_state(kairos_graph *g)
{
    for (SDState *s : g->sd_states) sd_state_free(s);
    g->sd_states.clear();
    dev_free(g->o2i);
    dev_free(g->o2k);
    g->o2i = nullptr;
    g->o2k = nullptr;
    g->sd_map_bytes = 0;
}

}  // namespace kairos
