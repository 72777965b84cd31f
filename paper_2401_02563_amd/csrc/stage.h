// Device helpers shared by the traversal kernels: LDS-staged frontier output
// and block-reduced work counters.
//
// Device-scope atomics on one address are executed one after another at the
// memory side, roughly 11 ns apiece on gfx950 (measured), while atomics on
// different addresses proceed in parallel.  A frontier counter bumped once per
// wavefront per edge group, or a work counter bumped by every wavefront at
// kernel exit, therefore costs tens of microseconds per round on its own.
// Frontier entries are instead collected per wavefront in LDS and written out
// with one global atomicAdd per flush (a full buffer, or the whole block at
// kernel exit), and work counters are summed per block and added to one of
// ST_SHARDS copies chosen by block index.
#pragma once

#include "internal.h"

namespace kairos {

// Orders LDS accesses of the lanes of one wavefront: what one lane wrote
// before the call is seen by every lane after it.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t lanes_below()
{
    const uint32_t lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// One step of a key-gated inclusive min-scan over the wavefront: mv takes
// the minimum with the value of the lane CTRL names (a DPP row shift or row
// broadcast, rows ROWS written) when that lane holds the same key.  Lanes
// without a source lane get the identity.
template <int CTRL, int ROWS>
__device__ __forceinline__ void gated_min_step(uint32_t &mv, uint32_t key)
{
    const uint32_t ms = (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)mv, CTRL, ROWS, 0xF, false);
    const uint32_t ks = (uint32_t)__builtin_amdgcn_update_dpp((int)key, (int)key, CTRL, ROWS, 0xF, false);
    if (ks == key) mv = min(mv, ms);
}

// gated_min_step with a 64-bit key given as two halves.
template <int CTRL, int ROWS>
__device__ __forceinline__ void gated_min_step2(uint32_t &mv, uint32_t klo, uint32_t khi)
{
    const uint32_t ms = (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)mv, CTRL, ROWS, 0xF, false);
    const uint32_t sl = (uint32_t)__builtin_amdgcn_update_dpp((int)klo, (int)klo, CTRL, ROWS, 0xF, false);
    const uint32_t sh = (uint32_t)__builtin_amdgcn_update_dpp((int)khi, (int)khi, CTRL, ROWS, 0xF, false);
    if (sl == klo && sh == khi) mv = min(mv, ms);
}

// Lanes of a wavefront that hold edges into the same (query, vertex) slot
// in a row -- a burst of one tail's adjacency -- need one atomic between
// them: a segmented minimum over each run leaves the run's least arrival in
// its last lane and drops the others' edges (none of them can beat it).
// `key` is the slot; a lane without an edge is a run of its own.  The
// minimum is the key-gated DPP scan of dedupe_runs32 below on the two
// halves of the key (a window may also take in an earlier run into the same
// slot, which only lowers the survivor to another of this group's arrivals
// for it).  Every lane of the wavefront must call this; without runs
// longer than one lane it returns after two ballots.
__device__ __forceinline__ void dedupe_runs(bool &ok, uint32_t &a, uint64_t key)
{
    // most edge groups improve nothing (their arrivals are not below the
    // heads' words): one ballot settles those
    const uint64_t m = __ballot(ok);
    if (m == 0ull) return;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t klo = (uint32_t)key, khi = (uint32_t)(key >> 32);
    const uint32_t dlo = __shfl_down(klo, 1), dhi = __shfl_down(khi, 1);
    const bool ok_dn = lane < 63 && ((m >> (lane + 1)) & 1ull);
    const bool last = !ok_dn || dlo != klo || dhi != khi;
    if (__ballot(ok && !last) == 0ull) return;  // no run longer than one lane
    uint32_t mv = ok ? a : 0xFFFFFFFFu;
    gated_min_step2<0x111, 0xF>(mv, klo, khi);  // row_shr:1
    gated_min_step2<0x112, 0xF>(mv, klo, khi);  // row_shr:2
    gated_min_step2<0x114, 0xF>(mv, klo, khi);  // row_shr:4
    gated_min_step2<0x118, 0xF>(mv, klo, khi);  // row_shr:8
    gated_min_step2<0x142, 0xA>(mv, klo, khi);  // row_bcast:15
    gated_min_step2<0x143, 0xC>(mv, klo, khi);  // row_bcast:31
    if (ok) {
        if (last)
            a = mv;
        else
            ok = false;
    }
}

// dedupe_runs for lanes that all relax edges of one query: the slot is the
// 32-bit head id.  A run is a maximal stretch of neighbouring lanes that
// have an edge and the same head; its last lane keeps the least arrival of
// the run and the run's other lanes drop their edges.  The minimum is a
// scan gated by key equality (DPP shifts by 1, 2, 4, 8 inside rows of 16
// lanes, then the last lane of a row to the next row and lane 31 to rows 2
// and 3): a run is contiguous, so its last lane's window covers the whole
// run; it may also take in an earlier run into the same head, which only
// lowers the survivor's value to another arrival of this group for that
// head.  Every lane of the wavefront must call this.
__device__ __forceinline__ void dedupe_runs32(bool &ok, uint32_t &a, uint32_t key)
{
    const uint64_t m = __ballot(ok);
    if (m == 0ull) return;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t dn = __shfl_down(key, 1);
    const bool ok_dn = lane < 63 && ((m >> (lane + 1)) & 1ull);
    const bool last = !ok_dn || dn != key;
    if (__ballot(ok && !last) == 0ull) return;  // no run longer than one lane
    uint32_t mv = ok ? a : 0xFFFFFFFFu;
    gated_min_step<0x111, 0xF>(mv, key);  // row_shr:1
    gated_min_step<0x112, 0xF>(mv, key);  // row_shr:2
    gated_min_step<0x114, 0xF>(mv, key);  // row_shr:4
    gated_min_step<0x118, 0xF>(mv, key);  // row_shr:8
    gated_min_step<0x142, 0xA>(mv, key);  // row_bcast:15
    gated_min_step<0x143, 0xC>(mv, key);  // row_bcast:31
    if (ok) {
        if (last)
            a = mv;
        else
            ok = false;
    }
}

// Per-wavefront output buffer of CAP entries in LDS.  `n` is wave-uniform.
// Entries past `cap` in the global array are counted but not written (the
// reader sees a length above cap and treats it as an overflow).
template <int CAP>
struct Stage {
    uint32_t *buf;       // this wavefront's CAP entries
    uint32_t n;          // entries held
    uint32_t *next;      // global frontier array
    uint32_t *next_cnt;  // its length counter
    uint32_t cap = 0xFFFFFFFFu;
};

// Writes the buffer out at a range reserved with one atomicAdd.
template <int CAP>
__device__ __forceinline__ void stage_flush_wave(Stage<CAP> &S)
{
    if (S.n == 0) return;
    const uint32_t lane = threadIdx.x & 63;
    wave_sync();
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(S.next_cnt, S.n);
    base = __shfl(base, 0);
    for (uint32_t j = lane; j < S.n; j += 64)
        if (base + j < S.cap) S.next[base + j] = S.buf[j];
    wave_sync();
    S.n = 0;
}

// Appends, for k < K, `item[k]` of every lane whose bit is set in the
// wave-uniform mask bal[k]; the entries of one k keep lane order.
template <int CAP, int K>
__device__ __forceinline__ void stage_append(Stage<CAP> &S, const unsigned long long (&bal)[K],
                                             const uint32_t (&item)[K])
{
    static_assert(K * 64 <= CAP, "a group must fit an empty buffer");
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) total += __popcll(bal[k]);
    if (total == 0) return;
    if (S.n + total > CAP) stage_flush_wave(S);
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t lt = lanes_below();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if ((bal[k] >> lane) & 1ull) S.buf[S.n + __popcll(bal[k] & lt)] = item[k];
        S.n += __popcll(bal[k]);
    }
}

// Kernel exit: every wavefront of the block calls this once; the block's
// remaining entries are written out behind a single atomicAdd.
template <int CAP, int WAVES>
__device__ __forceinline__ void stage_flush_block(Stage<CAP> &S)
{
    __shared__ uint32_t s_n[WAVES];
    __shared__ uint32_t s_base;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = threadIdx.x >> 6;
    wave_sync();
    if (lane == 0) s_n[w] = S.n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < WAVES; ++i) t += s_n[i];
        s_base = t ? atomicAdd(S.next_cnt, t) : 0u;
    }
    __syncthreads();
    uint32_t off = s_base;
    for (uint32_t i = 0; i < w; ++i) off += s_n[i];
    for (uint32_t j = lane; j < S.n; j += 64)
        if (off + j < S.cap) S.next[off + j] = S.buf[j];
    S.n = 0;
}

// Sums per-thread work counters over the block and adds the totals to the
// block's shard of `stats` (ST_SHARDS copies of ST_WORDS words).  Called by
// every thread of the block; no-op when stats is null.
template <int WAVES, int K>
__device__ __forceinline__ void block_stats(unsigned long long *stats, unsigned long long (&v)[K],
                                            const int (&slot)[K])
{
    if (!stats) return;
    __shared__ unsigned long long s_red[WAVES][K];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
        if (lane == 0) s_red[w][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < (uint32_t)K) {
        unsigned long long t = 0;
        for (int i = 0; i < WAVES; ++i) t += s_red[i][threadIdx.x];
        if (t) atomicAdd(&stats[(blockIdx.x % ST_SHARDS) * ST_WORDS + slot[threadIdx.x]], t);
    }
}

// Grid-wide barrier for a cooperative launch (all blocks resident).  Block b
// arrives on counter b % BAR_GROUPS; the last arrival of a group arrives on
// the top counter, and the last of those bumps the generation word that the
// others wait on.  Counters sit BAR_STRIDE words apart, so arrivals of
// different groups do not queue on one address.  `bar` holds BAR_WORDS
// zeroed words before the launch.  Every block must call this the same
// number of times.  The fences make each block's earlier writes visible to
// every block after the barrier.
//
// The wait is bounded: a block that polls more than `spin_limit` times
// raises the abort word, and every waiting block leaves as soon as it sees
// it.  Callers stop their round loop once grid_aborted() is true, so the
// launch always ends; the host reports the abort as an error.
constexpr uint32_t BAR_GROUPS = 16, BAR_STRIDE = 64;
constexpr size_t BAR_WORDS = (BAR_GROUPS + 3) * BAR_STRIDE;

__device__ __forceinline__ uint32_t *grid_abort_word(uint32_t *bar) { return bar + (BAR_GROUPS + 2) * BAR_STRIDE; }

__device__ __forceinline__ bool grid_aborted(uint32_t *bar)
{
    return __hip_atomic_load(grid_abort_word(bar), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

__device__ __forceinline__ void grid_barrier(uint32_t *bar, uint32_t spin_limit)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t *top = bar + BAR_GROUPS * BAR_STRIDE;
        uint32_t *gen = bar + (BAR_GROUPS + 1) * BAR_STRIDE;
        uint32_t *abort_w = grid_abort_word(bar);
        const uint32_t nb = gridDim.x;
        const uint32_t grp = blockIdx.x % BAR_GROUPS;
        const uint32_t members = (nb - grp + BAR_GROUPS - 1) / BAR_GROUPS;  // blocks b < nb, b % G == grp
        const uint32_t groups = nb < BAR_GROUPS ? nb : BAR_GROUPS;
        // read the generation before arriving: it cannot move until we arrive
        const uint32_t g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();  // release this block's writes; orders the load above before the arrival
        bool last = false;
        uint32_t *gc = bar + grp * BAR_STRIDE;
        if (__hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == members - 1) {
            __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == groups - 1) {
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last = true;
            }
        }
        if (last) {
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // relaxed polls (an acquire per poll would invalidate the cache
            // each time); the fence below is the acquire
            uint32_t polls = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
                if (__hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                if (++polls > spin_limit) {
                    __hip_atomic_store(abort_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __threadfence();  // acquire: later reads see every block's writes
    }
    __syncthreads();
}

}  // namespace kairos
