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

// Per-wavefront output buffer of CAP entries in LDS.  `n` is wave-uniform.
template <int CAP>
struct Stage {
    uint32_t *buf;       // this wavefront's CAP entries
    uint32_t n;          // entries held
    uint32_t *next;      // global frontier array
    uint32_t *next_cnt;  // its length counter
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
    for (uint32_t j = lane; j < S.n; j += 64) S.next[base + j] = S.buf[j];
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
    for (uint32_t j = lane; j < S.n; j += 64) S.next[off + j] = S.buf[j];
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

}  // namespace kairos
