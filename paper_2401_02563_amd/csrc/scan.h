// Exclusive prefix sum of a device array of uint32 words, in three launches
// (block scans, a one-block scan of the block totals, block offsets added),
// with the grand total written to a device word.  Shared by the kernels
// that turn per-item counts into output positions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kairos {
namespace {

constexpr int XSCAN_T = 256;                     // threads per block scan
constexpr int XSCAN_PER = 4;                     // entries per thread
constexpr int XSCAN_BLK = XSCAN_T * XSCAN_PER;  // entries per block
constexpr int XSCAN_TOP = 1024;                  // threads of the top-level scan

// Exclusive scan of `count` words, XSCAN_BLK per block; block totals to bsum.
// With count_p, the count is min(count, *count_p) (a device value bounded
// by the host's count, which sizes the grid).
__global__ __launch_bounds__(XSCAN_T) void xscan_block_kernel(uint32_t *data, uint32_t count, uint32_t *bsum,
                                                              const uint32_t *count_p = nullptr)
{
    if (count_p) count = min(count, *count_p);
    __shared__ uint32_t s_w[XSCAN_T / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t b0 = blockIdx.x * XSCAN_BLK + tid * XSCAN_PER;
    uint32_t v[XSCAN_PER];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < XSCAN_PER; ++j) {
        v[j] = b0 + j < count ? data[b0 + j] : 0u;
        s += v[j];
    }
    uint32_t x = s;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (uint32_t k = 0; k < XSCAN_T / 64; ++k) {
        if (k < w) off += s_w[k];
        tot += s_w[k];
    }
    uint32_t run = off + x - s;
#pragma unroll
    for (int j = 0; j < XSCAN_PER; ++j) {
        if (b0 + j < count) data[b0 + j] = run;
        run += v[j];
    }
    if (tid == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of the nb block totals in one block; the grand total to
// *total.
__global__ __launch_bounds__(XSCAN_TOP) void xscan_top_kernel(uint32_t *bsum, uint32_t nb, uint32_t *total,
                                                               const uint32_t *count_p = nullptr)
{
    __shared__ uint32_t part[XSCAN_TOP];
    if (count_p) nb = min(nb, (*count_p + XSCAN_BLK - 1) / XSCAN_BLK);
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (nb + XSCAN_TOP - 1) / XSCAN_TOP;
    const uint32_t beg = min(nb, tid * per), end = min(nb, beg + per);
    uint32_t s = 0;
    for (uint32_t i = beg; i < end; ++i) s += bsum[i];
    part[tid] = s;
    __syncthreads();
    for (uint32_t o = 1; o < XSCAN_TOP; o <<= 1) {
        const uint32_t y = tid >= o ? part[tid - o] : 0u;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    uint32_t run = part[tid] - s;
    for (uint32_t i = beg; i < end; ++i) {
        const uint32_t y = bsum[i];
        bsum[i] = run;
        run += y;
    }
    if (tid == XSCAN_TOP - 1) *total = part[XSCAN_TOP - 1];
}

__global__ __launch_bounds__(XSCAN_T) void xscan_add_kernel(uint32_t *data, uint32_t count, const uint32_t *bsum,
                                                            const uint32_t *count_p = nullptr)
{
    if (count_p) count = min(count, *count_p);
    if ((uint64_t)blockIdx.x * XSCAN_BLK >= count) return;
    const uint32_t add = bsum[blockIdx.x];
    const uint32_t b0 = blockIdx.x * XSCAN_BLK;
    for (uint32_t j = threadIdx.x; j < XSCAN_BLK; j += XSCAN_T)
        if (b0 + j < count) data[b0 + j] += add;
}

// Words of block-total scratch for a scan of `count` entries.
inline uint64_t scan_scratch_words(uint64_t count) { return count / XSCAN_BLK + 2; }

// In place: data[i] = sum of data[0..i); *total = sum of all (device word).
// bsum: scan_scratch_words(count) device words.  count == 0 writes 0.
inline void exclusive_scan(hipStream_t st, uint32_t *data, uint32_t count, uint32_t *bsum, uint32_t *total)
{
    const uint32_t nb = (count + XSCAN_BLK - 1) / XSCAN_BLK;
    if (nb) hipLaunchKernelGGL(xscan_block_kernel, dim3(nb), dim3(XSCAN_T), 0, st, data, count, bsum, nullptr);
    hipLaunchKernelGGL(xscan_top_kernel, dim3(1), dim3(XSCAN_TOP), 0, st, bsum, nb, total, nullptr);
    if (nb > 1) hipLaunchKernelGGL(xscan_add_kernel, dim3(nb), dim3(XSCAN_T), 0, st, data, count, bsum, nullptr);
}

// As exclusive_scan over the first *count_p (device) of at most max_count
// entries; the grid is sized for max_count.
inline void exclusive_scan_dev(hipStream_t st, uint32_t *data, uint32_t max_count, const uint32_t *count_p,
                               uint32_t *bsum, uint32_t *total)
{
    const uint32_t nb = (max_count + XSCAN_BLK - 1) / XSCAN_BLK;
    if (nb) hipLaunchKernelGGL(xscan_block_kernel, dim3(nb), dim3(XSCAN_T), 0, st, data, max_count, bsum, count_p);
    hipLaunchKernelGGL(xscan_top_kernel, dim3(1), dim3(XSCAN_TOP), 0, st, bsum, nb, total, count_p);
    if (nb > 1)
        hipLaunchKernelGGL(xscan_add_kernel, dim3(nb), dim3(XSCAN_T), 0, st, data, max_count, bsum, count_p);
}

}  // namespace
}  // namespace kairos
