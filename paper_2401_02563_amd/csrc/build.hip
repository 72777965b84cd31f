// Device builder of the temporal CSR index (paper §4.2).
//
// The paper sorts each high-degree vertex's edges by start time before
// building its interval tree (Alg. 1).  Here every adjacency is kept sorted
// by time instead, in both directions, so a traversal can binary-search the
// first edge it may use.  The whole edge list is sorted at once on the GPU
// by a stable least-significant-digit radix sort on 16-byte records
// {tail, head, t, a}:
//   out-index order (tail, t, a, head); in-index order (head, a, t, tail).
// Because a = t + lambda, ordering by a among equal t is ordering by lambda,
// and ordering by t among equal a is ordering by lambda descending; those
// keys need only as many bits as the spread of lambda (none when lambda is
// constant).  Each pass is histogram -> exclusive scan -> stable scatter,
// with no inter-block waiting.

#include "internal.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

namespace kairos {

namespace {

constexpr int SB = 256;            // threads per sort block
constexpr int SW = SB / 64;        // waves per sort block
constexpr int SK = 8;              // rows of 64 records per wave per tile
constexpr int STILE = SB * SK;     // records per tile
constexpr int SCAN_T = 1024;       // threads of the single-block scan

enum Field : int { F_SRC = 0, F_DST = 1, F_T = 2, F_A = 3, F_LAM = 4, F_LAMREV = 5 };

struct Pass {
    int field;
    int shift;
    int bits;
    uint32_t base;  // lambda offset for F_LAM (min) / F_LAMREV (max)
};

__device__ __forceinline__ uint32_t key_of(const uint4 &e, const Pass &p)
{
    uint32_t k;
    switch (p.field) {
    case F_SRC: k = e.x; break;
    case F_DST: k = e.y; break;
    case F_T: k = e.z; break;
    case F_A: k = e.w; break;
    case F_LAM: k = (e.w - e.z) - p.base; break;
    default: k = p.base - (e.w - e.z); break;
    }
    return (k >> p.shift) & ((1u << p.bits) - 1u);
}

// Validation and packing.  Flags: 1 id out of range, 2 lambda == 0,
// 4 t + lambda beyond the largest finite time.  stats: [0] flags, [1] max t,
// [2] max a, [3] min lambda, [4] max lambda.
__global__ void validate_pack_kernel(const uint32_t *__restrict__ src, const uint32_t *__restrict__ dst,
                                     const uint32_t *__restrict__ t, const uint32_t *__restrict__ lam,
                                     uint64_t m, uint32_t n, uint4 *__restrict__ out,
                                     uint32_t *stats)
{
    uint32_t flags = 0, mt = 0, ma = 0, mnl = 0xFFFFFFFFu, mxl = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t s = src[i], d = dst[i], tt = t[i], l = lam[i];
        uint64_t a = (uint64_t)tt + l;
        if (s >= n || d >= n) flags |= 1u;
        if (l == 0) flags |= 2u;
        if (a > TMAX) flags |= 4u;
        uint32_t a32 = (uint32_t)(a > TMAX ? TMAX : a);
        out[i] = make_uint4(s, d, tt, a32);
        mt = max(mt, tt);
        ma = max(ma, a32);
        mnl = min(mnl, l);
        mxl = max(mxl, l);
    }
    // wave reduction, then one atomic per wave
    for (int o = 32; o > 0; o >>= 1) {
        flags |= __shfl_xor(flags, o);
        mt = max(mt, (uint32_t)__shfl_xor(mt, o));
        ma = max(ma, (uint32_t)__shfl_xor(ma, o));
        mnl = min(mnl, (uint32_t)__shfl_xor(mnl, o));
        mxl = max(mxl, (uint32_t)__shfl_xor(mxl, o));
    }
    if ((threadIdx.x & 63) == 0) {
        if (flags) atomicOr(&stats[0], flags);
        atomicMax(&stats[1], mt);
        atomicMax(&stats[2], ma);
        atomicMin(&stats[3], mnl);
        atomicMax(&stats[4], mxl);
    }
}

__global__ __launch_bounds__(SB) void hist_kernel(const uint4 *__restrict__ in, uint64_t m, Pass p,
                                                  uint32_t *__restrict__ hist, uint32_t tiles_per_block,
                                                  uint32_t nblocks)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    uint64_t beg = (uint64_t)blockIdx.x * tiles_per_block * STILE;
    uint64_t end = min(m, beg + (uint64_t)tiles_per_block * STILE);
    for (uint64_t i = beg + tid; i < end; i += SB)
        atomicAdd(&h[key_of(in[i], p)], 1u);
    __syncthreads();
    if (tid < (1 << p.bits))
        hist[(uint64_t)tid * nblocks + blockIdx.x] = h[tid];
}

// Exclusive scan of `count` words in one block.
__global__ __launch_bounds__(SCAN_T) void scan_kernel(uint32_t *data, uint32_t count)
{
    __shared__ uint32_t part[SCAN_T];
    const int tid = threadIdx.x;
    uint32_t per = (count + SCAN_T - 1) / SCAN_T;
    uint32_t beg = min(count, tid * per), end = min(count, beg + per);
    uint32_t s = 0;
    for (uint32_t i = beg; i < end; ++i) s += data[i];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < SCAN_T; o <<= 1) {
        uint32_t v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = part[tid] - s;
    for (uint32_t i = beg; i < end; ++i) {
        uint32_t v = data[i];
        data[i] = run;
        run += v;
    }
}

// Stable scatter of one digit.  Each block owns a contiguous run of tiles and
// walks them in order.  Inside a tile, wave w owns records
// [w*SK*64, (w+1)*SK*64) and handles them 64 at a time; records of equal
// digit within those 64 are ranked by a ballot match over the digit bits, and
// a per-wave running count per digit carries the rank across rows.  Wave
// prefixes and a tile-wide digit scan then give each record its tile rank;
// records are staged in LDS in digit order and written out in runs.
__global__ __launch_bounds__(SB) void scatter_kernel(const uint4 *__restrict__ in,
                                                     uint4 *__restrict__ out, uint64_t m, Pass p,
                                                     const uint32_t *__restrict__ gscan,
                                                     uint32_t tiles_per_block, uint32_t nblocks)
{
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_wrun[SW][256];
    __shared__ uint32_t s_tstart[256];
    __shared__ uint32_t s_tcount[256];
    __shared__ uint32_t s_wsum[SW];
    __shared__ uint4 s_stage[STILE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const uint32_t nd = 1u << p.bits;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    s_base[tid] = (uint32_t)tid < nd ? gscan[(uint64_t)tid * nblocks + blockIdx.x] : 0u;

    for (uint32_t tile = 0; tile < tiles_per_block; ++tile) {
        const uint64_t tbase = ((uint64_t)blockIdx.x * tiles_per_block + tile) * STILE;
        if (tbase >= m) break;
        const uint32_t tn = (uint32_t)min((uint64_t)STILE, m - tbase);
        for (int k = tid; k < SW * 256; k += SB) (&s_wrun[0][0])[k] = 0u;
        __syncthreads();

        uint4 el[SK];
        uint32_t dg[SK], rk[SK];
#pragma unroll
        for (int j = 0; j < SK; ++j) {
            const uint32_t pos = (uint32_t)w * (SK * 64) + j * 64 + lane;
            const bool valid = pos < tn;
            el[j] = valid ? in[tbase + pos] : make_uint4(0, 0, 0, 0);
            const uint32_t d = valid ? key_of(el[j], p) : 0u;
            uint64_t mask = __ballot(valid);
            for (int b = 0; b < p.bits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                mask &= bit ? bb : ~bb;
            }
            const uint32_t rank = __popcll(mask & lt_mask);
            const uint32_t cnt = __popcll(mask);
            // every lane of the wave reads before the leader writes (lock-step LDS order)
            const uint32_t prev = valid ? s_wrun[w][d] : 0u;
            __builtin_amdgcn_wave_barrier();
            if (valid && rank == 0) s_wrun[w][d] = prev + cnt;
            __builtin_amdgcn_wave_barrier();
            dg[j] = d;
            rk[j] = prev + rank;
        }
        __syncthreads();
        // digit-wise prefix over waves, and tile count per digit
        {
            uint32_t run = 0;
#pragma unroll
            for (int w2 = 0; w2 < SW; ++w2) {
                uint32_t v = s_wrun[w2][tid];
                s_wrun[w2][tid] = run;
                run += v;
            }
            s_tcount[tid] = run;
        }
        __syncthreads();
        // exclusive scan of the 256 tile counts: wave scan + wave sums
        {
            uint32_t v = s_tcount[tid];
            uint32_t x = v;
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane == 63) s_wsum[w] = x;
            __syncthreads();
            uint32_t off = 0;
            for (int w2 = 0; w2 < w; ++w2) off += s_wsum[w2];
            s_tstart[tid] = off + x - v;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < SK; ++j) {
            const uint32_t pos = (uint32_t)w * (SK * 64) + j * 64 + lane;
            if (pos < tn) s_stage[s_tstart[dg[j]] + s_wrun[w][dg[j]] + rk[j]] = el[j];
        }
        __syncthreads();
        for (uint32_t k = tid; k < tn; k += SB) {
            const uint4 e = s_stage[k];
            const uint32_t d = key_of(e, p);
            out[(uint64_t)s_base[d] + (k - s_tstart[d])] = e;
        }
        __syncthreads();
        if ((uint32_t)tid < nd) s_base[tid] += s_tcount[tid];
        __syncthreads();
    }
}

// CSR arrays from records sorted by (key, ...).  which = 0: key = tail,
// writes t_out and {head, a}; which = 1: key = head, writes a_in and {tail, t}.
constexpr uint64_t kShortGap = 64;
constexpr uint32_t OFF_UNSET = 0xFFFFFFFFu;

__global__ void finalize_kernel(const uint4 *__restrict__ e, uint64_t m, uint32_t n, int which,
                                uint32_t *__restrict__ off, uint32_t *__restrict__ tk,
                                uint2 *__restrict__ pair)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 r = e[i];
        const uint32_t key = which == 0 ? r.x : r.y;
        if (which == 0) {
            tk[i] = r.z;
            pair[i] = make_uint2(r.y, r.w);
        } else {
            tk[i] = r.w;
            pair[i] = make_uint2(r.x, r.z);
        }
        // offsets of the keys in (previous key, key] start here.  A short
        // run of keys without records is filled here; a long one (vertices
        // without edges in this direction, which the relabelling can put
        // in one block) is left to gap_offsets_kernel, the keys after the
        // last one to tail_offsets_kernel
        const uint64_t first = i == 0 ? 0 : (uint64_t)(which == 0 ? e[i - 1].x : e[i - 1].y) + 1;
        if (key - first < kShortGap)
            for (uint64_t v = first; v <= key; ++v) off[v] = (uint32_t)i;
        else if (first <= key)
            off[key] = (uint32_t)i;
    }
}

// Offsets still unset (OFF_UNSET) after finalize_kernel: the first record
// whose key is at least v, by binary search over the sorted records.
__global__ void gap_offsets_kernel(const uint4 *__restrict__ e, uint64_t m, uint32_t n, int which,
                                   uint32_t *__restrict__ off)
{
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n;
         v += (uint64_t)gridDim.x * blockDim.x) {
        if (off[v] != OFF_UNSET) continue;
        uint64_t lo = 0, hi = m;
        while (lo < hi) {
            const uint64_t mid = lo + ((hi - lo) >> 1);
            if ((which == 0 ? e[mid].x : e[mid].y) < v)
                lo = mid + 1;
            else
                hi = mid;
        }
        off[v] = (uint32_t)lo;
    }
}

// off[v] = m for every key v after the last record's key (a long run when
// many vertices have no edge in this direction), grid-stride.
__global__ void tail_offsets_kernel(const uint4 *__restrict__ e, uint64_t m, uint32_t n, int which,
                                    uint32_t *__restrict__ off)
{
    const uint64_t last = which == 0 ? e[m - 1].x : e[m - 1].y;
    for (uint64_t v = last + 1 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n;
         v += (uint64_t)gridDim.x * blockDim.x)
        off[v] = (uint32_t)m;
}

__global__ void zero_offsets_kernel(uint32_t *off, uint32_t n)
{
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n;
         v += (uint64_t)gridDim.x * blockDim.x)
        off[v] = 0;
}

__global__ void max_degree_kernel(const uint32_t *__restrict__ off, uint32_t n, uint32_t *out)
{
    uint32_t best = 0;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * blockDim.x)
        best = max(best, off[v + 1] - off[v]);
    for (int o = 32; o > 0; o >>= 1) best = max(best, (uint32_t)__shfl_xor(best, o));
    if ((threadIdx.x & 63) == 0) atomicMax(out, best);
}

// Out-edges whose head equals the previous out-edge's head (runs of one
// pair's edges in a time-sorted adjacency, as in bursty contact data).
__global__ void repeat_heads_kernel(const uint2 *__restrict__ da, uint64_t m, unsigned long long *out)
{
    unsigned long long c = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; e < m;
         e += (uint64_t)gridDim.x * blockDim.x)
        c += da[e].x == da[e - 1].x;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

// Vertex relabelling: vertices with out-edges first, then those without;
// within each part in order of decreasing in-degree (ties by id), so the
// arrival words of the most-targeted heads share cache lines, and whether a
// head has anything to expand is one comparison of its id.
__global__ void indegree_kernel(const uint4 *__restrict__ e, uint64_t m, uint32_t *deg, uint32_t *has_out)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 r = e[i];
        atomicAdd(&deg[r.y], 1u);
        has_out[r.x] = 1u;  // racing stores of the same value
    }
}

// sort key: bit 31 set for a vertex without out-edges, below it the
// in-degree complemented (clamped to 31 bits), so ascending keys give the
// order above
__global__ void vertex_keys_kernel(const uint32_t *__restrict__ deg, const uint32_t *__restrict__ has_out, uint32_t n,
                                   uint4 *out)
{
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t key = (has_out[v] ? 0u : 0x80000000u) | (0x7FFFFFFFu - min(deg[v], 0x7FFFFFFFu));
        out[v] = make_uint4(key, (uint32_t)v, 0u, 0u);
    }
}

// Number of vertices with out-edges: after relabelling they are the ids
// below the first v with off_out[v] == m (one thread, binary search).
__global__ void live_count_kernel(const uint32_t *__restrict__ off_out, uint32_t n, uint32_t m, uint32_t *out)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (off_out[mid] < m)
            lo = mid + 1;
        else
            hi = mid;
    }
    *out = lo;
}

__global__ void perm_kernel(const uint4 *__restrict__ sorted, uint32_t n, uint32_t *perm, uint32_t *inv)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = sorted[i].y;
        perm[v] = (uint32_t)i;
        inv[i] = v;
    }
}

__global__ void remap_kernel(uint4 *e, uint64_t m, const uint32_t *__restrict__ perm)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint4 r = e[i];
        r.x = perm[r.x];
        r.y = perm[r.y];
        e[i] = r;
    }
}

__global__ void identity_perm_kernel(uint32_t n, uint32_t *perm, uint32_t *inv)
{
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x) {
        perm[v] = (uint32_t)v;
        inv[v] = (uint32_t)v;
    }
}

int bits_for(uint64_t x)
{
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

void add_field(std::vector<Pass> &ps, int field, int bits, uint32_t base)
{
    for (int sh = 0; sh < bits; sh += 8) ps.push_back(Pass{field, sh, std::min(8, bits - sh), base});
}

int grid_for(uint64_t work, int per_block, int cap)
{
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (uint64_t)cap) g = cap;
    return (int)g;
}

}  // namespace

int run_passes(kairos_graph *g, uint4 *&a, uint4 *&b, uint64_t m, const std::vector<Pass> &ps,
               uint32_t *hist, hipStream_t st)
{
    const uint64_t tiles = (m + STILE - 1) / STILE;
    const uint32_t nblocks = (uint32_t)std::min<uint64_t>(tiles, 1024);
    const uint32_t tpb = (uint32_t)((tiles + nblocks - 1) / nblocks);
    for (const Pass &p : ps) {
        hipEvent_t ev;
        prof_begin(g, st, &ev);
        hipLaunchKernelGGL(hist_kernel, dim3(nblocks), dim3(SB), 0, st, a, m, p, hist, tpb, nblocks);
        hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(SCAN_T), 0, st, hist,
                           (uint32_t)((1u << p.bits) * nblocks));
        hipLaunchKernelGGL(scatter_kernel, dim3(nblocks), dim3(SB), 0, st, a, b, m, p, hist, tpb,
                           nblocks);
        KAIROS_HIP(hipGetLastError());
        prof_end(g, st, KAIROS_K_SORT, ev);
        std::swap(a, b);
    }
    return KAIROS_OK;
}

int build_index(kairos_graph *g, const uint32_t *src, const uint32_t *dst, const uint32_t *t,
                 const uint32_t *lam, hipStream_t st)
{
    const uint64_t m = g->m;
    const uint32_t n = g->n;
    uint64_t *acct = &g->index_bytes;
    const size_t words = m ? m : 1;
    g->off_out = (uint32_t *)dev_alloc(sizeof(uint32_t) * ((size_t)n + 1), acct);
    g->off_in = (uint32_t *)dev_alloc(sizeof(uint32_t) * ((size_t)n + 1), acct);
    g->t_out = (uint32_t *)dev_alloc(sizeof(uint32_t) * words, acct);
    g->a_in = (uint32_t *)dev_alloc(sizeof(uint32_t) * words, acct);
    g->da_out = (uint2 *)dev_alloc(sizeof(uint2) * words, acct);
    g->st_in = (uint2 *)dev_alloc(sizeof(uint2) * words, acct);
    g->perm = (uint32_t *)dev_alloc(sizeof(uint32_t) * (size_t)n, acct);
    g->inv = (uint32_t *)dev_alloc(sizeof(uint32_t) * (size_t)n, acct);
    if (!g->off_out || !g->off_in || !g->t_out || !g->a_in || !g->da_out || !g->st_in || !g->perm || !g->inv)
        return KAIROS_ERR_NOMEM;
    if (m == 0) {
        hipLaunchKernelGGL(identity_perm_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, n, g->perm, g->inv);
        hipLaunchKernelGGL(zero_offsets_kernel, dim3(grid_for((uint64_t)n + 1, 256, 4096)), dim3(256),
                           0, st, g->off_out, n);
        hipLaunchKernelGGL(zero_offsets_kernel, dim3(grid_for((uint64_t)n + 1, 256, 4096)), dim3(256),
                           0, st, g->off_in, n);
        KAIROS_HIP(hipGetLastError());
        KAIROS_HIP(hipStreamSynchronize(st));
        g->max_out_degree = 0;
        g->h_perm.resize(n);
        for (uint32_t v = 0; v < n; ++v) g->h_perm[v] = v;
        return KAIROS_OK;
    }
    uint64_t scratch = 0;
    uint4 *a = (uint4 *)dev_alloc(sizeof(uint4) * m, &scratch);
    uint4 *b = (uint4 *)dev_alloc(sizeof(uint4) * m, &scratch);
    const uint64_t tiles = (m + STILE - 1) / STILE;
    const uint32_t nblocks = (uint32_t)std::min<uint64_t>(tiles, 1024);
    uint32_t *hist = (uint32_t *)dev_alloc(sizeof(uint32_t) * 256 * (size_t)nblocks + 64, &scratch);
    uint32_t *h_stats = nullptr;
    int rc = KAIROS_OK;
    do {
        if (!a || !b || !hist) {
            rc = KAIROS_ERR_NOMEM;
            break;
        }
        if (hipHostMalloc((void **)&h_stats, 64, hipHostMallocDefault) != hipSuccess) {
            rc = KAIROS_ERR_NOMEM;
            h_stats = nullptr;
            break;
        }
        uint32_t *d_stats = hist + 256 * (size_t)nblocks;
        const uint32_t init[8] = {0, 0, 0, 0xFFFFFFFFu, 0, 0, 0, 0};
        if (hipMemcpyAsync(d_stats, init, sizeof(init), hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = KAIROS_ERR_DEVICE;
            break;
        }
        hipEvent_t ev;
        prof_begin(g, st, &ev);
        hipLaunchKernelGGL(validate_pack_kernel, dim3(grid_for(m, 256, 8192)), dim3(256), 0, st, src,
                           dst, t, lam, m, n, a, d_stats);
        prof_end(g, st, KAIROS_K_SORT, ev);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(h_stats, d_stats, 32, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = KAIROS_ERR_DEVICE;
            break;
        }
        if (h_stats[0] != 0) {
            rc = KAIROS_ERR_RANGE;
            break;
        }
        const uint32_t max_t = h_stats[1], max_a = h_stats[2], min_l = h_stats[3], max_l = h_stats[4];
        g->max_t = max_t;
        g->max_a = max_a;
        const int nb = bits_for(n - 1);
        const int lb = bits_for(max_l - min_l);
        std::vector<Pass> out_p, in_p;
        add_field(out_p, F_DST, nb, 0);
        add_field(out_p, F_LAM, lb, min_l);
        add_field(out_p, F_T, bits_for(max_t), 0);
        add_field(out_p, F_SRC, nb, 0);
        add_field(in_p, F_SRC, nb, 0);
        add_field(in_p, F_LAMREV, lb, max_l);
        add_field(in_p, F_A, bits_for(max_a), 0);
        add_field(in_p, F_DST, nb, 0);
        {
            // relabel: in-degrees and out-edge marks, stable sort of the
            // vertices (out-edges first, then descending in-degree), then
            // remap both endpoints of every record
            uint64_t vs = 0;
            const uint64_t vtiles = ((uint64_t)n + STILE - 1) / STILE;
            const uint32_t vblocks = (uint32_t)std::min<uint64_t>(vtiles, 1024);
            uint32_t *deg = (uint32_t *)dev_alloc(sizeof(uint32_t) * (size_t)n, &vs);
            uint32_t *has_out = (uint32_t *)dev_alloc(sizeof(uint32_t) * (size_t)n, &vs);
            uint4 *va = (uint4 *)dev_alloc(sizeof(uint4) * (size_t)n, &vs);
            uint4 *vb = (uint4 *)dev_alloc(sizeof(uint4) * (size_t)n, &vs);
            uint32_t *vhist = (uint32_t *)dev_alloc(sizeof(uint32_t) * 256 * (size_t)vblocks, &vs);
            if (!deg || !has_out || !va || !vb || !vhist) {
                dev_free(deg);
                dev_free(has_out);
                dev_free(va);
                dev_free(vb);
                dev_free(vhist);
                rc = KAIROS_ERR_NOMEM;
                break;
            }
            prof_begin(g, st, &ev);
            const bool okm = hipMemsetAsync(deg, 0, sizeof(uint32_t) * (size_t)n, st) == hipSuccess &&
                             hipMemsetAsync(has_out, 0, sizeof(uint32_t) * (size_t)n, st) == hipSuccess;
            hipLaunchKernelGGL(indegree_kernel, dim3(grid_for(m, 256, 16384)), dim3(256), 0, st, a, m, deg, has_out);
            hipLaunchKernelGGL(vertex_keys_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, deg, has_out, n,
                               va);
            prof_end(g, st, KAIROS_K_SORT, ev);
            std::vector<Pass> vp;
            add_field(vp, F_SRC, 32, 0);
            rc = okm ? run_passes(g, va, vb, n, vp, vhist, st) : KAIROS_ERR_DEVICE;
            if (rc == KAIROS_OK) {
                hipLaunchKernelGGL(perm_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, va, n, g->perm,
                                   g->inv);
                hipLaunchKernelGGL(remap_kernel, dim3(grid_for(m, 256, 16384)), dim3(256), 0, st, a, m, g->perm);
                if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) rc = KAIROS_ERR_DEVICE;
            }
            hipStreamSynchronize(st);
            dev_free(deg);
            dev_free(has_out);
            dev_free(va);
            dev_free(vb);
            dev_free(vhist);
            if (rc != KAIROS_OK) break;
        }
        if ((rc = run_passes(g, a, b, m, out_p, hist, st)) != KAIROS_OK) break;
        const int fg = grid_for(m, 256, 16384);
        const int vg = grid_for((uint64_t)n + 1, 256, 4096);
        if (hipMemsetAsync(g->off_out, 0xFF, sizeof(uint32_t) * ((size_t)n + 1), st) != hipSuccess ||
            hipMemsetAsync(g->off_in, 0xFF, sizeof(uint32_t) * ((size_t)n + 1), st) != hipSuccess) {
            rc = KAIROS_ERR_DEVICE;
            break;
        }
        hipLaunchKernelGGL(finalize_kernel, dim3(fg), dim3(256), 0, st, a, m, n, 0, g->off_out,
                           g->t_out, g->da_out);
        hipLaunchKernelGGL(tail_offsets_kernel, dim3(vg), dim3(256), 0, st, a, m, n, 0, g->off_out);
        hipLaunchKernelGGL(gap_offsets_kernel, dim3(vg), dim3(256), 0, st, a, m, n, 0, g->off_out);
        if ((rc = run_passes(g, a, b, m, in_p, hist, st)) != KAIROS_OK) break;
        hipLaunchKernelGGL(finalize_kernel, dim3(fg), dim3(256), 0, st, a, m, n, 1, g->off_in,
                           g->a_in, g->st_in);
        hipLaunchKernelGGL(tail_offsets_kernel, dim3(vg), dim3(256), 0, st, a, m, n, 1, g->off_in);
        hipLaunchKernelGGL(gap_offsets_kernel, dim3(vg), dim3(256), 0, st, a, m, n, 1, g->off_in);
    } while (0);
    if (rc == KAIROS_OK) {
        // the 64 bytes past the histograms: max out-degree at byte 32, the
        // repeat count (8-byte aligned) at byte 40, vertices with out-edges
        // at byte 48
        uint32_t *d_max = hist + 256 * (size_t)nblocks + 8;
        unsigned long long *d_rep = (unsigned long long *)(hist + 256 * (size_t)nblocks + 10);
        uint32_t *d_live = hist + 256 * (size_t)nblocks + 12;
        hipMemsetAsync(d_max, 0, 4, st);
        hipMemsetAsync(d_rep, 0, 8, st);
        hipLaunchKernelGGL(max_degree_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st,
                           g->off_out, n, d_max);
        hipLaunchKernelGGL(repeat_heads_kernel, dim3(grid_for(m, 256 * 8, 8192)), dim3(256), 0, st, g->da_out, m,
                           d_rep);
        hipLaunchKernelGGL(live_count_kernel, dim3(1), dim3(64), 0, st, g->off_out, n, (uint32_t)m, d_live);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(h_stats, d_max, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(h_stats + 2, d_rep, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(h_stats + 4, d_live, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = KAIROS_ERR_DEVICE;
        } else {
            g->max_out_degree = h_stats[0];
            uint64_t rep;
            std::memcpy(&rep, h_stats + 2, 8);
            g->repeat_heads = rep;
            g->n_live = h_stats[4];
        }
    }
    if (rc == KAIROS_OK) {
        g->h_perm.resize(n);
        if (hipMemcpy(g->h_perm.data(), g->perm, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess)
            rc = KAIROS_ERR_DEVICE;
    }
    hipStreamSynchronize(st);
    dev_free(a);
    dev_free(b);
    dev_free(hist);
    if (h_stats) hipHostFree(h_stats);
    return rc;
}

namespace {

// Records {tail, head, t, a} of the out-index in its order, one wavefront
// per tail.
__global__ void out_records_kernel(const uint32_t *__restrict__ off_out, const uint32_t *__restrict__ t_out,
                                   const uint2 *__restrict__ da_out, uint32_t n_live, uint4 *__restrict__ rec)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t u = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); u < n_live; u += waves)
        for (uint32_t f = off_out[u] + lane; f < off_out[u + 1]; f += 64) {
            const uint2 va = da_out[f];
            rec[f] = make_uint4(u, va.x, t_out[f], va.y);
        }
}

}  // namespace

int build_time_order(kairos_graph *g, hipStream_t st, uint4 **out)
{
    const uint64_t m = g->m;
    *out = nullptr;
    if (m == 0) return KAIROS_OK;
    uint64_t scratch = 0;
    uint4 *a = (uint4 *)dev_alloc(sizeof(uint4) * m, nullptr);
    uint4 *b = (uint4 *)dev_alloc(sizeof(uint4) * m, &scratch);
    const uint64_t tiles = (m + STILE - 1) / STILE;
    const uint32_t nblocks = (uint32_t)std::min<uint64_t>(tiles, 1024);
    uint32_t *hist = (uint32_t *)dev_alloc(sizeof(uint32_t) * 256 * (size_t)nblocks + 64, &scratch);
    int rc = a && b && hist ? KAIROS_OK : KAIROS_ERR_NOMEM;
    if (rc == KAIROS_OK) {
        hipLaunchKernelGGL(out_records_kernel, dim3(grid_for(g->n_live, 4, 16384)), dim3(256), 0, st, g->off_out,
                           g->t_out, g->da_out, g->n_live, a);
        if (hipGetLastError() != hipSuccess) rc = KAIROS_ERR_DEVICE;
    }
    if (rc == KAIROS_OK) {
        // stable by departure; the out-index order breaks ties (tail, a, head)
        std::vector<Pass> ps;
        add_field(ps, F_T, bits_for(g->max_t), 0);
        rc = run_passes(g, a, b, m, ps, hist, st);  // leaves the sorted records in `a`
    }
    if (hipStreamSynchronize(st) != hipSuccess && rc == KAIROS_OK) rc = KAIROS_ERR_DEVICE;
    dev_free(b);
    dev_free(hist);
    if (rc != KAIROS_OK) {
        dev_free(a);
        return rc;
    }
    *out = a;
    return KAIROS_OK;
}

}  // namespace kairos
