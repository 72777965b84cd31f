// Destination-binned push rounds (propagation blocking) for single
// earliest-arrival queries with large frontiers.  Included by traverse.hip
// inside its anonymous namespace (it uses TravArgs and the claim helpers).
//
// A plain push round reads the head's arrival word for every claimed edge:
// one random 8-byte read per edge, which beyond L2 fetches a whole 128-byte
// line.  On graphs whose arrival array is much larger than L2 (2^24
// vertices: 128 MB) that read, not the edge stream, sets the round's time.
// A binned round moves the same edges through three streaming passes
// instead:
//   claim    one thread per frontier entry claims the newly usable range of
//            its adjacency (exactly as the push kernel does) and appends the
//            non-empty claims to a list; a scan gives each claim its first
//            edge in the round's edge sequence;
//   count    the edges are split evenly over the blocks; each block counts
//            the usable edges (arrival <= t_omega) per destination bin of
//            2^PB_BS vertices in LDS, and a scan over (bin, block) gives each
//            block a write position in every bin;
//   scatter  the same blocks read the same edges again and write the
//            candidates (head, arrival) to their bins, so each bin's
//            candidates are contiguous;
//   apply    one block per piece of a bin loads the bin's arrivals into LDS,
//            takes the minimum of its candidates there, and for every vertex
//            it lowered does one 64-bit atomicMin of (arrival, round stamp)
//            on the arrival word, which as in the push kernel says whether
//            the vertex improved and whether this round already enqueued it.
// Per edge that is 8 B read twice plus 8 B written and read once, all in
// order, against a 128-byte line per missed arrival read; the atomics shrink
// from one per improving edge to one per improved vertex and bin piece.
// Results are the same bits: a candidate is offered to its head exactly as
// the push kernel would offer it, and minimum is order-free.
//
// Measured on the scale-24 R-MAT graph (one query per call, a host check
// after every round for both forms): 6.70 ms per query binned from 16,384
// frontier entries against 4.58 ms with push rounds.  On the largest round
// claim / count / scatter / apply took 285 / 830 / 1953 / 663 us against
// 1161 + 1555 us for push + chunk: the passes run at 1.2-2.4 TB/s, far
// from the streaming rate the byte count assumes (the R-MAT hubs put most
// candidates into the first bins, and the scatter's writes spread over
// bins x blocks partial lines).  Count / scatter grids of 128 ... 16,384
// blocks were all slower than 2,048.  Off by default (tuning `binned` = 0).

constexpr int PB_T = 256;                  // threads per block of the claim, count and scatter passes
constexpr int PB_OWN = 512;                // claims held at a time in the LDS owner table
constexpr int PB_UNR = 4;                  // edges per thread in flight
constexpr int PB_BS = 14;                  // log2 vertices per bin (64 KB of arrivals in LDS)
constexpr uint32_t PB_SLICE = 1u << PB_BS;
constexpr int PB_AT = 1024;                // threads per apply block
constexpr uint32_t PB_MAX_BINS = 4096;     // bins of a count / scatter block's LDS table (n <= 2^26)
constexpr uint32_t PB_PIECE = 1u << 18;    // candidates per apply block at most
// device words of a binned round
enum : int { PBW_CLAIMS = 0, PBW_EDGES = 1, PBW_CANDS = 2, PBW_PIECES = 3, PBW_WORDS = 4 };

__global__ void pb_reset_kernel(uint32_t *words)
{
    if (threadIdx.x < PBW_WORDS) words[threadIdx.x] = 0u;
}

// Claim pass: the push kernel's claim of one frontier entry per thread (a
// single query: entries are vertices), non-empty claims appended with one
// atomicAdd per block.
__global__ __launch_bounds__(PB_T) void pb_claim_kernel(TravArgs A, uint2 *claims, uint32_t *lens, uint32_t *words)
{
    __shared__ uint32_t s_w[PB_T / 64];
    __shared__ uint32_t s_base;
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (blockIdx.x == 0 && tid == 0) {
        // the counter protocol of push_phase: clear the words of later rounds
        A.cnt[CNT_FRONT + (A.round + 2u) % 3u] = 0u;
        A.cnt[CNT_PULLVOL + (A.round + 2u) % 3u] = 0u;
        A.cnt[CNT_CHUNK + (A.round + 1u) % 3u] = 0u;
    }
    const uint32_t F = A.cnt[CNT_FRONT + A.round % 3u];
    const uint4 p = A.qp[0];
    const uint2 fpq = A.fpar[0];
    unsigned long long n_items = 0;
    for (uint32_t b0 = blockIdx.x * PB_T; b0 < F; b0 += gridDim.x * PB_T) {
        const uint32_t i = b0 + tid;
        uint32_t lo = 0, len = 0;
        if (i < F) {
            ++n_items;
            const uint32_t u = A.cur[i];
            // one thread per vertex and round: plain loads and stores
            const uint32_t r = arrival_of(A.av, u);
            const uint32_t b = A.off[u], e = A.off[u + 1];
            const uint32_t old = A.done[u];
            lo = lower_bound_u32(A.tt, b, old == INF ? e : min(old, e), departure_key(r, fpq.y, u, p.x));
            uint32_t end = old;
            if (old == INF) end = p.z > A.max_t ? e : lower_bound_u32(A.tt, lo, e, p.z);
            if (lo < end) {
                len = end - lo;
                A.done[u] = lo;
            }
        }
        const unsigned long long bal = __ballot(len > 0);
        if (lane == 0) s_w[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        if (tid == 0) {
            uint32_t t = 0;
            for (int k = 0; k < PB_T / 64; ++k) {
                const uint32_t c = s_w[k];
                s_w[k] = t;
                t += c;
            }
            s_base = t ? atomicAdd(&words[PBW_CLAIMS], t) : 0u;
        }
        __syncthreads();
        if (len > 0) {
            const uint32_t pos = s_base + s_w[w] + (uint32_t)__popcll(bal & lanes_below());
            claims[pos] = make_uint2(lo, len);
            lens[pos] = len;
        }
        __syncthreads();
    }
    unsigned long long v[1] = {n_items};
    const int slot[1] = {ST_BIN_ITEMS};
    block_stats<PB_T / 64>(A.stats, v, slot);
}

// Count (SCATTER = false) and scatter passes over the round's claimed edges,
// split evenly over the grid: block b takes edges [E b / G, E (b + 1) / G)
// of the sequence the claims form in list order.  Claims are walked through
// an LDS table of PB_OWN of them at a time; an edge's claim is found there
// by binary search.  hist is bin-major: hist[bin * G + b].
template <bool SCATTER>
__global__ __launch_bounds__(PB_T) void pb_bin_kernel(TravArgs A, const uint2 *__restrict__ claims,
                                                      const uint32_t *__restrict__ cbase,
                                                      const uint32_t *__restrict__ words, uint32_t *hist,
                                                      uint32_t nbins, uint2 *__restrict__ cand)
{
    __shared__ uint32_t s_bin[PB_MAX_BINS];  // counts, or write cursors
    __shared__ uint32_t s_first[PB_OWN];    // first edge (in the sequence) of each table claim
    __shared__ uint32_t s_lo[PB_OWN];       // its first adjacency position
    __shared__ uint32_t s_own0, s_end;
    const uint32_t tid = threadIdx.x;
    const uint32_t C = words[PBW_CLAIMS], E = words[PBW_EDGES];
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint32_t e0 = (uint32_t)((uint64_t)E * b / G), e1 = (uint32_t)((uint64_t)E * (b + 1) / G);
    const uint32_t tw = A.qp[0].z;
    for (uint32_t k = tid; k < nbins; k += PB_T) s_bin[k] = SCATTER ? hist[(size_t)k * G + b] : 0u;
    if (tid == 0) {
        // the last claim starting at or before e0
        uint32_t lo = 0, hi = C;
        while (lo < hi) {
            const uint32_t mid = lo + ((hi - lo) >> 1);
            if (cbase[mid] <= e0)
                lo = mid + 1;
            else
                hi = mid;
        }
        s_own0 = lo ? lo - 1u : 0u;
    }
    __syncthreads();
    unsigned long long n_edges = 0;
    uint32_t own = s_own0, cur = e0;
    while (cur < e1) {
        const uint32_t k = min((uint32_t)PB_OWN, C - own);
        if (k == 0) break;  // not reached: the claims cover every edge of the sequence
        for (uint32_t i = tid; i < k; i += PB_T) {
            s_first[i] = cbase[own + i];
            s_lo[i] = claims[own + i].x;
        }
        if (tid == 0) s_end = own + k < C ? cbase[own + k] : E;
        __syncthreads();
        const uint32_t hi = min(e1, s_end);
        for (uint32_t j0 = cur; j0 < hi; j0 += PB_T * PB_UNR) {
            uint32_t v[PB_UNR], a[PB_UNR];
            bool ok[PB_UNR];
#pragma unroll
            for (int u = 0; u < PB_UNR; ++u) {
                const uint32_t j = j0 + u * PB_T + tid;
                ok[u] = j < hi;
                uint32_t lo_k = 0, hi_k = k;  // last table claim whose first edge is <= j
                while (hi_k - lo_k > 1) {
                    const uint32_t mid = (lo_k + hi_k) >> 1;
                    if (s_first[mid] <= j)
                        lo_k = mid;
                    else
                        hi_k = mid;
                }
                const uint32_t e = ok[u] ? s_lo[lo_k] + (j - s_first[lo_k]) : 0u;
                const uint2 dv = A.da[e];
                v[u] = dv.x;
                a[u] = dv.y;
            }
#pragma unroll
            for (int u = 0; u < PB_UNR; ++u) {
                if (!ok[u]) continue;
                ++n_edges;
                if (a[u] > tw) continue;
                const uint32_t bin = v[u] >> PB_BS;
                if (SCATTER) {
                    const uint32_t pos = atomicAdd(&s_bin[bin], 1u);
                    cand[pos] = make_uint2(v[u], a[u]);
                } else {
                    atomicAdd(&s_bin[bin], 1u);
                }
            }
        }
        cur = hi;
        own += k;
        __syncthreads();  // the table is reloaded
    }
    if (!SCATTER) {
        for (uint32_t k = tid; k < nbins; k += PB_T) hist[(size_t)k * G + b] = s_bin[k];
        unsigned long long v[1] = {n_edges};
        const int slot[1] = {ST_BIN_EDGES};
        block_stats<PB_T / 64>(A.stats, v, slot);
    }
}

// Pieces of the bins: bin k's candidates are [hist[k G], hist[(k + 1) G])
// (the total for the last bin); it is cut into pieces of at most PB_PIECE.
// pbase[k] = first piece of bin k (exclusive scan), words[PBW_PIECES] the
// total.  One block.
__global__ __launch_bounds__(1024) void pb_pieces_kernel(const uint32_t *__restrict__ hist, uint32_t G,
                                                         uint32_t nbins, uint32_t *pbase, uint32_t *words)
{
    __shared__ uint32_t part[1024];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (nbins + 1023) / 1024;
    const uint32_t beg = min(nbins, tid * per), end = min(nbins, beg + per);
    const uint32_t total = words[PBW_CANDS];
    uint32_t s = 0;
    for (uint32_t k = beg; k < end; ++k) {
        const uint32_t c0 = hist[(size_t)k * G], c1 = k + 1 < nbins ? hist[(size_t)(k + 1) * G] : total;
        s += (c1 - c0 + PB_PIECE - 1) / PB_PIECE;
    }
    part[tid] = s;
    __syncthreads();
    for (uint32_t o = 1; o < 1024; o <<= 1) {
        const uint32_t y = tid >= o ? part[tid - o] : 0u;
        __syncthreads();
        part[tid] += y;
        __syncthreads();
    }
    uint32_t run = part[tid] - s;
    for (uint32_t k = beg; k < end; ++k) {
        pbase[k] = run;
        const uint32_t c0 = hist[(size_t)k * G], c1 = k + 1 < nbins ? hist[(size_t)(k + 1) * G] : total;
        run += (c1 - c0 + PB_PIECE - 1) / PB_PIECE;
    }
    if (tid == 1023) words[PBW_PIECES] = part[1023];
}

// Apply pass: one block per bin piece (grid-stride).  The bin's arrivals go
// to LDS, the piece's candidates lower them there (LDS atomicMin), and each
// lowered vertex takes one 64-bit atomicMin of (arrival, stamp) on its word:
// improved and not yet stamped by this round means a new frontier entry
// (vertices without out-edges excepted).  New entries are counted per block
// and appended behind one atomicAdd.
__global__ __launch_bounds__(PB_AT) void pb_apply_kernel(TravArgs A, const uint32_t *__restrict__ hist, uint32_t G,
                                                         uint32_t nbins, const uint32_t *__restrict__ pbase,
                                                         const uint2 *__restrict__ cand, const uint32_t *words)
{
    __shared__ uint32_t s_arr[PB_SLICE];
    __shared__ uint32_t s_low[PB_SLICE / 32];  // lowered by this piece
    __shared__ uint32_t s_push[PB_SLICE / 32]; // to enqueue
    __shared__ uint32_t s_wsum[PB_AT / 64];
    __shared__ uint32_t s_base;
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t P = words[PBW_PIECES], total = words[PBW_CANDS];
    uint32_t *next_cnt = &A.cnt[CNT_FRONT + (A.round + 1u) % 3u];
    unsigned long long n_relax = 0, n_att = 0;
    for (uint32_t piece = blockIdx.x; piece < P; piece += gridDim.x) {
        // the bin holding this piece: the last bin whose first piece is <= it
        uint32_t lo = 0, hi = nbins;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pbase[mid] <= piece)
                lo = mid;
            else
                hi = mid;
        }
        const uint32_t bin = lo;
        const uint32_t bc0 = hist[(size_t)bin * G], bc1 = bin + 1 < nbins ? hist[(size_t)(bin + 1) * G] : total;
        const uint32_t c0 = bc0 + (piece - pbase[bin]) * PB_PIECE, c1 = min(bc1, c0 + PB_PIECE);
        const uint32_t v0 = bin << PB_BS, nv = min(PB_SLICE, A.n - v0);
        for (uint32_t i = tid; i < nv; i += PB_AT) s_arr[i] = arrival_of(A.av, v0 + i);
        for (uint32_t i = tid; i < PB_SLICE / 32; i += PB_AT) s_low[i] = s_push[i] = 0u;
        __syncthreads();
        for (uint32_t c = c0 + tid; c < c1; c += PB_AT) {
            const uint2 x = cand[c];
            const uint32_t lv = x.x - v0;
            if (x.y < s_arr[lv] && x.y < atomicMin(&s_arr[lv], x.y)) atomicOr(&s_low[lv >> 5], 1u << (lv & 31));
        }
        __syncthreads();
        // one thread per word of 32 slice vertices
        uint32_t pushed = 0;
        if (tid < PB_SLICE / 32) {
            uint32_t m = s_low[tid];
            while (m) {
                const uint32_t bit = (uint32_t)__ffs(m) - 1u;
                m &= m - 1u;
                const uint32_t li = tid * 32u + bit, vtx = v0 + li;
                const uint32_t val = s_arr[li];
                ++n_att;
                const unsigned long long old = atomicMin(&A.av[vtx], av_word(val, A.stamp_val));
                if (val < (uint32_t)(old >> 32)) {
                    ++n_relax;
                    if ((uint32_t)old != A.stamp_val && vtx < A.n_live) pushed |= 1u << bit;
                }
            }
            s_push[tid] = pushed;
        }
        // block prefix over the pushed counts, one atomicAdd, then the entries
        uint32_t cntp = (uint32_t)__popc(pushed), x = cntp;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= (uint32_t)o) x += y;
        }
        if (lane == 63) s_wsum[w] = x;
        __syncthreads();
        if (tid == 0) {
            uint32_t t = 0;
            for (int k = 0; k < PB_AT / 64; ++k) {
                const uint32_t c = s_wsum[k];
                s_wsum[k] = t;
                t += c;
            }
            s_base = t ? atomicAdd(next_cnt, t) : 0u;
        }
        __syncthreads();
        if (pushed) {
            uint32_t pos = s_base + s_wsum[w] + x - cntp;
            uint32_t m = pushed;
            while (m) {
                const uint32_t bit = (uint32_t)__ffs(m) - 1u;
                m &= m - 1u;
                A.next[pos++] = v0 + tid * 32u + bit;
            }
        }
        __syncthreads();  // LDS is refilled for the next piece
    }
    unsigned long long v[2] = {n_relax, n_att};
    const int slot[2] = {ST_RELAX, ST_ATTEMPTS};
    block_stats<PB_AT / 64>(A.stats, v, slot);
}

// Device buffers of binned rounds, allocated with a single-query slot on
// its first binned round.
struct PBBufs {
    uint2 *claims = nullptr;   // n: non-empty claims {first position, length}
    uint32_t *lens = nullptr;  // n + 1: claim lengths, then their scan
    uint32_t *hist = nullptr;  // bins * PB grid: counts, then their scan
    uint32_t *pbase = nullptr; // bins: first piece of each bin
    uint2 *cand = nullptr;     // m: candidates {head, arrival}
    uint32_t *bsum = nullptr;  // scan scratch
    uint32_t *words = nullptr; // PBW_WORDS
    uint32_t grid = 0, nbins = 0;
};

bool binned_supported(const kairos_graph *g)
{
    return g->n <= PB_MAX_BINS * PB_SLICE && g->m > 0;
}

// One binned round of a single query: the claim of every entry of the
// current frontier, then count, scatter and apply.  Leaves the next frontier
// and its count where a push round leaves them.  Profiled as one unit
// (KAIROS_K_BINNED: all its launches, claim to apply).
PBBufs *pbufs(Slot *s) { return static_cast<PBBufs *>(s->pb); }

int binned_round(kairos_graph *g, Slot *s, const TravArgs &A, uint32_t F)
{
    hipStream_t st = s->stream;
    PBBufs &B = *pbufs(s);
    hipEvent_t ev;
    prof_begin(g, st, &ev);
    hipLaunchKernelGGL(pb_reset_kernel, dim3(1), dim3(64), 0, st, B.words);
    hipLaunchKernelGGL(pb_claim_kernel, dim3(grid_cap(F, PB_T, g->num_cus * 8)), dim3(PB_T), 0, st, A, B.claims,
                       B.lens, B.words);
    exclusive_scan_dev(st, B.lens, F, B.words + PBW_CLAIMS, B.bsum, B.words + PBW_EDGES);
    hipLaunchKernelGGL((pb_bin_kernel<false>), dim3(B.grid), dim3(PB_T), 0, st, A, B.claims, B.lens, B.words, B.hist,
                       B.nbins, B.cand);
    exclusive_scan(st, B.hist, B.nbins * B.grid, B.bsum, B.words + PBW_CANDS);
    hipLaunchKernelGGL(pb_pieces_kernel, dim3(1), dim3(1024), 0, st, B.hist, B.grid, B.nbins, B.pbase, B.words);
    hipLaunchKernelGGL((pb_bin_kernel<true>), dim3(B.grid), dim3(PB_T), 0, st, A, B.claims, B.lens, B.words, B.hist,
                       B.nbins, B.cand);
    hipLaunchKernelGGL(pb_apply_kernel, dim3(std::max(1, g->num_cus * 2)), dim3(PB_AT), 0, st, A, B.hist, B.grid,
                       B.nbins, B.pbase, B.cand, B.words);
    prof_end(g, st, KAIROS_K_BINNED, ev);
    KAIROS_HIP(hipGetLastError());
    return KAIROS_OK;
}

int binned_alloc(kairos_graph *g, Slot *s)
{
    if (s->pb) return KAIROS_OK;
    PBBufs *B = new PBBufs();
    const uint64_t n = g->n, m = std::max<uint64_t>(g->m, 1);
    B->grid = (uint32_t)std::max(1, g->num_cus * 8);
    B->nbins = (uint32_t)((n + PB_SLICE - 1) / PB_SLICE);
    const uint64_t hwords = (uint64_t)B->nbins * B->grid;
    bool ok = (B->claims = (uint2 *)dev_alloc(n * sizeof(uint2), &s->bytes)) != nullptr;
    ok = ok && (B->lens = (uint32_t *)dev_alloc((n + 1) * 4, &s->bytes)) != nullptr;
    ok = ok && (B->hist = (uint32_t *)dev_alloc(hwords * 4, &s->bytes)) != nullptr;
    ok = ok && (B->pbase = (uint32_t *)dev_alloc((uint64_t)B->nbins * 4, &s->bytes)) != nullptr;
    ok = ok && (B->cand = (uint2 *)dev_alloc(m * sizeof(uint2), &s->bytes)) != nullptr;
    ok = ok && (B->bsum = (uint32_t *)dev_alloc(scan_scratch_words(std::max<uint64_t>(n, hwords)) * 4, &s->bytes)) !=
                   nullptr;
    ok = ok && (B->words = (uint32_t *)dev_alloc(PBW_WORDS * 4, &s->bytes)) != nullptr;
    s->pb = B;
    return ok ? KAIROS_OK : KAIROS_ERR_NOMEM;
}

void binned_free(Slot *s)
{
    if (!s->pb) return;
    PBBufs *B = pbufs(s);
    dev_free(B->claims);
    dev_free(B->lens);
    dev_free(B->hist);
    dev_free(B->pbase);
    dev_free(B->cand);
    dev_free(B->bsum);
    dev_free(B->words);
    delete B;
    s->pb = nullptr;
}
