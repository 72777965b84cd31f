// Internal declarations of libkairos (not part of the C interface).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/kairos.h"

namespace kairos {

constexpr uint32_t INF = 0xFFFFFFFFu;
constexpr uint32_t TMAX = 0xFFFFFFFEu;

// Return-on-error helpers for host code.
#define KAIROS_HIP(call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) {                            \
            kairos::note_hip_error(e_, #call, __FILE__, __LINE__); \
            return KAIROS_ERR_DEVICE;                      \
        }                                                  \
    } while (0)

void note_hip_error(hipError_t e, const char *what, const char *file, int line);

// Device allocation with byte accounting; returns nullptr on failure.
void *dev_alloc(size_t bytes, uint64_t *account);
void dev_free(void *p);

// ---------------------------------------------------------------------------
// Per-query (or per-batch) device state.  One slot holds room for qcap
// queries over n vertices; the arrays are query-major (query i owns
// [i*n, (i+1)*n)).
struct Slot {
    uint32_t qcap = 0;
    uint32_t n = 0;
    uint32_t *done = nullptr;    // qcap*n: lowest claimed out-edge per vertex, INF = unvisited
    uint32_t *queue[2] = {nullptr, nullptr}; // qcap*n each: frontier items q*n+u
    uint4 *chunks = nullptr;     // split adjacency ranges {q, start, len, _}
    uint64_t chunk_cap = 0;
    uint4 *qp = nullptr;         // qcap: {src, t_alpha, t_omega, sweep departure}
    unsigned long long *av = nullptr; // qcap*n: arrival << 32 | stamp of the round that last lowered it
    uint8_t *filt = nullptr;     // qcap regions of filt_stride(n) bytes: packed arrival codes
    uint2 *fpar = nullptr;       // qcap: arrival-code parameters {base, shift | bits << 8}
    uint32_t *fa = nullptr;      // n: fastest duration (sweep)
    uint32_t *l1 = nullptr;      // n: latest departure + 1 (sweep), 0 = none
    uint32_t *steps = nullptr;   // sweep departure times, descending (max out-degree)
    uint32_t *cnt = nullptr;     // device counters, see CNT_* below
    unsigned long long *stats = nullptr; // device work counters, see ST_*
    uint32_t *bar = nullptr;     // grid barrier words of persistent launches
    uint32_t *h_pin = nullptr;   // pinned host mirror for counter read-back
    uint4 *h_q = nullptr;        // qcap: pinned staging of query parameters (read by the init kernel)
    // A slot over caller-provided memory (the allocation-free entry point):
    // h_pin is ordinary host memory, so query parameters are copied to
    // d_stage (device, qcap entries) instead of being read by the kernel
    // from the host, and the slot's launches are never profiled.
    uint4 *d_stage = nullptr;
    bool fixed = false;
    void *pb = nullptr;          // buffers of destination-binned rounds (traverse.hip), on first use
    uint32_t stamp_next = 2;     // next round stamp value (0 = never stamped, 1 = spare)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t bytes = 0;
};

// Bytes of one query's arrival-code region: room for 8-bit codes, rounded
// to whole words, so the layout does not depend on the code width.
inline size_t filt_stride(uint32_t n) { return ((size_t)n + 3) / 4 * 4; }

// Counter layout (uint32 words) in Slot::cnt.
enum : int {
    CNT_FRONT = 0,   // [0..2] rotating frontier sizes
    CNT_CHUNK = 3,   // [3..5] rotating chunk-list sizes
    CNT_STEP = 6,    // next departure step of a latest-departure / fastest sweep
    CNT_PULLVOL = 7, // [7..9] rotating: out-edges of the next frontier (saturating)
    CNT_ABORT = 10,  // set by a persistent launch whose barrier wait gave up
    CNT_TAIL_ROUND = 13, CNT_TAIL_WHICH = 14, CNT_TAIL_ROUNDS = 15,  // left by the tail and persistent kernels
    CNT_WORDS = 16
};
enum : int {
    ST_EDGES = 0, ST_ITEMS = 1, ST_RELAX = 2, ST_PULL_EDGES = 3, ST_PULL_VERTS = 4, ST_CHUNK_EDGES = 5, ST_ATTEMPTS = 6,
    ST_TAIL_EDGES = 7, ST_TAIL_ITEMS = 8, ST_BIN_EDGES = 9, ST_BIN_ITEMS = 10,
    ST_ROUNDS = 11,  // rounds run inside a kernel (the small-graph kernel)
    ST_WORDS = 16
};
// The work counters are kept in ST_SHARDS copies (a block adds to copy
// blockIdx % ST_SHARDS, so concurrent additions hit different addresses),
// followed by ST_SHARDS partial sums used by the traversed-edge count.
constexpr int ST_SHARDS = 64;
constexpr size_t ST_TOTAL_WORDS = (size_t)ST_SHARDS * ST_WORDS + ST_SHARDS;

// Sums the shards of a host copy of the work counters into h[ST_WORDS].
inline void stats_sum_shards(const unsigned long long *raw, unsigned long long *h)
{
    for (int k = 0; k < ST_WORDS; ++k) h[k] = 0;
    for (int sh = 0; sh < ST_SHARDS; ++sh)
        for (int k = 0; k < ST_WORDS; ++k) h[k] += raw[sh * ST_WORDS + k];
}

struct VBatch;
struct SDState;

struct ProfileAcc {
    bool on = false;
    uint64_t launches[KAIROS_K_COUNT] = {};
    double ms[KAIROS_K_COUNT] = {};
    uint64_t edges = 0, chunk_edges = 0, tail_edges = 0, tail_items = 0, attempts = 0, items = 0, relax = 0, pull_edges = 0, pull_verts = 0, rounds = 0;
    uint64_t bin_edges = 0, bin_items = 0;
    uint64_t sw_slabs = 0, sw_passes = 0, sw_fix = 0, sw_fallbacks = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> free_events;
    std::mutex mu;
};

}  // namespace kairos

struct kairos_graph {
    uint32_t n = 0;
    uint64_t m = 0;
    // out-index: edges grouped by tail, sorted by (tail, t, a, head)
    uint32_t *off_out = nullptr;  // n+1
    uint32_t *t_out = nullptr;    // m
    uint2 *da_out = nullptr;      // m: {head, arrival}
    // in-index: edges grouped by head, sorted by (head, a, t, tail)
    uint32_t *off_in = nullptr;   // n+1
    uint32_t *a_in = nullptr;     // m
    uint2 *st_in = nullptr;       // m: {tail, departure}
    // vertex labels: the index uses internal ids ordered by decreasing
    // in-degree; perm maps caller ids to internal ids, inv the reverse
    uint32_t *perm = nullptr;     // n
    uint32_t *inv = nullptr;      // n
    std::vector<uint32_t> h_perm; // host copy of perm
    uint32_t max_out_degree = 0;
    uint32_t n_live = 0;          // ids below have out-edges, ids from here none
    uint32_t max_t = 0;           // largest departure time (0 for an empty graph)
    uint32_t max_a = 0;           // largest arrival time
    uint64_t repeat_heads = 0;    // out-edges whose head repeats the previous out-edge's
    uint64_t index_bytes = 0;
    hipStream_t stream = nullptr; // caller's stream, or nullptr
    int device = 0;
    int num_cus = 256;
    kairos_tuning tuning{};
    std::mutex pool_mu;
    std::vector<kairos::Slot *> free_slots;   // single-query slots
    std::vector<kairos::Slot *> batch_slots;  // batch slots (any qcap)
    std::vector<kairos::VBatch *> vbatches;   // vertex-major batch state
    kairos::ProfileAcc prof;
    // the time-reversed graph (edge (u, v, t, lambda) -> (v, u, TMAX - t -
    // lambda, lambda)), built on the first single-target query
    kairos_graph *rev = nullptr;
    std::mutex rev_mu;
    // shortest duration: for each out-edge, the in-index position of the
    // same edge and that of the last in-edge of its tail arriving by its
    // departure (built on the first such query), and pooled query state
    uint32_t *o2i = nullptr;
    uint32_t *o2k = nullptr;
    uint64_t sd_map_bytes = 0;
    std::mutex sd_mu;
    std::vector<kairos::SDState *> sd_states;
    // every edge {tail, head, t, a} (internal ids) in departure order, for
    // the sweep form of batches (built on its first use)
    uint4 *tsorted = nullptr;
    std::mutex ts_mu;
};

namespace kairos {

// build.hip
int build_index(kairos_graph *g, const uint32_t *src, const uint32_t *dst, const uint32_t *t,
                const uint32_t *lam, hipStream_t st);
// The graph's edges {tail, head, t, a} sorted by departure (stable on the
// out-index order), in a new device array of m records (*out, null for m = 0).
int build_time_order(kairos_graph *g, hipStream_t st, uint4 **out);

// tiny.hip: one earliest-arrival query in one workgroup with its state in
// LDS, for graphs of at most TINY_N vertices (12 bytes of LDS per vertex)
constexpr uint32_t TINY_N = 10240;
bool tiny_eligible(const kairos_graph *g);
int run_tiny_earliest_arrival(kairos_graph *g, Slot *s, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out,
                              bool strict);

// traverse.hip
int slot_acquire(kairos_graph *g, uint32_t qcap, bool sweep, Slot **out);
void slot_release(kairos_graph *g, Slot *s);
void slot_destroy(Slot *s);
// strict: consecutive edges follow "Strictly succeeds" (§2.2) instead of
// "Succeeds"
int run_earliest_arrival(kairos_graph *g, Slot *s, uint32_t src, uint32_t ta, uint32_t tw,
                         uint32_t *out, bool strict = false);
int run_sweep(kairos_graph *g, Slot *s, int kind, uint32_t src, uint32_t ta, uint32_t tw,
              uint32_t *out, bool strict = false);
int run_earliest_arrival_path(kairos_graph *g, Slot *s, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out,
                              uint32_t *pred_tail, uint32_t *pred_dep);
int run_temporal_bfs(kairos_graph *g, Slot *s, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out,
                     bool strict = false);
// Edge list of the time-reversed graph of g, in caller ids, into four device
// arrays of g->m words.
int reverse_edge_list(kairos_graph *g, hipStream_t st, uint32_t *src, uint32_t *dst, uint32_t *t, uint32_t *lam);
// Latest departure towards `target` on g, answered on its time-reversed
// graph `rev` (slot s of rev): earliest arrival from the target over the
// reversed window, read back as TMAX - arrival.
int run_latest_departure_to(kairos_graph *rev, Slot *s, uint32_t target, uint32_t ta, uint32_t tw, uint32_t *out,
                            bool strict);
int run_batch(kairos_graph *g, Slot *s, uint32_t q, const uint32_t *src, const uint32_t *ta,
              const uint32_t *tw, uint32_t *out);
int count_traversed(kairos_graph *g, uint32_t ta, uint32_t tw, const uint32_t *ea, uint64_t *count);

// duration.hip: least total duration of a time-respecting path (Table 4's
// shortest duration); strict: "Strictly succeeds" between consecutive edges
int run_shortest_duration(kairos_graph *g, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out, bool strict);
void release_duration_state(kairos_graph *g);

// batch.hip: vertex-major batches of up to 64 queries per group
int vbatch_acquire(kairos_graph *g, uint32_t groups, VBatch **out);
void vbatch_release(kairos_graph *g, VBatch *b);
void vbatch_destroy(VBatch *b);
int run_vbatch(kairos_graph *g, VBatch *b, uint32_t q, const uint32_t *src, const uint32_t *ta,
               const uint32_t *tw, uint32_t *out);
// The sweep form (batch_layout 3): every edge of the groups' windows in
// departure order, one wavefront per edge and a lane per query.
int run_vbatch_sweep(kairos_graph *g, VBatch *b, uint32_t q, const uint32_t *src, const uint32_t *ta,
                     const uint32_t *tw, uint32_t *out);

// Device state of a multi-slot round loop driven by the server (query
// slots q in [0, qcap), query-major arrays of qcap*n words).
struct MultiState {
    uint32_t qcap = 0, n = 0;
    unsigned long long *av = nullptr;         // arrival << 32 | round stamp (see Slot)
    uint32_t *done = nullptr, *fa = nullptr, *l1 = nullptr;
    uint8_t *filt = nullptr;                  // qcap regions of filt_stride(n) bytes (see Slot)
    uint2 *fpar = nullptr;                    // qcap arrival-code parameters (see Slot)
    uint32_t *queue[2] = {nullptr, nullptr};  // queue[0] feeds the next round
    uint32_t *cnt = nullptr;                  // CNT_WORDS counters, then qcap activity flags
    uint4 *chunks = nullptr, *qp = nullptr;
    uint64_t chunk_cap = 0;
    unsigned long long *stats = nullptr;
    // sweep slots: row q of `steps` (step_cap words) holds the slot's
    // departure times ascending; step_cnt[q] of them, step_pos[q] started
    uint32_t *steps = nullptr, *step_cnt = nullptr, *step_pos = nullptr;
    uint32_t step_cap = 0;
    uint32_t round = 0, stamp_next = 2;
    hipStream_t stream = nullptr;
};
// One slot start: qp[q] = {src, ta, tw, sdep}; the source starts at sdep
// (ta when sdep == INF, a plain earliest-arrival query).  A sweep slot
// (sweep = 1) only takes its parameters: its steps start the source.
struct Inject {
    uint32_t q, src, ta, tw, sdep, sweep, pad1, pad2;
};
int multi_push_round(kairos_graph *g, MultiState *ms);
int multi_inject(kairos_graph *g, MultiState *ms, const Inject *host_pinned, uint32_t count);
int multi_init_slots(kairos_graph *g, MultiState *ms, const uint32_t *host_pinned, uint32_t count);
int multi_sweep_steps(kairos_graph *g, MultiState *ms, const uint32_t *host_pinned, uint32_t count);
int multi_advance(kairos_graph *g, MultiState *ms);
// A grouped sweep's next `width` departure times on slots lead .. lead +
// width - 1, from step pos0 of the lead's list.
struct GroupStart {
    uint32_t lead, width, pos0, src, tw, pad0, pad1, pad2;
};
int multi_group_start(kairos_graph *g, MultiState *ms, const GroupStart *host_pinned, uint32_t count);
int multi_group_reduce(kairos_graph *g, MultiState *ms, uint32_t lead, uint32_t width);
int multi_group_warm(kairos_graph *g, MultiState *ms, uint32_t lead, uint32_t width, uint32_t from);
int multi_finalize(kairos_graph *g, MultiState *ms, uint32_t q, int kind, uint32_t src, uint32_t tw,
                   uint32_t *out);

// A single-query slot laid out in `bytes` of device memory at `base`
// (256-byte aligned), with host read-back through `host_words` (>= 256
// words of ordinary host memory).  Returns the bytes it needs, and fills
// *s only if they fit.
uint64_t slot_layout(const kairos_graph *g, uint64_t chunk_cap, unsigned char *base, uint64_t bytes,
                     uint32_t *host_words, Slot *s);

// profiling (traverse.hip)
void set_unprofiled(bool on);  // this thread's launches skip profiling while on
void prof_begin(kairos_graph *g, hipStream_t st, hipEvent_t *ev0);
void prof_end(kairos_graph *g, hipStream_t st, int cls, hipEvent_t ev0);
void prof_add_stats(kairos_graph *g, const unsigned long long *h);

kairos_tuning default_tuning(const kairos_graph *g);

}  // namespace kairos
