// C entry points of libkairos: argument checks, handle lifetime, dispatch.
#include "internal.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace kairos {

void note_hip_error(hipError_t e, const char *what, const char *file, int line)
{
    static int verbose = -1;
    if (verbose < 0) {
        const char *s = std::getenv("KAIROS_LOG");
        verbose = (s && *s && *s != '0') ? 1 : 0;
    }
    if (verbose) std::fprintf(stderr, "kairos: %s failed: %s (%s:%d)\n", what, hipGetErrorString(e), file, line);
}

void *dev_alloc(size_t bytes, uint64_t *account)
{
    void *p = nullptr;
    if (bytes == 0) bytes = 4;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (account) *account += bytes;
    return p;
}

void dev_free(void *p)
{
    if (p) hipFree(p);
}

}  // namespace kairos

using namespace kairos;

extern "C" {

const char *kairos_status_string(int status)
{
    switch (status) {
    case KAIROS_OK: return "ok";
    case KAIROS_ERR_INVALID: return "invalid argument";
    case KAIROS_ERR_RANGE: return "value out of range";
    case KAIROS_ERR_NOMEM: return "out of memory";
    case KAIROS_ERR_DEVICE: return "device error";
    case KAIROS_ERR_BUSY: return "queue full";
    case KAIROS_ERR_SCRATCH: return "graph too large for the fixed scratch array";
    default: return "unknown status";
    }
}

static void graph_release(kairos_graph *g)
{
    if (!g) return;
    graph_release(g->rev);
    release_duration_state(g);
    dev_free(g->tsorted);
    for (Slot *s : g->free_slots) slot_destroy(s);
    for (Slot *s : g->batch_slots) slot_destroy(s);
    for (VBatch *b : g->vbatches) vbatch_destroy(b);
    g->free_slots.clear();
    g->batch_slots.clear();
    g->vbatches.clear();
    {
        std::lock_guard<std::mutex> lk(g->prof.mu);
        for (auto &p : g->prof.pending) {
            hipEventDestroy(p.second.first);
            hipEventDestroy(p.second.second);
        }
        for (hipEvent_t e : g->prof.free_events) hipEventDestroy(e);
        g->prof.pending.clear();
        g->prof.free_events.clear();
    }
    dev_free(g->off_out);
    dev_free(g->t_out);
    dev_free(g->da_out);
    dev_free(g->off_in);
    dev_free(g->a_in);
    dev_free(g->st_in);
    dev_free(g->perm);
    dev_free(g->inv);
    delete g;
}

int kairos_graph_build(const uint32_t *src, const uint32_t *dst, const uint32_t *t, const uint32_t *lambda,
                       uint64_t m, uint32_t n, void *hip_stream, kairos_graph **out)
{
    if (!out || n == 0) return KAIROS_ERR_INVALID;
    if (m > 0 && (!src || !dst || !t || !lambda)) return KAIROS_ERR_INVALID;
    if (m >= (1ull << 32)) return KAIROS_ERR_RANGE;
    kairos_graph *g = new (std::nothrow) kairos_graph();
    if (!g) return KAIROS_ERR_NOMEM;
    (void)hipGetLastError();
    g->n = n;
    g->m = m;
    g->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return KAIROS_ERR_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->device) == hipSuccess && prop.multiProcessorCount > 0)
        g->num_cus = prop.multiProcessorCount;
    g->tuning = default_tuning(g);
    hipStream_t st = g->stream;
    bool own = false;
    if (!st) {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            delete g;
            return KAIROS_ERR_DEVICE;
        }
        own = true;
    }
    int rc = build_index(g, src, dst, t, lambda, st);
    hipStreamSynchronize(st);
    if (own) hipStreamDestroy(st);
    g->tuning = default_tuning(g);  // again: some defaults depend on index statistics
    if (rc != KAIROS_OK) {
        graph_release(g);
        return rc;
    }
    *out = g;
    return KAIROS_OK;
}

void kairos_graph_free(kairos_graph *g)
{
    graph_release(g);
}

int kairos_graph_stats(const kairos_graph *g, uint32_t *n, uint64_t *m, uint64_t *device_bytes)
{
    if (!g) return KAIROS_ERR_INVALID;
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (device_bytes) *device_bytes = g->index_bytes + (g->rev ? g->rev->index_bytes : 0) + g->sd_map_bytes;
    return KAIROS_OK;
}

// The time-reversed graph of g, built once from g's own in-index on the
// first call (guarded: concurrent first calls build it once).
static int ensure_reverse(kairos_graph *g, kairos_graph **out)
{
    std::lock_guard<std::mutex> lk(g->rev_mu);
    if (!g->rev) {
        const size_t words = std::max<uint64_t>(g->m, 1);
        uint32_t *buf[4] = {nullptr, nullptr, nullptr, nullptr};
        bool ok = true;
        for (auto &b : buf) ok = ok && (b = (uint32_t *)dev_alloc(words * 4, nullptr)) != nullptr;
        int rc = ok ? KAIROS_OK : KAIROS_ERR_NOMEM;
        hipStream_t st = nullptr;
        if (rc == KAIROS_OK && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            st = nullptr;
            rc = KAIROS_ERR_DEVICE;
        }
        if (rc == KAIROS_OK) rc = reverse_edge_list(g, st, buf[0], buf[1], buf[2], buf[3]);
        if (rc == KAIROS_OK && hipStreamSynchronize(st) != hipSuccess) rc = KAIROS_ERR_DEVICE;
        kairos_graph *r = nullptr;
        if (rc == KAIROS_OK) rc = kairos_graph_build(buf[0], buf[1], buf[2], buf[3], g->m, g->n, g->stream, &r);
        if (st) hipStreamDestroy(st);
        for (auto b : buf) dev_free(b);
        if (rc != KAIROS_OK) return rc;
        r->tuning = g->tuning;
        g->rev = r;
    }
    *out = g->rev;
    return KAIROS_OK;
}

int kairos_graph_index(const kairos_graph *g, kairos_index_view *view)
{
    if (!g || !view) return KAIROS_ERR_INVALID;
    view->off_out = g->off_out;
    view->t_out = g->t_out;
    view->dst_a_out = (const uint32_t *)g->da_out;
    view->off_in = g->off_in;
    view->a_in = g->a_in;
    view->src_t_in = (const uint32_t *)g->st_in;
    view->perm = g->perm;
    view->n_live = g->n_live;
    return KAIROS_OK;
}

static int check_query(const kairos_graph *g, uint32_t src, uint32_t ta, uint32_t tw)
{
    if (src >= g->n || ta > tw || tw > KAIROS_TMAX) return KAIROS_ERR_RANGE;
    return KAIROS_OK;
}

// kind 0 earliest arrival, 1 latest departure, 2 fastest, 3 earliest
// arrival with predecessors (out2, out3), 4 temporal BFS hop counts
static int single_query(kairos_graph *g, int kind, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out,
                        uint32_t *out2 = nullptr, uint32_t *out3 = nullptr, bool strict = false)
{
    if (!g || !out || (kind == 3 && (!out2 || !out3))) return KAIROS_ERR_INVALID;
    (void)hipGetLastError();  // errors of unrelated earlier calls on this thread are not ours
    int rc = check_query(g, src, ta, tw);
    if (rc) return rc;
    Slot *s = nullptr;
    if ((rc = slot_acquire(g, 1, kind == 1 || kind == 2, &s))) return rc;
    switch (kind) {
    case 0:
        // small graphs: the whole query in one workgroup with its state in LDS
        rc = tiny_eligible(g) ? run_tiny_earliest_arrival(g, s, src, ta, tw, out, strict)
                              : run_earliest_arrival(g, s, src, ta, tw, out, strict);
        break;
    case 3: rc = run_earliest_arrival_path(g, s, src, ta, tw, out, out2, out3); break;
    case 4: rc = run_temporal_bfs(g, s, src, ta, tw, out, strict); break;
    default: rc = run_sweep(g, s, kind, src, ta, tw, out, strict); break;
    }
    if (rc == KAIROS_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = KAIROS_ERR_DEVICE;
    if (rc == KAIROS_OK) {
        slot_release(g, s);
    } else {
        hipStreamSynchronize(s->stream);
        slot_destroy(s);
    }
    return rc;
}

int kairos_earliest_arrival(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega, uint32_t *out)
{
    return single_query(g, 0, src, t_alpha, t_omega, out);
}

int kairos_latest_departure(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega, uint32_t *out)
{
    return single_query(g, 1, src, t_alpha, t_omega, out);
}

int kairos_fastest(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega, uint32_t *out)
{
    return single_query(g, 2, src, t_alpha, t_omega, out);
}

int kairos_earliest_arrival_path(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                                 uint32_t *out_arrival, uint32_t *out_pred_tail, uint32_t *out_pred_departure)
{
    return single_query(g, 3, src, t_alpha, t_omega, out_arrival, out_pred_tail, out_pred_departure);
}

int kairos_temporal_bfs(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega, uint32_t *out_hops)
{
    return single_query(g, 4, src, t_alpha, t_omega, out_hops);
}

static int latest_departure_to(kairos_graph *g, uint32_t target, uint32_t ta, uint32_t tw, uint32_t *out,
                               bool strict)
{
    if (!g || !out) return KAIROS_ERR_INVALID;
    (void)hipGetLastError();
    int rc = check_query(g, target, ta, tw);
    if (rc) return rc;
    kairos_graph *rev = nullptr;
    if ((rc = ensure_reverse(g, &rev))) return rc;
    Slot *s = nullptr;
    if ((rc = slot_acquire(rev, 1, false, &s))) return rc;
    rc = run_latest_departure_to(rev, s, target, ta, tw, out, strict);
    if (rc == KAIROS_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = KAIROS_ERR_DEVICE;
    if (rc == KAIROS_OK) {
        slot_release(rev, s);
    } else {
        hipStreamSynchronize(s->stream);
        slot_destroy(s);
    }
    return rc;
}

int kairos_latest_departure_to(kairos_graph *g, uint32_t target, uint32_t t_alpha, uint32_t t_omega,
                               uint32_t *out)
{
    return latest_departure_to(g, target, t_alpha, t_omega, out, false);
}

static int shortest_duration(kairos_graph *g, uint32_t src, uint32_t ta, uint32_t tw, uint32_t *out, bool strict)
{
    if (!g || !out) return KAIROS_ERR_INVALID;
    (void)hipGetLastError();
    int rc = check_query(g, src, ta, tw);
    if (rc) return rc;
    return run_shortest_duration(g, src, ta, tw, out, strict);
}

int kairos_shortest_duration(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega, uint32_t *out)
{
    return shortest_duration(g, src, t_alpha, t_omega, out, false);
}

int kairos_query(kairos_graph *g, int kind, uint32_t flags, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                 uint32_t *out)
{
    if ((flags & ~(uint32_t)KAIROS_STRICT) != 0) return KAIROS_ERR_INVALID;
    static const int internal[] = {0, 1, 2, 4};  // EA, LD, F, temporal BFS
    if (kind == KAIROS_LATEST_DEPARTURE_TO)
        return latest_departure_to(g, src, t_alpha, t_omega, out, (flags & KAIROS_STRICT) != 0);
    if (kind == KAIROS_SHORTEST_DURATION)
        return shortest_duration(g, src, t_alpha, t_omega, out, (flags & KAIROS_STRICT) != 0);
    if (kind < KAIROS_EARLIEST_ARRIVAL || kind > KAIROS_TEMPORAL_BFS) return KAIROS_ERR_INVALID;
    return single_query(g, internal[kind], src, t_alpha, t_omega, out, nullptr, nullptr,
                        (flags & KAIROS_STRICT) != 0);
}

int kairos_earliest_arrival_batch(kairos_graph *g, uint32_t q, const uint32_t *src, const uint32_t *t_alpha,
                                  const uint32_t *t_omega, uint32_t *out)
{
    if (!g) return KAIROS_ERR_INVALID;
    if (q == 0) return KAIROS_OK;
    if (!src || !t_alpha || !t_omega || !out) return KAIROS_ERR_INVALID;
    (void)hipGetLastError();
    for (uint32_t i = 0; i < q; ++i) {
        int rc = check_query(g, src[i], t_alpha[i], t_omega[i]);
        if (rc) return rc;
    }
    if (g->tuning.batch_layout != 1) {
        // groups of 64 queries; groups*n must fit the 32-bit frontier items
        const uint64_t max_groups = std::max<uint64_t>(1, 0xFFFFFFFEull / g->n);
        const uint64_t per_q = std::min<uint64_t>((uint64_t)q, max_groups * 64);
        for (uint64_t b = 0; b < q; b += per_q) {
            const uint32_t k = (uint32_t)std::min<uint64_t>(per_q, q - b);
            VBatch *vb = nullptr;
            int rc = vbatch_acquire(g, (k + 63) / 64, &vb);
            if (rc) return rc;
            rc = g->tuning.batch_layout == 3 ? run_vbatch_sweep(g, vb, k, src + b, t_alpha + b, t_omega + b, out + b * g->n)
                                             : run_vbatch(g, vb, k, src + b, t_alpha + b, t_omega + b, out + b * g->n);
            if (rc == KAIROS_OK) {
                vbatch_release(g, vb);
            } else {
                vbatch_destroy(vb);
                return rc;
            }
        }
        return KAIROS_OK;
    }
    // queries per launch: q*n must fit the 32-bit frontier item encoding
    const uint64_t per = std::max<uint64_t>(1, std::min<uint64_t>(q, 0xFFFFFFFEull / g->n));
    for (uint64_t b = 0; b < q; b += per) {
        const uint32_t k = (uint32_t)std::min<uint64_t>(per, q - b);
        Slot *s = nullptr;
        int rc = slot_acquire(g, k, false, &s);
        if (rc) return rc;
        rc = run_batch(g, s, k, src + b, t_alpha + b, t_omega + b, out + b * g->n);
        if (rc == KAIROS_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = KAIROS_ERR_DEVICE;
        if (rc == KAIROS_OK) {
            slot_release(g, s);
        } else {
            hipStreamSynchronize(s->stream);
            slot_destroy(s);
            return rc;
        }
    }
    return KAIROS_OK;
}

int kairos_traversed_edges(kairos_graph *g, uint32_t t_alpha, uint32_t t_omega, const uint32_t *ea,
                           uint64_t *count)
{
    if (!g || !ea || !count) return KAIROS_ERR_INVALID;
    if (t_alpha > t_omega || t_omega > KAIROS_TMAX) return KAIROS_ERR_RANGE;
    (void)hipGetLastError();
    return count_traversed(g, t_alpha, t_omega, ea, count);
}

int kairos_get_tuning(const kairos_graph *g, kairos_tuning *out)
{
    if (!g || !out) return KAIROS_ERR_INVALID;
    *out = g->tuning;
    return KAIROS_OK;
}

int kairos_set_tuning(kairos_graph *g, const kairos_tuning *in)
{
    if (!g || !in) return KAIROS_ERR_INVALID;
    if ((in->block != 256 && in->block != 512) || in->chunk < 16 || in->split < 16 ||
        in->rounds_per_sync < 1 || in->rounds_per_sync > 64 || in->sweep_group < 1 || in->sweep_group > 64 ||
        in->batch_layout > 3 || (in->arrival_filter != 0 && in->arrival_filter != 2 && in->arrival_filter != 4 && in->arrival_filter != 8) || in->batch_persistent > 1 || in->single_persistent > 1 || in->run_dedupe > 1 ||
        (in->binned != 0 && in->binned < 256))
        return KAIROS_ERR_INVALID;
    {
        // the reversed graph (if built) runs with the same parameters
        std::lock_guard<std::mutex> lr(g->rev_mu);
        if (g->rev) {
            int rc = kairos_set_tuning(g->rev, in);
            if (rc) return rc;
        }
    }
    std::lock_guard<std::mutex> lk(g->pool_mu);
    const bool resize = in->chunk < g->tuning.chunk || in->split < g->tuning.split ||
                        in->batch_layout != g->tuning.batch_layout;
    g->tuning = *in;
    if (resize) {
        // chunk lists are sized from these values: drop cached scratch
        for (Slot *s : g->free_slots) slot_destroy(s);
        for (Slot *s : g->batch_slots) slot_destroy(s);
        for (VBatch *b : g->vbatches) vbatch_destroy(b);
        g->free_slots.clear();
        g->batch_slots.clear();
        g->vbatches.clear();
    }
    return KAIROS_OK;
}

int kairos_profile_enable(kairos_graph *g, int on)
{
    if (!g) return KAIROS_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g->prof.mu);
    g->prof.on = on != 0;
    return KAIROS_OK;
}

int kairos_profile_read(kairos_graph *g, kairos_profile *out)
{
    if (!g || !out) return KAIROS_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g->prof.mu);
    std::memset(out, 0, sizeof(*out));
    for (auto &p : g->prof.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second.second) == hipSuccess &&
            hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess)
            g->prof.ms[p.first] += ms;
        g->prof.free_events.push_back(p.second.first);
        g->prof.free_events.push_back(p.second.second);
    }
    g->prof.pending.clear();
    for (int k = 0; k < KAIROS_K_COUNT; ++k) {
        out->launches[k] = g->prof.launches[k];
        out->ms[k] = g->prof.ms[k];
        g->prof.launches[k] = 0;
        g->prof.ms[k] = 0;
    }
    out->edges_scanned = g->prof.edges;
    out->chunk_edges = g->prof.chunk_edges;
    out->relax_attempts = g->prof.attempts;
    out->tail_edges = g->prof.tail_edges;
    out->tail_items = g->prof.tail_items;
    out->items = g->prof.items;
    out->relaxations = g->prof.relax;
    out->pull_edges = g->prof.pull_edges;
    out->pull_vertices = g->prof.pull_verts;
    out->rounds = g->prof.rounds;
    out->binned_edges = g->prof.bin_edges;
    out->binned_items = g->prof.bin_items;
    out->sweep_slabs = g->prof.sw_slabs;
    out->sweep_passes = g->prof.sw_passes;
    out->sweep_fix_edges = g->prof.sw_fix;
    out->sweep_fallbacks = g->prof.sw_fallbacks;
    g->prof.sw_slabs = g->prof.sw_passes = g->prof.sw_fix = g->prof.sw_fallbacks = 0;
    g->prof.edges = g->prof.chunk_edges = g->prof.tail_edges = g->prof.tail_items = g->prof.attempts = g->prof.items = g->prof.relax = g->prof.pull_edges = g->prof.pull_verts = 0;
    g->prof.rounds = 0;
    g->prof.bin_edges = g->prof.bin_items = 0;
    return KAIROS_OK;
}

}  // extern "C"
