// Continuous-batching query server.
//
// A scheduler thread owns a pool of query slots on the device.  Each
// iteration it (1) admits waiting queries into free slots, growing the slot
// pool when the device reports enough free memory, (2) starts them (slot
// state reset; an earliest-arrival source goes into the shared frontier, a
// latest-departure / fastest slot gets its departure times listed on the
// device), (3) runs a few push rounds, each over every active slot in one
// launch, and (4) reads back the per-slot activity flags.  A sweep either
// holds one slot, and a device kernel between rounds moves it to its next
// departure time once its frontier emptied (no host round trip per step),
// or, while the pool has room, holds a group of consecutive slots that run
// several departure times at once as earliest-arrival queries, folded into
// the first slot's accumulators when all ran dry and warm-started from the
// last for the next group.  A query with no frontier and no steps left is
// finished: its result is written to the caller's buffer and a completion
// with timestamps is queued for polling.  Queries that arrive while others run join at the next
// iteration, so their rounds overlap on the device with everyone else's.
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <cstring>

using namespace kairos;

namespace {

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Query {
    uint64_t ticket;
    int kind;
    uint32_t src, ta, tw;
    uint32_t *out;
    uint64_t t_submit;
};

struct SlotRun {
    bool busy = false;
    bool started = false;
    Query q{};
    // a grouped latest-departure / fastest query holds `width` consecutive
    // slots; the first (the lead) carries the query, the others point to it
    uint32_t width = 1;
    int32_t lead = -1;  // >= 0: member of the group led by that slot
    uint32_t pos0 = 0;  // lead: first step of the running group
};

}  // namespace

struct kairos_server {
    kairos_graph *g = nullptr;
    kairos_server_opts opts{};
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Query> waiting;
    std::deque<kairos_completion> done;
    std::thread th;
    bool stop = false;
    bool failed = false;
    uint64_t next_ticket = 1;
    kairos_server_stats stats{};
    uint64_t free_override = UINT64_MAX;
    // device side (scheduler thread only)
    MultiState ms;
    bool own_stream = false;
    uint32_t cap = 0;
    std::vector<SlotRun> slots;
    uint32_t *h_pin = nullptr;  // pinned, see pin_words
    uint64_t per_slot_chunks = 0;
    uint32_t rounds_per_check = 4;
};

namespace {

// Pinned host words: counters + activity flags (read back) | step counts
// (read back) | inject list | init list | sweep list | group starts at
// admission | group starts after a group.  Each list is written once per
// iteration, after the previous iteration's read-back synchronised.
struct PinLayout {
    size_t flags, step_cnt, inject, init, sweep, start_admit, start_next, total;
};

PinLayout pin_layout(uint32_t max_slots)
{
    const size_t m = max_slots;
    PinLayout p{};
    p.flags = 0;
    p.step_cnt = CNT_WORDS + m;
    p.inject = p.step_cnt + m;
    p.init = p.inject + 8 * m;
    p.sweep = p.init + m;
    p.start_admit = p.sweep + m;
    p.start_next = p.start_admit + 8 * m;
    p.total = p.start_next + 8 * m + 64;
    return p;
}

size_t pin_words(uint32_t max_slots)
{
    return pin_layout(max_slots).total;
}

uint64_t slot_bytes(kairos_server *s)
{
    return (uint64_t)s->g->n * (4 * 7) + filt_stride(s->g->n) + s->per_slot_chunks * sizeof(uint4) +
           sizeof(uint4) + sizeof(uint2) + 4 + 4ull * (s->g->max_out_degree + 2);
}

bool free_bytes_ok(kairos_server *s, uint64_t need)
{
    uint64_t fr = s->free_override;
    if (fr == UINT64_MAX) {
        size_t f = 0, t = 0;
        if (hipMemGetInfo(&f, &t) != hipSuccess) return false;
        fr = f;
    }
    return fr >= need + s->opts.mem_reserve_bytes;
}

void free_state(MultiState &m)
{
    dev_free(m.av);
    dev_free(m.filt);
    dev_free(m.fpar);
    dev_free(m.done);
    dev_free(m.fa);
    dev_free(m.l1);
    dev_free(m.queue[0]);
    dev_free(m.queue[1]);
    dev_free(m.cnt);
    dev_free(m.chunks);
    dev_free(m.qp);
    dev_free(m.stats);
    dev_free(m.steps);
    dev_free(m.step_cnt);
    dev_free(m.step_pos);
    m = MultiState{};
}

// Grow the slot pool to `ncap` slots, keeping the state of existing slots.
// Called between rounds only.  Returns false if memory is short.  The new
// pool is allocated whole while the old one is still live (its state is
// copied over), so the check charges all ncap slots, the transient peak.
bool grow(kairos_server *s, uint32_t ncap)
{
    if (ncap <= s->cap) return true;
    const uint64_t need = slot_bytes(s) * ncap;
    if (!free_bytes_ok(s, need)) return false;
    const size_t n = s->g->n;
    const size_t qn = (size_t)ncap * n, on = (size_t)s->cap * n;
    MultiState nm;
    nm.qcap = ncap;
    nm.n = (uint32_t)n;
    nm.round = s->ms.round;
    nm.stamp_next = s->ms.stamp_next;
    nm.stream = s->ms.stream;
    nm.chunk_cap = s->per_slot_chunks * ncap;
    nm.av = (unsigned long long *)dev_alloc(qn * 8, nullptr);
    nm.filt = (uint8_t *)dev_alloc((size_t)ncap * filt_stride(s->g->n), nullptr);
    nm.fpar = (uint2 *)dev_alloc((size_t)ncap * sizeof(uint2), nullptr);
    nm.done = (uint32_t *)dev_alloc(qn * 4, nullptr);
    nm.fa = (uint32_t *)dev_alloc(qn * 4, nullptr);
    nm.l1 = (uint32_t *)dev_alloc(qn * 4, nullptr);
    nm.queue[0] = (uint32_t *)dev_alloc(qn * 4 + 64, nullptr);
    nm.queue[1] = (uint32_t *)dev_alloc(qn * 4 + 64, nullptr);
    nm.cnt = (uint32_t *)dev_alloc((CNT_WORDS + (size_t)ncap) * 4, nullptr);
    nm.chunks = (uint4 *)dev_alloc(nm.chunk_cap * sizeof(uint4), nullptr);
    nm.qp = (uint4 *)dev_alloc((size_t)ncap * sizeof(uint4), nullptr);
    nm.stats = (unsigned long long *)dev_alloc(ST_TOTAL_WORDS * 8, nullptr);
    nm.step_cap = std::max<uint32_t>(s->g->max_out_degree, 1);
    nm.steps = (uint32_t *)dev_alloc((size_t)ncap * nm.step_cap * 4, nullptr);
    nm.step_cnt = (uint32_t *)dev_alloc((size_t)ncap * 4, nullptr);
    nm.step_pos = (uint32_t *)dev_alloc((size_t)ncap * 4, nullptr);
    hipStream_t st = s->ms.stream;
    bool ok = nm.av && nm.filt && nm.fpar && nm.done && nm.fa && nm.l1 && nm.queue[0] && nm.queue[1] && nm.cnt &&
              nm.chunks && nm.qp && nm.stats && nm.steps && nm.step_cnt && nm.step_pos;
    ok = ok && hipMemsetAsync(nm.av, 0, qn * 8, st) == hipSuccess &&
         hipMemsetAsync(nm.cnt, 0, (CNT_WORDS + (size_t)ncap) * 4, st) == hipSuccess &&
         hipMemsetAsync(nm.stats, 0, ST_TOTAL_WORDS * 8, st) == hipSuccess &&
         hipMemsetAsync(nm.step_cnt, 0, (size_t)ncap * 4, st) == hipSuccess &&
         hipMemsetAsync(nm.step_pos, 0, (size_t)ncap * 4, st) == hipSuccess;
    if (ok && s->cap) {
        const hipMemcpyKind k = hipMemcpyDeviceToDevice;
        ok = hipMemcpyAsync(nm.av, s->ms.av, on * 8, k, st) == hipSuccess &&
             hipMemcpyAsync(nm.filt, s->ms.filt, (size_t)s->cap * filt_stride(s->g->n), k, st) == hipSuccess &&
             hipMemcpyAsync(nm.fpar, s->ms.fpar, (size_t)s->cap * sizeof(uint2), k, st) == hipSuccess &&
             hipMemcpyAsync(nm.done, s->ms.done, on * 4, k, st) == hipSuccess &&
             hipMemcpyAsync(nm.fa, s->ms.fa, on * 4, k, st) == hipSuccess &&
             hipMemcpyAsync(nm.l1, s->ms.l1, on * 4, k, st) == hipSuccess &&
             hipMemcpyAsync(nm.queue[0], s->ms.queue[0], on * 4, k, st) == hipSuccess &&
             hipMemcpyAsync(nm.cnt, s->ms.cnt, (CNT_WORDS + (size_t)s->cap) * 4, k, st) == hipSuccess &&
             hipMemcpyAsync(nm.qp, s->ms.qp, (size_t)s->cap * sizeof(uint4), k, st) == hipSuccess &&
             hipMemcpyAsync(nm.steps, s->ms.steps, (size_t)s->cap * nm.step_cap * 4, k, st) == hipSuccess &&
             hipMemcpyAsync(nm.step_cnt, s->ms.step_cnt, (size_t)s->cap * 4, k, st) == hipSuccess &&
             hipMemcpyAsync(nm.step_pos, s->ms.step_pos, (size_t)s->cap * 4, k, st) == hipSuccess;
    }
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        hipStreamSynchronize(st);
        free_state(nm);
        (void)hipGetLastError();
        return false;
    }
    free_state(s->ms);  // nm already carries the stream
    s->ms = nm;
    s->cap = ncap;
    s->slots.resize(ncap);
    return true;
}

void complete(kairos_server *s, const Query &q, int status, uint64_t t_done)
{
    kairos_completion c{};
    c.ticket = q.ticket;
    c.status = status;
    c.kind = q.kind;
    c.t_submit_ns = q.t_submit;
    c.t_done_ns = t_done;
    s->done.push_back(c);
    s->stats.completed += 1;
}

// Fail everything in flight and waiting (after a device error).
void fail_all(kairos_server *s)
{
    const uint64_t t = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    s->failed = true;
    for (auto &sl : s->slots) {
        if (sl.busy && sl.lead < 0) complete(s, sl.q, KAIROS_ERR_DEVICE, t);
        sl = SlotRun{};
    }
    while (!s->waiting.empty()) {
        complete(s, s->waiting.front(), KAIROS_ERR_DEVICE, t);
        s->waiting.pop_front();
    }
    s->stats.active_slots = 0;
    s->stats.waiting = 0;
}

// First run of at least `want` free slots (start, length), else the longest
// run; length 0 when every slot is busy.
std::pair<uint32_t, uint32_t> free_run(const kairos_server *s, uint32_t want)
{
    uint32_t best_start = 0, best_len = 0;
    for (uint32_t i = 0; i < s->cap;) {
        if (s->slots[i].busy) {
            ++i;
            continue;
        }
        uint32_t j = i;
        while (j < s->cap && !s->slots[j].busy && j - i < want) ++j;
        if (j - i >= want) return {i, want};
        if (j - i > best_len) {
            best_start = i;
            best_len = j - i;
        }
        while (j < s->cap && !s->slots[j].busy) ++j;
        i = j;
    }
    return {best_start, best_len};
}

int iterate(kairos_server *s)
{
    kairos_graph *g = s->g;
    hipStream_t st = s->ms.stream;
    const PinLayout pl = pin_layout(s->opts.max_slots);
    const uint32_t group = std::min<uint32_t>(std::max<uint32_t>(g->tuning.sweep_group, 1u), 64u);
    std::vector<uint32_t> admitted;  // every slot taken, members included
    std::vector<uint32_t> leads;     // the slot that carries each new query
    {
        std::unique_lock<std::mutex> lk(s->mu);
        uint32_t active = 0;
        for (auto &sl : s->slots) active += sl.busy;
        if (active == 0 && s->waiting.empty()) {
            if (s->stop) return 1;
            s->cv.wait_for(lk, std::chrono::milliseconds(5));
            return 0;
        }
        uint32_t busy = active;
        while (!s->waiting.empty()) {
            // a sweep takes a group of slots only while the pool has room for
            // a group per waiting query: groups answer sooner but do more
            // work in all, so a saturated server steps on one slot.
            // rmat20-32m, 60/20/20 mix, 256 slots: one slot per sweep p99
            // 24.6 ms at 1k q/s, 6,159 q/s at saturation; groups of 8 always
            // 9.4 ms, 5,104 q/s; groups of 8 while there is room 9.6 ms,
            // 6,241 q/s
            const bool room = (uint64_t)s->waiting.size() * group + busy <= s->opts.max_slots;
            const uint32_t want = s->waiting.front().kind == 0 || !room ? 1u : group;
            std::pair<uint32_t, uint32_t> run = free_run(s, want);
            if (run.second < want && s->cap < s->opts.max_slots) {
                const uint32_t ncap = std::min<uint32_t>(s->opts.max_slots, std::max<uint32_t>(4, s->cap * 2));
                lk.unlock();
                const bool ok = grow(s, ncap);
                lk.lock();
                if (ok) continue;
                s->stats.admitted_waits_mem += 1;
            }
            if (run.second == 0) break;  // a sweep takes fewer slots rather than wait
            SlotRun &sl = s->slots[run.first];
            sl = SlotRun{};
            sl.busy = true;
            sl.started = true;
            sl.q = s->waiting.front();
            sl.width = run.second;
            s->waiting.pop_front();
            for (uint32_t j = 1; j < run.second; ++j) {
                SlotRun &m = s->slots[run.first + j];
                m = SlotRun{};
                m.busy = true;
                m.started = true;
                m.lead = (int32_t)run.first;
            }
            for (uint32_t j = 0; j < run.second; ++j) admitted.push_back(run.first + j);
            leads.push_back(run.first);
            busy += run.second;
        }
        uint32_t act = 0;
        for (auto &sl : s->slots) act += sl.busy;
        s->stats.active_slots = act;
        s->stats.waiting = (uint32_t)s->waiting.size();
        s->stats.max_slots_seen = std::max(s->stats.max_slots_seen, act);
        if (act == 0) {
            // nothing can run: queries wait for memory
            if (s->stop) {
                // shutting down and nothing will ever free memory for them
                while (!s->waiting.empty()) {
                    complete(s, s->waiting.front(), KAIROS_ERR_NOMEM, now_ns());
                    s->waiting.pop_front();
                }
                return 1;
            }
            s->cv.wait_for(lk, std::chrono::milliseconds(1));
            return 0;
        }
    }
    // start the new queries: reset their slots; an earliest-arrival source
    // joins the shared frontier; a sweep lists its departure times on the
    // device, then either steps through them on its one slot or runs them a
    // group at a time on its consecutive slots
    Inject *h_inj = (Inject *)(s->h_pin + pl.inject);
    uint32_t *h_init = s->h_pin + pl.init;
    uint32_t *h_sweep = s->h_pin + pl.sweep;
    GroupStart *h_admit = (GroupStart *)(s->h_pin + pl.start_admit);
    uint32_t n_inj = 0, n_sweep = 0, n_admit = 0;
    for (uint32_t slot : leads) {
        const SlotRun &sl = s->slots[slot];
        const uint32_t src = g->h_perm[sl.q.src];
        const uint32_t sweep = sl.q.kind != 0 ? 1u : 0u;
        h_inj[n_inj++] = Inject{slot, src, sl.q.ta, sl.q.tw, INF, sweep, 0, 0};
        if (sweep) h_sweep[n_sweep++] = slot;
        if (sweep && sl.width > 1) h_admit[n_admit++] = GroupStart{slot, sl.width, 0, src, sl.q.tw, 0, 0, 0};
    }
    for (size_t i = 0; i < admitted.size(); ++i) h_init[i] = admitted[i];
    int rc = multi_init_slots(g, &s->ms, h_init, (uint32_t)admitted.size());
    if (rc) return rc;
    if ((rc = multi_inject(g, &s->ms, h_inj, n_inj))) return rc;
    if ((rc = multi_sweep_steps(g, &s->ms, h_sweep, n_sweep))) return rc;
    if ((rc = multi_group_start(g, &s->ms, h_admit, n_admit))) return rc;
    bool stepping = false, grouped = false;
    for (uint32_t slot = 0; slot < s->cap; ++slot) {
        const SlotRun &sl = s->slots[slot];
        if (!sl.busy || sl.lead >= 0 || sl.q.kind == 0) continue;
        stepping |= sl.width == 1;
        grouped |= sl.width > 1;
    }
    // a few rounds per host check; single-slot sweeps step between rounds
    // on the device.  Every launch reads its frontier size on the device,
    // so a round whose frontier ran empty costs only its launches.
    if (stepping && (rc = multi_advance(g, &s->ms))) return rc;
    for (uint32_t k = 0; k < s->rounds_per_check; ++k) {
        if ((rc = multi_push_round(g, &s->ms))) return rc;
        if (stepping && (rc = multi_advance(g, &s->ms))) return rc;
    }
    const size_t rb = CNT_WORDS + s->cap;
    KAIROS_HIP(hipMemcpyAsync(s->h_pin + pl.flags, s->ms.cnt, rb * 4, hipMemcpyDeviceToHost, st));
    if (grouped)
        KAIROS_HIP(hipMemcpyAsync(s->h_pin + pl.step_cnt, s->ms.step_cnt, (size_t)s->cap * 4, hipMemcpyDeviceToHost,
                                  st));
    KAIROS_HIP(hipStreamSynchronize(st));
    const uint32_t *flags = s->h_pin + pl.flags + CNT_WORDS;
    const uint32_t *step_cnt = s->h_pin + pl.step_cnt;
    // finishing: a slot with no frontier work (and no step left); a group
    // whose members all ran dry folds into its lead, then takes the next
    // departure times (warm-started from its last member) or finishes
    std::vector<uint32_t> finished;
    GroupStart *h_next = (GroupStart *)(s->h_pin + pl.start_next);
    uint32_t n_next = 0;
    for (uint32_t slot = 0; slot < s->cap; ++slot) {
        SlotRun &sl = s->slots[slot];
        if (!sl.busy || !sl.started || sl.lead >= 0) continue;
        bool idle = true;
        for (uint32_t j = 0; j < sl.width; ++j) idle = idle && flags[slot + j] != s->ms.round;
        if (!idle) continue;
        if (sl.width == 1) {
            finished.push_back(slot);
            continue;
        }
        if ((rc = multi_group_reduce(g, &s->ms, slot, sl.width))) return rc;
        if (sl.pos0 + sl.width < step_cnt[slot]) {
            if ((rc = multi_group_warm(g, &s->ms, slot, sl.width, sl.width - 1))) return rc;
            sl.pos0 += sl.width;
            h_next[n_next++] = GroupStart{slot, sl.width, sl.pos0, g->h_perm[sl.q.src], sl.q.tw, 0, 0, 0};
        } else {
            finished.push_back(slot);
        }
    }
    if ((rc = multi_group_start(g, &s->ms, h_next, n_next))) return rc;
    if (!finished.empty()) {
        for (uint32_t slot : finished) {
            const Query &q = s->slots[slot].q;
            if ((rc = multi_finalize(g, &s->ms, slot, q.kind, q.src, q.tw, q.out))) return rc;
        }
        KAIROS_HIP(hipStreamSynchronize(st));
        const uint64_t t = now_ns();
        std::lock_guard<std::mutex> lk(s->mu);
        for (uint32_t slot : finished) {
            complete(s, s->slots[slot].q, KAIROS_OK, t);
            const uint32_t w = s->slots[slot].width;
            for (uint32_t j = 0; j < w; ++j) s->slots[slot + j] = SlotRun{};
        }
        uint32_t act = 0;
        for (auto &sl : s->slots) act += sl.busy;
        s->stats.active_slots = act;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.iterations += 1;
    }
    return 0;
}

void scheduler(kairos_server *s)
{
    for (;;) {
        int rc = iterate(s);
        if (rc == 1) break;
        if (rc != 0) {
            fail_all(s);
            std::unique_lock<std::mutex> lk(s->mu);
            while (!s->stop) {
                while (!s->waiting.empty()) {
                    complete(s, s->waiting.front(), KAIROS_ERR_DEVICE, now_ns());
                    s->waiting.pop_front();
                }
                s->cv.wait_for(lk, std::chrono::milliseconds(5));
            }
            while (!s->waiting.empty()) {
                complete(s, s->waiting.front(), KAIROS_ERR_DEVICE, now_ns());
                s->waiting.pop_front();
            }
            break;
        }
    }
}

}  // namespace

extern "C" {

int kairos_server_create(kairos_graph *g, const kairos_server_opts *opts, kairos_server **out)
{
    if (!g || !opts || !out || opts->max_slots == 0 || opts->queue_capacity == 0) return KAIROS_ERR_INVALID;
    if ((uint64_t)opts->max_slots * g->n >= 0xFFFFFFF0ull) return KAIROS_ERR_RANGE;
    kairos_server *s = new (std::nothrow) kairos_server();
    if (!s) return KAIROS_ERR_NOMEM;
    s->g = g;
    s->opts = *opts;
    // 4 rounds per check: rmat20-32m, 2,000 queries 60/20/20, Poisson at
    // 50k/s: 1/2/4/8 rounds 2,530/2,962/3,168/3,357 q/s; at 2k/s p50
    // 0.21/0.32/0.47/0.71 ms, p99 34/30/24/22 ms
    s->rounds_per_check = opts->rounds_per_check ? std::min<uint32_t>(opts->rounds_per_check, 64) : 4u;
    s->per_slot_chunks = g->m / std::max<uint32_t>(g->tuning.chunk, 64) +
                         g->m / std::max<uint32_t>(g->tuning.split, 64) + 1;
    if (opts->hip_stream) {
        s->ms.stream = (hipStream_t)opts->hip_stream;
    } else if (hipStreamCreateWithFlags(&s->ms.stream, hipStreamNonBlocking) == hipSuccess) {
        s->own_stream = true;
    } else {
        delete s;
        return KAIROS_ERR_DEVICE;
    }
    if (hipHostMalloc((void **)&s->h_pin, pin_words(opts->max_slots) * 4, hipHostMallocDefault) != hipSuccess) {
        if (s->own_stream) hipStreamDestroy(s->ms.stream);
        delete s;
        return KAIROS_ERR_NOMEM;
    }
    s->ms.n = g->n;
    s->th = std::thread(scheduler, s);
    *out = s;
    return KAIROS_OK;
}

int kairos_server_submit(kairos_server *s, int kind, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                         uint32_t *out, uint64_t *ticket)
{
    if (!s || !out || !ticket || kind < 0 || kind > 2) return KAIROS_ERR_INVALID;
    if (src >= s->g->n || t_alpha > t_omega || t_omega > KAIROS_TMAX) return KAIROS_ERR_RANGE;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->waiting.size() >= s->opts.queue_capacity) return KAIROS_ERR_BUSY;
    Query q{s->next_ticket++, kind, src, t_alpha, t_omega, out, now_ns()};
    *ticket = q.ticket;
    s->stats.submitted += 1;
    if (s->failed) {
        complete(s, q, KAIROS_ERR_DEVICE, now_ns());
        return KAIROS_OK;
    }
    s->waiting.push_back(q);
    s->stats.waiting = (uint32_t)s->waiting.size();
    s->cv.notify_one();
    return KAIROS_OK;
}

int kairos_server_poll(kairos_server *s, kairos_completion *done, uint32_t cap, uint32_t *n_done)
{
    if (!s || !n_done || (cap && !done)) return KAIROS_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    uint32_t k = 0;
    while (k < cap && !s->done.empty()) {
        done[k++] = s->done.front();
        s->done.pop_front();
    }
    *n_done = k;
    return KAIROS_OK;
}

int kairos_server_stats_read(kairos_server *s, kairos_server_stats *out)
{
    if (!s || !out) return KAIROS_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->pool_slots = s->cap;
    out->slot_bytes = slot_bytes(s);
    return KAIROS_OK;
}

int kairos_server_set_free_bytes_override(kairos_server *s, uint64_t bytes)
{
    if (!s) return KAIROS_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    s->free_override = bytes;
    return KAIROS_OK;
}

void kairos_server_free(kairos_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    hipStream_t st = s->ms.stream;  // free_state clears the struct
    (void)hipStreamSynchronize(st);
    free_state(s->ms);
    if (s->h_pin) (void)hipHostFree(s->h_pin);
    if (s->own_stream) (void)hipStreamDestroy(st);
    delete s;
}

}  // extern "C"
