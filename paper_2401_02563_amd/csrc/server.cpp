// Continuous-batching query server.
//
// A scheduler thread owns a pool of query slots on the device.  Each
// iteration it (1) admits waiting queries into free slots, growing the slot
// pool when the device reports enough free memory, (2) starts them (slot
// state reset; an earliest-arrival source goes into the shared frontier, a
// latest-departure / fastest slot gets its departure times listed on the
// device), (3) runs a few push rounds, each over every active slot in one
// launch, and (4) reads back the per-slot activity flags.  Between rounds a
// device kernel moves every sweep slot whose frontier emptied to its next
// departure time, so a sweep needs no host round trip per step.  A slot
// with no frontier and no steps left is finished: its result is written to
// the caller's buffer and a completion with timestamps is queued for
// polling.  Queries that arrive while others run join at the next
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
    uint32_t *h_pin = nullptr;  // pinned: counters+flags | inject list | init list | sweep list
    uint64_t per_slot_chunks = 0;
    uint32_t rounds_per_check = 4;
};

namespace {

size_t pin_words(uint32_t max_slots)
{
    return CNT_WORDS + (size_t)max_slots + 8 * (size_t)max_slots + 2 * (size_t)max_slots + 64;
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
// Called between rounds only.  Returns false if memory is short.
bool grow(kairos_server *s, uint32_t ncap)
{
    if (ncap <= s->cap) return true;
    const uint64_t need = slot_bytes(s) * (ncap - s->cap);
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
    for (auto &sl : s->slots)
        if (sl.busy) {
            complete(s, sl.q, KAIROS_ERR_DEVICE, t);
            sl = SlotRun{};
        }
    while (!s->waiting.empty()) {
        complete(s, s->waiting.front(), KAIROS_ERR_DEVICE, t);
        s->waiting.pop_front();
    }
    s->stats.active_slots = 0;
    s->stats.waiting = 0;
}

int iterate(kairos_server *s, std::vector<Inject> &pending, uint32_t &front)
{
    kairos_graph *g = s->g;
    hipStream_t st = s->ms.stream;
    std::vector<uint32_t> admitted;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        uint32_t active = 0;
        for (auto &sl : s->slots) active += sl.busy;
        if (active == 0 && s->waiting.empty() && pending.empty()) {
            if (s->stop) return 1;
            s->cv.wait_for(lk, std::chrono::milliseconds(5));
            return 0;
        }
        while (!s->waiting.empty()) {
            int slot = -1;
            for (uint32_t i = 0; i < s->cap; ++i)
                if (!s->slots[i].busy) {
                    slot = (int)i;
                    break;
                }
            if (slot < 0) {
                if (s->cap >= s->opts.max_slots) break;
                const uint32_t ncap = std::min<uint32_t>(s->opts.max_slots, std::max<uint32_t>(4, s->cap * 2));
                lk.unlock();
                const bool ok = grow(s, ncap);
                lk.lock();
                if (!ok) {
                    s->stats.admitted_waits_mem += 1;
                    break;
                }
                continue;
            }
            SlotRun &sl = s->slots[slot];
            sl = SlotRun{};
            sl.busy = true;
            sl.q = s->waiting.front();
            s->waiting.pop_front();
            admitted.push_back((uint32_t)slot);
        }
        uint32_t act = 0;
        for (auto &sl : s->slots) act += sl.busy;
        s->stats.active_slots = act;
        s->stats.waiting = (uint32_t)s->waiting.size();
        s->stats.max_slots_seen = std::max(s->stats.max_slots_seen, act);
        if (act == 0 && pending.empty()) {
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
    std::vector<uint32_t> sweeps;
    for (uint32_t slot : admitted) {
        SlotRun &sl = s->slots[slot];
        const uint32_t sweep = sl.q.kind != 0 ? 1u : 0u;
        pending.push_back(Inject{slot, g->h_perm[sl.q.src], sl.q.ta, sl.q.tw, INF, sweep, 0, 0});
        if (sweep) sweeps.push_back(slot);
        sl.started = true;
    }
    // pinned layout: [0, CNT_WORDS + max_slots) read-back | inject list |
    // init list | sweep list
    Inject *h_inj = (Inject *)(s->h_pin + CNT_WORDS + s->opts.max_slots);
    uint32_t *h_init = s->h_pin + CNT_WORDS + s->opts.max_slots + 8 * (size_t)s->opts.max_slots;
    uint32_t *h_sweep = h_init + s->opts.max_slots;
    for (size_t i = 0; i < admitted.size(); ++i) h_init[i] = admitted[i];
    for (size_t i = 0; i < sweeps.size(); ++i) h_sweep[i] = sweeps[i];
    int rc = multi_init_slots(g, &s->ms, h_init, (uint32_t)admitted.size());
    if (rc) return rc;
    for (size_t i = 0; i < pending.size(); ++i) h_inj[i] = pending[i];
    if ((rc = multi_inject(g, &s->ms, h_inj, (uint32_t)pending.size()))) return rc;
    if ((rc = multi_sweep_steps(g, &s->ms, h_sweep, (uint32_t)sweeps.size()))) return rc;
    front += (uint32_t)pending.size();
    pending.clear();
    bool any_sweep = false;
    for (uint32_t slot = 0; slot < s->cap; ++slot)
        any_sweep |= s->slots[slot].busy && s->slots[slot].q.kind != 0;
    // a few rounds per host check; sweep slots step between rounds on the
    // device.  Every launch reads its frontier size on the device, so a
    // round whose frontier ran empty costs only its launch.
    if (front > 0 || any_sweep) {
        if (any_sweep && (rc = multi_advance(g, &s->ms))) return rc;
        for (uint32_t k = 0; k < s->rounds_per_check; ++k) {
            if ((rc = multi_push_round(g, &s->ms))) return rc;
            if (any_sweep && (rc = multi_advance(g, &s->ms))) return rc;
        }
    }
    // finishing: slots with no frontier (and no step left) after the rounds
    const size_t rb = CNT_WORDS + s->cap;
    KAIROS_HIP(hipMemcpyAsync(s->h_pin, s->ms.cnt, rb * 4, hipMemcpyDeviceToHost, st));
    KAIROS_HIP(hipStreamSynchronize(st));
    front = s->h_pin[CNT_FRONT + s->ms.round % 3u];
    const uint32_t *flags = s->h_pin + CNT_WORDS;
    std::vector<uint32_t> finished;
    for (uint32_t slot = 0; slot < s->cap; ++slot) {
        SlotRun &sl = s->slots[slot];
        if (!sl.busy || !sl.started) continue;
        if (flags[slot] == s->ms.round) continue;  // still has frontier work
        finished.push_back(slot);
    }
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
            s->slots[slot] = SlotRun{};
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
    std::vector<Inject> pending;
    uint32_t front = 0;
    for (;;) {
        int rc = iterate(s, pending, front);
        if (rc == 1) break;
        if (rc != 0) {
            fail_all(s);
            pending.clear();
            front = 0;
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
