// Autotuner: picks the run-time parameters by measurement on a sample of
// the caller's own queries.  The paper fixes its equivalents (the cost
// constants c and c' of Eq. 1-2, the selectivity threshold of Eq. 3, the
// 2k-edge index cut-off of §5 and the parallel-loop grain of §6.1) by
// experiment; here they are the chunking of long adjacencies, the push/pull
// switch thresholds, the number of rounds queued between host checks and
// the batched launch mode.  None of them changes a result.
//
// Search: coordinate descent from the current setting, one parameter at a
// time over its candidate values, keeping a change only when the measured
// time (median of three runs of the sample: one query alone, or the sample as
// one batch) drops by more than 2%.
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <vector>

using namespace kairos;

namespace {

double seconds_now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int run_sample(kairos_graph *g, uint32_t q, const uint32_t *src, const uint32_t *ta, const uint32_t *tw,
               uint32_t *d_single, uint32_t *d_batch, double *secs)
{
    // a sample of one query tunes the single-query path, a larger sample the
    // batched path it will be answered with
    const double t0 = seconds_now();
    if (q == 1) {
        int rc = kairos_earliest_arrival(g, src[0], ta[0], tw[0], d_single);
        if (rc) return rc;
    } else {
        int rc = kairos_earliest_arrival_batch(g, q, src, ta, tw, d_batch);
        if (rc) return rc;
    }
    *secs = seconds_now() - t0;
    return KAIROS_OK;
}

int measure(kairos_graph *g, const kairos_tuning &t, uint32_t q, const uint32_t *src, const uint32_t *ta,
            const uint32_t *tw, uint32_t *d1, uint32_t *db, double *out)
{
    int rc = kairos_set_tuning(g, &t);
    if (rc) return rc;
    double warm;
    if ((rc = run_sample(g, q, src, ta, tw, d1, db, &warm))) return rc;
    double v[3];
    for (double &x : v)
        if ((rc = run_sample(g, q, src, ta, tw, d1, db, &x))) return rc;
    std::sort(v, v + 3);
    *out = v[1];
    return KAIROS_OK;
}

}  // namespace

extern "C" int kairos_autotune(kairos_graph *g, uint32_t q, const uint32_t *src, const uint32_t *t_alpha,
                               const uint32_t *t_omega, kairos_tuning *best_out)
{
    if (!g || (q && (!src || !t_alpha || !t_omega))) return KAIROS_ERR_INVALID;
    for (uint32_t i = 0; i < q; ++i)
        if (src[i] >= g->n || t_alpha[i] > t_omega[i] || t_omega[i] > KAIROS_TMAX) return KAIROS_ERR_RANGE;
    if (q == 0) {
        if (best_out) *best_out = g->tuning;
        return KAIROS_OK;
    }
    const uint32_t qb = (uint32_t)std::min<uint64_t>(q, std::max<uint64_t>(1, 0xFFFFFFFEull / g->n));
    uint32_t *d1 = (uint32_t *)dev_alloc((size_t)g->n * 4, nullptr);
    uint32_t *db = qb > 1 ? (uint32_t *)dev_alloc((size_t)qb * g->n * 4, nullptr) : nullptr;
    if (!d1 || (qb > 1 && !db)) {
        dev_free(d1);
        dev_free(db);
        return KAIROS_ERR_NOMEM;
    }
    kairos_tuning best = g->tuning;
    double best_t = 0;
    int rc = measure(g, best, qb, src, t_alpha, t_omega, d1, db, &best_t);
    struct Axis {
        uint32_t kairos_tuning::*field;
        std::vector<uint32_t> values;
    };
    const std::vector<Axis> axes = {
        {&kairos_tuning::batch_layout, {0, 1, 2}},
        {&kairos_tuning::split, {64, 128, 256, 1024}},
        {&kairos_tuning::chunk, {128, 256, 512, 2048}},
        {&kairos_tuning::tail_limit, {0, 1024, 4096, 16384}},
        {&kairos_tuning::dense_frontier, {0, 4, 16, 64}},
        {&kairos_tuning::arrival_filter, {0, 2, 4, 8}},
        {&kairos_tuning::batch_persistent, {0, 1}},
        {&kairos_tuning::single_persistent, {0, 1}},
        {&kairos_tuning::run_dedupe, {0, 1}},
        {&kairos_tuning::rounds_per_sync, {1, 2, 4}},
        {&kairos_tuning::pull_alpha, {0, 4, 14}},
        {&kairos_tuning::pull_beta, {8, 24, 64}},
    };
    for (const Axis &ax : axes) {
        if (rc) break;
        if (ax.field == &kairos_tuning::pull_beta && best.pull_alpha == 0) continue;
        for (uint32_t v : ax.values) {
            if (best.*(ax.field) == v) continue;
            kairos_tuning t = best;
            t.*(ax.field) = v;
            double secs;
            if ((rc = measure(g, t, qb, src, t_alpha, t_omega, d1, db, &secs))) break;
            if (secs < best_t * 0.98) {
                best_t = secs;
                best = t;
            }
        }
    }
    int rc2 = kairos_set_tuning(g, &best);
    dev_free(d1);
    dev_free(db);
    if (rc) return rc;
    if (rc2) return rc2;
    if (best_out) *best_out = best;
    return KAIROS_OK;
}
