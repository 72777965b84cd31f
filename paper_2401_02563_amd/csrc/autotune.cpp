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
// one batch) drops by more than 2%.  The workgroup size of the push and chunk
// kernels is one of the axes.  The sweep group width (departure times per
// group of a latest-departure / fastest sweep) is then tuned on its own
// objective: latest-departure queries from the first two sample sources.
//
// Cache: when KAIROS_TUNING_CACHE names a file, a setting found for a graph
// is stored there under a key of the device (architecture and compute units),
// the index's shape (n, m, vertices with out-edges, largest out-degree,
// repeated heads, largest departure) and the sample form (one query or a
// batch); a later call with the same key takes the stored setting without
// measuring.  One line per key: the key, then the 15 tuning fields in
// declaration order.
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

using namespace kairos;

namespace {

double seconds_now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int run_sample(kairos_graph *g, int form, uint32_t q, const uint32_t *src, const uint32_t *ta, const uint32_t *tw,
               uint32_t *d_single, uint32_t *d_batch, double *secs)
{
    // the one-query form answers the sample one query per call, the batch
    // form as one batch
    const double t0 = seconds_now();
    if (form == KAIROS_TUNE_SINGLE) {
        for (uint32_t i = 0; i < q; ++i) {
            int rc = kairos_earliest_arrival(g, src[i], ta[i], tw[i], d_single);
            if (rc) return rc;
        }
    } else {
        int rc = kairos_earliest_arrival_batch(g, q, src, ta, tw, d_batch);
        if (rc) return rc;
    }
    *secs = seconds_now() - t0;
    return KAIROS_OK;
}

int measure(kairos_graph *g, int form, const kairos_tuning &t, uint32_t q, const uint32_t *src, const uint32_t *ta,
            const uint32_t *tw, uint32_t *d1, uint32_t *db, double *out)
{
    int rc = kairos_set_tuning(g, &t);
    if (rc) return rc;
    double warm;
    if ((rc = run_sample(g, form, q, src, ta, tw, d1, db, &warm))) return rc;
    double v[3];
    for (double &x : v)
        if ((rc = run_sample(g, form, q, src, ta, tw, d1, db, &x))) return rc;
    std::sort(v, v + 3);
    *out = v[1];
    return KAIROS_OK;
}

int measure_sweep(kairos_graph *g, const kairos_tuning &t, uint32_t q, const uint32_t *src, const uint32_t *ta,
                  const uint32_t *tw, uint32_t *d1, double *out)
{
    int rc = kairos_set_tuning(g, &t);
    if (rc) return rc;
    const uint32_t k = std::min<uint32_t>(q, 2);
    double v[4];
    for (double &x : v) {
        const double t0 = seconds_now();
        for (uint32_t i = 0; i < k; ++i)
            if ((rc = kairos_latest_departure(g, src[i], ta[i], tw[i], d1))) return rc;
        x = seconds_now() - t0;
    }
    std::sort(v + 1, v + 4);  // v[0] warms the sweep state up
    *out = v[2];
    return KAIROS_OK;
}

constexpr int NFIELDS = 15;
uint32_t *field(kairos_tuning &t, int i)
{
    uint32_t *f[NFIELDS] = {&t.block, &t.chunk, &t.split, &t.pull_alpha, &t.pull_beta, &t.rounds_per_sync,
                            &t.batch_persistent, &t.sweep_group, &t.batch_layout, &t.tail_limit,
                            &t.dense_frontier, &t.arrival_filter, &t.single_persistent, &t.run_dedupe,
                            &t.binned};
    return f[i];
}

std::string cache_key(kairos_graph *g, int form)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch.resize(colon);
    }
    std::ostringstream k;
    k << arch << "/cu" << g->num_cus << "/n" << g->n << "/m" << g->m << "/live" << g->n_live << "/deg"
      << g->max_out_degree << "/rep" << g->repeat_heads << "/tmax" << g->max_t
      << (form == KAIROS_TUNE_SINGLE ? "/single" : "/batch");
    return k.str();
}

bool cache_lookup(const char *path, const std::string &key, kairos_tuning *t)
{
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string k;
        if (!(in >> k) || k != key) continue;
        kairos_tuning c{};
        bool ok = true;
        for (int i = 0; i < NFIELDS && ok; ++i) ok = static_cast<bool>(in >> *field(c, i));
        if (ok) {
            *t = c;  // the last line for a key wins
            found = true;
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &key, kairos_tuning t)
{
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line)) {
            std::istringstream in(line);
            std::string k;
            if ((in >> k) && k != key) keep.push_back(line);
        }
    }
    std::ostringstream row;
    row << key;
    for (int i = 0; i < NFIELDS; ++i) row << ' ' << *field(t, i);
    keep.push_back(row.str());
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp, std::ios::trunc);
        for (const std::string &l : keep) o << l << '\n';
        if (!o) return;  // the cache is an optimisation: a failed write is not an error
    }
    std::rename(tmp.c_str(), path);
}

}  // namespace

extern "C" int kairos_autotune(kairos_graph *g, uint32_t q, const uint32_t *src, const uint32_t *t_alpha,
                               const uint32_t *t_omega, kairos_tuning *best_out)
{
    return kairos_autotune_form(g, q == 1 ? KAIROS_TUNE_SINGLE : KAIROS_TUNE_BATCH, q, src, t_alpha, t_omega,
                                best_out);
}

extern "C" int kairos_autotune_form(kairos_graph *g, int form, uint32_t q, const uint32_t *src,
                                    const uint32_t *t_alpha, const uint32_t *t_omega, kairos_tuning *best_out)
{
    if (!g || (q && (!src || !t_alpha || !t_omega))) return KAIROS_ERR_INVALID;
    if (form != KAIROS_TUNE_SINGLE && form != KAIROS_TUNE_BATCH) return KAIROS_ERR_INVALID;
    for (uint32_t i = 0; i < q; ++i)
        if (src[i] >= g->n || t_alpha[i] > t_omega[i] || t_omega[i] > KAIROS_TMAX) return KAIROS_ERR_RANGE;
    if (q == 0) {
        if (best_out) *best_out = g->tuning;
        return KAIROS_OK;
    }
    const char *cache = std::getenv("KAIROS_TUNING_CACHE");
    const std::string key = cache && *cache ? cache_key(g, form) : std::string();
    if (!key.empty()) {
        kairos_tuning c{};
        if (cache_lookup(cache, key, &c) && kairos_set_tuning(g, &c) == KAIROS_OK) {
            if (best_out) *best_out = g->tuning;
            return KAIROS_OK;
        }
    }
    const uint32_t qb = form == KAIROS_TUNE_SINGLE
                            ? q
                            : (uint32_t)std::min<uint64_t>(q, std::max<uint64_t>(1, 0xFFFFFFFEull / g->n));
    const bool batch = form == KAIROS_TUNE_BATCH;
    uint32_t *d1 = (uint32_t *)dev_alloc((size_t)g->n * 4, nullptr);
    uint32_t *db = batch ? (uint32_t *)dev_alloc((size_t)qb * g->n * 4, nullptr) : nullptr;
    if (!d1 || (batch && !db)) {
        dev_free(d1);
        dev_free(db);
        return KAIROS_ERR_NOMEM;
    }
    kairos_tuning best = g->tuning;
    double best_t = 0;
    int rc = measure(g, form, best, qb, src, t_alpha, t_omega, d1, db, &best_t);
    struct Axis {
        uint32_t kairos_tuning::*field;
        std::vector<uint32_t> values;
    };
    const std::vector<Axis> axes = {
        {&kairos_tuning::block, {256, 512}},
        {&kairos_tuning::batch_layout, {0, 1, 2, 3}},
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
        {&kairos_tuning::binned, {0, 1u << 14, 1u << 16, 1u << 18, 1u << 20}},
    };
    for (const Axis &ax : axes) {
        if (rc) break;
        if (ax.field == &kairos_tuning::pull_beta && best.pull_alpha == 0) continue;
        for (uint32_t v : ax.values) {
            if (best.*(ax.field) == v) continue;
            kairos_tuning t = best;
            t.*(ax.field) = v;
            double secs;
            if ((rc = measure(g, form, t, qb, src, t_alpha, t_omega, d1, db, &secs))) break;
            if (secs < best_t * 0.98) {
                best_t = secs;
                best = t;
            }
        }
    }
    // the sweep group width, on latest-departure queries of the sample
    if (!rc) {
        double sweep_t = 0;
        rc = measure_sweep(g, best, q, src, t_alpha, t_omega, d1, &sweep_t);
        for (uint32_t v : {1u, 4u, 8u, 16u, 64u}) {
            if (rc || best.sweep_group == v) continue;
            kairos_tuning t = best;
            t.sweep_group = v;
            double secs;
            if ((rc = measure_sweep(g, t, q, src, t_alpha, t_omega, d1, &secs))) break;
            if (secs < sweep_t * 0.98) {
                sweep_t = secs;
                best = t;
            }
        }
    }
    int rc2 = kairos_set_tuning(g, &best);
    dev_free(d1);
    dev_free(db);
    if (rc) return rc;
    if (rc2) return rc2;
    if (!key.empty()) cache_store(cache, key, best);
    if (best_out) *best_out = best;
    return KAIROS_OK;
}
