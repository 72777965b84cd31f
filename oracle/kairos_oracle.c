/*
 * CPU oracle for temporal minimal-path queries -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct reference computations used by the test
 * suite, the smoke check and the CPU baseline of the benchmark to check the
 * GPU library.  Nothing in the library links or calls this file, and this
 * file uses nothing from the library.
 *
 * Model (paper §2.1, §2.2): a temporal edge e = (u, v, t, a) departs u at
 * time t and arrives at v at time a = t + lambda, lambda >= 1.  A path is
 * time-respecting when each edge departs no earlier than the previous one
 * arrives ("Succeeds": end(A) <= start(B)).  A query (src, [t_alpha,
 * t_omega]) only uses edges with t >= t_alpha and a <= t_omega (the closed
 * query interval of Alg. 2).
 *
 *   EA[v] = min arrival at v over such paths from src     (EA[src] = t_alpha)
 *   LD[v] = max departure from src over such paths to v   (LD[src] = t_omega)
 *   F[v]  = min (arrival at v - departure from src)        (F[src]  = 0)
 *   unreachable vertices get 0xFFFFFFFF in all three.
 *
 * The scans (earliest arrival, profiles, shortest duration) take the edge
 * list already sorted by departure time t (ascending; ties in any order) as
 * four parallel uint32 arrays; the traversed-edge count and the
 * earliest-arrival certificate take the edges in any order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_INF 0xFFFFFFFFu

/* first index in t[0..m) with t[i] >= key (t ascending) */
static uint64_t first_at_or_after(const uint32_t *t, uint64_t m, uint32_t key)
{
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (t[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/*
 * Earliest arrival by one pass over the edges in departure order, the
 * one-pass scheme the paper credits to its temporal-paths reference (§7).
 * When an edge departing at time t is examined, every edge that could
 * deliver a traveller to its tail by time t arrives at or before t and
 * therefore departed strictly earlier (lambda >= 1), so it has already been
 * examined: arr[u] is final as far as this edge is concerned.
 *
 * Returns the number of edges examined (those with t in [t_alpha, t_omega)).
 */
uint64_t oracle_earliest_arrival(uint64_t m, const uint32_t *src, const uint32_t *dst,
                                 const uint32_t *t, const uint32_t *a, uint32_t n,
                                 uint32_t source, uint32_t t_alpha, uint32_t t_omega,
                                 uint32_t *arr)
{
    for (uint32_t v = 0; v < n; ++v)
        arr[v] = ORACLE_INF;
    arr[source] = t_alpha;
    uint64_t e = first_at_or_after(t, m, t_alpha);
    uint64_t examined = 0;
    /* an edge departing at t >= t_omega arrives after t_omega: stop there */
    for (; e < m && t[e] < t_omega; ++e, ++examined) {
        uint32_t u = src[e], v = dst[e];
        if (a[e] <= t_omega && arr[u] <= t[e] && a[e] < arr[v])
            arr[v] = a[e];
    }
    return examined;
}

/*
 * Temporal edges traversed by a query: edges whose tail is reached and that
 * depart within the window no earlier than the tail's earliest arrival and
 * arrive within the window.  Uses the final EA array.
 */
uint64_t oracle_traversed_edges(uint64_t m, const uint32_t *src, const uint32_t *t,
                                const uint32_t *a, uint32_t t_alpha, uint32_t t_omega,
                                const uint32_t *arr)
{
    uint64_t count = 0;
    for (uint64_t e = 0; e < m; ++e) {
        uint32_t r = arr[src[e]];
        if (r == ORACLE_INF)
            continue;
        uint32_t lo = r > t_alpha ? r : t_alpha;
        if (t[e] >= lo && a[e] <= t_omega)
            ++count;
    }
    return count;
}

/* ---- Pareto profiles for latest departure and fastest path ---------------
 * Each vertex v keeps the non-dominated pairs (arr, dep): "a path leaving
 * src at dep reaches v at arr".  A pair (a1, s1) dominates (a2, s2) when
 * a1 <= a2 and s1 >= s2.  Kept sorted by arr ascending, which makes dep
 * ascending too.  Scanning edges in departure order, an edge (u, v, t, a)
 * extends the best pair of u that has arrived by t (the one with the latest
 * dep), or starts a new path when u is the source.
 */
typedef struct {
    uint32_t *arr;
    uint32_t *dep;
    uint32_t len, cap;
} profile_t;

static int profile_insert(profile_t *p, uint32_t a, uint32_t s)
{
    /* pairs with arr <= a form a prefix; its last has the largest dep */
    uint32_t lo = 0, hi = p->len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (p->arr[mid] <= a)
            lo = mid + 1;
        else
            hi = mid;
    }
    uint32_t k = lo; /* pairs [0,k) have arr <= a */
    if (k > 0 && p->dep[k - 1] >= s)
        return 0; /* dominated */
    /* the new pair dominates pairs with arr >= a and dep <= s: those with
     * arr == a sit at the end of the prefix, the rest at the start of the
     * suffix */
    uint32_t first = k;
    while (first > 0 && p->arr[first - 1] == a && p->dep[first - 1] <= s)
        --first;
    uint32_t last = k;
    while (last < p->len && p->dep[last] <= s)
        ++last;
    uint32_t removed = last - first;
    if (removed == 0) {
        if (p->len == p->cap) {
            uint32_t nc = p->cap ? 2 * p->cap : 4;
            uint32_t *na = realloc(p->arr, (size_t)nc * sizeof(uint32_t));
            if (!na)
                return -1;
            p->arr = na;
            uint32_t *nd = realloc(p->dep, (size_t)nc * sizeof(uint32_t));
            if (!nd)
                return -1;
            p->dep = nd;
            p->cap = nc;
        }
        memmove(p->arr + first + 1, p->arr + first, (size_t)(p->len - first) * sizeof(uint32_t));
        memmove(p->dep + first + 1, p->dep + first, (size_t)(p->len - first) * sizeof(uint32_t));
        p->len += 1;
    } else if (removed > 1) {
        memmove(p->arr + first + 1, p->arr + last, (size_t)(p->len - last) * sizeof(uint32_t));
        memmove(p->dep + first + 1, p->dep + last, (size_t)(p->len - last) * sizeof(uint32_t));
        p->len -= removed - 1;
    }
    p->arr[first] = a;
    p->dep[first] = s;
    return 1;
}

/* latest dep among pairs of p with arr <= t, or -1 */
static int64_t profile_best_by(const profile_t *p, uint32_t t)
{
    uint32_t lo = 0, hi = p->len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (p->arr[mid] <= t)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo ? (int64_t)p->dep[lo - 1] : -1;
}

/* Returns 0 on success, -1 on allocation failure.  Any output pointer may
 * be NULL. */
int oracle_profile(uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *t,
                   const uint32_t *a, uint32_t n, uint32_t source, uint32_t t_alpha,
                   uint32_t t_omega, uint32_t *ea, uint32_t *ld, uint32_t *fa)
{
    profile_t *P = calloc(n, sizeof(profile_t));
    if (!P)
        return -1;
    int rc = 0;
    uint64_t e = first_at_or_after(t, m, t_alpha);
    for (; e < m && t[e] < t_omega; ++e) {
        uint32_t u = src[e], v = dst[e];
        if (a[e] > t_omega || v == source)
            continue;
        int64_t s;
        if (u == source)
            s = t[e];
        else
            s = profile_best_by(&P[u], t[e]);
        if (s < 0)
            continue;
        if (profile_insert(&P[v], a[e], (uint32_t)s) < 0) {
            rc = -1;
            break;
        }
    }
    for (uint32_t v = 0; v < n; ++v) {
        uint32_t e_v = ORACLE_INF, l_v = ORACLE_INF, f_v = ORACLE_INF;
        if (v == source) {
            e_v = t_alpha;
            l_v = t_omega;
            f_v = 0;
        } else if (P[v].len) {
            e_v = P[v].arr[0];
            l_v = P[v].dep[P[v].len - 1];
            for (uint32_t i = 0; i < P[v].len; ++i) {
                uint32_t d = P[v].arr[i] - P[v].dep[i];
                if (d < f_v)
                    f_v = d;
            }
        }
        if (ea)
            ea[v] = e_v;
        if (ld)
            ld[v] = l_v;
        if (fa)
            fa[v] = f_v;
        free(P[v].arr);
        free(P[v].dep);
    }
    free(P);
    return rc;
}

/*
 * Earliest-arrival certificate: returns 1 iff A is exactly the
 * earliest-arrival array of the query, 0 otherwise.  Edges in any order.
 *   (i)   A[source] == t_alpha, and every finite A[v] lies in the window;
 *   (ii)  every finite A[v], v != source, equals the arrival of a usable
 *         edge (u, v, t, a) whose tail has arrived by its departure,
 *         A[u] <= t (a witness);
 *   (iii) no usable edge with A[u] <= t arrives before A[v].
 * By (ii) A strictly decreases back along witnesses to the source (lambda
 * >= 1), so each finite A[v] is the arrival of a real path: A >= EA.  By
 * (iii), induction along any time-respecting path gives A <= EA.  Usable:
 * t >= t_alpha and a <= t_omega.  `witnessed` is caller scratch of n bytes.
 */
int oracle_ea_certificate(uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *t,
                          const uint32_t *a, uint32_t n, uint32_t source, uint32_t t_alpha,
                          uint32_t t_omega, const uint32_t *A, uint8_t *witnessed)
{
    if (source >= n || A[source] != t_alpha)
        return 0;
    for (uint32_t v = 0; v < n; ++v) {
        witnessed[v] = 0;
        if (A[v] != ORACLE_INF && (A[v] < t_alpha || A[v] > t_omega))
            return 0;
    }
    for (uint64_t e = 0; e < m; ++e) {
        uint32_t u = src[e], v = dst[e];
        if (t[e] < t_alpha || a[e] > t_omega || A[u] == ORACLE_INF || A[u] > t[e])
            continue;
        if (a[e] < A[v])
            return 0; /* (iii) */
        if (a[e] == A[v])
            witnessed[v] = 1;
    }
    for (uint32_t v = 0; v < n; ++v)
        if (v != source && A[v] != ORACLE_INF && !witnessed[v])
            return 0; /* (ii) */
    return 1;
}

/* ---- Shortest duration ------------------------------------------------------
 * SD[v] = least total duration (sum of lambda over its edges) of a
 * time-respecting path from the source to v within the window; SD[src] = 0
 * (the "S. Duration" row of Table 4).  Waiting at a vertex costs nothing, so
 * a later arrival with a smaller total can still matter: each vertex keeps
 * the non-dominated pairs (arrival, duration) of the paths found so far.  A
 * pair (a1, d1) dominates (a2, d2) when a1 <= a2 and d1 <= d2.  Kept sorted
 * by arrival ascending, which makes duration strictly descending.  Scanning
 * edges in departure order, an edge (u, v, t, a) extends the pair of u with
 * the least duration among those that have arrived by t -- the last pair
 * with arrival <= t -- or starts at the source (duration 0 at any time from
 * t_alpha on).  Pairs of u that have arrived by t all come from edges that
 * departed before t (lambda >= 1), which the scan has already examined.
 */
typedef struct {
    uint32_t *arr;
    uint32_t *dur;
    uint32_t len, cap;
} dprofile_t;

/* index of the last pair with arr <= t, or -1 */
static int64_t dprofile_last_by(const dprofile_t *p, uint32_t t)
{
    uint32_t lo = 0, hi = p->len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (p->arr[mid] <= t)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (int64_t)lo - 1;
}

static int dprofile_insert(dprofile_t *p, uint32_t a, uint32_t d)
{
    int64_t k = dprofile_last_by(p, a); /* pairs [0, k] have arr <= a */
    if (k >= 0 && p->dur[k] <= d)
        return 0; /* dominated by a pair arriving no later and no longer */
    /* the new pair dominates the pairs with arr >= a and dur >= d: a pair
     * with arr == a at k (its dur is > d here), and the pairs after k whose
     * durations (descending) are still >= d */
    uint32_t first = (uint32_t)(k + 1);
    if (k >= 0 && p->arr[k] == a)
        first = (uint32_t)k;
    uint32_t last = (uint32_t)(k + 1);
    while (last < p->len && p->dur[last] >= d)
        ++last;
    uint32_t removed = last - first;
    if (removed == 0) {
        if (p->len == p->cap) {
            uint32_t nc = p->cap ? 2 * p->cap : 4;
            uint32_t *na = realloc(p->arr, (size_t)nc * sizeof(uint32_t));
            if (!na)
                return -1;
            p->arr = na;
            uint32_t *nd = realloc(p->dur, (size_t)nc * sizeof(uint32_t));
            if (!nd)
                return -1;
            p->dur = nd;
            p->cap = nc;
        }
        memmove(p->arr + first + 1, p->arr + first, (size_t)(p->len - first) * sizeof(uint32_t));
        memmove(p->dur + first + 1, p->dur + first, (size_t)(p->len - first) * sizeof(uint32_t));
        p->len += 1;
    } else if (removed > 1) {
        memmove(p->arr + first + 1, p->arr + last, (size_t)(p->len - last) * sizeof(uint32_t));
        memmove(p->dur + first + 1, p->dur + last, (size_t)(p->len - last) * sizeof(uint32_t));
        p->len -= removed - 1;
    }
    p->arr[first] = a;
    p->dur[first] = d;
    return 1;
}

/* Returns 0 on success, -1 on allocation failure.  sd: n entries.
 * strict != 0: consecutive edges follow "Strictly succeeds" (§2.2), so an
 * edge departing at t extends only paths that arrived by t - 1. */
int oracle_shortest_duration(uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *t,
                             const uint32_t *a, uint32_t n, uint32_t source, uint32_t t_alpha,
                             uint32_t t_omega, int strict, uint32_t *sd)
{
    dprofile_t *P = calloc(n, sizeof(dprofile_t));
    if (!P)
        return -1;
    int rc = 0;
    uint64_t e = first_at_or_after(t, m, t_alpha);
    for (; e < m && t[e] < t_omega; ++e) {
        uint32_t u = src[e], v = dst[e];
        if (a[e] > t_omega || v == source)
            continue;
        uint32_t lam = a[e] - t[e];
        uint32_t d;
        if (u == source) {
            d = lam;
        } else {
            if (strict && t[e] == 0)
                continue;
            int64_t k = dprofile_last_by(&P[u], strict ? t[e] - 1 : t[e]);
            if (k < 0)
                continue;
            d = P[u].dur[k] + lam;
        }
        if (dprofile_insert(&P[v], a[e], d) < 0) {
            rc = -1;
            break;
        }
    }
    for (uint32_t v = 0; v < n; ++v) {
        uint32_t s_v = ORACLE_INF;
        if (v == source)
            s_v = 0;
        else if (P[v].len)
            s_v = P[v].dur[P[v].len - 1]; /* durations descend with arrival */
        sd[v] = s_v;
        free(P[v].arr);
        free(P[v].dur);
    }
    free(P);
    return rc;
}
