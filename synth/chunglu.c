/*
 * Seeded synthetic inputs: directed Chung-Lu scale-free graphs and uniform
 * query sources.
 *
 * This module holds only input generation (random numbers, weights, sampling,
 * de-duplication, CSR layout).  It contains none of the PPR method's
 * arithmetic; both the oracle and the GPU path read the graphs it writes.
 *
 * Graph model (directed Chung-Lu with separate out- and in-weights):
 *   - rank weights w_i = c * (i+1)^(-1/(gamma-1)), i = 0..n-1, each capped at
 *     sqrt(m) (the Chung-Lu admissibility condition w_u * w_v <= sum(w));
 *     c is bisected so that sum_i min(c (i+1)^(-1/(gamma-1)), sqrt(m)) = m;
 *   - independent seeded permutations map ranks to node ids for the out- and
 *     the in-weights, so ids carry no degree order;
 *   - every node first receives one out-edge to a node v != u drawn
 *     proportionally to the in-weights (so every out-degree is >= 1, the
 *     no-dead-end assumption of the problem setting);
 *   - further candidate pairs (u ~ w_out, v ~ w_in) are drawn with a
 *     counter-based generator; self-loops and duplicates are rejected, and the
 *     first (m - n) distinct pairs in counter order are kept;
 *   - rows of the CSR are sorted ascending (canonical form).
 *
 * Random numbers: SplitMix64 finaliser (Steele, Lea, Flood 2014; constants as
 * published by Vigna) applied to a counter keyed on (seed, stream, index), so
 * the output does not depend on the number of threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>
#include <stdio.h>

/* Progress lines on stderr when PPR_SYNTH_VERBOSE is set (large graphs take minutes). */
static void progress(const char* what, int64_t a) {
    const char* v = getenv("PPR_SYNTH_VERBOSE");
    if (v && v[0] && v[0] != '0') {
        fprintf(stderr, "[synth] %s %lld\n", what, (long long)a);
        fflush(stderr);
    }
}

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Counter-based draw: independent 64-bit value for (seed, stream, index). */
static inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t index) {
    uint64_t key = sm64_mix(seed + 0x9E3779B97F4A7C15ULL * (stream + 1));
    return sm64_mix(key + 0x9E3779B97F4A7C15ULL * (index + 1));
}

static inline double unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* Uniform integer in [0, n) by multiply-high. */
static inline uint64_t below(uint64_t x, uint64_t n) {
    return (uint64_t)(((unsigned __int128)x * n) >> 64);
}

enum { ST_PERM_OUT = 1, ST_PERM_IN = 2, ST_MIN = 3, ST_U = 4, ST_V = 5, ST_SRC = 6 };

/* Uniform sources in [0, n): the i-th source is below(draw(seed, ST_SRC, i), n). */
void synth_sources(int32_t n, int32_t count, uint64_t seed, int32_t* out) {
    for (int32_t i = 0; i < count; ++i) out[i] = (int32_t)below(draw(seed, ST_SRC, (uint64_t)i), (uint64_t)n);
}

static double capped_total(double c, const double* t, const double* suf, int32_t n, double cap) {
    int32_t a = 0, b = n;   /* a = first rank with c t_a < cap */
    while (a < b) { int32_t mid = a + (b - a) / 2; if (c * t[mid] >= cap) a = mid + 1; else b = mid; }
    return (double)a * cap + c * suf[a];
}

/* Cumulative capped weights in rank order; returns the total.  The uncapped
   weights t_i = (i+1)^(-1/(gamma-1)) decrease in i, so the capped ranks form a
   prefix and sum_i min(c t_i, cap) = k cap + c sum_{i>=k} t_i, with k the
   number of ranks where c t_i >= cap. */
static double build_cdf(int32_t n, int64_t m, double gamma, double* cdf) {
    double e = 1.0 / (gamma - 1.0);
    double cap = sqrt((double)m);
    double* t = (double*)malloc(sizeof(double) * (size_t)n);
    double* suf = (double*)malloc(sizeof(double) * ((size_t)n + 1));
    if (!t || !suf) { free(t); free(suf); return -1.0; }
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) t[i] = pow((double)i + 1.0, -e);
    suf[n] = 0.0;
    for (int32_t i = n - 1; i >= 0; --i) suf[i] = suf[i + 1] + t[i];
    double lo = 0.0, hi = 1.0;
    while (capped_total(hi, t, suf, n, cap) < (double)m) { lo = hi; hi *= 2.0; }
    for (int it = 0; it < 200 && hi - lo > 1e-13 * hi; ++it) {
        double mid = 0.5 * (lo + hi);
        if (capped_total(mid, t, suf, n, cap) < (double)m) lo = mid; else hi = mid;
    }
    double c = hi, acc = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double w = c * t[i];
        acc += (w < cap) ? w : cap;
        cdf[i] = acc;
    }
    free(t); free(suf);
    return acc;
}

/* First i in [lo, hi] with cdf[i] > x (hi if none). */
static inline int32_t first_above(const double* cdf, int32_t lo, int32_t hi, double x) {
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > x) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* Rank drawn proportionally to the weights: first i with cdf[i] > x. */
static inline int32_t sample_rank(const double* cdf, int32_t n, double total, uint64_t r) {
    return first_above(cdf, 0, n - 1, unit(r) * total);
}

/* The same draw through a guide table (Chen and Asau): guide[k] is the answer
   for x = k * total / K, so the answer for x in bucket k lies in
   [guide[k], guide[k+1]]; the two checks catch a bucket index that rounding
   put next to the right one, and then the full search decides.  Returns
   exactly what sample_rank returns. */
typedef struct {
    const double* cdf;
    int32_t n;
    double total, inv;
    int64_t K;
    int32_t* guide;
} sampler_t;

static void sampler_init(sampler_t* S, const double* cdf, int32_t n, double total) {
    S->cdf = cdf;
    S->n = n;
    S->total = total;
    S->K = n;
    S->inv = (double)S->K / total;
    S->guide = (int32_t*)malloc(sizeof(int32_t) * ((size_t)S->K + 1));
    if (!S->guide) return;
    int32_t i = 0;
    for (int64_t k = 0; k <= S->K; ++k) {
        double x = (double)k * (total / (double)S->K);
        while (i < n - 1 && !(cdf[i] > x)) ++i;
        S->guide[k] = i;
    }
}

static inline int32_t sampler_draw(const sampler_t* S, uint64_t r) {
    double x = unit(r) * S->total;
    int64_t k = (int64_t)(x * S->inv);
    if (k < 0) k = 0;
    if (k >= S->K) k = S->K - 1;
    int32_t lo = S->guide[k], hi = S->guide[k + 1];
    if ((lo > 0 && S->cdf[lo - 1] > x) || (hi < S->n - 1 && !(S->cdf[hi] > x)))
        return first_above(S->cdf, 0, S->n - 1, x);
    return first_above(S->cdf, lo, hi, x);
}

static void permutation(int32_t n, uint64_t seed, uint64_t stream, int32_t* p) {
    for (int32_t i = 0; i < n; ++i) p[i] = i;
    for (int32_t i = n - 1; i > 0; --i) {
        int32_t j = (int32_t)below(draw(seed, stream, (uint64_t)i), (uint64_t)i + 1);
        int32_t t = p[i]; p[i] = p[j]; p[j] = t;
    }
}

typedef struct { int32_t v; uint32_t k; } cand_t;

static int cmp_cand(const void* a, const void* b) {
    const cand_t* x = (const cand_t*)a; const cand_t* y = (const cand_t*)b;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    return (x->k < y->k) ? -1 : (x->k > y->k);
}
static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* k-th smallest (0-based) of an array by quickselect (destructive). */
static uint32_t select_kth(uint32_t* a, int64_t len, int64_t k) {
    int64_t lo = 0, hi = len - 1;
    uint64_t state = 0x1234567ULL;
    while (lo < hi) {
        state = sm64_mix(state);
        uint32_t pivot = a[lo + (int64_t)below(state, (uint64_t)(hi - lo + 1))];
        int64_t i = lo, j = hi;
        while (i <= j) {
            while (a[i] < pivot) ++i;
            while (a[j] > pivot) --j;
            if (i <= j) { uint32_t t = a[i]; a[i] = a[j]; a[j] = t; ++i; --j; }
        }
        if (k <= j) hi = j; else if (k >= i) lo = i; else return a[k];
    }
    return a[k];
}

/*
 * Generate the graph.  row_ptr has n+1 entries, col has m entries (both
 * caller-allocated).  Returns 0 on success, -1 on bad arguments, -2 if memory
 * runs out, -3 if the requested m cannot be reached (too dense).
 * max_out / max_in (nullable) receive the realised maximum degrees.
 */
int synth_chunglu(int32_t n, int64_t m, double gamma_out, double gamma_in, uint64_t seed,
                  int64_t* row_ptr, int32_t* col, int32_t* max_out, int32_t* max_in) {
    if (n < 2 || m < n || gamma_out <= 1.0 || gamma_in <= 1.0) return -1;
    if ((double)m > 0.5 * (double)n * (double)(n - 1)) return -3;
    if (m - n > (int64_t)0xFFFFFFF0LL) return -1;
    int rc = 0;
    double* cdf_out = (double*)malloc(sizeof(double) * n);
    double* cdf_in = (double*)malloc(sizeof(double) * n);
    int32_t* perm_out = (int32_t*)malloc(sizeof(int32_t) * n);
    int32_t* perm_in = (int32_t*)malloc(sizeof(int32_t) * n);
    int32_t* first = (int32_t*)malloc(sizeof(int32_t) * n);
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    cand_t* cand = NULL; uint32_t* keys = NULL;
    sampler_t s_out, s_in;
    s_out.guide = NULL;
    s_in.guide = NULL;
    if (!cdf_out || !cdf_in || !perm_out || !perm_in || !first || !cnt || !fill) { rc = -2; goto done; }

    double tot_out = build_cdf(n, m, gamma_out, cdf_out);
    double tot_in = build_cdf(n, m, gamma_in, cdf_in);
    if (tot_out <= 0.0 || tot_in <= 0.0) { rc = -2; goto done; }
    sampler_init(&s_out, cdf_out, n, tot_out);
    sampler_init(&s_in, cdf_in, n, tot_in);
    if (!s_out.guide || !s_in.guide) { rc = -2; goto done; }
    permutation(n, seed, ST_PERM_OUT, perm_out);
    permutation(n, seed, ST_PERM_IN, perm_in);

    /* One guaranteed out-edge per node, target drawn from the in-weights, != u. */
    #pragma omp parallel for schedule(static)
    for (int32_t u = 0; u < n; ++u) {
        uint64_t att = 0;
        int32_t v;
        do {
            v = perm_in[sampler_draw(&s_in, draw(seed, ST_MIN, (uint64_t)u * 64 + att))];
            ++att;
        } while (v == u && att < 64);
        if (v == u) v = (u + 1) % n;
        first[u] = v;
    }

    int64_t target = m - n;
    int64_t K = target + target / 16 + 1024;
    for (int attempt = 0; attempt < 16; ++attempt) {
        if (K > (int64_t)0xFFFFFFF0LL) K = (int64_t)0xFFFFFFF0LL;
        free(cand); free(keys); cand = NULL; keys = NULL;
        progress("candidate draws", K);
        /* pass 1: count the non-self-loop candidates of each source row */
        memset(cnt, 0, sizeof(int64_t) * ((size_t)n + 1));
        #pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < K; ++k) {
            int32_t u = perm_out[sampler_draw(&s_out, draw(seed, ST_U, (uint64_t)k))];
            int32_t v = perm_in[sampler_draw(&s_in, draw(seed, ST_V, (uint64_t)k))];
            if (u != v) __atomic_fetch_add(&cnt[u + 1], 1, __ATOMIC_RELAXED);
        }
        for (int32_t u = 0; u < n; ++u) cnt[u + 1] += cnt[u];
        for (int32_t u = 0; u < n; ++u) fill[u] = cnt[u];
        cand = (cand_t*)malloc(sizeof(cand_t) * (size_t)(cnt[n] > 0 ? cnt[n] : 1));
        if (!cand) { rc = -2; goto done; }
        progress("pass 2, candidates", cnt[n]);
        /* pass 2: redraw and place (order inside a row is fixed by the sort below) */
        #pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < K; ++k) {
            int32_t u = perm_out[sampler_draw(&s_out, draw(seed, ST_U, (uint64_t)k))];
            int32_t v = perm_in[sampler_draw(&s_in, draw(seed, ST_V, (uint64_t)k))];
            if (u != v) {
                int64_t pos = __atomic_fetch_add(&fill[u], 1, __ATOMIC_RELAXED);
                cand[pos].v = v; cand[pos].k = (uint32_t)k;
            }
        }
        progress("dedup rows", n);
        /* per row: the first occurrence (smallest k) of each target survives,
           unless the target is the row's guaranteed edge; the rest get v = -1 */
        int64_t survivors = 0;
        #pragma omp parallel for schedule(dynamic, 1024) reduction(+:survivors)
        for (int32_t u = 0; u < n; ++u) {
            cand_t* row = cand + cnt[u];
            int64_t len = cnt[u + 1] - cnt[u];
            if (len > 1) qsort(row, (size_t)len, sizeof(cand_t), cmp_cand);
            int64_t i = 0;
            while (i < len) {
                int32_t v = row[i].v;
                int64_t j = i + 1;
                while (j < len && row[j].v == v) { row[j].v = -1; ++j; }
                if (v == first[u]) row[i].v = -1; else survivors++;
                i = j;
            }
        }
        if (survivors < target) { K = K + K / 4 + (target - survivors) * 2 + 1024; continue; }
        /* counter cutoff: keep the survivors whose k is among the first `target` */
        uint32_t kcut = 0;
        if (target > 0) {
            keys = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)survivors);
            if (!keys) { rc = -2; goto done; }
            int64_t ns = 0;
            for (int64_t i = 0; i < cnt[n]; ++i) if (cand[i].v >= 0) keys[ns++] = cand[i].k;
            kcut = select_kth(keys, ns, target - 1);
        }
        progress("assemble, survivors", survivors);
        /* assemble the CSR */
        row_ptr[0] = 0;
        for (int32_t u = 0; u < n; ++u) {
            int64_t d = 1;
            if (target > 0)
                for (int64_t i = cnt[u]; i < cnt[u + 1]; ++i) if (cand[i].v >= 0 && cand[i].k <= kcut) d++;
            row_ptr[u + 1] = row_ptr[u] + d;
        }
        if (row_ptr[n] != m) { rc = -3; goto done; }
        #pragma omp parallel for schedule(dynamic, 1024)
        for (int32_t u = 0; u < n; ++u) {
            int32_t* out = col + row_ptr[u];
            int64_t p = 0;
            out[p++] = first[u];
            if (target > 0)
                for (int64_t i = cnt[u]; i < cnt[u + 1]; ++i)
                    if (cand[i].v >= 0 && cand[i].k <= kcut) out[p++] = cand[i].v;
            if (p > 1) qsort(out, (size_t)p, sizeof(int32_t), cmp_i32);
        }
        int32_t mo = 0, mi = 0;
        int32_t* indeg = (int32_t*)calloc((size_t)n, sizeof(int32_t));
        if (!indeg) { rc = -2; goto done; }
        for (int32_t u = 0; u < n; ++u) {
            int32_t d = (int32_t)(row_ptr[u + 1] - row_ptr[u]);
            if (d > mo) mo = d;
        }
        for (int64_t e = 0; e < m; ++e) indeg[col[e]]++;
        for (int32_t u = 0; u < n; ++u) if (indeg[u] > mi) mi = indeg[u];
        free(indeg);
        if (max_out) *max_out = mo;
        if (max_in) *max_in = mi;
        rc = 0;
        goto done;
    }
    rc = -3;
done:
    free(cdf_out); free(cdf_in); free(perm_out); free(perm_in); free(first);
    free(cnt); free(fill); free(cand); free(keys); free(s_out.guide); free(s_in.guide);
    return rc;
}
