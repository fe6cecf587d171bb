/*
 * chung_lu.c -- seeded synthetic graph generator (workload inputs only; it
 * holds none of the diffusion arithmetic).
 *
 * Undirected Chung-Lu graphs with a power-law expected-degree sequence:
 * endpoints are drawn i.i.d. with probability proportional to a weight
 * vector w (Walker/Vose alias table), self-loops dropped, pairs canonicalised
 * to (min, max) and de-duplicated; sampling continues until exactly E_target
 * distinct edges exist (first occurrences in sampling order win).  Nodes are
 * then relabelled by a seeded random permutation and the graph is written as
 * a symmetric CSR with ascending neighbour lists.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) read at a counter position,
 * so every candidate edge has a fixed random stream regardless of threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t splitmix_at(uint64_t seed, uint64_t ctr) {
    uint64_t z = seed + (ctr + 1) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
static inline double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }
static inline uint64_t bounded(uint64_t r, uint64_t n) { return (uint64_t)(((__uint128_t)r * n) >> 64); }

typedef struct {
    int64_t n;
    double *prob;
    int64_t *alias;
} alias_t;

/* Vose's alias method, sequential and deterministic */
static int alias_build(alias_t *a, const double *w, int64_t n) {
    a->n = n;
    a->prob = (double *)malloc(sizeof(double) * n);
    a->alias = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *small = (int64_t *)malloc(sizeof(int64_t) * n), *large = (int64_t *)malloc(sizeof(int64_t) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    if (!a->prob || !a->alias || !small || !large || !p) return -1;
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += w[i];
    int64_t ns = 0, nl = 0;
    for (int64_t i = 0; i < n; i++) {
        p[i] = w[i] * (double)n / s;
        if (p[i] < 1.0) small[ns++] = i; else large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        int64_t l = small[--ns], g = large[--nl];
        a->prob[l] = p[l];
        a->alias[l] = g;
        p[g] = (p[g] + p[l]) - 1.0;
        if (p[g] < 1.0) small[ns++] = g; else large[nl++] = g;
    }
    while (nl > 0) { int64_t g = large[--nl]; a->prob[g] = 1.0; a->alias[g] = g; }
    while (ns > 0) { int64_t l = small[--ns]; a->prob[l] = 1.0; a->alias[l] = l; }
    free(small); free(large); free(p);
    return 0;
}
static inline int64_t alias_draw(const alias_t *a, uint64_t r1, uint64_t r2) {
    int64_t i = (int64_t)bounded(r1, (uint64_t)a->n);
    return u01(r2) < a->prob[i] ? i : a->alias[i];
}

/* candidate k -> canonical key (min << 32 | max), or UINT64_MAX for a self-loop */
static inline uint64_t candidate(const alias_t *a, uint64_t seed, uint64_t k) {
    int64_t u = alias_draw(a, splitmix_at(seed, 4 * k), splitmix_at(seed, 4 * k + 1));
    int64_t v = alias_draw(a, splitmix_at(seed, 4 * k + 2), splitmix_at(seed, 4 * k + 3));
    if (u == v) return UINT64_MAX;
    uint64_t lo = (uint64_t)(u < v ? u : v), hi = (uint64_t)(u < v ? v : u);
    return (lo << 32) | hi;
}

/* parallel LSD radix sort of 64-bit keys, four 16-bit digits */
static void radix_sort_u64(uint64_t *keys, uint64_t *tmp, int64_t m) {
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    const int R = 1 << 16;
    int64_t *hist = (int64_t *)malloc(sizeof(int64_t) * (size_t)R * nt);
    uint64_t *src = keys, *dst = tmp;
    for (int shift = 0; shift < 64; shift += 16) {
        memset(hist, 0, sizeof(int64_t) * (size_t)R * nt);
#pragma omp parallel num_threads(nt)
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            int64_t lo = m * tid / nt, hi = m * (tid + 1) / nt;
            int64_t *h = hist + (size_t)R * tid;
            for (int64_t i = lo; i < hi; i++) h[(src[i] >> shift) & 0xFFFF]++;
#pragma omp barrier
#pragma omp single
            {
                int64_t run = 0;
                for (int d = 0; d < R; d++)
                    for (int t = 0; t < nt; t++) {
                        int64_t c = hist[(size_t)R * t + d];
                        hist[(size_t)R * t + d] = run;
                        run += c;
                    }
            }
            for (int64_t i = lo; i < hi; i++) dst[h[(src[i] >> shift) & 0xFFFF]++] = src[i];
        }
        uint64_t *s = src; src = dst; dst = s;
    }
    free(hist);
}

static int64_t unique_sorted(uint64_t *k, int64_t m) {
    int64_t w = 0;
    for (int64_t i = 0; i < m; i++) {
        if (k[i] == UINT64_MAX) break;
        if (w == 0 || k[i] != k[w - 1]) k[w++] = k[i];
    }
    return w;
}

static int contains(const uint64_t *k, int64_t m, uint64_t key) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (k[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo < m && k[lo] == key;
}

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}
static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Draw exactly E distinct undirected edges and write them as a sorted array of
 * canonical keys (out_keys, capacity E).  Returns E, or -1 on failure.
 */
int64_t cl_sample_edges(int64_t n, const double *w, int64_t E, uint64_t seed, uint64_t *out_keys) {
    alias_t a;
    if (n < 2 || alias_build(&a, w, n)) return -1;
    int64_t U = 0;
    uint64_t ctr = 0;
    int64_t cap = E + E / 8 + 4096;
    uint64_t *buf = (uint64_t *)malloc(sizeof(uint64_t) * cap);
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (cap > E ? cap : E));
    if (!buf || !tmp) return -1;
    while (E - U > 4096) {
        int64_t M = E - U; /* at most E-U new distinct keys: never overshoots */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < M; k++) buf[k] = candidate(&a, seed, ctr + (uint64_t)k);
        ctr += (uint64_t)M;
        radix_sort_u64(buf, tmp, M);
        int64_t m = unique_sorted(buf, M);
        /* drop keys already present, merge the rest into out_keys */
        int64_t i = 0, j = 0, o = 0;
        while (i < U || j < m) {
            if (j >= m || (i < U && out_keys[i] < buf[j])) tmp[o++] = out_keys[i++];
            else if (i >= U || buf[j] < out_keys[i]) tmp[o++] = buf[j++];
            else { tmp[o++] = out_keys[i++]; j++; }
        }
        memcpy(out_keys, tmp, sizeof(uint64_t) * (size_t)o);
        U = o;
    }
    /* final exact round: first occurrences in sampling order */
    int64_t need = E - U, got = 0;
    uint64_t *fresh = (uint64_t *)malloc(sizeof(uint64_t) * (need > 0 ? need : 1));
    while (got < need) {
        uint64_t key = candidate(&a, seed, ctr++);
        if (key == UINT64_MAX || contains(out_keys, U, key)) continue;
        int dup = 0;
        for (int64_t t = 0; t < got; t++) if (fresh[t] == key) { dup = 1; break; }
        if (!dup) fresh[got++] = key;
    }
    qsort(fresh, (size_t)got, sizeof(uint64_t), cmp_u64);
    {
        int64_t i = 0, j = 0, o = 0;
        while (i < U || j < got) {
            if (j >= got || (i < U && out_keys[i] < fresh[j])) tmp[o++] = out_keys[i++];
            else tmp[o++] = fresh[j++];
        }
        memcpy(out_keys, tmp, sizeof(uint64_t) * (size_t)o);
        U = o;
    }
    free(fresh); free(buf); free(tmp); free(a.prob); free(a.alias);
    return U;
}

/* seeded Fisher-Yates permutation of 0..n-1 */
void cl_permutation(int64_t n, uint64_t seed, int32_t *perm) {
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)bounded(splitmix_at(seed, (uint64_t)i), (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/* relabel with perm and build the symmetric CSR (ascending neighbour lists) */
int cl_build_csr(int64_t n, int64_t E, const uint64_t *keys, const int32_t *perm, int32_t *row_ptr,
                 int32_t *col_idx) {
    int64_t *cur = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cur) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; e++) {
        int32_t u = perm[keys[e] >> 32], v = perm[keys[e] & 0xFFFFFFFFULL];
        __atomic_fetch_add(&cur[u + 1], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&cur[v + 1], 1, __ATOMIC_RELAXED);
    }
    for (int64_t i = 0; i < n; i++) cur[i + 1] += cur[i];
    for (int64_t i = 0; i <= n; i++) row_ptr[i] = (int32_t)cur[i];
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; e++) {
        int32_t u = perm[keys[e] >> 32], v = perm[keys[e] & 0xFFFFFFFFULL];
        int64_t pu = __atomic_fetch_add(&cur[u], 1, __ATOMIC_RELAXED);
        int64_t pv = __atomic_fetch_add(&cur[v], 1, __ATOMIC_RELAXED);
        col_idx[pu] = v;
        col_idx[pv] = u;
    }
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; u++)
        qsort(col_idx + row_ptr[u], (size_t)(row_ptr[u + 1] - row_ptr[u]), sizeof(int32_t), cmp_i32);
    free(cur);
    return 0;
}

/* connected components by union-find; label[u] = smallest node id of u's component */
void cl_components(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t *label) {
    for (int64_t i = 0; i < n; i++) label[i] = (int32_t)i;
    for (int64_t u = 0; u < n; u++) {
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
            int32_t a = (int32_t)u, b = col_idx[e];
            if (b <= a) continue;
            while (label[a] != a) { label[a] = label[label[a]]; a = label[a]; }
            while (label[b] != b) { label[b] = label[label[b]]; b = label[b]; }
            if (a != b) { if (a < b) label[b] = a; else label[a] = b; }
        }
    }
    for (int64_t i = 0; i < n; i++) {
        int32_t a = (int32_t)i;
        while (label[a] != a) a = label[a];
        label[i] = a;
    }
}
