/*
 * gde_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the local
 * diffusion solvers of "Faster Local Solvers for Graph Diffusion Equations"
 * (Bai, Zhou, Yang, Xiao; NeurIPS 2024).  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header or table with the GPU library.
 *
 * Every solver works on the generic linear system Q x = b with r = b - Q x
 * (Sec. 3.1, Eq. (4)) and the local diffusion process of Definition 3.1:
 * iterate (x, r, S_t) until the active set S_t is empty.
 *
 *   PPR : Q = I - (1-alpha) A D^-1, b = alpha s, active iff |r_u| >= alpha*eps*d_u
 *         (Eq. (2), Algorithm 1, Corollary 3.5).  Reported residual r/alpha.
 *   Katz: Q = I - beta A,           b = s,       active iff |r_u| >= eps*d_u
 *         (Eq. (3), stop rule of Sec. 5 / App. B).
 *   HK  : Taylor-truncated heat kernel solved level by level (the AHK push of
 *         Sec. 2 on the Kronecker system), see oracle_hk below.
 *
 * Readings of the paper that this file adopts:
 *   - S_0 = supp(s) is forced (Definition 3.1), whatever the threshold says.
 *   - active iff |r_u| >= theta_u AND r_u != 0; stop iff every |r_u| < theta_u.
 *   - theta_u = eps_eff * d_u with eps_eff = alpha*eps (PPR) or eps (Katz),
 *     all in FP64.
 *   - nodes inside one iteration are processed in ascending id order.
 *
 * Parity status: every exported function is pinned by tests in
 * tests/test_oracle_*.py against closed forms, truncated series, dense
 * solves, invariants of Theorem 3.4 / Corollary 3.5 and the stop-rule error
 * bound of Theorem 3.2.  oracle_replay_* is a checking tool whose arithmetic
 * is the same step functions as the free-run solvers.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_INVALID = 1, OR_NOT_CONVERGED = 4, OR_OOM = 5 };
enum { KIND_PPR = 0, KIND_KATZ = 1 };

typedef struct {
    int64_t n;
    const int64_t *rp; /* row pointer, n+1 entries */
    const int32_t *ci; /* column indices, rp[n] entries */
} graph_t;

static double deg(const graph_t *g, int64_t u) { return (double)(g->rp[u + 1] - g->rp[u]); }

/* ---- the set of nodes whose residual has ever been nonzero ---------------- */
typedef struct {
    int64_t *list;
    int64_t len;
    unsigned char *flag;
} touched_t;

static int touched_init(touched_t *t, int64_t n) {
    t->list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    t->flag = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    t->len = 0;
    return (t->list && t->flag) ? 0 : -1;
}
static void touched_free(touched_t *t) { free(t->list); free(t->flag); }
static void touch(touched_t *t, int64_t u) {
    if (!t->flag[u]) { t->flag[u] = 1; t->list[t->len++] = u; }
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* ---- the generic form of PPR and Katz (Sec. 3.1, Eq. (4)) ---------------- */
typedef struct {
    int kind;
    double param;   /* alpha (PPR) or beta (Katz) */
    double eps_eff; /* alpha*eps (PPR) or eps (Katz) */
} form_t;

static double form_b(const form_t *f, double s) { return f->kind == KIND_PPR ? f->param * s : s; }
/* weight of the edge u->w in beta*P: (1-alpha)/d_u for A D^-1, beta for A */
static double form_w(const form_t *f, const graph_t *g, int64_t u) {
    return f->kind == KIND_PPR ? (1.0 - f->param) / deg(g, u) : f->param;
}
static double form_theta(const form_t *f, const graph_t *g, int64_t u) { return f->eps_eff * deg(g, u); }
static double form_rscale(const form_t *f) { return f->kind == KIND_PPR ? 1.0 / f->param : 1.0; }

static int is_active(double r, double theta) { return r != 0.0 && fabs(r) >= theta; }

/* r <- r - Q h_S  with h supported on S:  r_u -= h_u ; r_w += w_u h_u  (w ~ u) */
static void apply_Q(const graph_t *g, const form_t *f, const int64_t *S, int64_t ns, const double *h,
                    double *r, touched_t *tch) {
    for (int64_t i = 0; i < ns; i++) {
        int64_t u = S[i];
        double hu = h[i];
        double wu = form_w(f, g, u);
        r[u] -= hu;
        for (int64_t e = g->rp[u]; e < g->rp[u + 1]; e++) {
            int64_t w = g->ci[e];
            r[w] += wu * hu;
            touch(tch, w);
        }
    }
}

/* ---- active-set selection: free run or replay of a recorded trace --------- */
typedef struct {
    const int64_t *off;   /* T_rec+1 offsets into nodes */
    const int32_t *nodes; /* concatenated S_t lists */
    int64_t T_rec;
    double kappa;
    int64_t flips, violations;
} replay_t;

/* S_t = {u : |r_u| >= theta_u, r_u != 0}, ascending ids.  Nodes outside the
 * touched set have r_u = 0 exactly, so scanning the touched set suffices. */
static int64_t select_free(const graph_t *g, const form_t *f, const double *r, const touched_t *tch,
                           int64_t *S) {
    int64_t ns = 0;
    for (int64_t i = 0; i < tch->len; i++) {
        int64_t u = tch->list[i];
        if (is_active(r[u], form_theta(f, g, u))) S[ns++] = u;
    }
    qsort(S, (size_t)ns, sizeof(int64_t), cmp_i64);
    return ns;
}

/* Use the recorded S_t (t >= 1) and grade every decision against the band
 * [theta(1-kappa), theta(1+kappa)).  A decision inside the band that differs
 * from the FP64 decision is a flip; one outside the band is a violation. */
static int64_t select_replay(const graph_t *g, const form_t *f, const double *r, const touched_t *tch,
                             replay_t *rp, int64_t t, int64_t *S, unsigned char *mark) {
    int64_t ns = 0;
    if (t < rp->T_rec) {
        for (int64_t i = rp->off[t]; i < rp->off[t + 1]; i++) S[ns++] = rp->nodes[i];
        qsort(S, (size_t)ns, sizeof(int64_t), cmp_i64);
    }
    for (int64_t i = 0; i < ns; i++) {
        int64_t u = S[i];
        double th = form_theta(f, g, u);
        if (i > 0 && S[i] == S[i - 1]) rp->violations++; /* duplicate entry */
        if (u < 0 || u >= g->n) { rp->violations++; continue; }
        mark[u] = 1;
        if (!(fabs(r[u]) >= th * (1.0 - rp->kappa)) || r[u] == 0.0) rp->violations++;
        else if (!is_active(r[u], th)) rp->flips++;
    }
    for (int64_t i = 0; i < tch->len; i++) {
        int64_t u = tch->list[i];
        if (mark[u]) continue;
        double th = form_theta(f, g, u);
        if (r[u] != 0.0 && fabs(r[u]) >= th * (1.0 + rp->kappa)) rp->violations++;
        else if (is_active(r[u], th)) rp->flips++;
    }
    for (int64_t i = 0; i < ns; i++)
        if (S[i] >= 0 && S[i] < g->n) mark[S[i]] = 0;
    return ns;
}

static void residual_norms(const graph_t *g, const form_t *f, const double *r, const touched_t *tch,
                           double *l1, double *dinf) {
    double a = 0.0, m = 0.0, sc = form_rscale(f);
    for (int64_t i = 0; i < tch->len; i++) {
        int64_t u = tch->list[i];
        double v = fabs(r[u]) * sc;
        a += v;
        double d = deg(g, u);
        if (d > 0 && v / d > m) m = v / d;
    }
    *l1 = a;
    *dinf = m;
}

/* trace record: |S_t|, vol(S_t), ||r_S||_1 and ||r||_1 at the start of t,
 * both residual norms in the reported scale */
typedef struct {
    int64_t cap;
    int64_t *size, *vol;
    double *rs_l1, *r_l1;
    int64_t nodes_cap; /* optional: the S_t lists themselves, concatenated */
    int32_t *nodes;
    int64_t nodes_len;
} trace_t;

static void trace_put(trace_t *tr, int64_t t, int64_t ns, int64_t vol, double rs, double r1, const int64_t *S) {
    if (!tr) return;
    if (tr->nodes) {
        for (int64_t i = 0; i < ns; i++) {
            if (tr->nodes_len < tr->nodes_cap) tr->nodes[tr->nodes_len] = (int32_t)S[i];
            tr->nodes_len++;
        }
    }
    if (t >= tr->cap) return;
    if (tr->size) tr->size[t] = ns;
    if (tr->vol) tr->vol[t] = vol;
    if (tr->rs_l1) tr->rs_l1[t] = rs;
    if (tr->r_l1) tr->r_l1[t] = r1;
}

static int check_seed(const graph_t *g, int32_t nnz, const int32_t *idx, const double *val) {
    if (nnz <= 0 || !idx || !val) return OR_INVALID;
    for (int32_t i = 0; i < nnz; i++) {
        if (idx[i] < 0 || idx[i] >= g->n) return OR_INVALID;
        if (i > 0 && idx[i] <= idx[i - 1]) return OR_INVALID;
        if (!(val[i] > 0.0) || !isfinite(val[i])) return OR_INVALID;
        if (deg(g, idx[i]) <= 0) return OR_INVALID;
    }
    return OR_OK;
}

/*
 * LocalGD (Eq. (9)) and LocalCH (Sec. 3.3 and App. B "Implementation
 * details"), sharing the selection and the Q-application above.
 *
 * LocalGD:  x <- x + r_S ,  r <- r - Q r_S .
 * LocalCH:  sigma = (L+mu)/(L-mu); with L + mu = 2 for both PPR
 *           (mu = alpha, L = 2 - alpha) and Katz (mu = 1 - beta*lam,
 *           L = 1 + beta*lam):
 *             t = 0 : h = (2/(L+mu)) r_S = r_S,    delta_1 = 1/sigma
 *             t >= 1: delta_{t+1} = 1/(2 sigma - delta_t)
 *                     h_u = (4 delta_{t+1}/(L-mu)) r_u + delta_t delta_{t+1} Delta_u,  u in S_t
 *             x <- x + h ;  r <- r - Q h ;  Delta <- h  (zero off S_t)
 *
 * method: 0 = LocalGD, 1 = LocalCH.  lam: spectral bound of A for Katz-CH.
 * x, r: dense n-vectors (output; r in the generic, unscaled form).
 * stats[0..3] = T, ops = sum vol(S_t), pushes = sum |S_t|, status.
 * norms[0..1] = reported ||r||_1 and ||D^-1 r||_inf.
 */
static int run_gd_ch(const graph_t *g, const form_t *f, int method, double lam, int32_t seed_nnz,
                     const int32_t *seed_idx, const double *seed_val, int32_t max_iters, double *x, double *r,
                     int64_t *stats, double *norms, trace_t *tr, replay_t *rp, int warm) {
    int64_t n = g->n;
    int rc = warm ? OR_OK : check_seed(g, seed_nnz, seed_idx, seed_val);
    if (rc) return rc;
    touched_t tch = {0};
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *h = (double *)malloc(sizeof(double) * (size_t)n);
    double *delta = (double *)calloc((size_t)n, sizeof(double)); /* previous update, dense */
    int64_t *prevS = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char *mark = (unsigned char *)calloc((size_t)n, 1);
    if (touched_init(&tch, n) || !S || !h || !delta || !prevS || !mark) {
        free(S); free(h); free(delta); free(prevS); free(mark); touched_free(&tch);
        return OR_OOM;
    }
    if (warm) { /* continue from the given (x, r): every node with r_u != 0 may be active */
        for (int64_t u = 0; u < n; u++)
            if (r[u] != 0.0) touch(&tch, u);
    } else {
        memset(x, 0, sizeof(double) * (size_t)n);
        memset(r, 0, sizeof(double) * (size_t)n);
        for (int32_t i = 0; i < seed_nnz; i++) {
            r[seed_idx[i]] = form_b(f, seed_val[i]);
            touch(&tch, seed_idx[i]);
        }
    }
    double sigma = 1.0, dlt = 0.0; /* Chebyshev state */
    if (method == 1) {
        double mu, L;
        if (f->kind == KIND_PPR) { mu = f->param; L = 2.0 - f->param; }
        else { mu = 1.0 - f->param * lam; L = 1.0 + f->param * lam; }
        sigma = (L + mu) / (L - mu);
        dlt = 1.0 / sigma; /* delta_1 */
    }
    double sc = form_rscale(f);
    int64_t T = 0, ops = 0, pushes = 0, nprev = 0;
    int status = OR_NOT_CONVERGED;
    for (int64_t t = 0;; t++) {
        int64_t ns;
        if (t == 0 && !warm) { /* S_0 = supp(s), forced (Definition 3.1) */
            ns = seed_nnz;
            for (int32_t i = 0; i < seed_nnz; i++) S[i] = seed_idx[i];
            if (rp && rp->T_rec > 0) {
                int64_t m = rp->off[1] - rp->off[0];
                int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
                for (int64_t i = 0; i < m; i++) tmp[i] = rp->nodes[rp->off[0] + i];
                qsort(tmp, (size_t)m, sizeof(int64_t), cmp_i64);
                if (m != ns) rp->violations++;
                else for (int64_t i = 0; i < m; i++) if (tmp[i] != S[i]) { rp->violations++; break; }
                free(tmp);
            }
        } else if (rp) {
            ns = select_replay(g, f, r, &tch, rp, t, S, mark);
        } else {
            ns = select_free(g, f, r, &tch, S);
        }
        if (ns == 0) { status = OR_OK; break; }
        if (t >= max_iters) break;
        /* the update h on S_t, from the residual at the start of iteration t */
        int64_t vol = 0;
        double rs = 0.0, r1 = 0.0;
        if (tr && tr->r_l1) /* only the trace reads ||r||_1; it feeds no arithmetic */
            for (int64_t i = 0; i < tch.len; i++) r1 += fabs(r[tch.list[i]]);
        for (int64_t i = 0; i < ns; i++) {
            int64_t u = S[i];
            vol += (int64_t)deg(g, u);
            rs += fabs(r[u]);
        }
        trace_put(tr, t, ns, vol, rs * sc, r1 * sc, S);
        if (method == 0 || t == 0) {
            for (int64_t i = 0; i < ns; i++) h[i] = r[S[i]];
        } else {
            double dnext = 1.0 / (2.0 * sigma - dlt);
            double c = 2.0 * sigma * dnext; /* = 4 delta_{t+1} / (L - mu) since L + mu = 2 */
            double m = dlt * dnext;
            for (int64_t i = 0; i < ns; i++) h[i] = c * r[S[i]] + m * delta[S[i]];
            dlt = dnext;
        }
        for (int64_t i = 0; i < ns; i++) x[S[i]] += h[i];
        apply_Q(g, f, S, ns, h, r, &tch);
        if (method == 1) { /* Delta^{(t+1)} = h restricted to S_t */
            for (int64_t i = 0; i < nprev; i++) delta[prevS[i]] = 0.0;
            for (int64_t i = 0; i < ns; i++) { delta[S[i]] = h[i]; prevS[i] = S[i]; }
            nprev = ns;
        }
        T++;
        ops += vol;
        pushes += ns;
    }
    if (rp && rp->T_rec != T) rp->violations++; /* the trace must have exactly T iterations */
    stats[0] = T; stats[1] = ops; stats[2] = pushes; stats[3] = status;
    residual_norms(g, f, r, &tch, &norms[0], &norms[1]);
    free(S); free(h); free(delta); free(prevS); free(mark); touched_free(&tch);
    return status;
}

static int make_form(int kind, double param, double eps, form_t *f) {
    if (kind != KIND_PPR && kind != KIND_KATZ) return OR_INVALID;
    if (!(eps > 0.0) || !isfinite(eps)) return OR_INVALID;
    if (kind == KIND_PPR && !(param > 0.0 && param < 1.0)) return OR_INVALID;
    if (kind == KIND_KATZ && !(param > 0.0)) return OR_INVALID;
    f->kind = kind;
    f->param = param;
    f->eps_eff = kind == KIND_PPR ? param * eps : eps;
    return OR_OK;
}

int oracle_localgd(int64_t n, const int64_t *rp, const int32_t *ci, int kind, double param, double eps,
                   int32_t seed_nnz, const int32_t *seed_idx, const double *seed_val, int32_t max_iters, double *x,
                   double *r, int64_t *stats, double *norms, int64_t trace_cap, int64_t *tr_size, int64_t *tr_vol,
                   double *tr_rs, double *tr_r1, int64_t nodes_cap, int32_t *tr_nodes, int64_t *nodes_len) {
    graph_t g = {n, rp, ci};
    form_t f;
    if (make_form(kind, param, eps, &f)) return OR_INVALID;
    trace_t tr = {trace_cap, tr_size, tr_vol, tr_rs, tr_r1, nodes_cap, tr_nodes, 0};
    int rc = run_gd_ch(&g, &f, 0, 0.0, seed_nnz, seed_idx, seed_val, max_iters, x, r, stats, norms, &tr, NULL, 0);
    if (nodes_len) *nodes_len = tr.nodes_len;
    return rc;
}

int oracle_localch(int64_t n, const int64_t *rp, const int32_t *ci, int kind, double param, double lam,
                   double eps, int32_t seed_nnz, const int32_t *seed_idx, const double *seed_val, int32_t max_iters,
                   double *x, double *r, int64_t *stats, double *norms, int64_t trace_cap, int64_t *tr_size,
                   int64_t *tr_vol, int64_t nodes_cap, int32_t *tr_nodes, int64_t *nodes_len) {
    graph_t g = {n, rp, ci};
    form_t f;
    if (make_form(kind, param, eps, &f)) return OR_INVALID;
    if (kind == KIND_KATZ && !(param * lam > 0.0 && param * lam < 1.0)) return OR_INVALID;
    trace_t tr = {trace_cap, tr_size, tr_vol, NULL, NULL, nodes_cap, tr_nodes, 0};
    int rc = run_gd_ch(&g, &f, 1, lam, seed_nnz, seed_idx, seed_val, max_iters, x, r, stats, norms, &tr, NULL, 0);
    if (nodes_len) *nodes_len = tr.nodes_len;
    return rc;
}

/* Replay of LocalGD (method 0) or LocalCH (method 1) on recorded active sets.
 * off has T_rec+1 entries; out_fv[0..1] = flips, violations. */
int oracle_replay_gd_ch(int64_t n, const int64_t *rp, const int32_t *ci, int method, int kind, double param,
                        double lam, double eps, int32_t seed_nnz, const int32_t *seed_idx, const double *seed_val,
                        int64_t T_rec, const int64_t *off, const int32_t *nodes, double kappa, double *x, double *r,
                        int64_t *stats, double *norms, int64_t *out_fv) {
    graph_t g = {n, rp, ci};
    form_t f;
    if (make_form(kind, param, eps, &f)) return OR_INVALID;
    replay_t rpl = {off, nodes, T_rec, kappa, 0, 0};
    int rc = run_gd_ch(&g, &f, method, lam, seed_nnz, seed_idx, seed_val, (int32_t)(T_rec + 1), x, r, stats, norms,
                       NULL, &rpl, 0);
    out_fv[0] = rpl.flips;
    out_fv[1] = rpl.violations;
    return rc;
}

/*
 * LocalGD continued from a given state (x, r) on the current graph: the
 * re-solve step of the dynamic algorithms of Sec. 4 (LocalGS(Dynamic) and
 * LocalSOR(Dynamic) return to their local solver after the Insert / Delete
 * corrections).  There is no forced S_0: S_t = {u : |r_u| >= theta_u, r_u != 0}
 * from t = 0, with signed residuals (a deletion can make r negative).
 * x, r: in / out, dense n-vectors in the generic form r = b - Q x.
 */
int oracle_localgd_warm(int64_t n, const int64_t *rp, const int32_t *ci, int kind, double param, double eps,
                        int32_t max_iters, double *x, double *r, int64_t *stats, double *norms) {
    graph_t g = {n, rp, ci};
    form_t f;
    if (make_form(kind, param, eps, &f)) return OR_INVALID;
    return run_gd_ch(&g, &f, 0, 0.0, 0, NULL, NULL, max_iters, x, r, stats, norms, NULL, NULL, 1);
}

/*
 * The standard (global) counterparts of LocalGD and LocalCH that Table 2 and the
 * eps sweep of Sec. 5 compare against: the same updates with S_t = V, the whole
 * node set, in every iteration.
 *
 *   GD : h = r                                  (Richardson / gradient step)
 *   CH : t = 0 h = r ; t >= 1 h = c_t r + m_t Delta  (Chebyshev, Sec. 3.3, with
 *        the coefficients of run_gd_ch above and Delta = the previous h)
 *   x <- x + h ,  r <- r - Q h   over all nodes
 *
 * The first iteration always runs (the forced S_0 of Definition 3.1); after it
 * the solver stops as soon as no node satisfies |r_u| >= theta_u (r_u != 0),
 * the stop rule of the local solvers.  Every iteration costs vol(V) = nnz edge
 * operations and |V| = n node updates (stats[1], stats[2]).
 * method: 0 = GD, 1 = CH.  x, r: dense outputs (r in the generic form).
 */
int oracle_global(int64_t n, const int64_t *rp, const int32_t *ci, int method, int kind, double param,
                  double lam, double eps, int32_t seed_nnz, const int32_t *seed_idx, const double *seed_val,
                  int32_t max_iters, double *x, double *r, int64_t *stats, double *norms) {
    graph_t g = {n, rp, ci};
    form_t f;
    if (make_form(kind, param, eps, &f)) return OR_INVALID;
    if (method == 1 && kind == KIND_KATZ && !(param * lam > 0.0 && param * lam < 1.0)) return OR_INVALID;
    int rc = check_seed(&g, seed_nnz, seed_idx, seed_val);
    if (rc) return rc;
    double *h = (double *)malloc(sizeof(double) * (size_t)n);
    double *rn = (double *)malloc(sizeof(double) * (size_t)n);
    if (!h || !rn) { free(h); free(rn); return OR_OOM; }
    memset(x, 0, sizeof(double) * (size_t)n);
    memset(r, 0, sizeof(double) * (size_t)n);
    memset(h, 0, sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < seed_nnz; i++) r[seed_idx[i]] = form_b(&f, seed_val[i]);
    double sigma = 1.0, dlt = 0.0;
    if (method == 1) {
        double mu, L;
        if (kind == KIND_PPR) { mu = param; L = 2.0 - param; }
        else { mu = 1.0 - param * lam; L = 1.0 + param * lam; }
        sigma = (L + mu) / (L - mu);
        dlt = 1.0 / sigma;
    }
    int64_t T = 0, nnz = rp[n];
    int status = OR_NOT_CONVERGED;
    for (int64_t t = 0;; t++) {
        if (t > 0) {
            int any = 0;
            for (int64_t u = 0; u < n && !any; u++) any = is_active(r[u], form_theta(&f, &g, u));
            if (!any) { status = OR_OK; break; }
        }
        if (t >= max_iters) break;
        if (method == 0 || t == 0) {
            for (int64_t u = 0; u < n; u++) h[u] = r[u];
        } else {
            double dnext = 1.0 / (2.0 * sigma - dlt);
            double c = 2.0 * sigma * dnext, m = dlt * dnext;
            for (int64_t u = 0; u < n; u++) h[u] = c * r[u] + m * h[u]; /* h still holds Delta */
            dlt = dnext;
        }
        /* r_new = r - Q h : r_new_w = r_w - h_w + sum_{u ~ w} w_u h_u */
        for (int64_t w = 0; w < n; w++) {
            double acc = r[w] - h[w];
            for (int64_t e = rp[w]; e < rp[w + 1]; e++) {
                int64_t u = ci[e];
                acc += form_w(&f, &g, u) * h[u];
            }
            rn[w] = acc;
        }
        for (int64_t u = 0; u < n; u++) { x[u] += h[u]; r[u] = rn[u]; }
        T++;
    }
    stats[0] = T; stats[1] = T * nnz; stats[2] = T * n; stats[3] = status;
    double a = 0.0, mx = 0.0, sc = form_rscale(&f);
    for (int64_t u = 0; u < n; u++) {
        double v = fabs(r[u]) * sc, d = deg(&g, u);
        a += v;
        if (d > 0 && v / d > mx) mx = v / d;
    }
    norms[0] = a;
    norms[1] = mx;
    free(h); free(rn);
    return status;
}

/*
 * Edge events on (x, r) in the generic form r = b - Q x (Sec. 4, the Insert and
 * Delete procedures of LocalGS(Dynamic) / LocalSOR(Dynamic)).  Each undirected
 * edge {a, c} is applied as the directed event a -> c and then c -> a; deg is the
 * current degree of every node and is updated event by event.
 *
 * PPR (Q = I - (1-alpha) A D^-1): a directed event a -> c changes column a of
 * A D^-1.  With d0 = deg[a] before and d1 after the event, x_a is rescaled to
 * x_a d1 / d0 so that the old neighbours keep receiving (1-alpha) x_a / d0;
 * with D = x_a / d0 (the change of x_a in magnitude):
 *   insert : x_a += D, r_a -= D, r_c += (1-alpha) D
 *   delete : x_a -= D, r_a += D, r_c -= (1-alpha) D
 * (the paper's procedures, written with the degree before the event, so that a
 * node left with degree 0 gets x_a = 0 instead of 0/0).  An isolated node's
 * column of A D^-1 is zero, so the first edge of a node with d0 = 0 only adds
 * (1-alpha) x_a to r_c.
 * Katz (Q = I - beta A, derived): the directed event a -> c adds or removes
 * A[c][a], so r_c += beta x_a (insert) or r_c -= beta x_a (delete).
 * sign: +1 insert, -1 delete.  The events must be valid for the graph they
 * are applied to (an inserted edge is new, a deleted edge exists).
 */
int oracle_edge_events(int64_t n, int kind, double param, double *x, double *r, int64_t *deg, int64_t k,
                       const int32_t *eu, const int32_t *ev, int sign) {
    if ((kind != KIND_PPR && kind != KIND_KATZ) || (sign != 1 && sign != -1)) return OR_INVALID;
    for (int64_t i = 0; i < k; i++) {
        for (int dir = 0; dir < 2; dir++) {
            int64_t a = dir == 0 ? eu[i] : ev[i];
            int64_t c = dir == 0 ? ev[i] : eu[i];
            if (a < 0 || a >= n || c < 0 || c >= n || a == c) return OR_INVALID;
            int64_t d0 = deg[a];
            if (sign < 0 && d0 < 1) return OR_INVALID;
            if (kind == KIND_PPR) {
                double alpha = param;
                if (d0 == 0) {
                    r[c] += (1.0 - alpha) * x[a];
                } else {
                    double D = x[a] / (double)d0;
                    x[a] += sign * D;
                    r[a] -= sign * D;
                    r[c] += sign * (1.0 - alpha) * D;
                }
            } else {
                r[c] += sign * param * x[a];
            }
            deg[a] = d0 + sign;
        }
    }
    return OR_OK;
}

/*
 * FIFO push (Algorithm 1 for APPR, the AKatz box of Sec. 2, LocalSOR of
 * Eq. (7) with q_uu = 1).  The queue starts with supp(s) in index order
 * (forced, Definition 3.1).  Pop u; v = r_u; x_u += omega v;
 * r_u -= omega v; r_w += omega w_u v for w in N(u); any node whose residual
 * is active and that is not queued joins the tail.  omega = 1 gives APPR /
 * AKatz.  stats[0..3] = pops, ops = sum of d_u over pops, epochs (queue
 * generations), status.  max_pops bounds the work (omega > 1 has no proof of
 * termination).
 */
int oracle_push_fifo(int64_t n, const int64_t *rp, const int32_t *ci, int kind, double param, double eps,
                     double omega, int32_t seed_nnz, const int32_t *seed_idx, const double *seed_val, int64_t max_pops,
                     double *x, double *r, int64_t *stats, double *norms) {
    graph_t g = {n, rp, ci};
    form_t f;
    if (make_form(kind, param, eps, &f)) return OR_INVALID;
    if (!(omega > 0.0 && omega < 2.0)) return OR_INVALID;
    int rc = check_seed(&g, seed_nnz, seed_idx, seed_val);
    if (rc) return rc;
    /* ring buffer of capacity n: a node is in the queue at most once */
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char *inq = (unsigned char *)calloc((size_t)n, 1);
    touched_t tch = {0};
    if (!q || !inq || touched_init(&tch, n)) { free(q); free(inq); touched_free(&tch); return OR_OOM; }
    memset(x, 0, sizeof(double) * (size_t)n);
    memset(r, 0, sizeof(double) * (size_t)n);
    int64_t head = 0, count = 0;
    for (int32_t i = 0; i < seed_nnz; i++) {
        int64_t u = seed_idx[i];
        r[u] = form_b(&f, seed_val[i]);
        touch(&tch, u);
        q[(head + count) % n] = u; count++; inq[u] = 1;
    }
    int64_t pops = 0, ops = 0, epochs = 0, epoch_left = count;
    int status = OR_OK;
    while (count > 0) {
        if (pops >= max_pops) { status = OR_NOT_CONVERGED; break; }
        if (epoch_left == 0) { epochs++; epoch_left = count; }
        int64_t u = q[head]; head = (head + 1) % n; count--; epoch_left--; inq[u] = 0;
        double v = r[u];
        double wu = form_w(&f, &g, u);
        x[u] += omega * v;
        r[u] -= omega * v;
        for (int64_t e = g.rp[u]; e < g.rp[u + 1]; e++) {
            int64_t w = g.ci[e];
            r[w] += omega * wu * v;
            touch(&tch, w);
            if (!inq[w] && is_active(r[w], form_theta(&f, &g, w))) {
                q[(head + count) % n] = w; count++; inq[w] = 1;
            }
        }
        if (!inq[u] && is_active(r[u], form_theta(&f, &g, u))) {
            q[(head + count) % n] = u; count++; inq[u] = 1;
        }
        pops++;
        ops += (int64_t)deg(&g, u);
    }
    stats[0] = pops; stats[1] = ops; stats[2] = epochs + (pops > 0); stats[3] = status;
    residual_norms(&g, &f, r, &tch, &norms[0], &norms[1]);
    free(q); free(inq); touched_free(&tch);
    return status;
}

/*
 * Heat kernel, level push (the AHK push of Sec. 2 on the Kronecker system,
 * processed one block at a time).  With M = A D^-1 the Taylor terms are
 * v_0 = e^{-tau} s, v_k = (tau/k) M v_{k-1}, f_K = sum_{k<=K} v_k.
 * Level k holds residual r_k (r_0 = e^{-tau} s).  Its active set is
 *   S_0 = supp(s) (forced),  S_k = {u : r_k[u] >= theta_{k,u}},
 *   theta_{k,u} = eps d_u / ((K+1) psi_k),  psi_k = sum_{j=k..K} tau^{j-k} k!/j!.
 * Each u in S_k moves r_k[u] into x and, for k < K, sends
 * (tau/(k+1)) r_k[u]/d_u to every neighbour in level k+1.  What stays in
 * level k is the leftover; ||f_K - x||_1 = sum_k psi_k ||leftover_k||_1.
 * norms[0] = that weighted sum, norms[1] = max_k (K+1) psi_k ||D^-1 leftover_k||_inf
 * (below eps iff every leftover is below its threshold).
 * stats = T (levels with a nonempty active set), ops, pushes, status.
 * run_level_push takes the series through c_0, the level ratios c_{k+1}/c_k
 * (ratio[k], k < K) and psi; oracle_hk and oracle_series below supply them.
 */
static int run_level_push(int64_t n, const int64_t *rp, const int32_t *ci, int32_t K, double c0,
                          const double *ratio, const double *psi, double eps, int32_t seed_nnz,
                          const int32_t *seed_idx, const double *seed_val, double *x, int64_t *stats, double *norms,
                          int64_t trace_cap, int64_t *tr_size, int64_t *tr_vol, int64_t nodes_cap,
                          int32_t *tr_nodes, int64_t *nodes_len, int64_t T_rec, const int64_t *off,
                          const int32_t *nodes, double kappa, int64_t *out_fv) {
    graph_t g = {n, rp, ci};
    int rc = check_seed(&g, seed_nnz, seed_idx, seed_val);
    if (rc) return rc;
    double *rk = (double *)calloc((size_t)n, sizeof(double));
    double *rk1 = (double *)calloc((size_t)n, sizeof(double));
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char *mark = (unsigned char *)calloc((size_t)n, 1);
    touched_t tk = {0}, tk1 = {0}; /* touched sets of the current and next level */
    if (!rk || !rk1 || !S || !mark || touched_init(&tk, n) || touched_init(&tk1, n)) return OR_OOM;
    memset(x, 0, sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < seed_nnz; i++) { rk[seed_idx[i]] = c0 * seed_val[i]; touch(&tk, seed_idx[i]); }
    replay_t rpl = {off, nodes, T_rec, kappa, 0, 0};
    int64_t T = 0, ops = 0, pushes = 0, rec = 0;
    double left_l1 = 0.0, left_dinf = 0.0;
    int stopped = 0;
    for (int32_t k = 0; k <= K; k++) {
        double th_k = eps / ((double)(K + 1) * psi[k]); /* theta_{k,u} = th_k * d_u */
        form_t fk = {KIND_KATZ, 0.0, th_k};              /* only its threshold is used */
        int64_t ns = 0;
        if (!stopped) {
            if (k == 0) {
                for (int32_t i = 0; i < seed_nnz; i++) S[ns++] = seed_idx[i];
                if (off && T_rec > 0) {
                    int64_t m = off[1] - off[0];
                    if (m != ns) rpl.violations++;
                }
            } else if (off) {
                ns = select_replay(&g, &fk, rk, &tk, &rpl, k, S, mark);
            } else {
                ns = select_free(&g, &fk, rk, &tk, S);
            }
        }
        if (ns == 0) stopped = 1;
        int64_t vol = 0;
        for (int64_t i = 0; i < ns; i++) {
            int64_t u = S[i];
            double v = rk[u];
            double d = deg(&g, u);
            vol += (int64_t)d;
            x[u] += v;
            rk[u] = 0.0;
            if (k < K) {
                double wgt = ratio[k] * v / d;
                for (int64_t ee = g.rp[u]; ee < g.rp[u + 1]; ee++) {
                    int64_t w = g.ci[ee];
                    rk1[w] += wgt;
                    touch(&tk1, w);
                }
            }
        }
        if (ns > 0) {
            if (T < trace_cap) { if (tr_size) tr_size[T] = ns; if (tr_vol) tr_vol[T] = vol; }
            for (int64_t i = 0; i < ns && tr_nodes; i++) {
                if (rec < nodes_cap) tr_nodes[rec] = (int32_t)S[i];
                rec++;
            }
            T++; ops += vol; pushes += ns;
        }
        /* leftover of level k */
        double l1 = 0.0, dinf = 0.0;
        for (int64_t i = 0; i < tk.len; i++) {
            int64_t u = tk.list[i];
            l1 += fabs(rk[u]);
            double d = deg(&g, u);
            if (d > 0 && fabs(rk[u]) / d > dinf) dinf = fabs(rk[u]) / d;
            rk[u] = 0.0;
            tk.flag[u] = 0;
        }
        tk.len = 0;
        left_l1 += psi[k] * l1;
        double wd = (double)(K + 1) * psi[k] * dinf;
        if (wd > left_dinf) left_dinf = wd;
        /* level k+1 becomes current */
        double *tmp = rk; rk = rk1; rk1 = tmp;
        touched_t tt = tk; tk = tk1; tk1 = tt;
    }
    if (off && T_rec != T) rpl.violations++;
    stats[0] = T; stats[1] = ops; stats[2] = pushes; stats[3] = OR_OK;
    norms[0] = left_l1; norms[1] = left_dinf;
    if (out_fv) { out_fv[0] = rpl.flips; out_fv[1] = rpl.violations; }
    if (nodes_len) *nodes_len = rec;
    free(rk); free(rk1); free(S); free(mark); touched_free(&tk); touched_free(&tk1);
    return OR_OK;
}

/* The heat kernel: c_k = e^{-tau} tau^k / k!, so c_0 = e^{-tau}, the level
 * ratio c_{k+1}/c_k = tau/(k+1) and psi_k = sum_{j=k..K} tau^{j-k} k!/j!.
 * psi_out (optional) receives psi. */
int oracle_hk(int64_t n, const int64_t *rp, const int32_t *ci, double tau, int32_t K, double eps, int32_t seed_nnz,
              const int32_t *seed_idx, const double *seed_val, double *x, int64_t *stats, double *norms,
              double *psi_out, int64_t trace_cap, int64_t *tr_size, int64_t *tr_vol, int64_t nodes_cap,
              int32_t *tr_nodes, int64_t *nodes_len, int64_t T_rec, const int64_t *off, const int32_t *nodes,
              double kappa, int64_t *out_fv) {
    if (!(tau >= 0.0) || !isfinite(tau) || K < 0 || K > 256 || !(eps > 0.0) || !isfinite(eps)) return OR_INVALID;
    double *psi = (double *)malloc(sizeof(double) * (size_t)(K + 1));
    double *ratio = (double *)malloc(sizeof(double) * (size_t)(K + 1));
    if (!psi || !ratio) { free(psi); free(ratio); return OR_OOM; }
    for (int32_t k = 0; k <= K; k++) {
        double s = 0.0, term = 1.0; /* term = tau^{j-k} k!/j! */
        for (int32_t j = k; j <= K; j++) {
            if (j > k) term *= tau / (double)j;
            s += term;
        }
        psi[k] = s;
        ratio[k] = tau / (double)(k + 1);
        if (psi_out) psi_out[k] = s;
    }
    int rc = run_level_push(n, rp, ci, K, exp(-tau), ratio, psi, eps, seed_nnz, seed_idx, seed_val, x, stats, norms,
                            trace_cap, tr_size, tr_vol, nodes_cap, tr_nodes, nodes_len, T_rec, off, nodes, kappa,
                            out_fv);
    free(psi); free(ratio);
    return rc;
}

/*
 * A general truncated series f_K = sum_{k=0..K} c_k (A D^-1)^k s (Eq. (1) with
 * M = A D^-1, Table 1), every c_k > 0 and finite: the same level push with
 * v_0 = c_0 s, level ratio c_{k+1}/c_k and psi_k = sum_{j=k..K} c_j / c_k (the
 * l1 weight of a unit of residual left at level k, since A D^-1 keeps mass).
 * With c_k = e^{-tau} tau^k/k! it is the heat kernel; with c_k = alpha
 * (1-alpha)^k the truncated PPR series.  psi_out as oracle_hk.
 */
int oracle_series(int64_t n, const int64_t *rp, const int32_t *ci, int32_t K, const double *c, double eps,
                  int32_t seed_nnz, const int32_t *seed_idx, const double *seed_val, double *x, int64_t *stats,
                  double *norms, double *psi_out, int64_t trace_cap, int64_t *tr_size, int64_t *tr_vol,
                  int64_t nodes_cap, int32_t *tr_nodes, int64_t *nodes_len, int64_t T_rec, const int64_t *off,
                  const int32_t *nodes, double kappa, int64_t *out_fv) {
    if (K < 0 || K > 256 || !c || !(eps > 0.0) || !isfinite(eps)) return OR_INVALID;
    for (int32_t k = 0; k <= K; k++)
        if (!(c[k] > 0.0) || !isfinite(c[k])) return OR_INVALID;
    double *psi = (double *)malloc(sizeof(double) * (size_t)(K + 1));
    double *ratio = (double *)malloc(sizeof(double) * (size_t)(K + 1));
    if (!psi || !ratio) { free(psi); free(ratio); return OR_OOM; }
    for (int32_t k = 0; k <= K; k++) {
        double s = 0.0;
        for (int32_t j = k; j <= K; j++) s += c[j] / c[k];
        psi[k] = s;
        ratio[k] = k < K ? c[k + 1] / c[k] : 0.0;
        if (psi_out) psi_out[k] = s;
    }
    int rc = run_level_push(n, rp, ci, K, c[0], ratio, psi, eps, seed_nnz, seed_idx, seed_val, x, stats, norms,
                            trace_cap, tr_size, tr_vol, nodes_cap, tr_nodes, nodes_len, T_rec, off, nodes, kappa,
                            out_fv);
    free(psi); free(ratio);
    return rc;
}
