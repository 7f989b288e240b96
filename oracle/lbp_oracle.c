/*
 * FP64 reference loopy belief propagation -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the oracle that the HIP implementation is checked against.
 * It shares no code with the HIP path and is never linked into it; only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * What it computes (PGMax, arXiv 2202.04110):
 *   - messages live in one flat array indexed by (edge, state), edges in
 *     factor order (Sec. "A fully flat array-based LBP implementation");
 *   - one iteration recomputes every factor-to-variable message from the
 *     previous iterate ("parallel message updates", Sec. "Package features")
 *     and then damps it [Pretti 2005];
 *   - enumeration factors are given by their valid configurations and one
 *     log-potential each (Sec. "Specifying complex factor graphs");
 *   - OR / AND logical factors use closed-form updates linear in the number
 *     of connected variables (Sec. "Package features", logical factors).
 * The paper prints no update equations; the reading used is textbook
 * log-domain loopy BP at temperature T (T = 0: max-product, T = 1:
 * sum-product):
 *   LSE_T(x) = max x                              (T = 0)
 *            = M + T log sum exp((x - M)/T)       (T > 0, M = max x)
 *   1. B[v,s]  = theta[v,s] + sum_{e in N(v)} m[e,s]
 *   2. n[e,s]  = B[var(e),s] - m[e,s]
 *   3. enum f: score(c) = phi_f(c) + sum_j n[e_j, c_j]
 *              u[e_j,s] = LSE_T{ score(c) : c_j = s } - n[e_j,s]
 *      OR / AND: closed forms (see or_update below)
 *   4. m'[e,s] = d m[e,s] + (1-d) u[e,s]
 *   5. m[e,s]  = m'[e,s] - max_s' m'[e,s']
 *   read-out: q[v,s] = B[v,s] - LSE_T,s(B[v,:]); MAP = lowest argmax_s B[v,s].
 * Messages start at 0.  The adjoint (og_backward) is plain reverse-mode
 * differentiation of N such iterations for T > 0 with every iterate stored.
 *
 * Every loop below is written for clarity, in the order of the steps above.
 * An optional OpenMP "parallel for" over variables / factors gives bitwise
 * the same result as one thread: every output element is owned by one
 * iteration of the loop and is computed in a fixed order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_ENUM 0
#define OG_OR 1
#define OG_AND 2

typedef struct {
    /* inputs (copied, FP64) */
    int32_t V, F, NT;
    int32_t *nst;          /* V   */
    double *theta;         /* VS  */
    int32_t *kind;         /* F   */
    int64_t *fe_off;       /* F+1 */
    int32_t *evar;         /* E   */
    int32_t *ftab;         /* F   */
    int32_t *tab_ncfg;     /* NT, 0 = dense */
    int64_t *tab_off;      /* NT+1 */
    int32_t *tab_states;   /* explicit tables */
    int64_t *lp_off;       /* F+1 */
    double *lp;            /* Tn  */
    /* derived */
    int64_t E, VS, ES, Tn;
    int64_t *vs_off;       /* V+1 */
    int64_t *es_off;       /* E+1 */
    int64_t *adj_off;      /* V+1, edges of each variable in increasing order */
    int64_t *adj;          /* E   */
} og_graph;

static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

void og_free(og_graph *g)
{
    if (!g) return;
    free(g->nst); free(g->theta); free(g->kind); free(g->fe_off); free(g->evar);
    free(g->ftab); free(g->tab_ncfg); free(g->tab_off); free(g->tab_states);
    free(g->lp_off); free(g->lp); free(g->vs_off); free(g->es_off);
    free(g->adj_off); free(g->adj);
    free(g);
}

/* Copies the graph (FP32 values are widened to FP64). Returns NULL on
 * allocation failure. Inputs are trusted: the tests hand in valid graphs. */
og_graph *og_create(int32_t V, const int32_t *nst, const float *theta,
                    int32_t F, const int32_t *kind, const int64_t *fe_off,
                    const int32_t *evar, const int32_t *ftab,
                    int32_t NT, const int32_t *tab_ncfg, const int64_t *tab_off,
                    const int32_t *tab_states, const int64_t *lp_off, const float *lp)
{
    og_graph *g = (og_graph *)calloc(1, sizeof(og_graph));
    if (!g) return NULL;
    g->V = V; g->F = F; g->NT = NT;
    g->E = fe_off[F];
    g->Tn = lp_off[F];
    g->nst = xcalloc(V, sizeof(int32_t));
    g->vs_off = xcalloc(V + 1, sizeof(int64_t));
    g->kind = xcalloc(F, sizeof(int32_t));
    g->fe_off = xcalloc(F + 1, sizeof(int64_t));
    g->evar = xcalloc(g->E, sizeof(int32_t));
    g->ftab = xcalloc(F, sizeof(int32_t));
    g->tab_ncfg = xcalloc(NT, sizeof(int32_t));
    g->tab_off = xcalloc(NT + 1, sizeof(int64_t));
    g->lp_off = xcalloc(F + 1, sizeof(int64_t));
    g->lp = xcalloc(g->Tn, sizeof(double));
    g->es_off = xcalloc(g->E + 1, sizeof(int64_t));
    g->adj_off = xcalloc(V + 1, sizeof(int64_t));
    g->adj = xcalloc(g->E, sizeof(int64_t));
    if (!g->nst || !g->vs_off || !g->kind || !g->fe_off || !g->evar || !g->ftab ||
        !g->tab_ncfg || !g->tab_off || !g->lp_off || !g->lp || !g->es_off ||
        !g->adj_off || !g->adj) { og_free(g); return NULL; }
    memcpy(g->nst, nst, sizeof(int32_t) * V);
    memcpy(g->kind, kind, sizeof(int32_t) * F);
    memcpy(g->fe_off, fe_off, sizeof(int64_t) * (F + 1));
    memcpy(g->evar, evar, sizeof(int32_t) * g->E);
    memcpy(g->ftab, ftab, sizeof(int32_t) * F);
    memcpy(g->tab_ncfg, tab_ncfg, sizeof(int32_t) * NT);
    memcpy(g->tab_off, tab_off, sizeof(int64_t) * (NT + 1));
    int64_t nts = tab_off[NT];
    g->tab_states = xcalloc(nts, sizeof(int32_t));
    if (!g->tab_states) { og_free(g); return NULL; }
    if (nts) memcpy(g->tab_states, tab_states, sizeof(int32_t) * nts);
    memcpy(g->lp_off, lp_off, sizeof(int64_t) * (F + 1));
    for (int64_t i = 0; i < g->Tn; ++i) g->lp[i] = (double)lp[i];

    for (int32_t v = 0; v < V; ++v) g->vs_off[v + 1] = g->vs_off[v] + nst[v];
    g->VS = g->vs_off[V];
    g->theta = xcalloc(g->VS, sizeof(double));
    if (!g->theta) { og_free(g); return NULL; }
    for (int64_t i = 0; i < g->VS; ++i) g->theta[i] = (double)theta[i];

    for (int64_t e = 0; e < g->E; ++e) g->es_off[e + 1] = g->es_off[e] + nst[evar[e]];
    g->ES = g->es_off[g->E];

    /* variable -> edges, edges in increasing index order */
    for (int64_t e = 0; e < g->E; ++e) g->adj_off[evar[e] + 1]++;
    for (int32_t v = 0; v < V; ++v) g->adj_off[v + 1] += g->adj_off[v];
    int64_t *fill = xcalloc(V, sizeof(int64_t));
    if (!fill) { og_free(g); return NULL; }
    for (int64_t e = 0; e < g->E; ++e) {
        int32_t v = evar[e];
        g->adj[g->adj_off[v] + fill[v]++] = e;
    }
    free(fill);
    return g;
}

int64_t og_num_edge_states(const og_graph *g) { return g->ES; }
int64_t og_num_var_states(const og_graph *g) { return g->VS; }

/* ---------------------------------------------------------------- helpers */

/* LSE_T over x[0..k-1]; -inf for an empty set. */
static double lse_t(const double *x, int64_t k, double T)
{
    if (k == 0) return -INFINITY;
    double M = -INFINITY;
    for (int64_t i = 0; i < k; ++i) if (x[i] > M) M = x[i];
    if (T == 0.0 || M == -INFINITY) return M;
    double s = 0.0;
    for (int64_t i = 0; i < k; ++i) s += exp((x[i] - M) / T);
    return M + T * log(s);
}

/* softplus at temperature T: T log(1 + e^{x/T}) = LSE_T(0, x) */
static double sp_t(double x, double T)
{
    if (x == -INFINITY) return 0.0;
    double a = fabs(x);
    return (x > 0 ? x : 0.0) + T * log1p(exp(-a / T));
}

/* T log(e^{a/T} - 1) for a >= 0, -inf at a = 0 */
static double lem_t(double a, double T)
{
    if (a <= 0.0) return -INFINITY;
    return a + T * log(-expm1(-a / T));
}

/* State of slot j in configuration c of factor f (dense tables: row-major,
 * last slot fastest). */
static int32_t cfg_state(const og_graph *g, int32_t f, int64_t c, int32_t j, int32_t arity)
{
    int32_t t = g->ftab[f];
    if (g->tab_ncfg[t] > 0) return g->tab_states[g->tab_off[t] + c * arity + j];
    int64_t r = c;
    for (int32_t l = arity - 1; l > j; --l) r /= g->nst[g->evar[g->fe_off[f] + l]];
    return (int32_t)(r % g->nst[g->evar[g->fe_off[f] + j]]);
}

static int64_t num_cfgs(const og_graph *g, int32_t f)
{
    return g->lp_off[f + 1] - g->lp_off[f];
}

/* step 1: beliefs */
static void beliefs(const og_graph *g, const double *m, double *B, int nthreads)
{
    (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads) if (nthreads > 1)
    for (int32_t v = 0; v < g->V; ++v) {
        for (int32_t s = 0; s < g->nst[v]; ++s) {
            double b = g->theta[g->vs_off[v] + s];
            for (int64_t k = g->adj_off[v]; k < g->adj_off[v + 1]; ++k)
                b += m[g->es_off[g->adj[k]] + s];
            B[g->vs_off[v] + s] = b;
        }
    }
}

/* step 3 for an enumeration factor: u[e_j, s] for all slots j and states s.
 * n points at the vtof rows (edge-state indexed), u is written at the same
 * positions. scratch holds num_cfgs doubles. */
static void enum_update(const og_graph *g, int32_t f, const double *n, double *u,
                        double T, double *score, double *sel)
{
    int64_t e0 = g->fe_off[f];
    int32_t k = (int32_t)(g->fe_off[f + 1] - e0);
    int64_t C = num_cfgs(g, f);
    for (int64_t c = 0; c < C; ++c) {
        double sc = g->lp[g->lp_off[f] + c];
        for (int32_t j = 0; j < k; ++j)
            sc += n[g->es_off[e0 + j] + cfg_state(g, f, c, j, k)];
        score[c] = sc;
    }
    for (int32_t j = 0; j < k; ++j) {
        int64_t e = e0 + j;
        int32_t ns = g->nst[g->evar[e]];
        for (int32_t s = 0; s < ns; ++s) {
            int64_t cnt = 0;
            for (int64_t c = 0; c < C; ++c)
                if (cfg_state(g, f, c, j, k) == s) sel[cnt++] = score[c];
            u[g->es_off[e] + s] = lse_t(sel, cnt, T) - n[g->es_off[e] + s];
        }
    }
}

/* step 3 for an OR factor (parents = all edges but the last, child = last).
 * Works on the differences delta = n[.,1] - n[.,0]; writes u[.,0] and u[.,1].
 * With flip = 1 the factor is AND: De Morgan, every variable complemented,
 * i.e. deltas negated on the way in and state roles swapped on the way out.
 *
 *   T = 0:  S = sum relu(delta_j), S_-i by prefix/suffix sums,
 *           M_-i = max_{j != i} delta_j (-inf if there is one parent)
 *           child:    u(0) = 0, u(1) = S + min(0, max_j delta_j)
 *           parent i: u(1) = delta_c + S_-i,
 *                     u(0) = max(0, delta_c + S_-i + min(0, M_-i))
 *   T > 0:  A = sum sp_T(delta_j), A_-i by prefix/suffix sums
 *           child:    u(0) = 0, u(1) = lem_T(A)
 *           parent i: u(1) = delta_c + A_-i, u(0) = sp_T(delta_c + lem_T(A_-i))
 * Each is the LSE_T of step 3 over the OR truth table, evaluated in closed
 * form (every joint state of the parents except all-zero maps to child 1). */
static void or_update(const og_graph *g, int32_t f, const double *n, double *u,
                      double T, int flip, double *buf)
{
    int64_t e0 = g->fe_off[f];
    int32_t k = (int32_t)(g->fe_off[f + 1] - e0);
    int32_t p = k - 1;
    double sgn = flip ? -1.0 : 1.0;
    double *delta = buf, *term = buf + k, *pre = buf + 2 * k, *suf = buf + 3 * k + 1;
    for (int32_t j = 0; j < k; ++j) {
        int64_t o = g->es_off[e0 + j];
        delta[j] = sgn * (n[o + 1] - n[o]);
    }
    double dc = delta[p];
    for (int32_t j = 0; j < p; ++j)
        term[j] = (T == 0.0) ? (delta[j] > 0 ? delta[j] : 0.0) : sp_t(delta[j], T);
    pre[0] = 0.0;
    for (int32_t j = 0; j < p; ++j) pre[j + 1] = pre[j] + term[j];
    suf[p] = 0.0;
    for (int32_t j = p - 1; j >= 0; --j) suf[j] = suf[j + 1] + term[j];
    double total = pre[p];
    double a0, a1;
    /* child */
    if (T == 0.0) {
        double mx = -INFINITY;
        for (int32_t j = 0; j < p; ++j) if (delta[j] > mx) mx = delta[j];
        a0 = 0.0;
        a1 = total + (mx < 0 ? mx : 0.0);
    } else {
        a0 = 0.0;
        a1 = lem_t(total, T);
    }
    {
        int64_t o = g->es_off[e0 + p];
        u[o + 0] = flip ? a1 : a0;
        u[o + 1] = flip ? a0 : a1;
    }
    /* parents; M_-i from the largest delta, its (first) index and the
     * largest delta among the other parents */
    int32_t amax = 0;
    for (int32_t j = 1; j < p; ++j) if (delta[j] > delta[amax]) amax = j;
    double max1 = p > 0 ? delta[amax] : -INFINITY, max2 = -INFINITY;
    for (int32_t j = 0; j < p; ++j) if (j != amax && delta[j] > max2) max2 = delta[j];
    for (int32_t i = 0; i < p; ++i) {
        double loo = pre[i] + suf[i + 1];
        if (T == 0.0) {
            double mo = (i == amax) ? max2 : max1;
            a1 = dc + loo;
            double alt = dc + loo + (mo < 0 ? mo : 0.0);
            a0 = alt > 0 ? alt : 0.0;
        } else {
            a1 = dc + loo;
            a0 = sp_t(dc + lem_t(loo, T), T);
        }
        int64_t o = g->es_off[e0 + i];
        u[o + 0] = flip ? a1 : a0;
        u[o + 1] = flip ? a0 : a1;
    }
}

static int64_t max_arity(const og_graph *g)
{
    int64_t mx = 1;
    for (int32_t f = 0; f < g->F; ++f) {
        int64_t k = g->fe_off[f + 1] - g->fe_off[f];
        if (k > mx) mx = k;
    }
    return mx;
}

static int64_t max_cfgs(const og_graph *g)
{
    int64_t mx = 1;
    for (int32_t f = 0; f < g->F; ++f) if (num_cfgs(g, f) > mx) mx = num_cfgs(g, f);
    return mx;
}

/* One iteration m -> m_next (steps 1-5). u receives the undamped update. */
static int iterate(const og_graph *g, const double *m, double *m_next, double *B, double *n,
                   double *u, double d, double T, int nthreads)
{
    beliefs(g, m, B, nthreads);
    /* step 2 */
#pragma omp parallel for schedule(static) num_threads(nthreads) if (nthreads > 1)
    for (int64_t e = 0; e < g->E; ++e) {
        int32_t v = g->evar[e];
        for (int32_t s = 0; s < g->nst[v]; ++s)
            n[g->es_off[e] + s] = B[g->vs_off[v] + s] - m[g->es_off[e] + s];
    }
    int64_t mc = max_cfgs(g), ma = max_arity(g);
    int err = 0;
    /* steps 3-5, one factor at a time */
#pragma omp parallel num_threads(nthreads) if (nthreads > 1)
    {
        double *score = (double *)malloc(sizeof(double) * mc);
        double *sel = (double *)malloc(sizeof(double) * mc);
        double *buf = (double *)malloc(sizeof(double) * (4 * ma + 4));
        if (!score || !sel || !buf) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (int32_t f = 0; f < g->F; ++f) {
                if (g->kind[f] == OG_ENUM) enum_update(g, f, n, u, T, score, sel);
                else or_update(g, f, n, u, T, g->kind[f] == OG_AND, buf);
                for (int64_t e = g->fe_off[f]; e < g->fe_off[f + 1]; ++e) {
                    int32_t ns = g->nst[g->evar[e]];
                    int64_t o = g->es_off[e];
                    double mx = -INFINITY;
                    for (int32_t s = 0; s < ns; ++s) {
                        m_next[o + s] = d * m[o + s] + (1.0 - d) * u[o + s];
                        if (m_next[o + s] > mx) mx = m_next[o + s];
                    }
                    for (int32_t s = 0; s < ns; ++s) m_next[o + s] -= mx;
                }
            }
        }
        free(score); free(sel); free(buf);
    }
    return err ? -2 : 0;
}

/* Runs `iters` iterations starting from m (ES doubles, updated in place).
 * resid (iters doubles, may be NULL) receives max|m_{t+1} - m_t| per iteration.
 * Returns 0, or -2 on allocation failure. */
int og_run(const og_graph *g, int32_t iters, double d, double T, int32_t nthreads,
           double *m, double *resid)
{
    double *B = xcalloc(g->VS, sizeof(double));
    double *n = xcalloc(g->ES, sizeof(double));
    double *u = xcalloc(g->ES, sizeof(double));
    double *mn = xcalloc(g->ES, sizeof(double));
    int rc = 0;
    if (!B || !n || !u || !mn) rc = -2;
    for (int32_t t = 0; t < iters && rc == 0; ++t) {
        rc = iterate(g, m, mn, B, n, u, d, T, nthreads);
        if (resid) {
            double r = 0.0;
            for (int64_t i = 0; i < g->ES; ++i) {
                double a = fabs(mn[i] - m[i]);
                if (a > r || a != a) r = a;
            }
            resid[t] = r;
        }
        memcpy(m, mn, sizeof(double) * g->ES);
    }
    free(B); free(n); free(u); free(mn);
    return rc;
}

/* One undamped, unnormalised factor update u(m) (steps 1-3) for tests of the
 * fixed-point property. */
int og_update(const og_graph *g, double T, const double *m, double *u)
{
    double *B = xcalloc(g->VS, sizeof(double));
    double *n = xcalloc(g->ES, sizeof(double));
    double *mn = xcalloc(g->ES, sizeof(double));
    int rc = (!B || !n || !mn) ? -2 : iterate(g, m, mn, B, n, u, 0.0, T, 1);
    free(B); free(n); free(mn);
    return rc;
}

/* Read-out from messages m: B (VS, may be NULL), q = B - LSE_T(B) (VS, may be
 * NULL), MAP = lowest-index argmax of B (V, may be NULL). */
int og_beliefs(const og_graph *g, const double *m, double T, double *Bout, double *q,
               int32_t *map)
{
    double *B = xcalloc(g->VS, sizeof(double));
    if (!B) return -2;
    beliefs(g, m, B, 1);
    for (int32_t v = 0; v < g->V; ++v) {
        const double *b = B + g->vs_off[v];
        int32_t ns = g->nst[v];
        if (q) {
            double z = lse_t(b, ns, T);
            for (int32_t s = 0; s < ns; ++s) q[g->vs_off[v] + s] = b[s] - z;
        }
        if (map) {
            int32_t best = 0;
            for (int32_t s = 1; s < ns; ++s) if (b[s] > b[best]) best = s;
            map[v] = best;
        }
    }
    if (Bout) memcpy(Bout, B, sizeof(double) * g->VS);
    free(B);
    return 0;
}

/* Log-score of a joint assignment x (V states): sum of evidence and factor
 * log-potentials, -inf if x violates a logical factor or matches no valid
 * configuration of an enumeration factor. */
double og_score(const og_graph *g, const int32_t *x)
{
    double sc = 0.0;
    for (int32_t v = 0; v < g->V; ++v) sc += g->theta[g->vs_off[v] + x[v]];
    for (int32_t f = 0; f < g->F; ++f) {
        int64_t e0 = g->fe_off[f];
        int32_t k = (int32_t)(g->fe_off[f + 1] - e0);
        if (g->kind[f] == OG_ENUM) {
            int64_t C = num_cfgs(g, f), hit = -1;
            for (int64_t c = 0; c < C && hit < 0; ++c) {
                int ok = 1;
                for (int32_t j = 0; j < k && ok; ++j)
                    ok = cfg_state(g, f, c, j, k) == x[g->evar[e0 + j]];
                if (ok) hit = c;
            }
            if (hit < 0) return -INFINITY;
            sc += g->lp[g->lp_off[f] + hit];
        } else {
            int any = 0, all = 1;
            for (int32_t j = 0; j < k - 1; ++j) {
                int b = x[g->evar[e0 + j]] != 0;
                any |= b; all &= b;
            }
            int child = x[g->evar[e0 + k - 1]] != 0;
            if (child != (g->kind[f] == OG_OR ? any : all)) return -INFINITY;
        }
    }
    return sc;
}

/* ------------------------------------------------------------- adjoint */

/* Reverse-mode derivative of L = sum_{v,s} gq[v,s] q[v,s], where q is the
 * read-out after `iters` iterations from m0 at temperature T > 0.
 * Outputs: gphi (Tn), gtheta (VS), gm0 (ES, may be NULL).
 * Only enumeration factors are supported (returns -1 otherwise); returns -2 on
 * allocation failure.  Every iterate is stored (plain, not memory-frugal). */
int og_backward(const og_graph *g, int32_t iters, double d, double T, const double *m0,
                const double *gq, double *gphi, double *gtheta, double *gm0)
{
    if (!(T > 0.0)) return -1;
    for (int32_t f = 0; f < g->F; ++f) if (g->kind[f] != OG_ENUM) return -1;
    int64_t ES = g->ES, VS = g->VS;
    double *ms = xcalloc((size_t)(iters + 1) * ES, sizeof(double));
    double *B = xcalloc(VS, sizeof(double));
    double *n = xcalloc(ES, sizeof(double));
    double *u = xcalloc(ES, sizeof(double));
    double *mp = xcalloc(ES, sizeof(double));  /* m' before normalisation */
    double *gm = xcalloc(ES, sizeof(double));  /* adjoint of m_{t+1} */
    double *gmp = xcalloc(ES, sizeof(double));
    double *gn = xcalloc(ES, sizeof(double));
    double *gB = xcalloc(VS, sizeof(double));
    int64_t mc = max_cfgs(g);
    double *score = xcalloc(mc, sizeof(double));
    double *sel = xcalloc(mc, sizeof(double));
    double *gscore = xcalloc(mc, sizeof(double));
    int rc = 0;
    if (!ms || !B || !n || !u || !mp || !gm || !gmp || !gn || !gB || !score || !sel || !gscore) {
        rc = -2;
        goto out;
    }
    memcpy(ms, m0, sizeof(double) * ES);
    for (int32_t t = 0; t < iters; ++t) {
        rc = iterate(g, ms + (size_t)t * ES, ms + (size_t)(t + 1) * ES, B, n, u, d, T, 1);
        if (rc) goto out;
    }
    memset(gphi, 0, sizeof(double) * g->Tn);
    memset(gtheta, 0, sizeof(double) * VS);
    /* read-out: q = B - LSE_T(B); dq/dB = I - p 1^T with p = softmax(B/T) */
    beliefs(g, ms + (size_t)iters * ES, B, 1);
    for (int32_t v = 0; v < g->V; ++v) {
        int32_t ns = g->nst[v];
        const double *b = B + g->vs_off[v];
        double z = lse_t(b, ns, T), tot = 0.0;
        for (int32_t s = 0; s < ns; ++s) tot += gq[g->vs_off[v] + s];
        for (int32_t s = 0; s < ns; ++s)
            gB[g->vs_off[v] + s] = gq[g->vs_off[v] + s] - exp((b[s] - z) / T) * tot;
    }
    /* B = theta + sum m */
    for (int64_t i = 0; i < VS; ++i) gtheta[i] += gB[i];
    for (int64_t e = 0; e < g->E; ++e) {
        int32_t v = g->evar[e];
        for (int32_t s = 0; s < g->nst[v]; ++s)
            gm[g->es_off[e] + s] = gB[g->vs_off[v] + s];
    }
    for (int32_t t = iters - 1; t >= 0; --t) {
        const double *m = ms + (size_t)t * ES;
        /* forward quantities of iteration t */
        beliefs(g, m, B, 1);
        for (int64_t e = 0; e < g->E; ++e) {
            int32_t v = g->evar[e];
            for (int32_t s = 0; s < g->nst[v]; ++s)
                n[g->es_off[e] + s] = B[g->vs_off[v] + s] - m[g->es_off[e] + s];
        }
        for (int32_t f = 0; f < g->F; ++f) enum_update(g, f, n, u, T, score, sel);
        for (int64_t e = 0; e < g->E; ++e) {
            int32_t ns = g->nst[g->evar[e]];
            int64_t o = g->es_off[e];
            for (int32_t s = 0; s < ns; ++s) mp[o + s] = d * m[o + s] + (1.0 - d) * u[o + s];
        }
        /* step 5: m_{t+1} = m' - m'[argmax] */
        for (int64_t e = 0; e < g->E; ++e) {
            int32_t ns = g->nst[g->evar[e]];
            int64_t o = g->es_off[e];
            int32_t am = 0;
            for (int32_t s = 1; s < ns; ++s) if (mp[o + s] > mp[o + am]) am = s;
            double tot = 0.0;
            for (int32_t s = 0; s < ns; ++s) tot += gm[o + s];
            for (int32_t s = 0; s < ns; ++s) gmp[o + s] = gm[o + s] - (s == am ? tot : 0.0);
        }
        /* step 4: m' = d m + (1-d) u ; gm now becomes the adjoint of m_t */
        for (int64_t i = 0; i < ES; ++i) {
            gm[i] = d * gmp[i];
            gn[i] = 0.0;
        }
        /* step 3: u[e_j,s] = LSE_T{score(c): c_j = s} - n[e_j,s] */
        for (int32_t f = 0; f < g->F; ++f) {
            int64_t e0 = g->fe_off[f];
            int32_t k = (int32_t)(g->fe_off[f + 1] - e0);
            int64_t C = num_cfgs(g, f);
            for (int64_t c = 0; c < C; ++c) {
                double sc = g->lp[g->lp_off[f] + c];
                for (int32_t j = 0; j < k; ++j)
                    sc += n[g->es_off[e0 + j] + cfg_state(g, f, c, j, k)];
                score[c] = sc;
                gscore[c] = 0.0;
            }
            for (int32_t j = 0; j < k; ++j) {
                int64_t o = g->es_off[e0 + j];
                int32_t ns = g->nst[g->evar[e0 + j]];
                for (int32_t s = 0; s < ns; ++s) {
                    double gu = (1.0 - d) * gmp[o + s];
                    int64_t cnt = 0;
                    for (int64_t c = 0; c < C; ++c)
                        if (cfg_state(g, f, c, j, k) == s) sel[cnt++] = score[c];
                    double z = lse_t(sel, cnt, T);
                    for (int64_t c = 0; c < C; ++c)
                        if (cfg_state(g, f, c, j, k) == s)
                            gscore[c] += gu * exp((score[c] - z) / T);
                    gn[o + s] -= gu;
                }
            }
            for (int64_t c = 0; c < C; ++c) {
                gphi[g->lp_off[f] + c] += gscore[c];
                for (int32_t j = 0; j < k; ++j)
                    gn[g->es_off[e0 + j] + cfg_state(g, f, c, j, k)] += gscore[c];
            }
        }
        /* step 2: n = B[var] - m */
        memset(gB, 0, sizeof(double) * VS);
        for (int64_t e = 0; e < g->E; ++e) {
            int32_t v = g->evar[e];
            for (int32_t s = 0; s < g->nst[v]; ++s) {
                gB[g->vs_off[v] + s] += gn[g->es_off[e] + s];
                gm[g->es_off[e] + s] -= gn[g->es_off[e] + s];
            }
        }
        /* step 1: B = theta + sum m */
        for (int64_t i = 0; i < VS; ++i) gtheta[i] += gB[i];
        for (int64_t e = 0; e < g->E; ++e) {
            int32_t v = g->evar[e];
            for (int32_t s = 0; s < g->nst[v]; ++s)
                gm[g->es_off[e] + s] += gB[g->vs_off[v] + s];
        }
    }
    if (gm0) memcpy(gm0, gm, sizeof(double) * ES);
out:
    free(ms); free(B); free(n); free(u); free(mp); free(gm); free(gmp); free(gn); free(gB);
    free(score); free(sel); free(gscore);
    return rc;
}
