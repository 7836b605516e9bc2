/*
 * Plain CPU oracle for BP-SF decoding.  TEST INFRASTRUCTURE ONLY: the tests,
 * the smoke check and the benchmark's CPU-baseline leg call it; the product
 * library never links, loads or calls it, and it shares no code with it.
 *
 * Method (paper: "Fully Parallelized BP Decoding for Quantum LDPC Codes Can
 * Outperform BP-OSD", arXiv 2507.00254):
 *   - Section II-B, steps 1-4: normalized min-sum BP on the Tanner graph of H
 *     with a flooding schedule (channel LLR init, variable-to-check sum over
 *     the other checks, check-to-variable min-sum rule Eq. (c2v), marginal and
 *     hard decision), stopped as soon as the hard decision reproduces the
 *     syndrome or after i_max iterations;
 *   - Algorithm 1: BP with per-bit oscillation counting, selection of the
 *     |Phi| most-flipped bits, trial vectors over Phi, syndrome flip
 *     s' = s + t H^T, an independent BP on every s', and undoing the flip on
 *     the output; Section IV: the result kept among successful trials.
 *
 * Written as plain loops in the paper's order so it can be checked by eye.
 * REAL is double by default; the same source is also built with REAL=float so
 * that hard decisions can be compared with a float implementation in the same
 * precision.  Built with -ffp-contract=off (no fused multiply-add).
 *
 * Readings where the paper is silent or garbled (each listed in the design
 * notes):
 *   - adaptive damping printed as "1 - 2^i" is read as alpha_i = 1 - 2^-i, i
 *     counted from 1 within each BP run; a positive fixed alpha overrides it;
 *   - sign(x) is -1 exactly when x < 0;
 *   - every iteration runs V2C, C2V, marginal + hard decision, then the
 *     oscillation update, then the syndrome test;
 *   - sums over a variable's checks run left to right in ascending check
 *     index, starting from the channel LLR;
 *   - c2v magnitude is alpha * (minimum over the other edges), one rounding;
 *   - top(flip_count, k) orders by count descending, then index ascending;
 *   - trial vectors: either all 2^k subsets of Phi (subset index = bit mask,
 *     bit j <-> Phi[j]) or all subsets of weight 1..w_max in combination order,
 *     or the caller's list of masks (|Phi| up to 64);
 *   - every trial BP starts from zero messages with its own iteration count;
 *   - result selection: minimum Hamming weight of the undone correction (ties
 *     to the lower trial index), or the lowest-index successful trial;
 *   - no successful trial: main BP's last hard decision, flagged not converged.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#define REAL double
#endif
#ifndef SUFFIX
#define SUFFIX _f64
#endif
typedef REAL real;

#define CAT2(a, b) a##b
#define CAT(a, b) CAT2(a, b)
#define FN(name) CAT(name, SUFFIX)

typedef struct {
    int32_t max_iter;       /* i_max of the first BP (with oscillation tracking) */
    int32_t cand_max_iter;  /* i_max of every trial BP */
    int32_t k;              /* |Phi| */
    int32_t cand_mode;      /* 0: all subsets of Phi; 1: subsets of weight 1..w_max */
    int32_t w_max;
    int32_t select_mode;    /* 0: minimum weight; 1: lowest successful trial index */
    double alpha;           /* > 0: fixed normalization; 0: adaptive 1 - 2^-i */
    int32_t flags;          /* bit0: never stop early; bit1: post-process even if BP converged */
    int32_t rule;           /* 0: normalized min-sum; 1: sum-product (tanh rule) */
} oracle_params;

#define OR_NO_EARLY_STOP 1
#define OR_FORCE_PP 2
#define OR_LAYERED 8      /* layered (row-serial) schedule instead of flooding */

/* ---------------------------------------------------------------- graph -- */

typedef struct {
    int M, N, E;
    const int32_t *row_ptr, *col_idx;   /* H by rows: edge e = position in col_idx */
    int32_t *var_ptr, *var_edge;        /* edges of each variable, ascending check */
    int32_t *order;                     /* checks in layered-schedule order */
    int n_layers;
} graph;

static int graph_build(graph *g, int M, int N, const int32_t *row_ptr, const int32_t *col_idx)
{
    g->M = M;
    g->N = N;
    g->row_ptr = row_ptr;
    g->col_idx = col_idx;
    g->E = row_ptr[M];
    g->var_ptr = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
    g->var_edge = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->E > 0 ? g->E : 1));
    int32_t *fill = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
    if (!g->var_ptr || !g->var_edge || !fill) {
        free(g->var_ptr); free(g->var_edge); free(fill);
        return -1;
    }
    for (int e = 0; e < g->E; e++) {
        if (col_idx[e] < 0 || col_idx[e] >= N) { free(g->var_ptr); free(g->var_edge); free(fill); return -1; }
        g->var_ptr[col_idx[e] + 1]++;
    }
    for (int v = 0; v < N; v++) g->var_ptr[v + 1] += g->var_ptr[v];
    /* Scanning rows in increasing order lists each variable's edges by ascending check. */
    for (int c = 0; c < M; c++)
        for (int e = row_ptr[c]; e < row_ptr[c + 1]; e++) {
            int v = col_idx[e];
            g->var_edge[g->var_ptr[v] + fill[v]++] = e;
        }
    free(fill);

    /* Layers of the layered schedule: in index order, each check takes the
     * smallest layer that no earlier check sharing a bit with it has. The
     * schedule visits the checks by layer, then by index. */
    int32_t *layer = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M > 0 ? M : 1));
    g->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M > 0 ? M : 1));
    uint8_t *used = (uint8_t *)calloc((size_t)M + 1, 1);
    if (!layer || !g->order || !used) {
        free(layer); free(g->order); free(used); free(g->var_ptr); free(g->var_edge);
        return -1;
    }
    g->n_layers = 0;
    for (int c = 0; c < M; c++) {
        memset(used, 0, (size_t)M + 1);
        for (int e = row_ptr[c]; e < row_ptr[c + 1]; e++) {
            int v = col_idx[e];
            for (int a = g->var_ptr[v]; a < g->var_ptr[v + 1]; a++) {
                int e2 = g->var_edge[a];
                int c2 = 0;
                while (row_ptr[c2 + 1] <= e2) c2++;   /* the check holding edge e2 */
                if (c2 < c) used[layer[c2]] = 1;
            }
        }
        int l = 0;
        while (used[l]) l++;
        layer[c] = l;
        if (l + 1 > g->n_layers) g->n_layers = l + 1;
    }
    int n = 0;
    for (int l = 0; l < g->n_layers; l++)
        for (int c = 0; c < M; c++)
            if (layer[c] == l) g->order[n++] = c;
    free(layer);
    free(used);
    return 0;
}

static void graph_free(graph *g)
{
    free(g->var_ptr);
    free(g->var_edge);
    free(g->order);
}

/* ------------------------------------------------------------------- BP -- */

typedef struct {
    real *c2v, *v2c, *lout;
    uint8_t *hard, *prev;
    int32_t *flips;
} bp_work;

typedef struct {          /* optional per-iteration records of one run */
    real *c2v;            /* [max_iter][E] (edge = CSR position) */
    real *v2c;            /* [max_iter][E] */
    real *lout;           /* [max_iter][N] */
    uint8_t *hard;        /* [max_iter][N] */
} bp_trace;

static real alpha_at(const oracle_params *prm, int iter)
{
    if (prm->alpha > 0.0) return (real)prm->alpha;
    return (real)(1.0 - ldexp(1.0, -iter));
}

/* One BP run on syndrome s.  Returns the number of iterations executed and
 * sets *converged.  With track != 0 the flip counts are accumulated. */
/* Step 3 for check c: c2v of its edges from the v2c of its edges. */
static void check_update(const graph *g, const uint8_t *s, const oracle_params *prm, real alpha, int c, bp_work *w)
{
    const int lo = g->row_ptr[c], hi = g->row_ptr[c + 1];
    if (prm->rule == 1) {
        /* Sum-product: 2 atanh of the product of tanh(x/2) over the other edges. */
        for (int e = lo; e < hi; e++) {
            double prod = 1.0;
            for (int e2 = lo; e2 < hi; e2++)
                if (e2 != e) prod *= tanh((double)w->v2c[e2] * 0.5);
            double val = 2.0 * atanh(prod);
            w->c2v[e] = (real)(s[c] ? -val : val);
        }
        return;
    }
    /* Min-sum: the minimum |v2c| over the other edges is the overall
     * minimum except on the edge holding it, where it is the second one. */
    real min1 = (real)INFINITY, min2 = (real)INFINITY;
    int arg = -1;
    int par = s[c] & 1;
    for (int e = lo; e < hi; e++) {
        real a = fabs(w->v2c[e]);
        if (a < min1) { min2 = min1; min1 = a; arg = e; }
        else if (a < min2) { min2 = a; }
        par ^= (w->v2c[e] < 0);
    }
    for (int e = lo; e < hi; e++) {
        real mag = (e == arg) ? min2 : min1;
        int neg = par ^ (w->v2c[e] < 0);   /* (-1)^s times the others' signs */
        real val = alpha * mag;
        w->c2v[e] = neg ? -val : val;
    }
}

/* Layered schedule: the checks in layer order, each one reading the current
 * posteriors of its bits, v2c = posterior - its previous c2v, and writing the
 * posteriors back as v2c + its new c2v before the next check reads them. */
static void layered_sweep(const graph *g, const uint8_t *s, const oracle_params *prm, real alpha, bp_work *w)
{
    for (int i = 0; i < g->M; i++) {
        const int c = g->order[i];
        for (int e = g->row_ptr[c]; e < g->row_ptr[c + 1]; e++)
            w->v2c[e] = w->lout[g->col_idx[e]] - w->c2v[e];
        check_update(g, s, prm, alpha, c, w);
        for (int e = g->row_ptr[c]; e < g->row_ptr[c + 1]; e++)
            w->lout[g->col_idx[e]] = w->v2c[e] + w->c2v[e];
    }
}

static int bp_run(const graph *g, const uint8_t *s, const real *L, const oracle_params *prm,
                  int max_iter, int track, bp_work *w, const bp_trace *tr, int *converged)
{
    const int M = g->M, N = g->N, E = g->E;
    *converged = 0;
    /* Messages from checks start at zero (step 2: "set to 0 for the first iteration"). */
    for (int e = 0; e < E; e++) w->c2v[e] = (real)0;
    for (int v = 0; v < N; v++) { w->prev[v] = 0; if (track) w->flips[v] = 0; }

    const int layered = (prm->flags & OR_LAYERED) != 0;
    if (layered) for (int v = 0; v < N; v++) w->lout[v] = L[v];
    int it = 0;
    for (it = 1; it <= max_iter; it++) {
        if (layered) {
            layered_sweep(g, s, prm, alpha_at(prm, it), w);
            for (int v = 0; v < N; v++) w->hard[v] = (w->lout[v] > 0) ? 0 : 1;
            goto decided;
        }
        /* Step 2, V2C: channel LLR plus the messages of all other checks. */
        for (int v = 0; v < N; v++) {
            for (int a = g->var_ptr[v]; a < g->var_ptr[v + 1]; a++) {
                int e = g->var_edge[a];
                real acc = L[v];
                for (int b = g->var_ptr[v]; b < g->var_ptr[v + 1]; b++) {
                    int e2 = g->var_edge[b];
                    if (e2 != e) acc = acc + w->c2v[e2];
                }
                w->v2c[e] = acc;
            }
        }
        /* Step 3, C2V. */
        const real alpha = alpha_at(prm, it);
        for (int c = 0; c < M; c++) check_update(g, s, prm, alpha, c, w);
        /* Step 4: marginal LLR and hard decision. */
        for (int v = 0; v < N; v++) {
            real acc = L[v];
            for (int a = g->var_ptr[v]; a < g->var_ptr[v + 1]; a++) acc = acc + w->c2v[g->var_edge[a]];
            w->lout[v] = acc;
            w->hard[v] = (acc > 0) ? 0 : 1;
        }
    decided:
        /* Algorithm 1: oscillation tracking against the previous hard decision. */
        for (int v = 0; v < N; v++) {
            if (track) w->flips[v] += (w->hard[v] ^ w->prev[v]);
            w->prev[v] = w->hard[v];
        }
        if (tr) {
            if (tr->c2v) memcpy(tr->c2v + (size_t)(it - 1) * E, w->c2v, sizeof(real) * (size_t)E);
            if (tr->v2c) memcpy(tr->v2c + (size_t)(it - 1) * E, w->v2c, sizeof(real) * (size_t)E);
            if (tr->lout) memcpy(tr->lout + (size_t)(it - 1) * N, w->lout, sizeof(real) * (size_t)N);
            if (tr->hard) memcpy(tr->hard + (size_t)(it - 1) * N, w->hard, (size_t)N);
        }
        /* Stop when e H^T = s. */
        int ok = 1;
        for (int c = 0; c < M && ok; c++) {
            int par = s[c] & 1;
            for (int e = g->row_ptr[c]; e < g->row_ptr[c + 1]; e++) par ^= w->hard[g->col_idx[e]];
            if (par) ok = 0;
        }
        /* The flag describes the hard decision that is returned. */
        *converged = ok;
        if (ok && !(prm->flags & OR_NO_EARLY_STOP)) return it;
    }
    return max_iter;
}

static int work_alloc(bp_work *w, int N, int E)
{
    w->c2v = (real *)malloc(sizeof(real) * (size_t)(E > 0 ? E : 1));
    w->v2c = (real *)malloc(sizeof(real) * (size_t)(E > 0 ? E : 1));
    w->lout = (real *)malloc(sizeof(real) * (size_t)(N > 0 ? N : 1));
    w->hard = (uint8_t *)malloc((size_t)(N > 0 ? N : 1));
    w->prev = (uint8_t *)malloc((size_t)(N > 0 ? N : 1));
    w->flips = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    return (w->c2v && w->v2c && w->lout && w->hard && w->prev && w->flips) ? 0 : -1;
}

static void work_free(bp_work *w)
{
    free(w->c2v); free(w->v2c); free(w->lout); free(w->hard); free(w->prev); free(w->flips);
}

static int priors_to_llr(const double *priors, int N, real *L)
{
    for (int v = 0; v < N; v++) {
        double p = priors[v];
        if (!(p > 0.0 && p < 1.0)) return -1;
        /* Step 1: channel LLR, computed in double and then held in REAL. */
        L[v] = (real)log((1.0 - p) / p);
    }
    return 0;
}

/* kmax: 24 for generated trial lists (2^k masks at most 2^24), up to 64 for
 * a caller's list (a 64-bit mask per trial). */
static int check_params(const oracle_params *prm, int N, int kmax)
{
    if (prm->max_iter < 1 || prm->cand_max_iter < 0) return -1;
    if (prm->k < 0 || prm->k > N || prm->k > kmax) return -1;
    if (prm->cand_mode != 0 && prm->cand_mode != 1) return -1;
    if (prm->cand_mode == 1 && (prm->w_max < 1 || prm->w_max > prm->k)) return -1;
    if (prm->select_mode != 0 && prm->select_mode != 1) return -1;
    if (!(prm->alpha >= 0.0) || prm->rule < 0 || prm->rule > 1) return -1;
    return 0;
}

/* ---------------------------------------------------------- trial list -- */

/* Number of trial vectors and, if masks != NULL, the masks in trial order. */
static int64_t trial_masks(const oracle_params *prm, uint64_t *masks)
{
    const int k = prm->k;
    if (k == 0) return 0;
    if (prm->cand_mode == 0) {
        int64_t n = (int64_t)1 << k;
        if (masks) for (int64_t i = 0; i < n; i++) masks[i] = (uint64_t)i;
        return n;
    }
    /* Weight 1, then weight 2, ...: combinations of positions in lexicographic order. */
    int64_t n = 0;
    int pos[32];
    for (int wgt = 1; wgt <= prm->w_max; wgt++) {
        for (int j = 0; j < wgt; j++) pos[j] = j;
        for (;;) {
            if (masks) {
                uint64_t m = 0;
                for (int j = 0; j < wgt; j++) m |= 1ull << pos[j];
                masks[n] = m;
            }
            n++;
            int j = wgt - 1;
            while (j >= 0 && pos[j] == k - wgt + j) j--;
            if (j < 0) break;
            pos[j]++;
            for (int q = j + 1; q < wgt; q++) pos[q] = pos[q - 1] + 1;
        }
    }
    return n;
}

/* ---------------------------------------------------------------- BP-SF -- */

typedef struct {
    uint8_t converged;
    int32_t iterations;       /* main iterations (+ winning trial's, if a trial won) */
    int32_t main_iterations;
    uint8_t main_converged;
    int32_t winner;           /* trial index, or -1 */
    int64_t trial_iterations; /* iterations summed over every trial run */
} shot_result;

typedef struct {
    uint8_t *conv;      /* [n_trials] or NULL */
    int32_t *iters;     /* [n_trials] or NULL */
    int32_t *weight;    /* [n_trials] or NULL (-1 when not converged) */
} trial_record;

static int bpsf_one(const graph *g, const uint8_t *s, const real *L, const oracle_params *prm,
                    const uint64_t *masks, int64_t n_trials, bp_work *w, uint8_t *s2, uint8_t *best,
                    uint8_t *corr, int32_t *phi_out, int32_t *flips_out, const bp_trace *tr,
                    trial_record *rec, shot_result *res)
{
    const int N = g->N, M = g->M;
    int conv = 0;
    int it = bp_run(g, s, L, prm, prm->max_iter, 1, w, tr, &conv);
    res->main_iterations = it;
    res->main_converged = (uint8_t)conv;
    res->winner = -1;
    res->trial_iterations = 0;
    memcpy(corr, w->hard, (size_t)N);
    if (flips_out) memcpy(flips_out, w->flips, sizeof(int32_t) * (size_t)N);
    res->converged = (uint8_t)conv;
    res->iterations = it;
    if (phi_out) for (int j = 0; j < prm->k; j++) phi_out[j] = -1;
    if ((conv && !(prm->flags & OR_FORCE_PP)) || prm->k == 0) return 0;

    /* top(flip_count, |Phi|): count descending, index ascending. */
    int32_t phi[64];
    uint8_t *t_vec = best;   /* trial vector t as a 0/1 array over the bits */
    memset(t_vec, 0, (size_t)N);
    for (int j = 0; j < prm->k; j++) {
        int bi = -1;
        for (int v = 0; v < N; v++) {
            if (t_vec[v]) continue;
            if (bi < 0 || w->flips[v] > w->flips[bi]) bi = v;
        }
        phi[j] = bi;
        t_vec[bi] = 1;   /* marks "already chosen" while selecting */
    }
    if (phi_out) for (int j = 0; j < prm->k; j++) phi_out[j] = phi[j];

    uint8_t *t = (uint8_t *)malloc((size_t)N + 1);
    if (!t) return -1;
    int have = 0;
    int32_t best_w = 0, best_it = 0;
    int64_t best_idx = -1;
    for (int64_t ti = 0; ti < n_trials; ti++) {
        uint64_t mask = masks[ti];
        memset(t, 0, (size_t)N);
        for (int j = 0; j < prm->k; j++)
            if ((mask >> j) & 1ull) t[phi[j]] = 1;
        /* s' = s + t H^T: row c of H dotted with t, added to s_c. */
        for (int c = 0; c < M; c++) {
            int par = s[c] & 1;
            for (int e = g->row_ptr[c]; e < g->row_ptr[c + 1]; e++) par ^= t[g->col_idx[e]];
            s2[c] = (uint8_t)par;
        }
        int tconv = 0;
        int tit = bp_run(g, s2, L, prm, prm->cand_max_iter, 0, w, NULL, &tconv);
        res->trial_iterations += tit;
        int32_t wt = -1;
        if (tconv) {
            /* Undo the flip on the output: e = e' + t. */
            for (int v = 0; v < N; v++) w->hard[v] ^= t[v];
            wt = 0;
            for (int v = 0; v < N; v++) wt += w->hard[v];
            int take = 0;
            if (!have) take = 1;
            else if (prm->select_mode == 0 && wt < best_w) take = 1;
            if (take) {
                have = 1;
                best_w = wt;
                best_it = tit;
                best_idx = ti;
                memcpy(best, w->hard, (size_t)N);
            }
        }
        if (rec) {
            if (rec->conv) rec->conv[ti] = (uint8_t)tconv;
            if (rec->iters) rec->iters[ti] = tit;
            if (rec->weight) rec->weight[ti] = wt;
        }
        if (have && prm->select_mode == 1 && !rec) break;   /* first success in trial order */
    }
    free(t);
    if (have) {
        memcpy(corr, best, (size_t)N);
        res->converged = 1;
        res->iterations = res->main_iterations + best_it;
        res->winner = (int32_t)best_idx;
    }
    return 0;
}

/* ------------------------------------------------------------- exports -- */

/* One BP run (no post-processing) with optional per-iteration records.
 * flips_out counts oscillations over the iterations executed. */
int FN(oracle_bp)(int32_t M, int32_t N, const int32_t *row_ptr, const int32_t *col_idx,
                  const uint8_t *syndrome, const double *priors, const oracle_params *prm,
                  int32_t max_iter, uint8_t *hard_out, real *lout_out, int32_t *flips_out,
                  real *trace_c2v, real *trace_v2c, real *trace_lout, uint8_t *trace_hard,
                  int32_t *iters_out, uint8_t *converged_out)
{
    if (M < 0 || N < 0 || !row_ptr || max_iter < 1) return -1;
    if (!(prm->alpha >= 0.0) || prm->rule < 0 || prm->rule > 1) return -1;
    graph g;
    if (graph_build(&g, M, N, row_ptr, col_idx)) return -1;
    bp_work w;
    real *L = (real *)malloc(sizeof(real) * (size_t)(N > 0 ? N : 1));
    int rc = -1;
    if (!L || work_alloc(&w, N, g.E)) { free(L); graph_free(&g); return -1; }
    if (priors_to_llr(priors, N, L) == 0) {
        bp_trace tr = {trace_c2v, trace_v2c, trace_lout, trace_hard};
        int conv = 0;
        int it = bp_run(&g, syndrome, L, prm, max_iter, 1, &w, &tr, &conv);
        if (hard_out) memcpy(hard_out, w.hard, (size_t)N);
        if (lout_out) memcpy(lout_out, w.lout, sizeof(real) * (size_t)N);
        if (flips_out) memcpy(flips_out, w.flips, sizeof(int32_t) * (size_t)N);
        *iters_out = it;
        *converged_out = (uint8_t)conv;
        rc = 0;
    }
    work_free(&w);
    free(L);
    graph_free(&g);
    return rc;
}

/* Number of trial vectors the parameters produce (or -1 if invalid). */
int64_t FN(oracle_num_trials)(const oracle_params *prm, uint32_t *masks_out)
{
    if (prm->k < 0 || prm->k > 24) return -1;
    if (prm->cand_mode == 1 && (prm->w_max < 1 || prm->w_max > prm->k)) return -1;
    const int64_t n = trial_masks(prm, NULL);
    if (masks_out && n > 0) {
        uint64_t *m = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
        if (!m) return -1;
        trial_masks(prm, m);
        for (int64_t i = 0; i < n; i++) masks_out[i] = (uint32_t)m[i];   /* k <= 24: no bit lost */
        free(m);
    }
    return n;
}

/* BP-SF on one syndrome with every intermediate exposed (tests). */
int FN(oracle_bpsf_detail)(int32_t M, int32_t N, const int32_t *row_ptr, const int32_t *col_idx,
                           const uint8_t *syndrome, const double *priors, const oracle_params *prm,
                           uint8_t *corr_out, int32_t *phi_out, int32_t *flips_out,
                           uint8_t *trial_conv, int32_t *trial_iters, int32_t *trial_weight,
                           int32_t *summary /* converged, iterations, main_iters, main_conv, winner */,
                           int64_t *trial_iter_total)
{
    if (M < 0 || N < 0 || !row_ptr || check_params(prm, N, 24)) return -1;
    graph g;
    if (graph_build(&g, M, N, row_ptr, col_idx)) return -1;
    int64_t nt = trial_masks(prm, NULL);
    uint64_t *masks = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nt > 0 ? nt : 1));
    real *L = (real *)malloc(sizeof(real) * (size_t)(N > 0 ? N : 1));
    uint8_t *s2 = (uint8_t *)malloc((size_t)(M > N ? M : N) + 1);
    uint8_t *best = (uint8_t *)malloc((size_t)N + 1);
    bp_work w;
    int rc = -1;
    if (masks && L && s2 && best && work_alloc(&w, N, g.E) == 0) {
        trial_masks(prm, masks);
        if (priors_to_llr(priors, N, L) == 0) {
            shot_result res;
            trial_record rec = {trial_conv, trial_iters, trial_weight};
            rc = bpsf_one(&g, syndrome, L, prm, masks, nt, &w, s2, best, corr_out, phi_out, flips_out,
                          NULL, &rec, &res);
            summary[0] = res.converged;
            summary[1] = res.iterations;
            summary[2] = res.main_iterations;
            summary[3] = res.main_converged;
            summary[4] = res.winner;
            if (trial_iter_total) *trial_iter_total = res.trial_iterations;
        }
        work_free(&w);
    }
    free(masks); free(L); free(s2); free(best);
    graph_free(&g);
    return rc;
}

typedef struct {
    const graph *g;
    const uint8_t *syn;
    const real *L;
    const oracle_params *prm;
    const uint64_t *masks;
    int64_t n_trials, mask_stride, lo, hi;
    uint8_t *corr, *conv;
    int32_t *iters, *winner, *phi, *main_iters;
    int64_t *trial_iters;
    int rc;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *j = (batch_job *)arg;
    const int N = j->g->N, M = j->g->M, k = j->prm->k;
    bp_work w;
    uint8_t *s2 = (uint8_t *)malloc((size_t)(M > N ? M : N) + 1);
    uint8_t *best = (uint8_t *)malloc((size_t)N + 1);
    j->rc = -1;
    if (!s2 || !best || work_alloc(&w, N, j->g->E)) { free(s2); free(best); return NULL; }
    j->rc = 0;
    for (int64_t i = j->lo; i < j->hi; i++) {
        shot_result res;
        int32_t phi_tmp[64];
        if (bpsf_one(j->g, j->syn + (size_t)i * M, j->L, j->prm, j->masks + i * j->mask_stride, j->n_trials,
                     &w, s2, best,
                     j->corr + (size_t)i * N, phi_tmp, NULL, NULL, NULL, &res)) { j->rc = -1; break; }
        j->conv[i] = res.converged;
        j->iters[i] = res.iterations;
        if (j->winner) j->winner[i] = res.winner;
        if (j->main_iters) j->main_iters[i] = res.main_iterations;
        if (j->trial_iters) j->trial_iters[i] = res.trial_iterations;
        if (j->phi) for (int q = 0; q < k; q++) j->phi[(size_t)i * k + q] = phi_tmp[q];
    }
    work_free(&w);
    free(s2);
    free(best);
    return NULL;
}

static int run_batch(const graph *g, const uint8_t *syndromes, int64_t shots, const real *L,
                     const oracle_params *prm, const uint64_t *masks, int64_t nt, int64_t mask_stride,
                     uint8_t *corr, uint8_t *conv, int32_t *iters, int32_t *winner, int32_t *phi,
                     int32_t *main_iters, int64_t *trial_iters, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > shots) nthreads = (int32_t)shots;
    batch_job jobs[256];
    pthread_t tid[256];
    for (int t = 0; t < nthreads; t++) {
        batch_job *j = &jobs[t];
        j->g = g; j->syn = syndromes; j->L = L; j->prm = prm; j->masks = masks; j->n_trials = nt;
        j->mask_stride = mask_stride;
        j->lo = shots * t / nthreads; j->hi = shots * (t + 1) / nthreads;
        j->corr = corr; j->conv = conv; j->iters = iters; j->winner = winner; j->phi = phi;
        j->main_iters = main_iters; j->trial_iters = trial_iters; j->rc = 0;
    }
    int started = 0;
    for (int t = 1; t < nthreads; t++)
        if (pthread_create(&tid[t], NULL, batch_worker, &jobs[t]) == 0) started = t; else { jobs[t].rc = -1; break; }
    batch_worker(&jobs[0]);
    for (int t = 1; t <= started; t++) pthread_join(tid[t], NULL);
    int rc = 0;
    for (int t = 0; t < nthreads; t++) if (jobs[t].rc) rc = -1;
    return rc;
}

/* BP-SF over a batch of syndromes; shots are split statically over threads. */
int FN(oracle_bpsf_batch)(int32_t M, int32_t N, const int32_t *row_ptr, const int32_t *col_idx,
                          const uint8_t *syndromes, int64_t shots, const double *priors,
                          const oracle_params *prm, uint8_t *corr, uint8_t *conv, int32_t *iters,
                          int32_t *winner, int32_t *phi, int32_t *main_iters, int64_t *trial_iters,
                          int32_t nthreads)
{
    if (M < 0 || N < 0 || shots < 0 || !row_ptr || check_params(prm, N, 24)) return -1;
    if (shots == 0) return 0;
    graph g;
    if (graph_build(&g, M, N, row_ptr, col_idx)) return -1;
    int64_t nt = trial_masks(prm, NULL);
    uint64_t *masks = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nt > 0 ? nt : 1));
    real *L = (real *)malloc(sizeof(real) * (size_t)(N > 0 ? N : 1));
    int rc = -1;
    if (masks && L && priors_to_llr(priors, N, L) == 0) {
        trial_masks(prm, masks);
        rc = run_batch(&g, syndromes, shots, L, prm, masks, nt, 0, corr, conv, iters, winner, phi, main_iters,
                       trial_iters, nthreads);
    }
    free(masks);
    free(L);
    graph_free(&g);
    return rc;
}

/* As oracle_bpsf_batch with the trial vectors given by the caller instead of
 * prm->cand_mode: shot i tries masks[i * mask_stride + t] for t < n_trials,
 * in that order (bit j <-> Phi[j]; bits at or above k are ignored). A stride
 * of 0 gives every shot the same list. 64-bit masks, |Phi| up to 64. */
int FN(oracle_bpsf_batch_table64)(int32_t M, int32_t N, const int32_t *row_ptr, const int32_t *col_idx,
                                  const uint8_t *syndromes, int64_t shots, const double *priors,
                                  const oracle_params *prm, const uint64_t *masks, int64_t n_trials,
                                  int64_t mask_stride, uint8_t *corr, uint8_t *conv, int32_t *iters,
                                  int32_t *winner, int32_t *phi, int32_t *main_iters, int64_t *trial_iters,
                                  int32_t nthreads)
{
    oracle_params q = *prm;
    q.cand_mode = 0;   /* validated as such; the list comes from the caller */
    if (M < 0 || N < 0 || shots < 0 || !row_ptr || check_params(&q, N, 64)) return -1;
    if (n_trials < 0 || mask_stride < 0 || (n_trials > 0 && !masks)) return -1;
    if (shots == 0) return 0;
    graph g;
    if (graph_build(&g, M, N, row_ptr, col_idx)) return -1;
    real *L = (real *)malloc(sizeof(real) * (size_t)(N > 0 ? N : 1));
    int rc = -1;
    if (L && priors_to_llr(priors, N, L) == 0)
        rc = run_batch(&g, syndromes, shots, L, prm, masks, n_trials, mask_stride, corr, conv, iters, winner, phi,
                       main_iters, trial_iters, nthreads);
    free(L);
    graph_free(&g);
    return rc;
}

/* The same with 32-bit masks (|Phi| up to 32): the list is widened. */
int FN(oracle_bpsf_batch_table)(int32_t M, int32_t N, const int32_t *row_ptr, const int32_t *col_idx,
                                const uint8_t *syndromes, int64_t shots, const double *priors,
                                const oracle_params *prm, const uint32_t *masks, int64_t n_trials,
                                int64_t mask_stride, uint8_t *corr, uint8_t *conv, int32_t *iters,
                                int32_t *winner, int32_t *phi, int32_t *main_iters, int64_t *trial_iters,
                                int32_t nthreads)
{
    if (prm->k > 32 || n_trials < 0 || mask_stride < 0 || shots < 0 || (n_trials > 0 && !masks)) return -1;
    const int64_t n = mask_stride > 0 ? shots * mask_stride : n_trials;
    uint64_t *wide = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    if (!wide) return -1;
    for (int64_t i = 0; i < n; i++) wide[i] = masks ? masks[i] : 0;
    const int rc = FN(oracle_bpsf_batch_table64)(M, N, row_ptr, col_idx, syndromes, shots, priors, prm,
                                                 n > 0 ? wide : NULL, n_trials, mask_stride, corr, conv, iters,
                                                 winner, phi, main_iters, trial_iters, nthreads);
    free(wide);
    return rc;
}
