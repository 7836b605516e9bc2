/*
 * Sanitizer driver for the CPU oracle (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer together with
 * oracle/bpsf_oracle.c, it calls every exported entry point on small codes
 * (a path, the [7,4] Hamming code, the [[72,12,6]] bivariate-bicycle check
 * matrix, a random column-weight-2 matrix) with the option combinations the
 * tests use, including rejected arguments. Any invalid access or undefined
 * operation aborts the run; a wrong result is not its concern.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t max_iter, cand_max_iter, k, cand_mode, w_max, select_mode;
    double alpha;
    int32_t flags, rule;
} oracle_params;

int oracle_bp_f64(int32_t, int32_t, const int32_t *, const int32_t *, const uint8_t *, const double *,
                  const oracle_params *, int32_t, uint8_t *, double *, int32_t *, double *, double *, double *,
                  uint8_t *, int32_t *, uint8_t *);
int64_t oracle_num_trials_f64(const oracle_params *, uint32_t *);
int oracle_bpsf_detail_f64(int32_t, int32_t, const int32_t *, const int32_t *, const uint8_t *, const double *,
                           const oracle_params *, uint8_t *, int32_t *, int32_t *, uint8_t *, int32_t *, int32_t *,
                           int32_t *, int64_t *);
int oracle_bpsf_batch_f64(int32_t, int32_t, const int32_t *, const int32_t *, const uint8_t *, int64_t,
                          const double *, const oracle_params *, uint8_t *, uint8_t *, int32_t *, int32_t *,
                          int32_t *, int32_t *, int64_t *, int32_t);
int oracle_bpsf_batch_table64_f64(int32_t, int32_t, const int32_t *, const int32_t *, const uint8_t *, int64_t,
                                  const double *, const oracle_params *, const uint64_t *, int64_t, int64_t,
                                  uint8_t *, uint8_t *, int32_t *, int32_t *, int32_t *, int32_t *, int64_t *,
                                  int32_t);
int oracle_bpsf_batch_table_f64(int32_t, int32_t, const int32_t *, const int32_t *, const uint8_t *, int64_t,
                                const double *, const oracle_params *, const uint32_t *, int64_t, int64_t,
                                uint8_t *, uint8_t *, int32_t *, int32_t *, int32_t *, int32_t *, int64_t *,
                                int32_t);

typedef struct {
    int M, N;
    int32_t *row_ptr, *col_idx;
} csr;

static uint64_t rng_state = 0x2507002540ull;
static uint64_t rnd(void)   /* xorshift64*: a source of test data only */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 0x2545F4914F6CDD1Dull;
}

static csr from_dense(int M, int N, const uint8_t *h)
{
    csr c = {M, N, malloc(sizeof(int32_t) * (size_t)(M + 1)), malloc(sizeof(int32_t) * (size_t)(M * N + 1))};
    int e = 0;
    for (int r = 0; r < M; r++) {
        c.row_ptr[r] = e;
        for (int v = 0; v < N; v++)
            if (h[r * N + v]) c.col_idx[e++] = v;
    }
    c.row_ptr[M] = e;
    return c;
}

/* H_X = [A | B] of the bivariate-bicycle code with l = m = 6,
 * A = x^3 + y + y^2, B = y^3 + x + x^2, x = S_6 (x) I_6, y = I_6 (x) S_6 */
static csr bb72(void)
{
    const int l = 6, m = 6, n = l * m;
    uint8_t *h = calloc((size_t)n * 2 * n, 1);
    for (int i = 0; i < l; i++)
        for (int j = 0; j < m; j++) {
            const int r = i * m + j;
            /* x^a y^b maps row (i, j) to column ((i + a) mod l, (j + b) mod m) */
            const int A[3][2] = {{3, 0}, {0, 1}, {0, 2}}, B[3][2] = {{0, 3}, {1, 0}, {2, 0}};
            for (int t = 0; t < 3; t++) {
                h[r * 2 * n + ((i + A[t][0]) % l) * m + (j + A[t][1]) % m] ^= 1;
                h[r * 2 * n + n + ((i + B[t][0]) % l) * m + (j + B[t][1]) % m] ^= 1;
            }
        }
    csr c = from_dense(n, 2 * n, h);
    free(h);
    return c;
}

static void run_code(const csr *c, int shots, double p)
{
    const int M = c->M, N = c->N;
    uint8_t *syn = calloc((size_t)shots * M, 1), *corr = calloc((size_t)shots * N, 1), *conv = calloc(shots, 1);
    int32_t *it = calloc(shots, 4), *win = calloc(shots, 4), *mit = calloc(shots, 4), *phi = calloc((size_t)shots * 64, 4);
    int64_t *tit = calloc(shots, 8);
    double *pri = malloc(sizeof(double) * N);
    for (int v = 0; v < N; v++) pri[v] = p * (0.5 + (double)(rnd() % 1000) / 1000.0);
    for (int s = 0; s < shots; s++)
        for (int r = 0; r < M; r++) {
            int par = 0;
            for (int e = c->row_ptr[r]; e < c->row_ptr[r + 1]; e++) par ^= (rnd() % 1000) < (uint64_t)(p * 1000);
            syn[s * M + r] = (uint8_t)par;
        }
    const oracle_params variants[] = {
        {30, 10, 4, 0, 1, 0, 0.625, 0, 0}, {30, 10, 5, 1, 2, 1, 0.0, 0, 0}, {20, 8, 4, 0, 1, 0, 0.625, 1, 0},
        {20, 8, 3, 0, 1, 0, 0.625, 2, 0},  {20, 8, 4, 0, 1, 0, 0.625, 8, 0}, {25, 0, 0, 0, 1, 0, 0.625, 0, 0},
        {15, 5, 3, 1, 3, 1, 1.0, 0, 1},
    };
    for (size_t vi = 0; vi < sizeof variants / sizeof variants[0]; vi++) {
        oracle_params prm = variants[vi];
        if (prm.k > N) continue;
        const int64_t nt = oracle_num_trials_f64(&prm, NULL);
        uint32_t *masks = malloc(sizeof(uint32_t) * (size_t)(nt > 0 ? nt : 1));
        if (nt > 0) oracle_num_trials_f64(&prm, masks);
        /* one shot with every intermediate and the per-iteration records */
        const int im = prm.max_iter;
        double *tc = calloc((size_t)im * c->row_ptr[M], 8), *tv = calloc((size_t)im * c->row_ptr[M], 8),
               *tl = calloc((size_t)im * N, 8), *lout = calloc(N, 8);
        uint8_t *th = calloc((size_t)im * N, 1), *hard = calloc(N, 1), *tconv = calloc(nt > 0 ? nt : 1, 1), bc = 0;
        int32_t *flips = calloc(N, 4), *titer = calloc(nt > 0 ? nt : 1, 4), *twt = calloc(nt > 0 ? nt : 1, 4),
                pphi[64], summary[5], bit = 0;
        int64_t ttot = 0;
        if (oracle_bp_f64(M, N, c->row_ptr, c->col_idx, syn, pri, &prm, im, hard, lout, flips, tc, tv, tl, th, &bit, &bc))
            abort();
        if (oracle_bpsf_detail_f64(M, N, c->row_ptr, c->col_idx, syn, pri, &prm, corr, pphi, flips, tconv, titer, twt,
                                   summary, &ttot))
            abort();
        if (oracle_bpsf_batch_f64(M, N, c->row_ptr, c->col_idx, syn, shots, pri, &prm, corr, conv, it, win, phi, mit,
                                  tit, 3))
            abort();
        if (nt > 0) {
            if (oracle_bpsf_batch_table_f64(M, N, c->row_ptr, c->col_idx, syn, shots, pri, &prm, masks, nt, 0, corr,
                                            conv, it, win, phi, mit, tit, 2))
                abort();
            /* one list per shot, widened to 64 bits */
            uint64_t *per = malloc(sizeof(uint64_t) * (size_t)(nt * shots));
            for (int64_t i = 0; i < nt * shots; i++) per[i] = masks[i % nt];
            if (oracle_bpsf_batch_table64_f64(M, N, c->row_ptr, c->col_idx, syn, shots, pri, &prm, per, nt, nt, corr,
                                              conv, it, win, phi, mit, tit, 2))
                abort();
            free(per);
        }
        free(masks); free(tc); free(tv); free(tl); free(lout); free(th); free(hard); free(tconv); free(flips);
        free(titer); free(twt);
    }
    /* |Phi| = 40 with 64-bit single-bit masks (caller lists reach 64) */
    if (N >= 40) {
        oracle_params big = {20, 10, 40, 0, 1, 0, 0.625, 0, 0};
        uint64_t one[3] = {1ull << 35, 1ull << 39, 3ull};
        if (oracle_bpsf_batch_table64_f64(M, N, c->row_ptr, c->col_idx, syn, shots, pri, &big, one, 3, 0, corr, conv, it,
                                          win, phi, mit, tit, 2))
            abort();
    }
    /* rejected arguments: each must return an error, touching nothing */
    oracle_params bad = {0, 10, 4, 0, 1, 0, 0.625, 0, 0};
    if (!oracle_bpsf_batch_f64(M, N, c->row_ptr, c->col_idx, syn, shots, pri, &bad, corr, conv, it, win, phi, mit, tit, 1))
        abort();
    bad.max_iter = 10;
    bad.k = N + 1;
    if (!oracle_bpsf_detail_f64(M, N, c->row_ptr, c->col_idx, syn, pri, &bad, corr, phi, it, conv, it, it, it, tit))
        abort();
    pri[0] = 0.0;
    oracle_params ok = {10, 5, 2, 0, 1, 0, 0.625, 0, 0};
    if (!oracle_bpsf_batch_f64(M, N, c->row_ptr, c->col_idx, syn, shots, pri, &ok, corr, conv, it, win, phi, mit, tit, 1))
        abort();
    free(syn); free(corr); free(conv); free(it); free(win); free(mit); free(phi); free(tit); free(pri);
}

int main(void)
{
    uint8_t path[4 * 5] = {0}, ham[3 * 7] = {1, 0, 1, 0, 1, 0, 1, 0, 1, 1, 0, 0, 1, 1, 0, 0, 0, 1, 1, 1, 1},
            rand2[6 * 12] = {0};
    for (int r = 0; r < 4; r++) path[r * 5 + r] = path[r * 5 + r + 1] = 1;
    for (int v = 0; v < 12; v++) {
        const int a = (int)(rnd() % 6), b = (a + 1 + (int)(rnd() % 5)) % 6;
        rand2[a * 12 + v] = rand2[b * 12 + v] = 1;
    }
    csr codes[4] = {from_dense(4, 5, path), from_dense(3, 7, ham), from_dense(6, 12, rand2), bb72()};
    for (int i = 0; i < 4; i++) {
        run_code(&codes[i], i == 3 ? 60 : 20, i == 3 ? 0.06 : 0.15);
        free(codes[i].row_ptr);
        free(codes[i].col_idx);
    }
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
