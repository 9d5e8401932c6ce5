/*
 * bzref.c -- reference (oracle) minimum distance of linear codes over F_3 / F_7.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the GPU library.  Plain mod-p integers,
 * one byte per symbol, every codeword formed from its rows and counted.
 *
 * What is computed (arXiv 2603.29942):
 *   d = min{ wt(c) : c in C \ {0} }                               (Sec. 3)
 * reached with the Brouwer-Zimmermann rounds of Algorithm 6 (Sec. 3.1):
 *   L := 1, U := n-k+1, g := 1; while g <= k and L < U: for every matrix
 *   Gamma_j take the minimum weight of all combinations of g of its rows;
 *   then L := (m-1)(g+1) + max{0, g+1-k+k_m}; g := g+1.
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *   - the combinations of Algorithm 6 range over F_p (the listing writes F_2),
 *     with the coefficient of the lowest-indexed row fixed to 1 because scalar
 *     multiples have equal weight (Sec. 4.2); a stage therefore has
 *     C(k,g) (p-1)^(g-1) combinations;
 *   - information sets: Gamma_j is the reduced row echelon form of G with the
 *     columns not used by Gamma_1..Gamma_{j-1} placed first (ascending) and the
 *     used ones after them (ascending); k_j is the number of its pivots among
 *     the unused columns.  Matrices with k_j = k are kept; the first one with
 *     0 < k_j < k is kept as the last matrix; none is kept once k_j = 0 or no
 *     column is left (Algorithm 6 assumes only Gamma_m may be partial);
 *   - early termination (Sec. 4.4) is tested after every stage (g, j) with
 *     L_{g,j} = sum_{i<=j} c_i(g) + sum_{i>j} c_i(g-1), c_i(g) = max(0, g+1-(k-k_i)),
 *     which equals the bound of Algorithm 6 at j = m; BZREF_CHECK_ROUND tests
 *     only at j = m, as the listing does.
 */
#include "bzref.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* F_p helpers: plain integers                                              */

static int mod_inverse(int a, int p) {
    /* Fermat: a^(p-2) mod p, p prime, a != 0 */
    int r = 1, b = a % p, e = p - 2;
    while (e > 0) {
        if (e & 1) r = (r * b) % p;
        b = (b * b) % p;
        e >>= 1;
    }
    return r;
}

static int args_ok(int p, int n, int k, const void *G) {
    if (p != 3 && p != 7) return 0;
    if (n < 1 || n > BZREF_MAX_N || k < 1 || k > BZREF_MAX_K || k > n) return 0;
    if (!G) return 0;
    return 1;
}

static int values_ok(int p, int n, int k, const uint8_t *G) {
    for (int i = 0; i < n * k; i++)
        if (G[i] >= p) return 0;
    return 1;
}

/* Gauss-Jordan elimination of the k x n matrix A (row-major) over F_p, in
 * place.  Columns are taken left to right; each pivot is scaled to 1 and
 * cleared from every other row.  pivcol[t] receives the column of the pivot of
 * row t.  Returns the rank. */
static int rref(int p, int k, int n, uint8_t *A, int *pivcol) {
    int rank = 0;
    for (int c = 0; c < n && rank < k; c++) {
        int r = -1;
        for (int i = rank; i < k; i++)
            if (A[i * n + c] != 0) { r = i; break; }
        if (r < 0) continue;
        if (r != rank)
            for (int t = 0; t < n; t++) {
                uint8_t x = A[r * n + t];
                A[r * n + t] = A[rank * n + t];
                A[rank * n + t] = x;
            }
        int inv = mod_inverse(A[rank * n + c], p);
        for (int t = 0; t < n; t++) A[rank * n + t] = (uint8_t)((A[rank * n + t] * inv) % p);
        for (int i = 0; i < k; i++) {
            if (i == rank) continue;
            int f = A[i * n + c];
            if (f == 0) continue;
            for (int t = 0; t < n; t++)
                A[i * n + t] = (uint8_t)((A[i * n + t] + (p - f) * A[rank * n + t]) % p);
        }
        pivcol[rank] = c;
        rank++;
    }
    return rank;
}

int bzref_rank(int p, int n, int k, const uint8_t *G) {
    if (!args_ok(p, n, k, G)) return BZREF_ERR_ARG;
    if (!values_ok(p, n, k, G)) return BZREF_ERR_VALUE;
    uint8_t *A = malloc((size_t)k * n);
    int piv[BZREF_MAX_K];
    memcpy(A, G, (size_t)k * n);
    int r = rref(p, k, n, A, piv);
    free(A);
    return r;
}

int bzref_decompose(int p, int n, int k, const uint8_t *G, uint8_t *gammas,
                    int32_t *ranks, int32_t *pivots) {
    if (!args_ok(p, n, k, G) || !gammas || !ranks) return BZREF_ERR_ARG;
    if (!values_ok(p, n, k, G)) return BZREF_ERR_VALUE;
    int used[BZREF_MAX_N] = {0};
    int order[BZREF_MAX_N], piv[BZREF_MAX_K];
    uint8_t *A = malloc((size_t)k * n);
    int m = 0;
    for (;;) {
        int nu = 0;
        for (int c = 0; c < n; c++)
            if (!used[c]) order[nu++] = c;
        if (nu == 0) break;
        int t = nu;
        for (int c = 0; c < n; c++)
            if (used[c]) order[t++] = c;
        /* A = G with its columns permuted into the order above */
        for (int i = 0; i < k; i++)
            for (int s = 0; s < n; s++) A[i * n + s] = G[i * n + order[s]];
        int rank = rref(p, k, n, A, piv);
        if (rank < k) { free(A); return BZREF_ERR_RANK; }
        int kj = 0;
        for (int i = 0; i < k; i++)
            if (piv[i] < nu) kj++;
        if (kj == 0) break;
        /* store Gamma_j back in the original column order */
        uint8_t *Gj = gammas + (size_t)m * k * n;
        for (int i = 0; i < k; i++)
            for (int s = 0; s < n; s++) Gj[i * n + order[s]] = A[i * n + s];
        if (pivots)
            for (int i = 0; i < k; i++) pivots[m * k + i] = order[piv[i]];
        ranks[m] = kj;
        m++;
        for (int i = 0; i < k; i++)
            if (piv[i] < nu) used[order[piv[i]]] = 1;
        if (kj < k || m == BZREF_MAX_M) break;
    }
    free(A);
    return m;
}

/* ------------------------------------------------------------------------ */
/* One stage: every combination sum_t a_t row_{i_t}, i_1 < ... < i_g,       */
/* a_1 = 1, a_t in {1..p-1}; weight = number of nonzero coordinates.        */

typedef struct {
    int p, n, k, g;
    const uint8_t *gam;
    /* work items: (i1, i2) pairs, or single rows when g == 1 */
    int n_tasks;
    int *task_i1, *task_i2;
    int next_task;
    int first_row_lo, first_row_hi;
    pthread_mutex_t lock;
    /* merged tallies */
    uint64_t count;
    int minw;
    uint64_t *hist; /* n+1, may be NULL */
} stage_ctx;

typedef struct {
    stage_ctx *ctx;
    uint64_t count;
    int minw;
    uint64_t *hist; /* n+1 local counters */
    uint8_t *partial; /* (g+1) x n partial sums, one vector per depth */
} stage_worker;

static void record(stage_worker *w, const uint8_t *c) {
    int n = w->ctx->n, wt = 0;
    for (int t = 0; t < n; t++) wt += (c[t] != 0);
    w->count++;
    if (wt < w->minw) w->minw = wt;
    w->hist[wt]++;
}

/* partial sum of depth rows is in partial[depth*n ..]; extend with rows > last */
static void extend(stage_worker *w, int depth, int last) {
    stage_ctx *x = w->ctx;
    int n = x->n, p = x->p;
    const uint8_t *base = w->partial + (size_t)depth * n;
    uint8_t *next = w->partial + (size_t)(depth + 1) * n;
    for (int i = last + 1; i < x->k; i++) {
        const uint8_t *row = x->gam + (size_t)i * n;
        for (int a = 1; a < p; a++) {
            for (int t = 0; t < n; t++) next[t] = (uint8_t)((base[t] + a * row[t]) % p);
            if (depth + 1 == x->g) record(w, next);
            else extend(w, depth + 1, i);
        }
    }
}

static void run_task(stage_worker *w, int i1, int i2) {
    stage_ctx *x = w->ctx;
    int n = x->n, p = x->p;
    const uint8_t *r1 = x->gam + (size_t)i1 * n;
    /* depth 1: the lowest row with coefficient 1 */
    memcpy(w->partial + n, r1, (size_t)n);
    if (x->g == 1) { record(w, w->partial + n); return; }
    const uint8_t *r2 = x->gam + (size_t)i2 * n;
    for (int a = 1; a < p; a++) {
        uint8_t *two = w->partial + 2 * (size_t)n;
        for (int t = 0; t < n; t++) two[t] = (uint8_t)((r1[t] + a * r2[t]) % p);
        if (x->g == 2) record(w, two);
        else extend(w, 2, i2);
    }
}

static void *stage_thread(void *arg) {
    stage_worker *w = (stage_worker *)arg;
    stage_ctx *x = w->ctx;
    for (;;) {
        pthread_mutex_lock(&x->lock);
        int t = x->next_task++;
        pthread_mutex_unlock(&x->lock);
        if (t >= x->n_tasks) break;
        run_task(w, x->task_i1[t], x->task_i2[t]);
    }
    pthread_mutex_lock(&x->lock);
    x->count += w->count;
    if (w->minw < x->minw) x->minw = w->minw;
    if (x->hist)
        for (int t = 0; t <= x->n; t++) x->hist[t] += w->hist[t];
    pthread_mutex_unlock(&x->lock);
    return NULL;
}

int bzref_threads(int nthreads) {
    if (nthreads > 0) return nthreads;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

int bzref_stage_enum(int p, int n, int k, const uint8_t *gam, int g, int nthreads,
                     int first_row_lo, int first_row_hi, uint64_t *count, uint64_t *hist) {
    if (!args_ok(p, n, k, gam) || g < 1 || g > k) return BZREF_ERR_ARG;
    stage_ctx x;
    memset(&x, 0, sizeof x);
    x.p = p; x.n = n; x.k = k; x.g = g; x.gam = gam;
    x.first_row_lo = first_row_lo; x.first_row_hi = first_row_hi;
    x.minw = n + 1;
    x.hist = hist;
    pthread_mutex_init(&x.lock, NULL);
    x.task_i1 = malloc(sizeof(int) * k * k);
    x.task_i2 = malloc(sizeof(int) * k * k);
    int lo = 0, hi = k;
    if (first_row_hi > first_row_lo) { lo = first_row_lo; hi = first_row_hi < k ? first_row_hi : k; }
    for (int i1 = lo; i1 < hi; i1++) {
        if (g == 1) {
            x.task_i1[x.n_tasks] = i1; x.task_i2[x.n_tasks] = -1; x.n_tasks++;
        } else {
            for (int i2 = i1 + 1; i2 < k; i2++) {
                x.task_i1[x.n_tasks] = i1; x.task_i2[x.n_tasks] = i2; x.n_tasks++;
            }
        }
    }
    int T = bzref_threads(nthreads);
    if (T > x.n_tasks) T = x.n_tasks > 0 ? x.n_tasks : 1;
    stage_worker *ws = calloc((size_t)T, sizeof(stage_worker));
    pthread_t *th = calloc((size_t)T, sizeof(pthread_t));
    for (int t = 0; t < T; t++) {
        ws[t].ctx = &x;
        ws[t].minw = n + 1;
        ws[t].hist = calloc((size_t)n + 1, sizeof(uint64_t));
        ws[t].partial = calloc((size_t)(g + 2) * n, 1);
    }
    for (int t = 1; t < T; t++) pthread_create(&th[t], NULL, stage_thread, &ws[t]);
    stage_thread(&ws[0]);
    for (int t = 1; t < T; t++) pthread_join(th[t], NULL);
    for (int t = 0; t < T; t++) { free(ws[t].hist); free(ws[t].partial); }
    free(ws); free(th);
    free(x.task_i1); free(x.task_i2);
    pthread_mutex_destroy(&x.lock);
    if (count) *count += x.count;
    return x.minw;
}

/* ------------------------------------------------------------------------ */
/* Brouwer-Zimmermann driver                                                 */

static uint64_t sat_mul(uint64_t a, uint64_t b) {
    if (a == 0 || b == 0) return 0;
    if (a > UINT64_MAX / b) return UINT64_MAX;
    return a * b;
}

static uint64_t sat_add(uint64_t a, uint64_t b) { return a > UINT64_MAX - b ? UINT64_MAX : a + b; }

static uint64_t binom_sat(int n, int r) {
    if (r < 0 || r > n) return 0;
    uint64_t v = 1;
    for (int i = 1; i <= r; i++) {
        /* v = v * (n - r + i) / i, exact at every step; saturate on overflow */
        uint64_t num = (uint64_t)(n - r + i);
        if (v > UINT64_MAX / num) return UINT64_MAX;
        v = v * num / (uint64_t)i;
    }
    return v;
}

static int bound_c(int g, int k, int kj) {
    int v = g + 1 - (k - kj);
    return v > 0 ? v : 0;
}

int bzref_min_distance(int p, int n, int k, const uint8_t *G, int flags, int nthreads,
                       uint64_t max_codewords, uint64_t *hist, bzref_result *out) {
    if (!out || !args_ok(p, n, k, G)) return BZREF_ERR_ARG;
    memset(out, 0, sizeof *out);
    if (!values_ok(p, n, k, G)) return BZREF_ERR_VALUE;
    uint8_t *gammas = malloc((size_t)BZREF_MAX_M * k * n);
    int m = bzref_decompose(p, n, k, G, gammas, out->ranks, NULL);
    if (m < 0) { free(gammas); return m; }
    out->m = m;
    int U = n - k + 1, L = 1;
    int status = BZREF_OK;
    out->terminated_by = 2;
    int round_mode = (flags & BZREF_CHECK_ROUND) != 0;
    int no_term = (flags & BZREF_NO_TERMINATION) != 0;
    for (int g = 1; g <= k && (no_term || L < U); g++) {
        int done = 0;
        out->terminated_by = 1;
        for (int j = 1; j <= m; j++) {
            uint64_t expect = sat_mul(binom_sat(k, g), (uint64_t)1);
            for (int t = 1; t < g; t++) expect = sat_mul(expect, (uint64_t)(p - 1));
            if (max_codewords && sat_add(out->codewords_total, expect) > max_codewords) {
                status = BZREF_ERR_LIMIT;
                done = 1;
                break;
            }
            if (out->n_stages >= BZREF_MAX_STAGES) { status = BZREF_ERR_LIMIT; done = 1; break; }
            int s = out->n_stages;
            uint64_t cnt = 0;
            uint64_t *h = hist ? hist + (size_t)s * (n + 1) : NULL;
            int smin = bzref_stage_enum(p, n, k, gammas + (size_t)(j - 1) * k * n, g, nthreads,
                                        0, 0, &cnt, h);
            if (smin < U) U = smin;
            int Lgj = 0;
            for (int i = 1; i <= m; i++) Lgj += bound_c(i <= j ? g : g - 1, k, out->ranks[i - 1]);
            bzref_stage *st = &out->stages[s];
            st->g = g; st->j = j; st->codewords = cnt; st->stage_min = smin;
            st->upper_after = U; st->lower_after = Lgj;
            out->n_stages++;
            out->codewords_total += cnt;
            if (!no_term && (!round_mode || j == m) && Lgj >= U) {
                out->terminated_by = 0;
                done = 1;
                break;
            }
        }
        if (done) break;
        /* Algorithm 6: L := (m-1)(g+1) + max{0, g+1-k+k_m}, i.e. L_{g,m} */
        L = 0;
        for (int i = 1; i <= m; i++) L += bound_c(g, k, out->ranks[i - 1]);
    }
    out->d = U;
    free(gammas);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Brute force over every message                                            */

int bzref_brute_force(int p, int n, int k, const uint8_t *G, uint64_t *hist) {
    if (!args_ok(p, n, k, G) || !hist) return BZREF_ERR_ARG;
    if (!values_ok(p, n, k, G)) return BZREF_ERR_VALUE;
    for (int w = 0; w <= n; w++) hist[w] = 0;
    int msg[BZREF_MAX_K] = {0};
    int d = n + 1;
    for (;;) {
        int wt = 0, any = 0;
        for (int t = 0; t < n; t++) {
            int s = 0;
            for (int i = 0; i < k; i++) s += msg[i] * G[i * n + t];
            wt += (s % p) != 0;
        }
        for (int i = 0; i < k; i++) any |= msg[i];
        hist[wt]++;
        if (any && wt < d) d = wt;
        /* next message in mixed radix p */
        int i = 0;
        while (i < k && msg[i] == p - 1) msg[i++] = 0;
        if (i == k) break;
        msg[i]++;
    }
    return d;
}
