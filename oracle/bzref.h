/*
 * bzref.h -- reference (oracle) minimum-distance computation over F_3 and F_7.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU library
 * against a plain, slow, obviously correct implementation.  It shares no code,
 * header, table or constant with the GPU library, and the GPU library must
 * never call it.
 *
 * Everything here is ordinary mod-p integer arithmetic, one byte per symbol:
 * no bit slicing, no isometric additions, no identity-column shortcuts.
 *
 * Paper: Hernando & Quintana-Orti, "Implementing Basic Arithmetic in F_p via
 * F_2, and Its Application for Computing the Hamming Distance of Linear Codes"
 * (arXiv 2603.29942).
 *   - problem statement, d = min{wt(c) : c in C \ {0}}: Sec. 3;
 *   - Brouwer-Zimmermann bounds and rounds: Sec. 3.1, Algorithm 6;
 *   - one coefficient fixed to 1 per combination (scalar multiples are
 *     isometric): Sec. 4.2;
 *   - early termination between generator matrices: Sec. 4.4.
 */
#ifndef BZREF_H
#define BZREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BZREF_MAX_N 128
#define BZREF_MAX_K 64
#define BZREF_MAX_M 128
#define BZREF_MAX_STAGES 256

/* status codes (the same numeric values as the GPU library documents) */
#define BZREF_OK 0
#define BZREF_ERR_ARG (-1)   /* p not in {3,7}, n/k out of range, NULL pointer */
#define BZREF_ERR_VALUE (-2) /* a generator entry >= p */
#define BZREF_ERR_RANK (-3)  /* rank(G) < k */
#define BZREF_ERR_LIMIT (-6) /* the next required stage would exceed max_codewords */

/* flags for bzref_min_distance */
#define BZREF_CHECK_ROUND 1 /* test L >= U only after the last matrix of a round */
#define BZREF_NO_TERMINATION 2 /* run every stage g = 1..k, j = 1..m (for the histogram identity) */

typedef struct {
    int32_t g, j;           /* round (number of rows combined) and matrix index, 1-based */
    uint64_t codewords;     /* combinations enumerated in this stage */
    int32_t stage_min;      /* minimum weight seen in this stage */
    int32_t upper_after;    /* U after the stage */
    int32_t lower_after;    /* L_{g,j} after the stage */
} bzref_stage;

typedef struct {
    int32_t d;              /* minimum distance (valid when status == BZREF_OK) */
    int32_t m;              /* number of generator matrices Gamma_j kept */
    int32_t ranks[BZREF_MAX_M]; /* k_j: pivots of Gamma_j inside the columns not used before */
    int32_t n_stages;
    int32_t terminated_by;  /* 0: L >= U after a stage; 1: every round done; 2: no stage needed */
    uint64_t codewords_total;
    bzref_stage stages[BZREF_MAX_STAGES];
} bzref_result;

/* rank of the k x n row-major matrix G over F_p (p prime, entries < p) */
int bzref_rank(int p, int n, int k, const uint8_t *G);

/* Information-set decomposition: gammas[j][k][n] (row-major, original column
 * order), ranks[j], pivots[j][k] (original column index of the pivot of each
 * row).  Returns m >= 1, or a negative status. */
int bzref_decompose(int p, int n, int k, const uint8_t *G, uint8_t *gammas,
                    int32_t *ranks, int32_t *pivots);

/* Brouwer-Zimmermann with the reading of Algorithm 6 documented in the .c file.
 * hist: NULL, or BZREF_MAX_STAGES x (n+1) uint64 counters (stage-major), zeroed
 * by the caller; hist[s*(n+1)+w] counts the weight-w combinations of stage s.
 * max_codewords: 0 for no limit.  nthreads <= 0: one per online CPU. */
int bzref_min_distance(int p, int n, int k, const uint8_t *G, int flags, int nthreads,
                       uint64_t max_codewords, uint64_t *hist, bzref_result *out);

/* One stage alone: all g-row combinations of the k x n matrix gam with the
 * lowest-indexed coefficient 1.  Returns the minimum weight; count and hist
 * (n+1 entries, may be NULL, accumulated into) receive the tallies.  When
 * first_row_hi > first_row_lo, only combinations whose lowest row lies in
 * [first_row_lo, first_row_hi) are enumerated (bounded samples). */
int bzref_stage_enum(int p, int n, int k, const uint8_t *gam, int g, int nthreads,
                     int first_row_lo, int first_row_hi, uint64_t *count, uint64_t *hist);

/* Brute force over all p^k messages: hist[w] = A_w (n+1 entries).  Returns d. */
int bzref_brute_force(int p, int n, int k, const uint8_t *G, uint64_t *hist);

/* number of threads bzref_min_distance uses for a given request */
int bzref_threads(int nthreads);

#ifdef __cplusplus
}
#endif

#endif
