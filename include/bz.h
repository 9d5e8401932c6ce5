/*
 * bz.h -- C ABI of the MI355X (gfx950) Brouwer-Zimmermann minimum-distance library.
 *
 * Computes the minimum Hamming distance d = min{wt(c) : c in C \ {0}} of a
 * linear code over F_3 or F_7 given by a k x n generator matrix (problem
 * statement: Hernando & Quintana-Orti, arXiv 2603.29942, Sec. 3), with the
 * Brouwer-Zimmermann rounds of Algorithm 6 (Sec. 3.1).  Every step of the
 * path runs on the GPU: the information-set decomposition into systematic
 * matrices Gamma_j, the bit-sliced packing in the natural encoding (Sec. 2 and
 * 4.1), the enumeration of all g-row combinations with the lowest coefficient
 * fixed to 1 (Sec. 4.2), exact prefix sums with the F_3 / F_7 additions of
 * Algorithms 3 and 4 (for the rounds g >= 4 of the batched and served calls
 * and of F_7 plain calls, the sums of the two highest rows of a combination
 * come from a per-set table of all row pairs that the decomposition builds), the
 * isometric last addition (Sec. 4.3), the popcount
 * weight, the min-reduce against the upper bound U, and the stage-by-stage
 * lower-bound test with early termination (Sec. 4.4).
 *
 * Conventions
 *   - Every function returns BZ_OK (0) or a negative bz_status; nothing throws
 *     or aborts across the ABI.
 *   - G is k x n, row-major, one uint8 per symbol, entries in [0, p).
 *   - Limits: p in {3, 7}; 1 <= k <= n; n <= BZ_MAX_N; k <= BZ_MAX_K.
 *   - The caller owns every buffer it passes in; the library copies or reads
 *     them during the call and keeps no pointer to them afterwards.  Device
 *     memory for intermediate state is allocated once per device by the library
 *     and reused by later calls.
 *   - Calls on one device are serialised by a per-device lock.
 *
 * Readings of points the paper leaves open (all shared with the oracle):
 *   - combinations range over F_p with the coefficient of the lowest-indexed
 *     row fixed to 1; a round-g stage has C(k,g) (p-1)^(g-1) combinations;
 *   - Gamma_j is the reduced row echelon form of G with the columns unused by
 *     Gamma_1..Gamma_{j-1} first (ascending) and the used ones after
 *     (ascending); k_j counts its pivots among the unused columns; matrices
 *     with k_j = k are kept, the first partial one (0 < k_j < k) is kept as the
 *     last, and none once k_j = 0 or no column is left;
 *   - the early-termination test L_{g,j} >= U runs after every stage (g, j)
 *     with L_{g,j} = sum_{i<=j} c_i(g) + sum_{i>j} c_i(g-1),
 *     c_i(g) = max(0, g+1-(k-k_i)); BZ_CHECK_ROUND tests only at j = m.
 */
#ifndef BZ_H
#define BZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BZ_MAX_N 128
#define BZ_MAX_K 64
#define BZ_MAX_M 128
#define BZ_MAX_STAGES 256

typedef enum {
    BZ_OK = 0,
    BZ_ERR_ARG = -1,    /* p not in {3,7}, n or k out of range, NULL pointer, bad option */
    BZ_ERR_VALUE = -2,  /* a generator entry >= p */
    BZ_ERR_RANK = -3,   /* rank(G) < k */
    BZ_ERR_DEVICE = -4, /* a HIP runtime error, or no gfx950 device */
    BZ_ERR_NOMEM = -5,  /* a device or pinned-host allocation failed */
    BZ_ERR_LIMIT = -6   /* the next required stage would exceed max_codewords, or a
                           stage lies outside the kernel's index ranges */
} bz_status;

enum { BZ_CHECK_STAGE = 0, BZ_CHECK_ROUND = 1 };

/* One stage: all combinations of g rows of Gamma_j. */
typedef struct {
    int32_t g, j;         /* round and matrix index, both 1-based */
    uint64_t codewords;   /* combinations the kernel evaluated in this stage */
    int32_t stage_min;    /* minimum weight seen in this stage */
    int32_t upper_after;  /* U after the stage */
    int32_t lower_after;  /* L_{g,j} */
} bz_stage;

typedef struct {
    int32_t d;                    /* minimum distance (valid when the call returns BZ_OK) */
    int32_t m;                    /* number of matrices Gamma_j */
    int32_t ranks[BZ_MAX_M];      /* k_j */
    int32_t n_stages;             /* stages run (and reported) */
    int32_t terminated_by;        /* 0: L >= U after a stage; 1: every round done; 2: no stage needed (k = n) */
    uint64_t codewords_total;
    bz_stage stages[BZ_MAX_STAGES];
    /* with options.timing: device time of the two kernels of the call, measured
       with HIP events on the call's stream (milliseconds); else 0 */
    float decompose_ms;
    float enum_ms;
    int32_t info;                 /* BZ_INFO_* bits: how the run was carried out (never its result) */
} bz_result;

/* bz_result.info: the second information set was computed ahead by a second
 * workgroup of the decomposition launch and handed over (see bz_options.no_ahead) */
#define BZ_INFO_AHEAD 1
/* bz_result.info: the rounds g >= 4 took the sums of their two highest rows
 * from the information sets' pair tables (see bz_options.pair_tables) */
#define BZ_INFO_PAIRS 2

typedef struct {
    int32_t check;            /* BZ_CHECK_STAGE (default) or BZ_CHECK_ROUND */
    int32_t no_termination;   /* 1: run every stage g = 1..k, j = 1..m (weight spectra) */
    int32_t identity_skip;    /* 1 (default): weight = g + popcount over the n-k non-pivot
                                 columns (Gamma_j is the identity on its k pivot columns);
                                 0: popcount over all n columns */
    int32_t histograms;       /* 1: fill hist_out */
    uint64_t *hist_out;       /* host buffer, BZ_MAX_STAGES x (n+1) uint64, row s = stage s:
                                 number of combinations of weight w; written when histograms */
    uint64_t max_codewords;   /* work limit; 0 = default (2^44) */
    void *hip_stream;         /* hipStream_t to run on; NULL = the library's stream */
    int32_t device;           /* HIP device ordinal */
    int32_t blocks_per_cu;    /* enumeration grid: workgroups per compute unit; 0 = as many
                                 as the kernel's registers and LDS allow */
    int32_t timing;           /* 1: fill bz_result.decompose_ms / enum_ms */
    int32_t wait_timeout_s;   /* workgroups that wait for earlier stages give up (BZ_ERR_DEVICE)
                                 after this many seconds; 0 = default (120) */
    uint64_t *trace_out;      /* NULL, or a host buffer of (BZ_MAX_STAGES + 2) x 4 uint64 that
                                 receives a device wall-clock timeline in nanoseconds from the
                                 start of the decomposition kernel: row 0 = decomposition
                                 {start, rows loaded, matrices reduced, end}; row 1 =
                                 enumeration kernel {first workgroup start, last workgroup end};
                                 row 2+s = stage s {first workgroup start, last workgroup
                                 end, checked, last workgroup start}.  Workgroup times
                                 are those of every seventh workgroup (the device's one
                                 real-time counter slows down when a thousand workgroups
                                 read it at once); "checked" is exact */
    int32_t cooperative;      /* reserved, must be 0 (BZ_ERR_ARG otherwise).  The persistent
                                 launch is an ordinary one, sized to the device's occupancy;
                                 a cooperative launch (co-residency guaranteed by the runtime)
                                 is not offered: it started the kernel about 11 us later and
                                 processes that made one ended in a crash inside the profiler's
                                 shutdown when run under rocprofv3.  The plain path deals its
                                 tiles to fixed workgroups; a workgroup kept off the device by
                                 other processes' kernels delays the run until it starts (or
                                 until wait_timeout_s: BZ_ERR_DEVICE) */
    int32_t no_ahead;         /* 1: the decomposition computes every information set itself;
                                 0 (default): when the first set's pivots are the columns
                                 0 .. k-1, the second set (columns k .. n-1 first) is taken
                                 from a second workgroup that computed it in parallel, if it
                                 has finished (BZ_INFO_AHEAD).  Results never depend on it */
    int32_t pair_tables;      /* 0 (default): the decomposition builds each information set's
                                 table of row-pair sums for F_7 codes, not for F_3 ones (the
                                 plain F_3 runs measured no faster with it); 1: always; -1:
                                 never (BZ_INFO_PAIRS tells which ran).  Results never depend
                                 on it; bz_min_distance_noalloc never builds tables */
} bz_options;

/* Fill *o with the defaults above. */
void bz_default_options(bz_options *o);

/* Minimum distance d = min{wt(c) : c in C \ {0}} of the code generated by the
 * host matrix G (k x n), default options: the problem statement of Sec. 3,
 * computed with the rounds of Algorithm 6 (Sec. 3.1) over the information sets
 * Gamma_j, the arithmetic of Sec. 2 (Algorithms 3, 4), the isometric last
 * addition (Sec. 4.3) and the stage-by-stage termination test of Sec. 4.4.
 * Returns BZ_OK and fills *out (d, m, the ranks k_j and the stage trace), or
 * BZ_ERR_ARG / VALUE / RANK / LIMIT / DEVICE / NOMEM. */
int bz_min_distance(int p, int n, int k, const uint8_t *G, bz_result *out);

/* As bz_min_distance (Sec. 3; Algorithm 6 of Sec. 3.1), with options.
 * G_is_device = 1: G is a device pointer (already resident in GPU memory on
 * options->device, readable from the stream); 0: a host pointer, copied to
 * the device inside the call.  On return *out is complete and G is no longer
 * read.  Without histograms or a trace, the check that ends the run writes the
 * result block to host memory and the call returns as soon as it has, while
 * workgroups of the launch may still be retiring; the next call on this
 * device waits for them (on the same stream by stream order, on another
 * stream through an event).  With histograms or a trace the stream has been
 * synchronised.  A call waits for the round in flight of every server on its
 * device to yield (see bz_server_*) and keeps them from starting another
 * until it returns: its persistent launch needs the whole device. */
int bz_min_distance_ex(int p, int n, int k, const uint8_t *G, int G_is_device,
                       const bz_options *o, bz_result *out);

/* For callers that cannot allocate (code that runs under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): bz_min_distance_ex on a
 * device generator G (G_is_device = 1) whose device state lives in one fixed
 * array of the library (BZ_NOALLOC_SCRATCH_BYTES per device, held until the
 * process ends; sized for the largest problem the library accepts: n <= BZ_MAX_N,
 * k <= BZ_MAX_K, m <= BZ_MAX_M).  The call allocates nothing: no device, pinned
 * or mapped memory, no stream, no event (the first call on a device looks up the
 * array's address and fills its binomial table).  It runs on options->hip_stream
 * (NULL: the null stream) and synchronises it before returning.  Supported
 * options: check, no_termination, identity_skip, max_codewords, hip_stream,
 * device, blocks_per_cu, wait_timeout_s, no_ahead; histograms, trace_out, timing
 * or cooperative set, n > BZ_MAX_N, k > BZ_MAX_K or a NULL pointer give
 * BZ_ERR_ARG.  Every such call on one device shares the one array: calls are
 * serialised by the device's lock within a process, and calls that overlap on
 * one device from several processes race.  Results equal bz_min_distance_ex's. */
#define BZ_NOALLOC_SCRATCH_BYTES (640u * 1024u)
int bz_min_distance_noalloc(int p, int n, int k, const uint8_t *G_dev, const bz_options *o, bz_result *out);

/* Releases what the library holds for a device (the library stream and
 * events, the device workspace, pinned and mapped host buffers, the per-shape
 * tables, the batch workspace) after waiting for its work; the next call on the
 * device sets it up again.  BZ_ERR_ARG while a server runs on the device (stop
 * it first).  Call it before the HIP runtime shuts down, e.g. at process exit. */
int bz_release(int device);

/* Human-readable name of a status code. */
const char *bz_status_str(int status);

/* ---------------------------------------------------------------------- */
/* Batches: many codes of different p, n and k in one call (one decomposition
 * launch and one persistent enumeration launch for the whole batch).  Each
 * code's d and stage trace are those of bz_min_distance_ex on that code with
 * the same options (Algorithm 6 per code; the codes only share the GPU). */

#define BZ_MAX_BATCH 65536

typedef struct {
    int32_t p, n, k;      /* as for bz_min_distance */
    int32_t sweep_ops;    /* VALU operations per lane and task (the size of a unit of
                             work), 0 = default 4500; chosen per (p, words) by the
                             autotuner; results do not depend on it */
    uint64_t g_offset;    /* byte offset of this code's k x n row-major generator in G */
} bz_code;

typedef struct {
    int32_t check;           /* BZ_CHECK_STAGE (default) or BZ_CHECK_ROUND */
    int32_t no_termination;  /* 1: every stage of every code (no L >= U exit) */
    int32_t identity_skip;   /* 1 (default) */
    int32_t blocks_per_cu;   /* enumeration grid: workgroups per compute unit; 0 = as many
                                as the kernel's registers and LDS allow */
    uint64_t max_codewords;  /* per-code work limit; 0 = default (2^44) */
    void *hip_stream;        /* NULL = library stream */
    int32_t device;
    int32_t wait_timeout_s;  /* the launch gives up (BZ_ERR_DEVICE) if no work appears for this
                                long while codes remain; 0 = default (120) */
    int32_t timing;          /* 1: fill the two fields below (HIP events on the stream) */
    float decompose_ms;      /* out: decomposition launch */
    float enum_ms;           /* out: enumeration launch */
    int32_t cooperative;     /* reserved, must be 0 (BZ_ERR_ARG otherwise); the persistent
                                launch is an ordinary one (the batched kernel hands out work
                                dynamically, so it never waits for a workgroup that has not
                                started) */
    float *code_ms_out;      /* NULL, or a host array of ncodes floats: per code, the device
                                time in ms from the start of the decomposition launch to the
                                check that ended the code (its time to d within the batch) */
} bz_batch_options;

void bz_default_batch_options(bz_batch_options *o);

/* Minimum distance of ncodes codes.  G holds all generators (g_bytes bytes,
 * host memory, or device memory when G_is_device); code i reads its k x n
 * bytes at codes[i].g_offset.  out[i] and status_out[i] receive each code's
 * result and status (the values bz_min_distance_ex returns: BZ_OK, VALUE,
 * RANK, LIMIT).  Returns BZ_OK when the batch ran, BZ_ERR_ARG for an invalid
 * batch or code descriptor (nothing runs), BZ_ERR_NOMEM, or BZ_ERR_DEVICE.
 * The library keeps a batch workspace per device that grows to the largest
 * batch seen (about 28 KB per code plus the packed rows and the pair tables:
 * (n/k + 1) k(k-1)/2 W 16 bytes per code for F_3, six times that for F_7,
 * W = ceil((n-k)/32) with the identity skip, else ceil(n/32)). */
int bz_min_distance_batch(int ncodes, const bz_code *codes, const uint8_t *G, uint64_t g_bytes, int G_is_device,
                          bz_batch_options *o, bz_result *out, int32_t *status_out);

/* ---------------------------------------------------------------------- */
/* Serving with continuous batching.  Requests (one code each) are queued by
 * bz_server_submit and run by bz_server_poll, which the caller calls in its
 * loop: a round admits queued requests into free slots (the device memory of
 * one code each: admission by memory), decomposes them, orders all active
 * codes (arrival order, or shortest predicted work first with the predictor
 * network) and runs them together in one persistent launch.  With the
 * predicted policy, queued requests are admitted shortest predicted work first
 * (when they outnumber the free slots) and within a per-round budget of
 * predicted work (admit_budget) when one is set.  Requests that
 * arrive while a round runs make it yield at the next part boundary and join
 * the next round with the unfinished codes, which keep their progress.  Codes
 * that end are returned by the next poll, also while their round runs.  Each
 * result equals bz_min_distance_ex's on that code with the same options
 * (Algorithm 6 per code; the ordering only changes when it ends).  One server
 * per thread of control: calls on one server must not overlap. */

typedef struct bz_server bz_server;
enum { BZ_SERVE_FIFO = 0, BZ_SERVE_PREDICTED = 1 };

typedef struct {
    int32_t slots;            /* codes resident on the device at once, 0 -> 1024 */
    int32_t policy;           /* BZ_SERVE_FIFO or BZ_SERVE_PREDICTED */
    const float *mlp_params;  /* host, BZ_MLP_PARAMS floats: the network for BZ_SERVE_PREDICTED */
    int32_t check;            /* BZ_CHECK_STAGE (default) or BZ_CHECK_ROUND */
    int32_t identity_skip;    /* 1 (default) */
    uint64_t max_codewords;   /* per-code work limit, 0 = default (2^44) */
    int32_t blocks_per_cu;    /* persistent launch: workgroups per compute unit, 0 = as many as fit */
    int32_t device;
    int32_t wait_timeout_s;   /* as in bz_batch_options */
    int32_t max_n;            /* largest n accepted, 0 = 128; sizes each slot */
    int32_t cooperative;      /* reserved, must be 0 (as in bz_batch_options) */
    double admit_budget;      /* BZ_SERVE_PREDICTED: predicted combinations admitted per round
                                 (at least one request per round); 0 = no budget (slots only).
                                 Queued requests are admitted shortest predicted work first;
                                 their estimate uses p, n, k (the rank deficit is not known
                                 before the decomposition and is taken as 0) */
} bz_server_options;

void bz_default_server_options(bz_server_options *o);
/* Allocates the slots (about 28 KB + 4 KB x min(128, max_n) + 64 max_n bytes
 * each, plus the pair tables of the largest code a slot may hold: 0.39 MB for
 * max_n = 64, 1.7 MB for max_n = 128 with the identity skip, 0.77 / 2.3 MB
 * without). */
int bz_server_start(const bz_server_options *o, bz_server **out);
/* Queues one code (G: host, k x n row-major, copied); tag is returned with its result.
 * BZ_ERR_ARG for an invalid shape or n > max_n; the code's own errors (VALUE,
 * RANK, LIMIT) come back as its status. */
int bz_server_submit(bz_server *s, int p, int n, int k, const uint8_t *G, uint64_t tag);
/* Progresses the server without blocking on running work; returns up to
 * max_out finished codes (tags, results, statuses, *n_out) and, in
 * *in_flight (may be NULL), the requests queued or running. */
int bz_server_poll(bz_server *s, int max_out, uint64_t *tags, bz_result *results, int32_t *statuses, int *n_out,
                   int *in_flight);
/* Rounds launched and rounds asked to yield so far. */
int bz_server_stats(bz_server *s, uint64_t *rounds, uint64_t *yields);
/* Ends the running round at its next part boundary, waits for it and frees everything. */
int bz_server_stop(bz_server *s);

/* ---------------------------------------------------------------------- */
/* Work predictor: a 4 -> 64 -> 64 -> 1 FP32 multilayer perceptron with ReLU
 * hidden layers that maps features of a code to log10 of the combinations the
 * method evaluates on it.  It is only used to order and admit work (the
 * stage-by-stage L >= U test still decides d).  Not from the paper.
 *
 * Parameters: BZ_MLP_PARAMS floats, W1[64][4], b1[64], W2[64][64], b2[64],
 * w3[64], b3 (row-major).  x: n x 4 features, row-major.  All pointers are
 * device pointers; calls are asynchronous on `stream`.  Sums run in a fixed
 * order, so results are reproducible bit for bit.  BZ_ERR_ARG for NULL or
 * negative sizes. */
#define BZ_MLP_PARAMS 4545

/* y[n] = network(x); cache (n x 128 floats, or NULL) receives the hidden
 * activations the backward pass needs. */
int bz_mlp_forward(const float *params, const float *x, int n, float *y, float *cache, void *stream);
/* Gradient of L = mean_i (y_i - target_i)^2 with respect to the parameters
 * (grad[BZ_MLP_PARAMS]), from y and cache of bz_mlp_forward; dz is scratch of
 * n x 129 floats; loss (1 float, or NULL) receives L. */
int bz_mlp_backward(const float *params, const float *x, const float *target, int n, const float *y,
                    const float *cache, float *dz, float *grad, float *loss, void *stream);
/* One Adam step (bias-corrected, step >= 1) on params with moment buffers m, v
 * (BZ_MLP_PARAMS floats each, zero before step 1). */
int bz_mlp_adam(float *params, const float *grad, float *m, float *v, int step, float lr, float beta1, float beta2,
                float eps, void *stream);

/* ---------------------------------------------------------------------- */
/* Bit-sliced F_p vector arithmetic on the device (Sec. 2; Tables 1-2 of the
 * paper time these additions).  Vectors of nsym symbols are stored sliced:
 * planes[v][b][w], b < r planes (r = 2 for F_3, 3 for F_7), w < ceil(nsym/32)
 * words; bit t of word w of plane b is bit b of symbol 32w+t; bits beyond
 * nsym are zero.  Natural encoding (value = sum_b bit_b 2^b) unless stated.
 * All pointers are device pointers; calls are asynchronous on `stream`
 * (NULL: the null stream). */

enum {
    BZ_OP_ADD = 0,     /* a + b, Algorithm 3 (F_3) / Algorithm 4 (F_7) */
    BZ_OP_SUB = 1,     /* a - b = a + (-b); -b is a plane swap (F_3) or masked complement (F_7) */
    BZ_OP_DOUBLE = 2,  /* 2a as a circular shift of the planes (Sec. 4.2); b unused */
    BZ_OP_ISO_ADD = 3, /* nonzero mask of a + b (isometric addition, Sec. 4.3) in plane 0, other planes 0 */
    BZ_OP_ISO_SUB = 4, /* nonzero mask of a - b (isometric subtraction, Sec. 4.3) */
    BZ_OP_KAT_ADD = 5  /* F_3 only: Algorithm 2 on planes in its encoding 0=(1,1), 1=(0,1), 2=(1,0) */
};

enum { BZ_ENC_NATURAL = 0, BZ_ENC_KAT = 1 };

/* symbols (nvec x nsym uint8, row-major) -> planes; encoding BZ_ENC_KAT is for F_3 only */
int bz_sliced_pack(int p, int encoding, int nvec, int nsym, const uint8_t *sym, uint32_t *planes,
                   void *stream);
/* planes -> symbols (inverse of bz_sliced_pack; a plane pattern outside the
 * encoding decodes to 255) */
int bz_sliced_unpack(int p, int encoding, int nvec, int nsym, const uint32_t *planes, uint8_t *sym,
                     void *stream);
/* out = op applied `reps` times to a with operand b, x <- op(x, b) starting
 * from x = a: a + reps*b (BZ_OP_ADD, BZ_OP_KAT_ADD), a - reps*b (BZ_OP_SUB),
 * 2^reps * a (BZ_OP_DOUBLE); the isometric masks need reps = 1.  The chain
 * runs in registers, so reps > 1 times the arithmetic of Tables 1-2 and
 * reps = 1 a single pass over memory.  out may alias a.  BZ_ERR_ARG for
 * p, op or sizes out of range. */
int bz_sliced_op(int p, int op, int nvec, int nsym, const uint32_t *a, const uint32_t *b,
                 uint32_t *out, int reps, void *stream);

/* ---------------------------------------------------------------------- */
/* VALU issue-rate probe (not from the paper; it measures the rates behind the
 * roofline): one launch of blocks_per_cu (1..8) workgroups of 256 threads per
 * compute unit, each thread running eight independent chains of one VALU
 * instruction `iters` times.  op: 0 v_xor_b32, 1 v_add_u32, 2 v_bitop3_b32,
 * 3 v_bcnt_u32_b32, 4 v_min_u32, 5 v_fma_f32.  out: device buffer of
 * blocks x 256 uint32 (one store per thread); *ms: the launch's time from HIP
 * events on `stream`; *lane_ops: lane-operations executed.  Synchronous. */
int bz_valu_rate(int op, int iters, int blocks_per_cu, uint32_t *out, float *ms, double *lane_ops, void *stream);

#ifdef __cplusplus
}
#endif

#endif
