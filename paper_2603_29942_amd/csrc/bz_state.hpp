// bz_state.hpp -- per-code state shared by the decomposition and enumeration
// kernels, and the stage schedule (built identically on the device and, for
// reading the results back, on the host).
#pragma once
#include <stdint.h>

#include "../../include/bz.h"

#ifndef BZ_HD
#define BZ_HD __host__ __device__ __forceinline__
#endif

namespace bz {

typedef uint64_t u64;

// Row storage: Gamma_j row i, word w, plane b at rows[(j*BZ_MAX_K + i)*ROW_WORDS + w*4 + b]
// for b < 3; slot b = 3 holds the OR of the planes (the row's nonzero mask).  The
// W words of a row are one contiguous, 16-byte aligned run that scalar loads
// fetch in one go.
constexpr int ROW_WORDS = 16;
constexpr uint64_t DEFAULT_LIMIT = 1ull << 44;

// Pair tables: for each information set, the exact sums of two of its rows,
// R_s + c R_L for s < L and every c in F_p^* up to the sign that the isometric
// subtraction supplies (Sec. 4.2-4.3): F_3 keeps R_s + R_L and R_s - R_L
// (planes 0 and 1 of each, one 16-byte unit per word), F_7 keeps c = 1..6 (six
// units per pair, each word planes 0..2 and their OR).  A combination
// base + h_s R_s + h_L R_L equals base + h_s T with T = R_s + (h_L / h_s) R_L,
// so a lane with an exact base finishes all (p-1)^2 multipliers of the pair
// from these units without an exact addition of its own.  Pairs are stored
// row-major in s (all L > s of row s, ascending), so the pairs of a run of
// rows s form one contiguous range.  Unit u of pair e, word w: at (e * units +
// u) * W + w, in units of 16 bytes.
BZ_HD int pair_units(int p) { return p == 3 ? 1 : p - 1; }
// pairs (s', L) with s' < s: those of rows 0 .. s-1
BZ_HD u64 pair_first(int s, int k) { return (u64)s * (u64)(k - 1) - (u64)s * (u64)(s - 1) / 2; }
BZ_HD u64 pair_table_units(int p, int k, int W) { return (u64)k * (u64)(k - 1) / 2 * (u64)pair_units(p) * (u64)W; }
// pair e = (s, s + 1 + rem) in that order: advance (s, rem) by d pairs
BZ_HD void pair_advance(int k, int &s, int &rem, int d) {
    rem += d;
    while (s < k - 1 && rem >= k - 1 - s) {
        rem -= k - 1 - s;
        s++;
    }
}
// units past the last table of a buffer that a sweep's group of loads may
// read (a group of UR units of W words, at most 8 of 16 bytes, is loaded whole)
constexpr int PAIR_PAD_UNITS = 16;
// information sets a decomposition can produce: every full-rank set takes k
// unused columns and the first deficient one ends it
BZ_HD int pair_sets(int n, int k) { return n / k + 1 < BZ_MAX_M ? n / k + 1 : BZ_MAX_M; }

// One stage (g, j) of Algorithm 6, and how its work is cut into wave tasks
// (64 lanes each):
//   g = 1: a task covers 64 rows i (one combination per lane).
//   g = 2: a task covers 64 pairs of rows s < L (colex rank L(L-1)/2 + s), one
//           pair per lane, with every nonzero multiplier of L.
//   g >= 3: a combination is  base + h_s R_s + h_L R_L  with a base of g-2 rows
//           whose top row is q (its lowest row has coefficient 1, the others any
//           of the (p-1)^(g-3) nonzero choices), then a row s > q with every
//           nonzero coefficient and a last row L > s with every nonzero
//           multiplier.  Bases are grouped by q.  A task is (q, a chunk of 64
//           bases, a block of consecutive rows s): each lane holds one base, and
//           all lanes share q and the rows s, so the sweeps over L are
//           wave-uniform.  Row s sweeps k-1-s last rows, so the rows of a
//           q-group weigh len, len-1, ..., 1 (len = k-2-q); the blocks split
//           that total into nearly equal parts of at most about `cap` (s, L)
//           steps, which keeps every task of a stage about equally long.
// Tasks are dealt four at a time (one per wavefront of a workgroup), round by
// round, to the workgroups of the grid.  The deal of stage s starts at
// workgroup off_s mod grid, off_s being the tiles of all stages before s, so
// that the stages whose deal starts within the first pass over the grid
// (off_s < grid) begin on workgroups of their own, at once and side by side,
// without waiting for the checks of earlier stages ("nowait"); every later
// stage waits (see LOOKAHEAD).
constexpr int WAVES_PER_GROUP = 4;

struct StageDesc {
    int32_t g, j;
    int32_t L;          // L_{g,j}
    int16_t check;      // 1: test L >= U after this stage
    int16_t nowait;     // 1: off_s < grid, starts without waiting for checks
    u64 tasks;          // wave tasks in the stage
    u64 tiles;          // ceil(tasks / WAVES_PER_GROUP)
    u64 codewords;      // C(k,g) (p-1)^(g-1)
    uint32_t coef_combos;  // (p-1)^(g-3) for g >= 3, else 1
    uint32_t parts;        // workgroups that own at least one tile: min(grid, tiles)
    uint32_t sweep_cap;    // g >= 3: target (s, L) steps per lane and task
    uint32_t rot;          // (grid - off_s mod grid) mod grid, see tile_of
    uint32_t vcap;         // step budget of a lane's run of bases (qgroup_digits);
                           // 0: one base per lane
    uint32_t pad;
};


// Bases with top row q (g >= 3): how many, and how their rows s are blocked.
struct QEntry {
    u64 first;     // first task of the group
    u64 bases;     // C(q, g-3) (p-1)^(g-3)
    uint32_t nb;   // blocks of rows s, see qgroup_blocks
    uint32_t vd;   // a lane takes (p-1)^vd consecutive bases, see qgroup_digits
};

// The plain enumeration kernel hands out the stages that start at once as
// one pool of tiles, claimed by POOL_SLICES counters (see pool_stages).
constexpr uint32_t POOL_SLICES = 32;

// Results the host reads back (kept contiguous and first in CodeState).
struct CodeResult {
    int32_t status;       // BZ_OK or a negative status
    int32_t m;
    int32_t n_table;      // stages in the schedule
    int32_t table_complete;  // 1: the schedule reaches g = k, j = m; 0: cut by the work limit
    u64 ctl;              // checker state, see ctl_make
    u64 t_end;            // batches: wall_clock64() when the code ended (its last check)
    int32_t W;            // words per plane of the packed rows
    int32_t info;         // BZ_INFO_* bits of bz_result.info
    int32_t ranks[BZ_MAX_M];
    int32_t stage_min[BZ_MAX_STAGES];
    u64 stage_count[BZ_MAX_STAGES];
};

// Progress word of the wake copies: stages checked (bits 0-31), terminating
// stage + 1 (bits 32-63).  It only grows (checked grows, the terminating stage
// is set once), so the checkers publish it with atomic max in any order.
constexpr int WAKE_COPIES = 16;
BZ_HD u64 wake_make(int checked, int term) { return ((u64)(uint32_t)(term + 1) << 32) | (uint32_t)checked; }
BZ_HD int wake_checked(u64 w) { return (int)(uint32_t)w; }
BZ_HD int wake_term(u64 w) { return (int)(w >> 32) - 1; }

struct CodeState {
    CodeResult res;
    // inputs of this run
    int32_t p, n, k, flags;
    int32_t U0;           // n - k + 1
    int32_t pair_slot1;   // slot of the second set's pair table (1, or pair_sets(n, k): built ahead)
    u64 max_codewords;
    // completion tracking: workgroups done with each stage
    uint32_t stage_done[BZ_MAX_STAGES];
    // wall-clock trace (FLAG_TRACE): row 0 = decomposition start, its phases
    // (rows loaded, matrices reduced, schedule built); row 1 = enumeration kernel
    // first start / last end; row 2+s = stage s: first start, last end, checked,
    // last start
    u64 trace[BZ_MAX_STAGES + 2][4];
    StageDesc stages[BZ_MAX_STAGES];
    // copies of the checker's progress for the workgroups that wait on it,
    // one per 128-byte line (workgroup b reads copy b mod WAKE_COPIES), so
    // that a thousand pollers do not queue on one address; see wake_make
    u64 wake[WAKE_COPIES][16];
    // claim counters of the pool, one per 128-byte line (see pool_stages)
    uint32_t pool_next[POOL_SLICES][32];
};

// Claim word of a code in a batch: stage + 1 (bits 48-63, 0 = nothing to
// claim), parts of that stage (bits 24-47) and the next part to hand out
// (bits 0-23, advanced by atomic add; values >= parts are failed claims).
// The claim words of a batch are one contiguous array (code i at [i]), so
// that a wavefront scanning 64 codes reads 512 consecutive bytes.
BZ_HD u64 claim_make(int stage, uint32_t parts) { return ((u64)(uint32_t)(stage + 1) << 48) | ((u64)parts << 24); }
BZ_HD int claim_stage(u64 c) { return (int)(c >> 48) - 1; }
BZ_HD uint32_t claim_parts(u64 c) { return (uint32_t)(c >> 24) & 0xffffffu; }
BZ_HD uint32_t claim_next(u64 c) { return (uint32_t)c & 0xffffffu; }

// One code of a batch, filled by the host.
struct BatchCode {
    u64 g_offset;    // byte offset of its k x n generator in the batch's G
    u64 row_offset;  // word offset of its packed rows
    u64 max_codewords;
    int32_t p, n, k, flags;
    int32_t U0, WF, W;    // words per plane of G, and processed per combination
    uint32_t sweep_ops;  // VALU operations per lane and task
    uint32_t pair_stride;  // 16-byte units per pair table (pair_table_units(p, k, W))
    u64 pair_offset;       // 16-byte offset of its first pair table
};

// Batch-wide state: codes with stages left, the error flag of a time-out, and
// the wall_clock64() start of the decomposition launch (the earliest
// workgroup's), from which the codes' end times are counted.
struct BatchState {
    uint32_t remaining;
    int32_t status;
    u64 t0;
};

enum { FLAG_ROUND = 1, FLAG_NO_TERM = 2, FLAG_SKIP = 4, FLAG_HIST = 8, FLAG_TRACE = 16 };

// Checker state in one 64-bit word, so that it is read and advanced with a
// single atomic: stages checked (bits 0-15), terminating stage + 1 (bits
// 16-31, 0 = none), U after the checked stages (bits 32-47).
BZ_HD u64 ctl_make(int checked, int term, int U) {
    return (u64)(uint32_t)checked | ((u64)(uint32_t)(term + 1) << 16) | ((u64)(uint32_t)U << 32);
}
BZ_HD int ctl_checked(u64 c) { return (int)(c & 0xffff); }
BZ_HD int ctl_term(u64 c) { return (int)((c >> 16) & 0xffff) - 1; }
BZ_HD int ctl_U(u64 c) { return (int)((c >> 32) & 0xffff); }


// Workgroups start a stage that is not "nowait" only once every stage more
// than LOOKAHEAD places before it has been checked.  0 (the default) runs
// those stages one at a time: work on a stage beyond the current one competes
// with it for the vector ALUs and is thrown away when the current stage ends
// the run, which measured slower than draining each stage first.
#ifndef BZ_LOOKAHEAD
#define BZ_LOOKAHEAD 0
#endif
constexpr int LOOKAHEAD = BZ_LOOKAHEAD;

BZ_HD u64 sat_mul(u64 a, u64 b) {
    u64 r;
    return __builtin_mul_overflow(a, b, &r) ? ~0ull : r;
}
BZ_HD u64 sat_add(u64 a, u64 b) { return a > ~0ull - b ? ~0ull : a + b; }
// sat_mul(a, b) for b < 2^32, from two 32 x 32 -> 64 products
BZ_HD u64 sat_mul32(u64 a, uint32_t b) {
    const u64 lo = (u64)(uint32_t)a * b, hi = (a >> 32) * (u64)b + (lo >> 32);
    return (hi >> 32) ? ~0ull : (hi << 32) | (uint32_t)lo;
}

// off_s of stage (g, j): m times the tiles of the rounds before g, plus j - 1
// times the tiles of round g (saturating; tiles_before = the first sum).
BZ_HD u64 deal_offset(int m, u64 tiles_before, int j, u64 tiles) {
    return sat_add(sat_mul((u64)m, tiles_before), sat_mul((u64)(j - 1), tiles));
}
BZ_HD uint32_t deal_rot(u64 off, uint32_t grid) { return (uint32_t)((grid - off % grid) % grid); }

BZ_HD u64 binom_sat(int n, int r) {
    if (r < 0 || r > n) return 0;
    u64 v = 1;
    for (int i = 1; i <= r; i++) {
        u64 num = (u64)(n - r + i);
        if (v > ~0ull / num) return ~0ull;
        v = v * num / (u64)i;
    }
    return v;
}

BZ_HD int bound_c(int g, int k, int kj) {
    int v = g + 1 - (k - kj);
    return v > 0 ? v : 0;
}

// Target (s, L) steps per lane in one task: about `ops` VALU operations, from
// the per-step cost of the completions (F_3: two prefixes, add and subtract;
// F_7: six prefixes, three rotations, add and subtract).
#ifndef BZ_SWEEP_OPS
#define BZ_SWEEP_OPS 4500
#endif
constexpr uint32_t DEFAULT_SWEEP_OPS = BZ_SWEEP_OPS;
// Task size of the plain path: F_3 tasks of 3000 operations (the F_3 [72,36]
// codes run 3% faster than with 4500, F_7 [48,24] 4% slower); F_7 tasks of
// 6000 (with the pair tables the F_7 [48,24] codes run 2% faster than with
// 4500 or 9000, 18% slower with 3000).
BZ_HD uint32_t plain_sweep_ops(int p) { return p == 3 ? 3000u : 6000u; }
BZ_HD uint32_t sweep_cap_for(int p, int W, uint32_t ops = DEFAULT_SWEEP_OPS) {
    const uint32_t per = (p == 3) ? 2u * (6u * (uint32_t)W + 1u) : 6u * (25u * (uint32_t)W + 3u);
    const uint32_t cap = (ops ? ops : DEFAULT_SWEEP_OPS) / per;
    return cap < 4u ? 4u : cap;
}

// The q-group of bases with top row q (g >= 3): its number of bases and the
// blocking of its rows s = q+1 .. k-2.  Row q+1+i sweeps len-i last rows
// (len = k-2-q), so the first i rows hold P(i) = i len - i(i-1)/2 steps and
// all of them T = len(len+1)/2.  nb = min(len, ceil(T / cap)) blocks; block
// b starts at row offset max(b, the least i with nb P(i) >= b T): equal
// shares of T, except that a row heavier than a share is a block of its own
// (the rows get lighter as s grows, so those come first, and every block
// holds at least one row).
BZ_HD uint32_t qgroup_blocks(int k, uint32_t cap, int q) {
    const uint32_t len = (uint32_t)(k - 2 - q), T = len * (len + 1) / 2;
    const uint32_t nb = (T + cap - 1) / cap;
    return nb > len ? len : (nb < 1 ? 1 : nb);
}
BZ_HD int qgroup_block_start(int k, int q, uint32_t nb, uint32_t b) {
    const uint32_t len = (uint32_t)(k - 2 - q), T = len * (len + 1) / 2;
    const uint32_t target = b * T;  // <= 62 * 1953: fits 32 bits
    uint32_t lo = 0, hi = len;      // nb P(len) = nb T >= target
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint32_t P = mid * len - mid * (mid - 1) / 2;
        if (nb * P >= target) hi = mid;
        else lo = mid + 1;
    }
    return (int)(lo > b ? lo : b);
}
// Low coefficient digits a lane runs through itself: a lane takes
// (p-1)^vd consecutive bases, which differ only in the coefficients of their
// first vd rows in decoding order (the top row q first), so one decoding and
// one row addition per further base serve them all.  F_3 (vd <= 3): the
// coefficients 1 or 2 of vd rows, walked in Gray-code order.  F_7 (vd <= 1):
// the coefficient 1, 2, ..., 6 of row q, one addition of row q per step.  vd
// is the largest d <= min(g-3, max_digits(p)) with T (p-1)^d <= vcap (the
// lane's (s, L) steps stay within the run budget; with vcap <= cap the group
// is then one block) and bases >= 64 (p-1)^d (the group still fills a
// wavefront); T = len (len + 1) / 2 as in qgroup_blocks.  vcap = 0: no runs.
constexpr int BZ_MAX_VD = 3;
BZ_HD uint32_t max_digits(int p) { return p == 3 ? (uint32_t)BZ_MAX_VD : 1u; }
// bases per lane, (p-1)^vd
BZ_HD uint32_t run_len(int p, uint32_t vd) { return p == 3 ? (1u << vd) : (vd ? (uint32_t)(p - 1) : 1u); }
// the largest d with T (p-1)^d <= vcap, 0 if none (vcap >= 1)
BZ_HD uint32_t digits_by_steps(int p, int k, int q, uint32_t vcap) {
    const uint32_t len = (uint32_t)(k - 2 - q), T = len * (len + 1) / 2;
    if (p == 3) return vcap >= T ? 31u - (uint32_t)__builtin_clz(vcap / T) : 0u;
    return vcap / T >= (uint32_t)(p - 1) ? 1u : 0u;  // (d = 1 is the most F_7 takes)
}
// the largest d with bases >= 64 (p-1)^d, 0 if none
BZ_HD uint32_t digits_by_bases(int p, u64 bases) {
    if (p == 3) return bases >= 128 ? 57u - (uint32_t)__builtin_clzll(bases) : 0u;
    return bases >= 64u * (u64)(p - 1) ? 1u : 0u;
}
BZ_HD uint32_t digits_of(int p, int g, uint32_t by_steps, u64 bases) {
    uint32_t d = (uint32_t)(g - 3) < max_digits(p) ? (uint32_t)(g - 3) : max_digits(p);
    d = by_steps < d ? by_steps : d;
    const uint32_t b = digits_by_bases(p, bases);
    return b < d ? b : d;
}
BZ_HD uint32_t qgroup_digits(int p, int k, int g, uint32_t vcap, int q, u64 bases) {
    if (vcap == 0) return 0;
    return digits_of(p, g, digits_by_steps(p, k, q, vcap), bases);
}
// Run budget of a round: runs shorten the work of a stage but lengthen its
// tasks and cut their number, so a round takes them only when its stages
// still have a tile for every workgroup with them (measured: the stages that
// leave workgroups idle run slower with runs).
BZ_HD uint32_t run_budget(int p, uint32_t cap) { return cap; }
BZ_HD bool runs_pay(u64 tasks_with_runs, uint32_t grid) {
    return (tasks_with_runs + WAVES_PER_GROUP - 1) / WAVES_PER_GROUP >= (u64)grid;
}
BZ_HD void qgroup(int k, int g, u64 M, uint32_t cap, uint32_t vcap, const u64 *binom, int q, u64 *bases,
                  uint32_t *nb, uint32_t *vd, int p) {
    *bases = sat_mul(binom[q * 65 + (g - 3)], M);
    *nb = qgroup_blocks(k, cap, q);
    *vd = qgroup_digits(p, k, g, vcap, q, *bases);
}
// chunks of 64 bases (no overflow at the saturated value)
BZ_HD u64 ceil64(u64 bases) { return (bases >> 6) + ((bases & 63) != 0); }
// tasks of a q-group: chunks of 64 lanes of (p-1)^vd bases each, times the
// blocks ((p-1)^vd divides the bases whenever vd > 0)
BZ_HD u64 qgroup_tasks(int p, u64 bases, uint32_t nb, uint32_t vd) {
    const u64 lanes = p == 3 ? bases >> vd : (vd ? bases / (u64)(p - 1) : bases);
    return ceil64(lanes) * (u64)nb;
}

// Number of tasks of a stage with g >= 3 (saturating); with tab != NULL also
// fills the q-groups (entries for q = g-3 .. k-3, index q-(g-3)).
BZ_HD u64 fill_qtable(int p, int k, int g, u64 M, uint32_t cap, uint32_t vcap, const u64 *binom, QEntry *tab) {
    u64 first = 0;
    for (int q = g - 3; q <= k - 3; q++) {
        u64 bases;
        uint32_t nb, vd;
        qgroup(k, g, M, cap, vcap, binom, q, &bases, &nb, &vd, p);
        if (tab) {
            QEntry &e = tab[q - (g - 3)];
            e.first = first;
            e.bases = bases;
            e.nb = nb;
            e.vd = vd;
        }
        first = sat_add(first, qgroup_tasks(p, bases, nb, vd));
    }
    return first;
}

// The pair s < L of colex rank r (r = L(L-1)/2 + s), r < k(k-1)/2.
BZ_HD void pair_of(int r, int k, int *s, int *L) {
    int lo = 1, hi = k - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (mid * (mid - 1) / 2 <= r) lo = mid;
        else hi = mid - 1;
    }
    *L = lo;
    *s = r - lo * (lo - 1) / 2;
}

// Locate task t among the q-groups (binary search on .first): returns the
// index of its group.
BZ_HD int qtable_find(const QEntry *tab, int nq, u64 t) {
    int lo = 0, hi = nq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].first <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The largest c in [i-1, hi] with C(c, i) <= rho, given rho < C(hi+1, i):
// the next row of a colex unranking.  For i = 1 that is rho itself; larger i
// search the table (measured faster than starting from the root of
// C(c, i) = rho and stepping to the exact answer).
template <typename Bin>
BZ_HD int top_row(u64 rho, int i, int hi, Bin bin) {
    if (i == 1) return (int)rho;
    int lo = i - 1, h = hi;
    while (lo < h) {
        const int mid = (lo + h + 1) >> 1;
        if (bin(mid, i) <= rho) lo = mid;
        else h = mid - 1;
    }
    return lo;
}

// Decode base number bi (< bases) of the group with top row q: its lower rows
// (the (g-3)-subset of {0..q-1} of colex rank bi / M, M = (p-1)^(g-3)) and the
// coefficients from the base-(p-1) digits of bi % M, least significant first.
// The lowest row of the base gets coefficient 1.  BaseCursor yields the rows
// one at a time, the top row q first: first() then next() for i = g-3 .. 1.
struct BaseCursor {
    u64 rho;      // colex rank still to decode
    uint32_t ci;  // coefficient digits still to use
    int hi;       // the next row is below hi + 1
};
template <int P>
BZ_HD BaseCursor base_first(int g, int q, u64 M, u64 bi, int *coef) {
    const int t = g - 3;  // lower rows
    BaseCursor c;
    if (P == 3) {
        c.rho = bi >> t;
        c.ci = (uint32_t)bi & (uint32_t)(M - 1);
    } else if ((bi >> 32) == 0) {
        const uint32_t b32 = (uint32_t)bi, r = b32 / (uint32_t)M;
        c.rho = r;
        c.ci = b32 - r * (uint32_t)M;
    } else {
        c.rho = bi / M;
        c.ci = (uint32_t)(bi - c.rho * M);
    }
    *coef = 1;
    if (t > 0) {
        *coef = (int)(c.ci % (uint32_t)(P - 1)) + 1;
        c.ci /= (uint32_t)(P - 1);
    }
    c.hi = q - 1;
    return c;
}
template <int P, typename Bin>
BZ_HD int base_next(BaseCursor &c, int i, Bin bin, int *coef) {
    const int lo = top_row(c.rho, i, c.hi, bin);
    c.rho -= bin(lo, i);
    c.hi = lo - 1;
    *coef = 1;
    if (i > 1) {
        *coef = (int)(c.ci % (uint32_t)(P - 1)) + 1;
        c.ci /= (uint32_t)(P - 1);
    }
    return lo;
}
// visit(row, coef) for every row of the base, the top row q first.
template <int P, typename Bin, typename Visit>
BZ_HD void decode_base(int g, int q, u64 M, u64 bi, Bin bin, Visit visit) {
    int coef;
    BaseCursor c = base_first<P>(g, q, M, bi, &coef);
    visit(q, coef);
    for (int i = g - 3; i >= 1; i--) {
        const int row = base_next<P>(c, i, bin, &coef);
        visit(row, coef);
    }
}

// (p-1)^e, saturating (p - 1 = 2: a shift; p - 1 = 6: at most 25 steps
// before it saturates, each a constant multiply and compare)
BZ_HD u64 pow_sat(int p, int e) {
    if (e <= 0) return 1;
    if (p == 3) return e >= 64 ? ~0ull : (1ull << e);
    u64 r = 1;
    for (int t = 0; t < e; t++) {
        if (r > ~0ull / 6u) return ~0ull;
        r *= 6u;
    }
    return r;
}
// Round g of the schedule (its m stages (g, 1..m) share these): the
// combinations of one stage, C(k, g) (p-1)^(g-1), and the coefficient
// combinations (p-1)^(g-3) of one base of g-3 rows (1 for g < 3); saturating.
BZ_HD u64 round_codewords(int p, int k, int g, const u64 *binom) { return sat_mul(binom[k * 65 + g], pow_sat(p, g - 1)); }
BZ_HD u64 round_combos(int p, int g) { return pow_sat(p, g - 3); }
// Stages of round g within the codeword limit, given cum = the (saturated)
// codewords of all earlier rounds: the largest j <= m with
// sat(cum + j cw) <= max_codewords, or 0 when the coefficient combinations do
// not fit 32 bits.  The same decision as build_schedule stage by stage.
BZ_HD int round_stages(int m, u64 cum, u64 cw, u64 combos, u64 max_codewords) {
    if (combos >= (1ull << 32)) return 0;
    if (max_codewords == ~0ull) return m;
    if (cum > max_codewords) return 0;
    if (sat_mul(cw, (u64)m) <= max_codewords - cum) return m;  // the usual case, without a division
    const u64 j = (max_codewords - cum) / cw;
    return j < (u64)m ? (int)j : m;
}
// The last-row sweep of a prefix built on row s: every row L = s+1 .. k-1 is
// combined with it, UR rows at a time (the kernel issues the loads of a group
// together).  group(L0, nr) combines rows L0 .. L0+nr-1 (nr <= UR).  Returns
// the rows combined: the kernel's per-stage combination counts are taken from
// this number, and the host replay drives the same loop, so a row skipped or
// repeated here shows up in both.
template <int UR, typename Group>
BZ_HD int sweep_last_rows(int s, int k, Group &&group) {
    int done = 0;
    for (int L = s + 1; L < k; L += UR) {
        const int nr = k - L < UR ? k - L : UR;
        group(L, nr);
        done += nr;
    }
    return done;
}

// Rounds g <= SUBSET_G give each lane one g-subset of the rows (all its
// coefficient vectors); larger rounds give it a base of g-2 rows and sweep the
// last two rows (see StageDesc).  Round 4 takes bases of two rows: with the
// pair tables its sweep needs no exact addition, and the four-row subsets
// held the most registers of the batched kernel (119 VGPRs: four workgroups
// per CU instead of five).
constexpr int SUBSET_G = 3;

// Tasks of a stage with g <= SUBSET_G: 64 subsets per task.
BZ_HD u64 small_stage_tasks(int k, int g) { return (binom_sat(k, g) + 63) / 64; }

// The g-subset of the rows 0..k-1 of colex rank r (r < C(k, g)), ascending in
// rows[0..g-1]: the top row is the largest c with C(c, g) <= r, and so on down.
template <int G, typename Bin>
BZ_HD void decode_subset(u64 r, int k, Bin bin, int (&rows)[G]) {
    int hi = k - 1;
#pragma unroll
    for (int t = G; t >= 1; t--) {
        const int lo = top_row(r, t, hi, bin);
        rows[t - 1] = lo;
        r -= bin(lo, t);
        hi = lo - 1;
    }
}

// Build the schedule: stages (g, j) for g = 1..k, j = 1..m in order, while the
// cumulative combination count stays within max_codewords, at most
// BZ_MAX_STAGES stages, and every index fits the kernel ((p-1)^(g-3) < 2^32,
// tasks < 2^62 counted without runs of bases; the last condition only when
// count_tasks).  The deal of a stage starts at off_s = the tiles of all earlier
// stages; stages with off_s < grid start at once (nowait), the others wait for
// the checks.  Rounds take runs of bases where runs_pay.  grid: workgroups
// of the enumeration launch; W: words per plane of the packed rows.  Returns the
// number of stages; *complete = 1 if the schedule reaches (k, m).
// binom[c*65+i] = C(c, i) for c, i <= 64.
BZ_HD int build_schedule(int p, int k, int m, const int32_t *ranks, int flags, u64 max_codewords,
                         uint32_t grid, int W, const u64 *binom, StageDesc *st, int *complete,
                         bool count_tasks = true, uint32_t sweep_ops = DEFAULT_SWEEP_OPS) {
    int ns = 0;
    u64 cum = 0, off = 0;
    *complete = 1;
    const uint32_t cap = sweep_cap_for(p, W, sweep_ops);
    for (int g = 1; g <= k; g++) {
        const u64 cw = round_codewords(p, k, g, binom);
        u64 tasks0, tasks;  // without runs of bases; the round's own
        uint32_t vcap = 0;
        const u64 combos = round_combos(p, g);
        if (g <= SUBSET_G) tasks0 = tasks = small_stage_tasks(k, g);
        else if (combos >= (1ull << 32)) tasks0 = tasks = ~0ull;
        else if (count_tasks) {
            tasks0 = tasks = fill_qtable(p, k, g, combos, cap, 0, binom, nullptr);
            const uint32_t budget = run_budget(p, cap);
            if (budget) {
                const u64 tv = fill_qtable(p, k, g, combos, cap, budget, binom, nullptr);
                if (runs_pay(tv, grid)) {
                    tasks = tv;
                    vcap = budget;
                }
            }
        } else {
            tasks0 = tasks = 0;  // the caller fills tasks, tiles and parts of these stages
        }
        for (int j = 1; j <= m; j++) {
            if (ns >= BZ_MAX_STAGES || sat_add(cum, cw) > max_codewords || combos >= (1ull << 32) ||
                tasks0 >= (1ull << 62)) {
                *complete = 0;
                return ns;
            }
            StageDesc &d = st[ns];
            d.g = g;
            d.j = j;
            int L = 0;
            for (int i = 1; i <= m; i++) L += bound_c(i <= j ? g : g - 1, k, ranks[i - 1]);
            d.L = L;
            d.check = (flags & FLAG_NO_TERM) ? 0 : ((flags & FLAG_ROUND) ? (j == m) : 1);
            d.nowait = off < (u64)grid;
            d.vcap = vcap;
            d.pad = 0;
            d.tasks = tasks;
            d.tiles = (d.tasks + WAVES_PER_GROUP - 1) / WAVES_PER_GROUP;
            d.codewords = cw;
            d.coef_combos = (uint32_t)combos;
            d.parts = (uint32_t)(d.tiles < (u64)grid ? d.tiles : (u64)grid);
            d.sweep_cap = cap;
            d.rot = deal_rot(off, grid);
            off = sat_add(off, d.tiles);
            cum = sat_add(cum, cw);
            ns++;
        }
    }
    return ns;
}

// The second information set computed ahead (plain path): a second
// workgroup eliminates G with the column order {k, ..., n-1}, {0, ..., k-1},
// which is the second set's order whenever the first set's pivots are columns
// 0 .. k-1, and leaves the packed rows and the set's pivot columns and size
// here; flag = the call's epoch once they are complete (and ok = 1).
struct SpecBuf {
    u32 rows[BZ_MAX_K * 16];
    u32 pivmask[4];
    int32_t kj, ok;
    u32 flag, pad;
};

// The task counts of the rounds g > SUBSET_G and their run budgets depend on
// (p, k, W, grid, task size) only, not on the generator: the plain path
// computes them once per shape on the host and the decomposition reads them
// (the same values as build_schedule's and as the kernel's own loop).
// cut_g: the first round whose count without runs reaches 2^62 (k + 1: none).
struct RoundTable {
    u64 tasks[BZ_MAX_K];     // round g at [g - 1]
    uint32_t vcap[BZ_MAX_K];
    int32_t cut_g;
    uint32_t pad;
};
BZ_HD void fill_round_table(int p, int k, int W, uint32_t grid, uint32_t sweep_ops, const u64 *binom,
                            RoundTable *t) {
    const uint32_t cap = sweep_cap_for(p, W, sweep_ops), budget = run_budget(p, cap);
    t->cut_g = k + 1;
    t->pad = 0;
    for (int g = 1; g <= BZ_MAX_K; g++) {
        t->tasks[g - 1] = 0;
        t->vcap[g - 1] = 0;
        if (g <= SUBSET_G || g > k) continue;
        const u64 combos = round_combos(p, g);
        if (combos >= (1ull << 32)) continue;  // such rounds are never in a schedule
        const u64 t0 = fill_qtable(p, k, g, combos, cap, 0, binom, nullptr);
        if (t0 >= (1ull << 62) && t->cut_g > k) t->cut_g = g;
        t->tasks[g - 1] = t0;
        if (budget) {
            const u64 tv = fill_qtable(p, k, g, combos, cap, budget, binom, nullptr);
            if (runs_pay(tv, grid)) {
                t->tasks[g - 1] = tv;
                t->vcap[g - 1] = budget;
            }
        }
    }
}

// Tile owned by workgroup b in round r of a stage whose deal is rotated by
// rot.  Rounds alternate direction so that the heavy-first order of the items
// spreads evenly over the workgroups; in round 0 workgroup off_s mod grid
// takes tile 0, the next one tile 1, and so on.
BZ_HD u64 tile_of(u64 r, uint32_t b, uint32_t grid, uint32_t rot) {
    const uint32_t bb = (uint32_t)(((u64)b + rot) % grid);
    return r * grid + ((r & 1) ? (grid - 1 - bb) : bb);
}

// The pool of the plain enumeration kernel.  The stages that start at once
// (nowait) are a prefix of the schedule, and all of them but the last have
// fewer tiles than the grid (each starts within the first pass).  These
// stages, without the last one when it holds more than pool_stage_cap tiles,
// are numbered as one sequence of "pool tiles" in schedule order (the tiles of
// stage s are off_s .. off_s + tiles_s - 1).  Workgroup b runs pool tile b
// first; the tiles from grid on are handed out one at a time while the
// workgroups last: slice c of C = pool_slices(grid) counters hands out the
// pool tiles grid + c, grid + c + C, grid + c + 2C, ... in this order, and
// workgroup b claims from slice b mod C.  Every slice thus holds the same mix
// of heavy and light tiles, no counter serves more than grid / C workgroups,
// and a workgroup that drew light tiles simply claims more.
BZ_HD uint32_t pool_slices(uint32_t grid) { return grid < POOL_SLICES ? grid : POOL_SLICES; }
BZ_HD u64 pool_stage_cap(uint32_t grid) { return 32ull * grid; }
// off_s of a stage that starts at once (off_s < grid), from its rotation
BZ_HD u64 nowait_offset(uint32_t rot, uint32_t grid) { return (u64)((grid - rot) % grid); }
// The number of pool stages; *tiles = their tiles (< grid + pool_stage_cap).
BZ_HD int pool_stages(const StageDesc *st, int ns, uint32_t grid, u64 *tiles) {
    int lo = 0, hi = ns;  // the first stage that waits (nowait is a prefix)
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (st[mid].nowait) lo = mid + 1;
        else hi = mid;
    }
    int sp = lo;
    if (sp > 0 && st[sp - 1].tiles > pool_stage_cap(grid)) sp--;
    *tiles = sp > 0 ? nowait_offset(st[sp - 1].rot, grid) + st[sp - 1].tiles : 0;
    return sp;
}
// pool tile number i of slice c, counted from the first claimed tile (grid)
BZ_HD u64 pool_tile(uint32_t c, uint32_t i, uint32_t C) { return (u64)c + (u64)C * i; }
// The pool stage of pool tile u (< the pool's tiles), searching upward from
// stage s (a stage at or before it).
BZ_HD int pool_stage_of(const StageDesc *st, int sp, int s, u64 u, uint32_t grid) {
    while (s + 1 < sp && nowait_offset(st[s + 1].rot, grid) <= u) s++;
    return s;
}

BZ_HD void fill_binomials(u64 *tab) {
    for (int a = 0; a <= 64; a++)
        for (int b = 0; b <= 64; b++) tab[a * 65 + b] = (b > a) ? 0 : (b == 0 || b == a) ? 1 : 0;
    for (int a = 2; a <= 64; a++)
        for (int b = 1; b < a; b++) tab[a * 65 + b] = tab[(a - 1) * 65 + b - 1] + tab[(a - 1) * 65 + b];
}

}  // namespace bz
