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

// Row storage: Gamma_j row i, plane b, word w at rows[((j*BZ_MAX_K + i)*3 + b)*4 + w].
constexpr int ROW_WORDS = 12;
constexpr uint64_t DEFAULT_LIMIT = 1ull << 44;

// One stage (g, j) of Algorithm 6, and how its work is cut into queue chunks.
//   g = 1: an item is a row i (one combination).
//   g = 2: an item is the lowest row s; the kernel adds every later row.
//   g >= 3: an item is a "base" of g-2 rows (lowest coefficient 1, the others
//           any of the (p-1)^(g-3) nonzero choices); the kernel extends it by a
//           row s above the base with any nonzero coefficient, and then by a last
//           row above s with every nonzero multiplier.
struct StageDesc {
    int32_t g, j;
    int32_t L;          // L_{g,j}
    int32_t check;      // 1: test L >= U after this stage
    u64 items;          // work items in the stage
    u64 items_per_chunk;
    u64 chunk_begin;    // first global chunk index of the stage
    u64 n_chunks;
    u64 codewords;      // C(k,g) (p-1)^(g-1)
    uint32_t coef_combos;  // (p-1)^(g-3) for g >= 3, else 1
    uint32_t pad;
};

// Results the host reads back (kept contiguous and first in CodeState).
struct CodeResult {
    int32_t status;       // BZ_OK or a negative status from the decomposition
    int32_t m;
    int32_t n_table;      // stages in the schedule
    int32_t table_complete;  // 1: the schedule reaches g = k, j = m; 0: cut by the work limit
    int32_t term_stage;   // stage after which L >= U held, or -1
    int32_t checked;      // stages checked without termination
    int32_t W;            // words per plane of the packed rows
    int32_t pad;
    int32_t ranks[BZ_MAX_M];
    int32_t stage_min[BZ_MAX_STAGES];
    u64 stage_count[BZ_MAX_STAGES];
};

struct CodeState {
    CodeResult res;
    // inputs of this run
    int32_t p, n, k, flags;
    int32_t U0;           // n - k + 1
    int32_t pad0;
    u64 max_codewords;
    u64 total_chunks;
    // queue and completion tracking
    u64 next_chunk;
    u64 stage_done[BZ_MAX_STAGES];
    int32_t U_after[BZ_MAX_STAGES];
    StageDesc stages[BZ_MAX_STAGES];
};

enum { FLAG_ROUND = 1, FLAG_NO_TERM = 2, FLAG_SKIP = 4, FLAG_HIST = 8 };

BZ_HD u64 sat_mul(u64 a, u64 b) {
    if (a == 0 || b == 0) return 0;
    if (a > ~0ull / b) return ~0ull;
    return a * b;
}
BZ_HD u64 sat_add(u64 a, u64 b) { return a > ~0ull - b ? ~0ull : a + b; }

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

// Colex unranking: the t-subset c_1 < ... < c_t of {0, ..., hi} whose rank is
// sr = sum_i C(c_i, i).  Elements come out from the largest (i = t) to the
// smallest; visit(i, c_i) is called for each.  binom[c * 65 + i] = C(c, i).
template <typename Visit>
BZ_HD void colex_unrank(u64 sr, int t, int hi, const u64 *binom, Visit visit) {
    for (int i = t; i >= 1; i--) {
        int lo = i - 1, h = hi;
        while (lo < h) {
            const int mid = (lo + h + 1) >> 1;
            if (binom[mid * 65 + i] <= sr) lo = mid;
            else h = mid - 1;
        }
        sr -= binom[lo * 65 + i];
        hi = lo - 1;
        visit(i, lo);
    }
}

// Build the schedule: stages (g, j) for g = 1..k, j = 1..m in order, while the
// cumulative combination count stays within max_codewords, at most
// BZ_MAX_STAGES stages, and every index fits the kernel (items < 2^62,
// (p-1)^(g-3) < 2^32).  lanes_target: aim for about this many chunks per
// large stage.  Returns the number of stages; *complete = 1 if the schedule
// reaches (k, m).
BZ_HD int build_schedule(int p, int k, int m, const int32_t *ranks, int flags, u64 max_codewords,
                         u64 target_chunks, StageDesc *st, int *complete, u64 *total_chunks) {
    int ns = 0;
    u64 cum = 0, chunk = 0;
    *complete = 1;
    for (int g = 1; g <= k; g++) {
        u64 pw = 1;  // (p-1)^(g-1)
        for (int t = 1; t < g; t++) pw = sat_mul(pw, (u64)(p - 1));
        u64 cw = sat_mul(binom_sat(k, g), pw);
        u64 items;
        u64 combos = 1;
        if (g == 1) items = (u64)k;
        else if (g == 2) items = (u64)(k - 1);
        else {
            for (int t = 3; t < g; t++) combos = sat_mul(combos, (u64)(p - 1));
            items = sat_mul(binom_sat(k - 2, g - 2), combos);
        }
        for (int j = 1; j <= m; j++) {
            if (ns >= BZ_MAX_STAGES || sat_add(cum, cw) > max_codewords || combos >= (1ull << 32) ||
                items >= (1ull << 62)) {
                *complete = 0;
                *total_chunks = chunk;
                return ns;
            }
            StageDesc &d = st[ns];
            d.g = g;
            d.j = j;
            int L = 0;
            for (int i = 1; i <= m; i++) L += bound_c(i <= j ? g : g - 1, k, ranks[i - 1]);
            d.L = L;
            d.check = (flags & FLAG_NO_TERM) ? 0 : ((flags & FLAG_ROUND) ? (j == m) : 1);
            d.items = items;
            // chunks of 64 * t items; t grows for stages with far more items than lanes
            u64 t = items / (64ull * target_chunks);
            if (t < 1) t = 1;
            if (t > 64) t = 64;
            d.items_per_chunk = 64ull * t;
            d.n_chunks = (items + d.items_per_chunk - 1) / d.items_per_chunk;
            d.chunk_begin = chunk;
            d.codewords = cw;
            d.coef_combos = (uint32_t)combos;
            d.pad = 0;
            chunk += d.n_chunks;
            cum = sat_add(cum, cw);
            ns++;
        }
    }
    *total_chunks = chunk;
    return ns;
}

}  // namespace bz
