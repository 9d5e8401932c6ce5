// Host-side checks of the library's shared (host/device) code, built with g++.
//
//   arith     exhaustive: every pair of symbols, at every bit position of a
//             word, through the bit-sliced F_3 / F_7 functions, against
//             plain mod-p integers
//   schedule  stage counts, work items, tile dealing and bounds L_{g,j}
//   unrank    the work decomposition visits every g-row combination with the
//             lowest coefficient 1 exactly once
//
// Prints "OK <check>" per passing check; exits 1 on the first failure.
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <random>
#include <map>
#include <set>
#include <vector>

#include "bz_arith.hpp"
#include "bz_state.hpp"

using namespace bz;

static int fails = 0;
#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);            \
            if (++fails > 20) std::exit(1);                                    \
        }                                                                      \
    } while (0)

static int sym_at(const u32 *pl, int r, int t) {
    int v = 0;
    for (int b = 0; b < r; b++) v |= ((pl[b] >> t) & 1) << b;
    return v;
}

static void put(u32 *pl, int r, int t, int v) {
    for (int b = 0; b < r; b++) pl[b] |= (u32)((v >> b) & 1) << t;
}

static void check_arith() {
    for (int P : {3, 7}) {
        const int r = P == 3 ? 2 : 3;
        // fill words with all pairs (a, b), shifted through every bit position
        std::vector<std::pair<int, int>> pairs;
        for (int a = 0; a < P; a++)
            for (int b = 0; b < P; b++) pairs.push_back({a, b});
        for (int shift = 0; shift < 32; shift++) {
            u32 A[3] = {0, 0, 0}, B[3] = {0, 0, 0};
            std::vector<int> pos(pairs.size());
            for (size_t i = 0; i < pairs.size() && i < 32; i++) {
                int t = (int)((i + shift) % 32);
                pos[i] = t;
                put(A, r, t, pairs[i].first);
                put(B, r, t, pairs[i].second);
            }
            const size_t npairs = pairs.size() < 32 ? pairs.size() : 32;
            u32 S[3] = {0, 0, 0}, D[3] = {0, 0, 0}, N[3] = {0, 0, 0}, X2[3] = {0, 0, 0};
            u32 iso_a, iso_s;
            if (P == 3) {
                f3_add(A[0], A[1], B[0], B[1], S[0], S[1]);
                u32 nb0, nb1;
                f3_neg(B[0], B[1], nb0, nb1);
                f3_add(A[0], A[1], nb0, nb1, D[0], D[1]);
                f3_neg(A[0], A[1], N[0], N[1]);
                X2[0] = N[0]; X2[1] = N[1];
                iso_a = f3_iso_add(A[0], A[1], B[0], B[1]);
                iso_s = f3_iso_sub(A[0], A[1], B[0], B[1]);
            } else {
                f7_add(A[0], A[1], A[2], B[0], B[1], B[2], S[0], S[1], S[2]);
                u32 nb[3];
                f7_neg(B[0], B[1], B[2], nb[0], nb[1], nb[2]);
                f7_add(A[0], A[1], A[2], nb[0], nb[1], nb[2], D[0], D[1], D[2]);
                f7_neg(A[0], A[1], A[2], N[0], N[1], N[2]);
                f7_double(A[0], A[1], A[2], X2[0], X2[1], X2[2]);
                iso_a = f7_iso_add(A[0], A[1], A[2], B[0], B[1], B[2]);
                iso_s = f7_iso_sub(A[0], A[1], A[2], B[0], B[1], B[2]);
            }
            u32 used = 0;
            for (size_t i = 0; i < npairs; i++) {
                const int t = pos[i], a = pairs[i].first, b = pairs[i].second;
                used |= 1u << t;
                CHECK(sym_at(S, r, t) == (a + b) % P);
                CHECK(sym_at(D, r, t) == (a - b + P) % P);
                CHECK(sym_at(N, r, t) == (P - a) % P);
                CHECK(sym_at(X2, r, t) == (2 * a) % P);
                CHECK((int)((iso_a >> t) & 1) == ((a + b) % P != 0));
                CHECK((int)((iso_s >> t) & 1) == ((a - b + P) % P != 0));
                for (int h = 1; h < P; h++) {
                    u32 x[3] = {A[0], A[1], A[2]}, y[3] = {0, 0, 0};
                    scale<3>(1, x, y);  // keep both instantiations referenced
                    if (P == 3) scale<3>(h, x, y);
                    else scale<7>(h, x, y);
                    CHECK(sym_at(y, r, t) == (h * a) % P);
                }
            }
            // padding stays zero
            for (int b = 0; b < r; b++) {
                CHECK((S[b] & ~used) == 0);
                CHECK((D[b] & ~used) == 0);
                CHECK((N[b] & ~used) == 0);
            }
            CHECK((iso_a & ~used) == 0);
            CHECK((iso_s & ~used) == 0);
        }
    }
    // F_7 addition also tolerates the non-canonical 7 = (1,1,1) as an input
    for (int a = 0; a < 8; a++)
        for (int b = 0; b < 8; b++) {
            u32 A[3] = {0, 0, 0}, B[3] = {0, 0, 0}, S[3];
            put(A, 3, 5, a);
            put(B, 3, 5, b);
            f7_add(A[0], A[1], A[2], B[0], B[1], B[2], S[0], S[1], S[2]);
            CHECK(sym_at(S, 3, 5) == (a + b) % 7);
        }
    if (!fails) std::printf("OK arith\n");
}

static u64 C(int n, int r) { return binom_sat(n, r); }
static u64 BINOM[65 * 65];

// The pool of the plain enumeration kernel (pool_stages): the nowait prefix
// (without its last stage when that one is over the cap), numbered from
// off_0 = 0 on; the first tile of every workgroup plus the slices' claims hand
// out every pool tile exactly once, and the stage walk finds each tile's stage.
static void check_pool(const StageDesc *st, int ns, uint32_t grid) {
    u64 ptiles = 0;
    const int sp = pool_stages(st, ns, grid, &ptiles);
    int nw = 0;
    while (nw < ns && st[nw].nowait) nw++;
    for (int s = nw; s < ns; s++) CHECK(!st[s].nowait);
    CHECK(sp == nw || (nw > 0 && sp == nw - 1 && st[nw - 1].tiles > pool_stage_cap(grid)));
    u64 off = 0;
    for (int s = 0; s < sp; s++) {
        CHECK(nowait_offset(st[s].rot, grid) == off);
        if (s + 1 < sp) CHECK(st[s].tiles < grid);
        CHECK(st[s].tiles >= 1 && st[s].tiles <= pool_stage_cap(grid));
        off += st[s].tiles;
    }
    CHECK(ptiles == off);
    if (ptiles > 4000000) return;
    std::vector<int> seen(ptiles, 0);
    const uint32_t C = pool_slices(grid);
    for (u64 b = 0; b < grid && b < ptiles; b++) seen[b]++;
    for (uint32_t c = 0; c < C; c++) {
        u64 last = 0;
        for (uint32_t i = 0;; i++) {
            const u64 u = grid + pool_tile(c, i, C);
            if (u >= ptiles) break;
            CHECK(u > last);
            last = u;
            seen[u]++;
        }
    }
    for (u64 u = 0; u < ptiles; u++) CHECK(seen[u] == 1);
    int prev = 0;
    for (u64 u = 0; u < ptiles; u++) {
        const int s0 = pool_stage_of(st, sp, 0, u, grid);
        const u64 o = nowait_offset(st[s0].rot, grid);
        CHECK(s0 < sp && o <= u && u < o + st[s0].tiles);
        CHECK(pool_stage_of(st, sp, prev, u, grid) == s0);
        prev = s0;
    }
}

static void check_schedule() {
    const int before = fails;
    struct Case { int p, k, m; std::vector<int> ranks; };
    std::vector<Case> cases = {{3, 10, 4, {10, 10, 10, 10}}, {3, 36, 2, {36, 35}}, {7, 24, 2, {24, 24}},
                               {7, 20, 4, {20, 20, 20, 2}}, {3, 5, 3, {5, 5, 3}}, {7, 1, 1, {1}},
                               {3, 64, 2, {64, 64}}};
    for (auto &c : cases) {
        for (int flags : {0, (int)FLAG_ROUND, (int)FLAG_NO_TERM}) {
            StageDesc st[BZ_MAX_STAGES];
            int complete = 0;
            const uint32_t grid = 1000;
            int ns = build_schedule(c.p, c.k, c.m, c.ranks.data(), flags, ~0ull, grid, 2, BINOM, st, &complete);
            u64 cum = 0, off = 0;
            std::vector<int> owner(grid, -1);  // nowait stages that fit the grid own disjoint workgroups
            for (int s = 0; s < ns; s++) {
                const StageDesc &d = st[s];
                CHECK(d.g == s / c.m + 1 && d.j == s % c.m + 1);
                u64 pw = 1;
                for (int t = 1; t < d.g; t++) pw *= (u64)(c.p - 1);
                CHECK(d.codewords == sat_mul(C(c.k, d.g), pw));
                if (d.g >= 3) {
                    // each base of g-2 rows with top row q has (p-1)^2 C(k-1-q, 2) completions
                    u64 sum = 0;
                    for (int q = d.g - 3; q <= c.k - 3; q++)
                        sum = sat_add(sum, sat_mul(sat_mul(C(q, d.g - 3), (u64)d.coef_combos),
                                                   (u64)(c.p - 1) * (c.p - 1) * C(c.k - 1 - q, 2)));
                    CHECK(sum == d.codewords || d.codewords == ~0ull);
                }
                CHECK(d.tiles * WAVES_PER_GROUP >= d.tasks && (d.tiles - 1) * WAVES_PER_GROUP < d.tasks);
                CHECK(d.parts == std::min<u64>(d.tiles, grid));
                // the rounds of tile_of() deal every tile exactly once
                if (d.tiles <= 50000) {
                    std::vector<int> seen(d.tiles, 0);
                    for (uint32_t b = 0; b < grid; b++)
                        for (u64 r = 0;; r++) {
                            const u64 t = tile_of(r, b, grid, d.rot);
                            if (t >= d.tiles) break;
                            seen[t]++;
                        }
                    for (u64 t = 0; t < d.tiles; t++) CHECK(seen[t] == 1);
                    // the workgroups that own a round-0 tile are exactly d.parts many,
                    // the ones from off_s mod grid on
                    uint32_t owners = 0;
                    for (uint32_t b = 0; b < grid; b++) {
                        const bool own = tile_of(0, b, grid, d.rot) < d.tiles;
                        owners += own;
                        CHECK(own == ((b + grid - (uint32_t)(off % grid)) % grid < d.parts));
                    }
                    CHECK(owners == d.parts);
                }
                // the deal starts where the previous stage's ended; the stages that
                // start within the first pass over the grid do not wait
                CHECK(d.rot == (grid - off % grid) % grid);
                CHECK(d.nowait == (off < grid));
                if (d.nowait && off + d.tiles <= grid) {
                    for (uint32_t b = 0; b < grid; b++) {
                        const bool own = tile_of(0, b, grid, d.rot) < d.tiles;
                        CHECK(own == (b >= off && b < off + d.tiles));
                        if (own) CHECK(owner[b] == -1);
                        if (own) owner[b] = s;
                    }
                }
                off = sat_add(off, d.tiles);
                cum = sat_add(cum, d.codewords);
                // L_{g,j} at j = m is Algorithm 6's (m-1)(g+1) + max(0, g+1-k+k_m) when only
                // the last matrix may be partial
                bool only_last_partial = true;
                for (int i = 0; i + 1 < c.m; i++) only_last_partial &= c.ranks[i] == c.k;
                if (d.j == c.m && only_last_partial) {
                    int alg6 = (c.m - 1) * (d.g + 1) + std::max(0, d.g + 1 - c.k + c.ranks[c.m - 1]);
                    CHECK(d.L == alg6);
                }
                CHECK(d.check == ((flags & FLAG_NO_TERM) ? 0 : (flags & FLAG_ROUND) ? (d.j == c.m) : 1));
            }
            if (complete) CHECK(ns == c.k * c.m);
            check_pool(st, ns, grid);
            for (uint32_t g2 : {1u, 7u, 64u, 1280u, 1536u}) {
                for (uint32_t ops : {plain_sweep_ops(c.p), 700u}) {
                    StageDesc st2[BZ_MAX_STAGES];
                    int ns2 = build_schedule(c.p, c.k, c.m, c.ranks.data(), flags, ~0ull, g2, 2, BINOM, st2, &complete,
                                             true, ops);
                    check_pool(st2, ns2, g2);
                }
            }
        }
        // the work limit cuts the schedule before the stage that would exceed it
        StageDesc st[BZ_MAX_STAGES];
        int complete = 1;
        int ns = build_schedule(c.p, c.k, c.m, c.ranks.data(), 0, 1000, 64, 2, BINOM, st, &complete);
        u64 cum = 0;
        for (int s = 0; s < ns; s++) cum += st[s].codewords;
        CHECK(cum <= 1000);
        if (!complete && ns < BZ_MAX_STAGES) {
            u64 pw = 1;
            int g = ns / c.m + 1;
            for (int t = 1; t < g; t++) pw *= (u64)(c.p - 1);
            CHECK(cum + sat_mul(C(c.k, g), pw) > 1000);
        }
    }
    if (fails == before) std::printf("OK schedule\n");
}

// The decomposition kernel builds the schedule with one round g per lane (a
// saturating scan of the codewords of the rounds, then one stage per lane),
// the rounds' task counts from its own loop or from the per-shape table of the
// plain path; replayed here both ways, it gives the same table as build_schedule.
static int lane_parallel_schedule(int p, int k, int m, const int *ranks, int flags, u64 max_cw, uint32_t grid,
                                  int W, StageDesc *st, int *complete, uint32_t sweep_ops, bool table) {
    u64 cw[64], inc[64], tasks[64];
    uint32_t combos[64], vcaps[64];
    int js[64];
    for (int l = 0; l < 64; l++) {
        const int g = l + 1;
        const bool in = g <= k;
        cw[l] = in ? round_codewords(p, k, g, BINOM) : 0;
        const u64 cb = round_combos(p, g);
        combos[l] = (uint32_t)cb;
        const u64 mine = sat_mul(cw[l], (u64)m);
        inc[l] = l ? sat_add(inc[l - 1], mine) : mine;
        const u64 before = l ? inc[l - 1] : 0;
        js[l] = in ? round_stages(m, before, cw[l], cb, max_cw) : m;
        tasks[l] = (g <= SUBSET_G) ? small_stage_tasks(k, g) : 0;
        vcaps[l] = 0;
    }
    int ns = k * m;
    *complete = 1;
    for (int l = 0; l < k; l++)
        if (js[l] < m) {
            ns = l * m + js[l];
            *complete = 0;
            break;
        }
    const uint32_t cap = sweep_cap_for(p, W, sweep_ops);
    const int last_g = (ns + m - 1) / m;
    if (table) {
        // the plain path: the rounds' counts from the per-shape table
        static RoundTable rt;
        fill_round_table(p, k, W, grid, sweep_ops, BINOM, &rt);
        for (int g = SUBSET_G + 1; g <= last_g; g++) {
            if (g >= rt.cut_g) {
                ns = std::min(ns, (g - 1) * m);
                *complete = 0;
                break;
            }
            tasks[g - 1] = rt.tasks[g - 1];
            vcaps[g - 1] = rt.vcap[g - 1];
        }
    }
    for (int g = SUBSET_G + 1; g <= last_g && !table; g++) {
        // the kernel's per-q loop, with and without runs of bases (the digit
        // count from its table of digits_by_steps)
        const uint32_t budget = run_budget(p, cap);
        u64 t = 0, tv = 0;
        for (int q = g - 3; q <= k - 3; q++) {
            const u64 bases = sat_mul32(BINOM[q * 65 + (g - 3)], combos[g - 1]);
            const uint32_t nb = qgroup_blocks(k, cap, q);
            t = sat_add(t, qgroup_tasks(p, bases, nb, 0));
            tv = sat_add(tv, qgroup_tasks(p, bases, nb, digits_of(p, g, digits_by_steps(p, k, q, budget), bases)));
        }
        if (t >= (1ull << 62)) {
            ns = std::min(ns, (g - 1) * m);
            *complete = 0;
            break;
        }
        const bool runs = runs_pay(tv, grid);
        tasks[g - 1] = runs ? tv : t;
        vcaps[g - 1] = runs ? budget : 0u;
    }
    if (ns > BZ_MAX_STAGES) {
        ns = BZ_MAX_STAGES;
        *complete = 0;
    }
    // tiles of the rounds before each round: an inclusive saturating scan over
    // the lanes in the kernel's order (offsets 1, 2, 4, ...), then shifted by one
    u64 scan[64];
    for (int l = 0; l < 64; l++) scan[l] = (l < k) ? (tasks[l] + WAVES_PER_GROUP - 1) / WAVES_PER_GROUP : 0;
    for (int off = 1; off < 64; off <<= 1) {
        u64 nxt[64];
        for (int l = 0; l < 64; l++) nxt[l] = l >= off ? sat_add(scan[l], scan[l - off]) : scan[l];
        std::memcpy(scan, nxt, sizeof scan);
    }
    for (int s = 0; s < ns; s++) {
        const int g = s / m + 1, j = s % m + 1;
        int L = 0;
        for (int i = 1; i <= m; i++) L += bound_c(i <= j ? g : g - 1, k, ranks[i - 1]);
        StageDesc &d = st[s];
        d.g = g;
        d.j = j;
        d.L = L;
        d.check = (flags & FLAG_NO_TERM) ? 0 : ((flags & FLAG_ROUND) ? (j == m) : 1);
        d.tasks = tasks[g - 1];
        d.tiles = (d.tasks + WAVES_PER_GROUP - 1) / WAVES_PER_GROUP;
        d.codewords = cw[g - 1];
        d.coef_combos = combos[g - 1];
        d.parts = (uint32_t)(d.tiles < (u64)grid ? d.tiles : (u64)grid);
        d.sweep_cap = cap;
        d.vcap = vcaps[g - 1];
        d.pad = 0;
        const u64 off = deal_offset(m, g >= 2 ? scan[g - 2] : 0, j, d.tiles);
        d.nowait = off < (u64)grid;
        d.rot = deal_rot(off, grid);
    }
    return ns;
}

static void check_parallel_schedule() {
    const int before = fails;
    std::mt19937_64 rng(12345);
    int cases = 0;
    for (int it = 0; it < 4000; it++) {
        const int p = (rng() & 1) ? 3 : 7;
        const int k = 1 + (int)(rng() % 64);
        const int m = (it % 10 == 0) ? 1 + (int)(rng() % 128) : 1 + (int)(rng() % 6);
        std::vector<int> ranks(m);
        for (int i = 0; i < m; i++) ranks[i] = (int)(rng() % (k + 1));
        const int flags = (int)(rng() % 3) == 0 ? 0 : (int)(rng() % 3) == 0 ? (int)FLAG_ROUND : (int)FLAG_NO_TERM;
        u64 max_cw;
        switch (it % 5) {
        case 0: max_cw = ~0ull; break;
        case 1: max_cw = rng() % 100000; break;
        case 2: max_cw = 1ull << (rng() % 64); break;
        case 3: max_cw = rng(); break;
        default: max_cw = (1ull << 44); break;
        }
        const uint32_t grid = 1 + (uint32_t)(rng() % 2048);
        const int W = 1 + (int)(rng() % 4);
        static StageDesc a[BZ_MAX_STAGES], b[BZ_MAX_STAGES];
        int ca = -1, cb = -1;
        const uint32_t ops = (it % 3 == 0) ? DEFAULT_SWEEP_OPS : 500u + (uint32_t)(rng() % 20000);
        const int na = build_schedule(p, k, m, ranks.data(), flags, max_cw, grid, W, BINOM, a, &ca, true, ops);
        for (bool table : {false, true}) {
            const int nb = lane_parallel_schedule(p, k, m, ranks.data(), flags, max_cw, grid, W, b, &cb, ops, table);
            CHECK(na == nb && ca == cb);
            if (na != nb) {
                std::printf("  p=%d k=%d m=%d max=%llu table=%d: %d vs %d\n", p, k, m, (unsigned long long)max_cw,
                            (int)table, na, nb);
                continue;
            }
            for (int s = 0; s < na; s++) CHECK(std::memcmp(&a[s], &b[s], sizeof(StageDesc)) == 0);
        }
        cases++;
    }
    if (fails == before) std::printf("OK parallel schedule (%d cases)\n", cases);
}

// The kernel's work decomposition, replayed on the host: every g-row
// combination with lowest coefficient 1 is visited exactly once, and the
// per-task counts the kernel adds up equal the combinations visited.
static void check_unrank() {
    const int before = fails;
    int vd_seen[BZ_MAX_VD + 1] = {0, 0, 0, 0}, vd7_seen = 0;
    for (int P : {3, 7}) {
        for (int W : {1, 2, 4}) {
            for (int k = 3; k <= (P == 3 && W == 4 ? 13 : 10); k++) {
                for (int g = 1; g <= k && g <= (P == 3 && W == 4 ? 7 : 6); g++) {
                  // grid 1: every stage after the first waits (runs of bases);
                  // a huge grid: every stage starts at once (one base per lane)
                  for (uint32_t grid : {1u, 1u << 30}) {
                    StageDesc st[BZ_MAX_STAGES];
                    int complete;
                    int32_t ranks[1] = {k};
                    int ns = build_schedule(P, k, 1, ranks, FLAG_NO_TERM, ~0ull, grid, W, BINOM, st, &complete);
                    CHECK(ns == k);
                    const StageDesc &d = st[g - 1];
                    CHECK(d.vcap == ((g > SUBSET_G && grid == 1) ? d.sweep_cap : 0u));
                    std::map<std::vector<int>, int> seen;
                    u64 counted = 0;
                    auto add = [&](std::vector<int> rows, std::vector<int> coefs) {
                        // canonical key: rows ascending with their coefficients
                        std::vector<std::pair<int, int>> rc;
                        for (size_t i = 0; i < rows.size(); i++) rc.push_back({rows[i], coefs[i]});
                        std::sort(rc.begin(), rc.end());
                        std::vector<int> key;
                        for (auto &x : rc) { key.push_back(x.first); key.push_back(x.second); }
                        seen[key]++;
                    };
                    if (g == 1) {
                        for (u64 t = 0; t < d.tasks; t++)
                            for (int l = 0; l < 64; l++) {
                                int i = (int)(t * 64) + l;
                                if (i < k) { add({i}, {1}); counted++; }
                            }
                    } else if (g == 2) {
                        for (u64 t = 0; t < d.tasks; t++)
                            for (int l = 0; l < 64; l++) {
                                const int r = (int)(t * 64) + l;
                                if (r >= k * (k - 1) / 2) continue;
                                int s, L;
                                pair_of(r, k, &s, &L);
                                CHECK(0 <= s && s < L && L < k);
                                for (int h = 1; h < P; h++) { add({s, L}, {1, h}); counted++; }
                            }
                    } else if (g <= SUBSET_G) {
                        // one subset per lane, every coefficient vector with the lowest row's 1
                        CHECK(d.tasks == (C(k, g) + 63) / 64);
                        auto bin = [&](int c, int i) { return BINOM[c * 65 + i]; };
                        for (u64 t = 0; t < d.tasks; t++)
                            for (int l = 0; l < 64; l++) {
                                const u64 r = t * 64 + (u64)l;
                                if (r >= C(k, g)) continue;
                                std::vector<int> rows(g);
                                if (g == 3) {
                                    int rr[3];
                                    decode_subset<3>(r, k, bin, rr);
                                    rows.assign(rr, rr + 3);
                                } else {
                                    int rr[4];
                                    decode_subset<4>(r, k, bin, rr);
                                    rows.assign(rr, rr + 4);
                                }
                                for (int i = 0; i + 1 < g; i++) CHECK(rows[i] < rows[i + 1]);
                                CHECK(rows[0] >= 0 && rows[g - 1] < k);
                                std::vector<int> coefs(g, 1);
                                // coefficients of rows 1..g-1 in 1..P-1, as a counter
                                for (u64 cv = 0; cv < (u64)std::pow(P - 1, g - 1); cv++) {
                                    u64 x = cv;
                                    for (int i = 1; i < g; i++) { coefs[i] = (int)(x % (P - 1)) + 1; x /= (P - 1); }
                                    add(rows, coefs);
                                    counted++;
                                }
                            }
                    } else {
                        std::vector<QEntry> tab(BZ_MAX_K);
                        const u64 tasks = fill_qtable(P, k, g, d.coef_combos, d.sweep_cap, d.vcap, BINOM, tab.data());
                        CHECK(tasks == d.tasks);
                        const int nq = k - 2 - (g - 3);
                        for (u64 t = 0; t < d.tasks; t++) {
                            const int qi = qtable_find(tab.data(), nq, t);
                            const int q = g - 3 + qi;
                            const QEntry &e = tab[qi];
                            CHECK(e.first <= t && (qi + 1 == nq || tab[qi + 1].first > t));
                            const u64 local = t - e.first;
                            const u64 chunk = local / e.nb;
                            const int block = (int)(local - chunk * e.nb);
                            const int s_lo = q + 1 + qgroup_block_start(k, q, e.nb, (uint32_t)block);
                            const int s_hi = q + 1 + qgroup_block_start(k, q, e.nb, (uint32_t)block + 1);
                            CHECK(s_lo < s_hi && s_hi <= k - 1);
                            if (block == 0) CHECK(s_lo == q + 1);
                            if (block + 1 == (int)e.nb) CHECK(s_hi == k - 1);
                            // a lane's (s, L) steps in one task: at most one share of the
                            // group's total plus one row, or a single row
                            int steps = 0;
                            for (int s = s_lo; s < s_hi; s++) steps += k - 1 - s;
                            const int len = k - 2 - q, T = len * (len + 1) / 2;
                            CHECK(steps <= std::max(len, (T + (int)e.nb - 1) / (int)e.nb + len));
                            CHECK(s_hi - s_lo == 1 || steps <= 2 * (int)d.sweep_cap);
                            // a lane's run of (p-1)^vd bases: a whole group in one block,
                            // within the step budget, every lane's run inside the group
                            const int nv = (int)run_len(P, e.vd);
                            CHECK(e.vd <= max_digits(P) && (int)e.vd <= g - 3);
                            CHECK(nv == (int)std::pow(P - 1, (int)e.vd));
                            if (e.vd > 0) {
                                if (P == 3) vd_seen[e.vd]++;
                                else vd7_seen++;
                                CHECK(e.nb == 1 && (u64)nv * (u64)T <= d.sweep_cap);
                                CHECK(e.bases % (u64)nv == 0 && e.bases >= 64 * (u64)nv);
                            }
                            u64 nvalid = 0;
                            auto bin = [&](int c, int i) { return BINOM[c * 65 + i]; };
                            auto decode = [&](u64 bi, std::vector<int> &rows, std::vector<int> &coefs) {
                                rows.clear();
                                coefs.clear();
                                auto visit = [&](int row, int coef) { rows.push_back(row); coefs.push_back(coef); };
                                if (P == 3) decode_base<3>(g, q, d.coef_combos, bi, bin, visit);
                                else decode_base<7>(g, q, d.coef_combos, bi, bin, visit);
                            };
                            for (int l = 0; l < 64; l++) {
                                const u64 bi0 = (chunk * 64 + (u64)l) * (u64)nv;
                                if (bi0 >= e.bases) continue;
                                // the kernel's walk: decode the first base, then per step v
                                // F_3: flip digit t = ctz(v) (coefficient 1 -> 2 or 2 -> 1 of
                                // the t-th decoded row); F_7: add 1 to the coefficient of the
                                // top row.  The walk must meet the decodings of bi0 ..
                                // bi0 + (p-1)^vd - 1, each once
                                std::vector<int> rows, coefs, r1, c1;
                                decode(bi0, rows, coefs);
                                std::set<std::vector<int>> walked, direct;
                                uint32_t cur = 0;
                                for (int v = 0; v < nv; v++) {
                                    if (v > 0 && P == 3) {
                                        const int t = __builtin_ctz((uint32_t)v);
                                        const int h = ((cur >> t) & 1u) ? 2 : 1;
                                        cur ^= 1u << t;
                                        coefs[t] = (coefs[t] + h) % 3;
                                    }
                                    if (v > 0 && P == 7) coefs[0] = (coefs[0] + 1) % 7;
                                    nvalid++;
                                    decode(bi0 + (u64)v, r1, c1);
                                    CHECK(r1 == rows);
                                    walked.insert(coefs);
                                    direct.insert(c1);
                                    CHECK((int)rows.size() == g - 2);
                                    CHECK(rows[0] == q);
                                    for (size_t i = 1; i < rows.size(); i++) CHECK(rows[i] < rows[i - 1]);
                                    // the kernel's last-row sweep (the same loop, groups of
                                    // UR rows), each row with every coefficient a of row s and
                                    // every multiplier h; the count is taken from the rows the
                                    // sweep combined, as the kernel takes it
                                    for (int s = s_lo; s < s_hi; s++) {
                                        auto group = [&](int L0, int nr) {
                                            for (int u = 0; u < nr; u++)
                                                for (int a = 1; a < P; a++)
                                                    for (int h = 1; h < P; h++) {
                                                        std::vector<int> r2(rows), c2(coefs);
                                                        r2.push_back(s); c2.push_back(a);
                                                        r2.push_back(L0 + u); c2.push_back(h);
                                                        add(r2, c2);
                                                    }
                                        };
                                        const int done = (W <= 2) ? sweep_last_rows<4>(s, k, group)
                                                                  : sweep_last_rows<2>(s, k, group);
                                        counted += (u64)((P - 1) * (P - 1)) * (u64)done;
                                    }
                                }
                                CHECK(walked == direct && (int)walked.size() == nv);
                            }
                            (void)nvalid;
                        }
                    }
                    u64 expect = C(k, g);
                    for (int t = 1; t < g; t++) expect *= (u64)(P - 1);
                    CHECK((u64)seen.size() == expect);
                    CHECK(counted == expect);
                    for (auto &kv : seen) {
                        CHECK(kv.second == 1);
                        CHECK(kv.first[1] == 1);  // coefficient of the lowest row
                    }
                  }
                }
            }
        }
    }
    // every run length occurred (F_3 at W = 4 has the smallest step budget)
    for (int v = 1; v <= BZ_MAX_VD; v++) CHECK(vd_seen[v] > 0);
    CHECK(vd7_seen > 0);
    if (fails == before) std::printf("OK unrank\n");
}

// Bit helpers of the decomposition against plain definitions: compress (the
// masked bits of x in order, to the low end), the saturating products and
// powers against step-by-step saturation.
// The digit count of a run of bases (closed form) against its definition: the
// largest d <= min(g-3, 3) (F_3; 1 for F_7) with T (p-1)^d <= vcap and
// bases >= 64 (p-1)^d.
static void check_digits() {
    const int before = fails;
    std::mt19937_64 rng(99);
    for (int it = 0; it < 200000; it++) {
        const int k = 4 + (int)(rng() % 61), g = 3 + (int)(rng() % 12), q = (int)(rng() % (k - 2));
        const uint32_t vcap = (it % 7 == 0) ? 0u : 1u + (uint32_t)(rng() % 5000);
        const u64 bases = (it % 3 == 0) ? rng() >> (rng() % 64) : rng() % 4096;
        const uint32_t len = (uint32_t)(k - 2 - q), T = len * (len + 1) / 2;
        uint32_t d = 0;
        if (vcap)
            while ((int)d < std::min(g - 3, BZ_MAX_VD) && (u64)T << (d + 1) <= vcap && (bases >> (d + 1)) >= 64) d++;
        CHECK(qgroup_digits(3, k, g, vcap, q, bases) == d);
        // F_7: one digit at most (6 bases per lane)
        const uint32_t d7 = (vcap && g >= 4 && 6ull * T <= vcap && bases >= 384) ? 1u : 0u;
        CHECK(qgroup_digits(7, k, g, vcap, q, bases) == d7);
    }
    if (fails == before) std::printf("OK digits\n");
}

static void check_bits() {
    const int before = fails;
    std::mt19937_64 rng(777);
    for (int it = 0; it < 200000; it++) {
        u32 x = (u32)rng(), m = (u32)rng();
        if (it % 4 == 1) m &= (u32)rng();
        if (it % 4 == 2) m |= (u32)rng();
        if (it % 97 == 0) m = 0;
        if (it % 89 == 0) m = ~0u;
        u32 want = 0;
        int o = 0;
        for (int i = 0; i < 32; i++)
            if ((m >> i) & 1u) want |= ((x >> i) & 1u) << o++;
        CHECK(compress_apply(x, m, compress_plan(m)) == want);
    }
    for (int it = 0; it < 200000; it++) {
        const u64 a = rng() >> (rng() % 64);
        const uint32_t b = (uint32_t)(rng() >> (rng() % 32 + 32));
        CHECK(sat_mul32(a, b) == sat_mul(a, (u64)b));
    }
    for (int p : {3, 7})
        for (int e = -2; e <= 70; e++) {
            u64 r = 1;
            for (int t = 0; t < e; t++) r = sat_mul(r, (u64)(p - 1));
            CHECK(pow_sat(p, e) == r);
        }
    if (fails == before) std::printf("OK bits\n");
}

// The blocks of rows s of every q-group: they partition the rows in order,
// none is empty, and each holds at most one share of the group's steps plus
// one row (or is a single row).
static void check_blocks() {
    const int before = fails;
    for (int k = 3; k <= 64; k++)
        for (int q = 0; q <= k - 3; q++)
            for (uint32_t cap : {1u, 2u, 4u, 7u, 17u, 57u, 115u, 300u, 2000u, 100000u}) {
                const uint32_t nb = qgroup_blocks(k, cap, q);
                const int len = k - 2 - q, T = len * (len + 1) / 2;
                CHECK(nb >= 1 && (int)nb <= len);
                CHECK((int)nb == std::min(len, (T + (int)cap - 1) / (int)cap));
                int prev = qgroup_block_start(k, q, nb, 0);
                CHECK(prev == 0);
                for (uint32_t b = 1; b <= nb; b++) {
                    const int st = qgroup_block_start(k, q, nb, b);
                    CHECK(st > prev);
                    int steps = 0;
                    for (int i = prev; i < st; i++) steps += len - i;
                    CHECK(st - prev == 1 || steps <= (T + (int)nb - 1) / (int)nb + len);
                    prev = st;
                }
                CHECK(prev == len);
            }
    if (fails == before) std::printf("OK blocks\n");
}

// Pair tables: the walk of pair_advance visits the pairs s < L row-major in s,
// each once, at index pair_first(s, k) + (L - s - 1), from any start and in
// steps of one or of 64; the pairs of a block of rows s of a q-group are the
// index range [pair_first(s_lo), pair_first(s_hi)), consecutive blocks abut,
// and a table holds exactly units x W x pairs entries.
static void check_pairs() {
    const int before = fails;
    for (int k = 1; k <= 64; k++) {
        const int np = k * (k - 1) / 2;
        CHECK(pair_first(k - 1, k) == (u64)np && pair_first(0, k) == 0);
        int s = 0, rem = 0, e = 0;
        pair_advance(k, s, rem, 0);
        for (int a = 0; a < k; a++)
            for (int b = a + 1; b < k; b++, e++) {
                CHECK(s == a && s + 1 + rem == b);
                CHECK(pair_first(a, k) + (u64)(b - a - 1) == (u64)e);
                pair_advance(k, s, rem, 1);
            }
        CHECK(e == np);
        for (int t = 0; t < 64; t++) {
            int s2 = 0, r2 = 0;
            pair_advance(k, s2, r2, t);
            for (int e2 = t; e2 < np; e2 += 64) {
                const int L = s2 + 1 + r2;
                CHECK(s2 < L && L < k && pair_first(s2, k) + (u64)r2 == (u64)e2);
                pair_advance(k, s2, r2, 64);
            }
        }
        for (int p : {3, 7})
            for (int W = 1; W <= 4; W++)
                CHECK(pair_table_units(p, k, W) == (u64)np * (u64)(p == 3 ? 1 : 6) * (u64)W);
        for (int q = 0; q <= k - 3; q++)
            for (uint32_t cap : {1u, 7u, 57u, 2000u}) {
                const uint32_t nb = qgroup_blocks(k, cap, q);
                u64 prev = pair_first(q + 1, k);
                for (uint32_t b = 0; b < nb; b++) {
                    const int lo = q + 1 + qgroup_block_start(k, q, nb, b);
                    const int hi = q + 1 + qgroup_block_start(k, q, nb, b + 1);
                    u64 want = 0;
                    for (int r = lo; r < hi; r++) want += (u64)(k - 1 - r);
                    CHECK(pair_first(lo, k) == prev && pair_first(hi, k) - pair_first(lo, k) == want);
                    prev = pair_first(hi, k);
                }
                CHECK(prev == (u64)np);
            }
    }
    for (int n = 1; n <= BZ_MAX_N; n++)
        for (int k = 1; k <= n && k <= BZ_MAX_K; k++) CHECK(pair_sets(n, k) >= 1 && pair_sets(n, k) * k >= n);
    // a pair's units cover its (p-1)^2 coefficient pairs once each: unit c
    // holds R_s + c R_L (F_3: c = 1 and c = 2 = -1 in one unit), and a lane
    // takes Q + h T_c for every h in F_p^*, i.e. coefficients (h, h c) on (s, L)
    for (int P : {3, 7}) {
        std::vector<int> seen(P * P, 0);
        for (int c = 1; c < P; c++)
            for (int h = 1; h < P; h++) seen[h * P + (h * c) % P]++;
        for (int hs = 1; hs < P; hs++)
            for (int hl = 1; hl < P; hl++) CHECK(seen[hs * P + hl] == 1);
        CHECK((int)pair_units(P) * (P == 3 ? 2 : 1) == P - 1);
    }
    if (fails == before) std::printf("OK pairs\n");
}

// The next row of a colex unranking (direct for i = 1, a table search above)
// against a plain scan for the largest c with C(c, i) <= rho.
static void check_top_row() {
    const int before = fails;
    auto bin = [](int c, int i) { return BINOM[c * 65 + i]; };
    std::mt19937_64 rng(99);
    for (int i = 1; i <= 6; i++)
        for (int hi = i - 1; hi <= 63; hi++) {
            const u64 lim = BINOM[(hi + 1) * 65 + i];  // rho < C(hi + 1, i)
            for (int it = 0; it < 300; it++) {
                u64 rho = (it < 100 && (u64)it < lim) ? (u64)it : (lim > 1 ? rng() % lim : 0);
                if (it == 299) rho = lim - 1;
                int want = i - 1;
                for (int c = i - 1; c <= hi; c++)
                    if (BINOM[c * 65 + i] <= rho) want = c;
                CHECK(top_row(rho, i, hi, bin) == want);
            }
        }
    if (fails == before) std::printf("OK top row\n");
}

int main() {
    fill_binomials(BINOM);
    check_top_row();
    check_bits();
    check_blocks();
    check_pairs();
    check_digits();
    for (int a = 0; a <= 64; a++)
        for (int b = 0; b <= 64; b++) CHECK(binom_sat(a, b) == ~0ull || BINOM[a * 65 + b] == binom_sat(a, b));
    check_arith();
    check_schedule();
    check_parallel_schedule();
    check_unrank();
    return fails ? 1 : 0;
}
