// Host-side checks of the library's shared (host/device) code, built with g++.
//
//   arith     exhaustive: every pair of symbols, at every bit position of a
//             word, through the bit-sliced F_3 / F_7 functions, against
//             plain mod-p integers
//   schedule  stage counts, work items, chunk accounting and bounds L_{g,j}
//   unrank    the work decomposition visits every g-row combination with the
//             lowest coefficient 1 exactly once
//
// Prints "OK <check>" per passing check; exits 1 on the first failure.
#include <cstdio>
#include <cstdlib>
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
            u64 total = 0;
            int ns = build_schedule(c.p, c.k, c.m, c.ranks.data(), flags, ~0ull, 64, st, &complete, &total);
            u64 chunk = 0, cum = 0;
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
                CHECK(d.chunk_begin == chunk);
                CHECK(d.n_chunks * d.items_per_chunk >= d.items && (d.n_chunks - 1) * d.items_per_chunk < d.items);
                chunk += d.n_chunks;
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
            CHECK(chunk == total);
            if (complete) CHECK(ns == c.k * c.m);
        }
        // the work limit cuts the schedule before the stage that would exceed it
        StageDesc st[BZ_MAX_STAGES];
        int complete = 1;
        u64 total = 0;
        int ns = build_schedule(c.p, c.k, c.m, c.ranks.data(), 0, 1000, 64, st, &complete, &total);
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

static void check_unrank() {
    const int before = fails;
    static u64 binom[65 * 65];
    for (int a = 0; a <= 64; a++)
        for (int b = 0; b <= 64; b++) binom[a * 65 + b] = C(a, b);
    for (int P : {3, 7}) {
        for (int k = 3; k <= 9; k++) {
            for (int g = 3; g <= k && g <= 6; g++) {
                StageDesc st[BZ_MAX_STAGES];
                int complete;
                u64 total;
                int32_t ranks[1] = {k};
                int ns = build_schedule(P, k, 1, ranks, FLAG_NO_TERM, ~0ull, 64, st, &complete, &total);
                CHECK(ns == k);
                const StageDesc &d = st[g - 1];
                std::map<std::vector<int>, int> seen;  // (rows..., coefs...) -> count
                for (u64 item = 0; item < d.items; item++) {
                    const u64 sr = item / d.coef_combos;
                    u32 ci = (u32)(item - sr * d.coef_combos);
                    std::vector<int> rows(g - 2), coef(g - 2);
                    int q = -1;
                    colex_unrank(sr, g - 2, k - 3, binom, [&](int i, int c) {
                        rows[i - 1] = c;
                        int h = 1;
                        if (i > 1) {
                            h = (int)(ci % (u32)(P - 1)) + 1;
                            ci /= (u32)(P - 1);
                        }
                        coef[i - 1] = h;
                        if (i == g - 2) q = c;
                    });
                    for (int i = 1; i < g - 2; i++) CHECK(rows[i - 1] < rows[i]);
                    // extensions as the kernel makes them: row s with every nonzero
                    // coefficient, last row L with every nonzero multiplier
                    for (int s = q + 1; s < k - 1; s++)
                        for (int a = 1; a < P; a++)
                            for (int L = s + 1; L < k; L++)
                                for (int h = 1; h < P; h++) {
                                    std::vector<int> key(rows);
                                    key.push_back(s);
                                    key.push_back(L);
                                    key.insert(key.end(), coef.begin(), coef.end());
                                    key.push_back(a);
                                    key.push_back(h);
                                    seen[key]++;
                                }
                }
                // every g-subset, lowest coefficient 1, others nonzero: exactly once
                u64 expect = C(k, g);
                for (int t = 1; t < g; t++) expect *= (u64)(P - 1);
                CHECK((u64)seen.size() == expect);
                for (auto &kv : seen) {
                    CHECK(kv.second == 1);
                    CHECK(kv.first[g] == 1);  // the coefficient of the lowest row
                }
            }
        }
    }
    if (fails == before) std::printf("OK unrank\n");
}

int main() {
    check_arith();
    check_schedule();
    check_unrank();
    return fails ? 1 : 0;
}
