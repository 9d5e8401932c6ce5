// bz_kernels.hpp -- gfx950 kernels of the Brouwer-Zimmermann path.
//
//   decompose_kernel  one wavefront per code: validates G, packs it into bit
//                     planes, computes the information-set decomposition
//                     Gamma_1..Gamma_m by Gauss-Jordan on bit-sliced rows (one
//                     row per lane), packs each Gamma_j for the enumeration, and
//                     writes the stage schedule and the initial queue state.
//   enum_kernel       persistent: every wavefront pulls chunks of work from a
//                     global queue that runs through the stages in order,
//                     builds exact prefix sums in registers, finishes every
//                     combination with the isometric addition, takes the weight
//                     by popcount and min-reduces it; the wavefront that
//                     completes a stage's last chunk applies the L >= U test and
//                     stops the queue when it holds.
//
// Paper: Hernando & Quintana-Orti, arXiv 2603.29942 (Sec. 2-4, Algorithm 6).
#pragma once
#include <hip/hip_runtime.h>

#include "bz_arith.hpp"
#include "bz_state.hpp"

namespace bz {

constexpr u32 BIG = 0x7fffffffu;

__device__ __forceinline__ u32 uni(u32 x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ u64 uni64(u64 x) {
    u32 lo = __builtin_amdgcn_readfirstlane((u32)x);
    u32 hi = __builtin_amdgcn_readfirstlane((u32)(x >> 32));
    return ((u64)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T ld_acq(T *p) {
    return __hip_atomic_load(p, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_rel(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
}

// select word q of a small register array with a uniform index (no dynamic
// register indexing)
template <int N>
__device__ __forceinline__ u32 pick(const u32 (&a)[N], int q) {
    u32 v = a[0];
#pragma unroll
    for (int i = 1; i < N; i++) v = (q == i) ? a[i] : v;
    return v;
}

// =====================================================================
// Decomposition: one wavefront per code, lane i holds row i.
// =====================================================================
struct RunArgs {
    int32_t n, k, flags, U0;
    u64 max_codewords;
    u64 target_chunks;
};

template <int P, int WF>
__global__ __launch_bounds__(64) void decompose_kernel(const uint8_t *__restrict__ G, CodeState *cs,
                                                       u32 *__restrict__ rows, RunArgs args) {
    constexpr int R = (P == 3) ? 2 : 3;
    const int lane = threadIdx.x;
    const int n = args.n, k = args.k, flags = args.flags;
    const u64 target_chunks = args.target_chunks;
    CodeResult &res = cs->res;
    if (lane == 0) {
        cs->p = P;
        cs->n = n;
        cs->k = k;
        cs->flags = flags;
        cs->U0 = args.U0;
        cs->max_codewords = args.max_codewords;
    }

    // -- load G: lanes walk 64 columns of one row, ballots transpose the bits
    u32 x[3][4];
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
        for (int w = 0; w < 4; w++) x[b][w] = 0;
    bool bad = false;
    for (int i = 0; i < k; i++) {
#pragma unroll
        for (int cb = 0; cb < WF; cb += 2) {
            const int c = cb * 32 + lane;
            const int v = (c < n) ? (int)G[(size_t)i * n + c] : 0;
            bad |= (v >= P);
#pragma unroll
            for (int b = 0; b < R; b++) {
                const u64 msk = __ballot((v >> b) & 1);
                if (lane == i) {
                    x[b][cb] = (u32)msk;
                    if (cb + 1 < WF) x[b][cb + 1] = (u32)(msk >> 32);
                }
            }
        }
    }
    u32 colmask[4];
#pragma unroll
    for (int w = 0; w < 4; w++) {
        const int lo = w * 32;
        colmask[w] = (n >= lo + 32) ? 0xffffffffu : (n > lo ? ((1u << (n - lo)) - 1u) : 0u);
    }

    int status = BZ_OK;
    if (__any(bad)) status = BZ_ERR_VALUE;

    int m = 0;
    u32 used[4] = {0, 0, 0, 0};
    const bool skip = (flags & FLAG_SKIP) != 0;
    const int W = skip ? (n - k + 31) / 32 : WF;

    while (status == BZ_OK) {
        u32 unused[4];
        bool anyu = false;
#pragma unroll
        for (int w = 0; w < 4; w++) {
            unused[w] = colmask[w] & ~used[w];
            anyu |= unused[w] != 0;
        }
        if (!anyu) break;
        int piv_lane = -1, npiv = 0, kj = 0;
        u32 pivmask[4] = {0, 0, 0, 0};
        for (int pass = 0; pass < 2 && npiv < k; pass++) {
#pragma unroll
            for (int w = 0; w < WF; w++) {
                u32 bits = pass == 0 ? unused[w] : (colmask[w] & used[w]);
                while (bits && npiv < k) {
                    const int t = __builtin_ctz(bits);
                    bits &= bits - 1;
                    int v = 0;
#pragma unroll
                    for (int b = 0; b < R; b++) v |= (int)((x[b][w] >> t) & 1u) << b;
                    const bool cand = lane < k && piv_lane < 0 && v != 0;
                    const u64 cm = __ballot(cand);
                    if (cm == 0) continue;
                    const int pl = __ffsll((unsigned long long)cm) - 1;
                    const int pv = __shfl(v, pl);
                    const int inv = inv_mod(P, pv);
                    // normalised pivot row, wave-uniform
                    u32 pr[3][4];
#pragma unroll
                    for (int ww = 0; ww < WF; ww++) {
                        u32 raw[3] = {0, 0, 0}, sc[3] = {0, 0, 0};
#pragma unroll
                        for (int b = 0; b < R; b++) raw[b] = __shfl(x[b][ww], pl);
                        scale<P>(inv, raw, sc);
#pragma unroll
                        for (int b = 0; b < 3; b++) pr[b][ww] = sc[b];
                    }
                    if (lane == pl) {
#pragma unroll
                        for (int ww = 0; ww < WF; ww++)
#pragma unroll
                            for (int b = 0; b < R; b++) x[b][ww] = pr[b][ww];
                        piv_lane = npiv;
                    } else if (v != 0) {
                        // row -= v * pivot  ==  row + (p - v) * pivot
#pragma unroll
                        for (int ww = 0; ww < WF; ww++) {
                            u32 src[3] = {pr[0][ww], pr[1][ww], pr[2][ww]}, sc[3] = {0, 0, 0};
                            scale<P>(P - v, src, sc);
                            if (P == 3) {
                                f3_add(x[0][ww], x[1][ww], sc[0], sc[1], x[0][ww], x[1][ww]);
                            } else {
                                f7_add(x[0][ww], x[1][ww], x[2][ww], sc[0], sc[1], sc[2], x[0][ww],
                                       x[1][ww], x[2][ww]);
                            }
                        }
                    }
                    npiv++;
                    if (pass == 0) kj++;
                    pivmask[w] |= 1u << t;
                }
            }
        }
        if (npiv < k) {
            status = BZ_ERR_RANK;
            break;
        }
        if (kj == 0) break;
        // -- pack Gamma_m: row piv_lane of matrix m
        if (lane < k) {
            u32 *dst = rows + ((size_t)(m * BZ_MAX_K + piv_lane) * 3) * 4;
            if (skip) {
                u32 out[3][4];
#pragma unroll
                for (int b = 0; b < 3; b++)
#pragma unroll
                    for (int w = 0; w < 4; w++) out[b][w] = 0;
                int ob = 0;
#pragma unroll
                for (int w = 0; w < WF; w++) {
                    u32 bits = colmask[w] & ~pivmask[w];
                    while (bits) {
                        const int t = __builtin_ctz(bits);
                        bits &= bits - 1;
                        const int q = ob >> 5, sh = ob & 31;
#pragma unroll
                        for (int b = 0; b < R; b++) {
                            const u32 bit = ((x[b][w] >> t) & 1u) << sh;
#pragma unroll
                            for (int qq = 0; qq < 4; qq++)
                                if (qq == q) out[b][qq] |= bit;
                        }
                        ob++;
                    }
                }
#pragma unroll
                for (int b = 0; b < 3; b++)
#pragma unroll
                    for (int w = 0; w < 4; w++) dst[b * 4 + w] = out[b][w];
            } else {
#pragma unroll
                for (int b = 0; b < 3; b++)
#pragma unroll
                    for (int w = 0; w < 4; w++) dst[b * 4 + w] = (w < WF) ? x[b][w] : 0u;
            }
        }
        if (lane == 0) res.ranks[m] = kj;
        m++;
#pragma unroll
        for (int w = 0; w < 4; w++) used[w] |= pivmask[w] & unused[w];
        if (kj < k || m == BZ_MAX_M) break;
    }
    __syncthreads();  // ranks written by lane 0 are read back below by lane 0 only

    // -- schedule and queue state
    if (lane == 0) {
        res.status = status;
        res.m = m;
        res.W = W;
        res.term_stage = -1;
        res.checked = 0;
        cs->next_chunk = 0;
        int complete = 1;
        u64 total = 0;
        int ns = 0;
        if (status == BZ_OK) {
            const bool no_term = (flags & FLAG_NO_TERM) != 0;
            if (no_term || args.U0 > 1)
                ns = build_schedule(P, k, m, res.ranks, flags, args.max_codewords, target_chunks, cs->stages,
                                    &complete, &total);
        }
        res.n_table = ns;
        res.table_complete = complete;
        cs->total_chunks = total;
    }
    __syncthreads();
    const int ns = res.n_table;
    for (int s = lane; s < ns; s += 64) {
        res.stage_min[s] = (int)BIG;
        res.stage_count[s] = 0;
        cs->stage_done[s] = 0;
        cs->U_after[s] = 0;
    }
}

// =====================================================================
// Enumeration
// =====================================================================

// weights of the 2 (F_3) or 6 (F_7) completions of prefix Pv by row Rl
template <int P, int W, bool HIST>
__device__ __forceinline__ void complete(const u32 (&Pv)[3][W], const u32 (&anyP)[W], const u32 (&Rl)[3][W],
                                         u32 &lmin, u32 *lh, u32 woff) {
    if constexpr (P == 3) {
        u32 wa = 0, ws = 0;
#pragma unroll
        for (int w = 0; w < W; w++) {
            wa += __builtin_popcount(f3_iso_add(Pv[0][w], Pv[1][w], Rl[0][w], Rl[1][w]));
            ws += __builtin_popcount(f3_iso_sub(Pv[0][w], Pv[1][w], Rl[0][w], Rl[1][w]));
        }
        lmin = min(lmin, min(wa, ws));
        if constexpr (HIST) {
            atomicAdd(&lh[wa + woff], 1u);
            atomicAdd(&lh[ws + woff], 1u);
        }
    } else {
        u32 anyPR[W];
#pragma unroll
        for (int w = 0; w < W; w++) anyPR[w] = anyP[w] | Rl[0][w] | Rl[1][w] | Rl[2][w];
#pragma unroll
        for (int e = 0; e < 3; e++) {
            u32 wa = 0, ws = 0;
#pragma unroll
            for (int w = 0; w < W; w++) {
                // rotation by e: S_i = R_{i-e}  (times 2^e, Sec. 4.2)
                const u32 s0 = Rl[(3 - e) % 3][w], s1 = Rl[(4 - e) % 3][w], s2 = Rl[(5 - e) % 3][w];
                const u32 x0 = Pv[0][w] ^ s0, x1 = Pv[1][w] ^ s1, x2 = Pv[2][w] ^ s2;
                ws += __builtin_popcount(x0 | x1 | x2);             // P - 2^e R
                wa += __builtin_popcount(~(x0 & x1 & x2) & anyPR[w]);  // P + 2^e R
            }
            lmin = min(lmin, min(wa, ws));
            if constexpr (HIST) {
                atomicAdd(&lh[wa + woff], 1u);
                atomicAdd(&lh[ws + woff], 1u);
            }
        }
    }
}

template <int P, int W>
__device__ __forceinline__ void load_row(const u32 *__restrict__ rows, int j, int i, u32 (&r)[3][W]) {
    const u32 *src = rows + ((size_t)(j * BZ_MAX_K + i) * 3) * 4;
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
        for (int w = 0; w < W; w++) r[b][w] = (b < ((P == 3) ? 2 : 3)) ? src[b * 4 + w] : 0u;
}

template <int P, int W>
__device__ __forceinline__ void add_scaled(u32 (&x)[3][W], const u32 (&r)[3][W], int h) {
#pragma unroll
    for (int w = 0; w < W; w++) {
        u32 src[3] = {r[0][w], r[1][w], r[2][w]}, sc[3] = {0, 0, 0};
        scale<P>(h, src, sc);
        if constexpr (P == 3) f3_add(x[0][w], x[1][w], sc[0], sc[1], x[0][w], x[1][w]);
        else f7_add(x[0][w], x[1][w], x[2][w], sc[0], sc[1], sc[2], x[0][w], x[1][w], x[2][w]);
    }
}

template <int W>
__device__ __forceinline__ void any_planes(const u32 (&x)[3][W], u32 (&a)[W]) {
#pragma unroll
    for (int w = 0; w < W; w++) a[w] = x[0][w] | x[1][w] | x[2][w];
}

// the lane's combinations of one chunk; returns the number of combinations
// the wavefront evaluated (wave-uniform)
template <int P, int W, bool HIST>
__device__ u64 run_chunk(const StageDesc &sd, int k, int j, const u32 *__restrict__ rows,
                         const u64 *__restrict__ binom, u64 first, u64 last, u32 &lmin, u32 *lh, u32 woff) {
    const int lane = __lane_id();
    const int g = sd.g;
    u64 cnt = 0;
    for (u64 base = first; base < last; base += 64) {
        const u64 item = base + (u64)lane;
        const bool valid = item < last;
        if (g == 1) {
            if (valid) {
                u32 r[3][W], a[W];
                load_row<P, W>(rows, j, (int)item, r);
                any_planes<W>(r, a);
                u32 wt = 0;
#pragma unroll
                for (int w = 0; w < W; w++) wt += __builtin_popcount(a[w]);
                lmin = min(lmin, wt);
                if constexpr (HIST) atomicAdd(&lh[wt + woff], 1u);
            }
            cnt += (u64)__popcll(__ballot(valid));
            continue;
        }
        int q;  // highest row of the lane's prefix
        u32 Q[3][W], anyQ[W];
        if (g == 2) {
            q = valid ? (int)item : k;
            if (valid) load_row<P, W>(rows, j, q, Q);
            else {
#pragma unroll
                for (int b = 0; b < 3; b++)
#pragma unroll
                    for (int w = 0; w < W; w++) Q[b][w] = 0;
            }
            any_planes<W>(Q, anyQ);
            const int qmin = uni(q);
            for (int L = qmin + 1; L < k; L++) {
                const bool act = valid && L > q;
                u32 Rl[3][W];
                load_row<P, W>(rows, j, uni(L), Rl);
                if (act) complete<P, W, HIST>(Q, anyQ, Rl, lmin, lh, woff);
                cnt += (u64)(P - 1) * (u64)__popcll(__ballot(act));
            }
            continue;
        }
        // g >= 3: base of g-2 rows c_1 < ... < c_{g-2} from colex rank sr,
        // coefficients of c_2.. from the digits of ci in base p-1
        const int t = g - 2;
        const u32 M = sd.coef_combos;
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
            for (int w = 0; w < W; w++) Q[b][w] = 0;
        q = k;
        if (valid) {
            const u64 sr = item / M;
            u32 ci = (u32)(item - sr * M);
            colex_unrank(sr, t, k - 3, binom, [&](int i, int c) {
                u32 r[3][W];
                load_row<P, W>(rows, j, c, r);
                int coef = 1;
                if (i > 1) {
                    coef = (int)(ci % (u32)(P - 1)) + 1;
                    ci /= (u32)(P - 1);
                }
                if (i == t) {
                    q = c;
#pragma unroll
                    for (int w = 0; w < W; w++) {
                        u32 src[3] = {r[0][w], r[1][w], r[2][w]}, sc[3] = {0, 0, 0};
                        scale<P>(coef, src, sc);
#pragma unroll
                        for (int b = 0; b < 3; b++) Q[b][w] = sc[b];
                    }
                } else {
                    add_scaled<P, W>(Q, r, coef);
                }
            });
        }
        const int qmin = uni(q);
        for (int s = qmin + 1; s < k - 1; s++) {
            const bool act = valid && s > q;
            const u64 nact = (u64)__popcll(__ballot(act));
            if (nact == 0) continue;
            u32 Rs[3][W];
            load_row<P, W>(rows, j, uni(s), Rs);
            for (int a = 1; a < P; a++) {
                u32 Pv[3][W], anyP[W];
#pragma unroll
                for (int b = 0; b < 3; b++)
#pragma unroll
                    for (int w = 0; w < W; w++) Pv[b][w] = Q[b][w];
                add_scaled<P, W>(Pv, Rs, a);
                any_planes<W>(Pv, anyP);
                for (int L = s + 1; L < k; L++) {
                    u32 Rl[3][W];
                    load_row<P, W>(rows, j, uni(L), Rl);
                    if (act) complete<P, W, HIST>(Pv, anyP, Rl, lmin, lh, woff);
                    cnt += (u64)(P - 1) * nact;
                }
            }
        }
    }
    return cnt;
}

// stage-completion check (lane 0 of a wavefront): advance over every stage
// whose chunks are all done, in stage order, applying L_{g,j} >= U
__device__ void run_checker(CodeState *cs) {
    const int ns = cs->res.n_table;
    for (int guard = 0; guard <= BZ_MAX_STAGES; guard++) {
        const int c = ld_acq(&cs->res.checked);
        if (c >= ns) return;
        if (ld_acq(&cs->res.term_stage) >= 0) return;
        if (ld_acq(&cs->stage_done[c]) != cs->stages[c].n_chunks) return;
        const int Uprev = (c == 0) ? cs->U0 : ld_acq(&cs->U_after[c - 1]);
        const int smin = ld_acq(&cs->res.stage_min[c]);
        const int Uc = min(Uprev, smin);
        st_rel(&cs->U_after[c], Uc);
        if (cs->stages[c].check && cs->stages[c].L >= Uc) {
            int expect = -1;
            __hip_atomic_compare_exchange_strong(&cs->res.term_stage, &expect, c, __ATOMIC_SEQ_CST,
                                                 __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        int expect = c;
        __hip_atomic_compare_exchange_strong(&cs->res.checked, &expect, c + 1, __ATOMIC_SEQ_CST,
                                             __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int P, int W, bool HIST>
__global__ __launch_bounds__(256) void enum_kernel(CodeState *cs, const u32 *__restrict__ rows,
                                                   const u64 *__restrict__ binom, u64 *__restrict__ hist) {
    __shared__ u32 lhist[HIST ? 4 * (BZ_MAX_N + 1) : 1];
    const int lane = __lane_id();
    const int wid = threadIdx.x >> 6;
    if (cs->res.status != BZ_OK) return;
    const int k = cs->k, n = cs->n;
    const int ns = cs->res.n_table;
    const u64 total = cs->total_chunks;
    const bool skip = (cs->flags & FLAG_SKIP) != 0;
    u32 *lh = HIST ? &lhist[wid * (BZ_MAX_N + 1)] : nullptr;
    int s = 0;
    for (;;) {
        u64 ch = 0;
        if (lane == 0) ch = atomicAdd((unsigned long long *)&cs->next_chunk, 1ull);
        ch = uni64(__shfl(ch, 0));
        if (ch >= total) break;
        while (s + 1 < ns && cs->stages[s + 1].chunk_begin <= ch) s++;
        s = uni(s);
        const int term = uni(ld_acq(&cs->res.term_stage));
        if (term >= 0 && s > term) break;
        const StageDesc sd = cs->stages[s];
        const u64 first = (ch - sd.chunk_begin) * sd.items_per_chunk;
        const u64 last = min(first + sd.items_per_chunk, sd.items);
        const u32 woff = skip ? (u32)sd.g : 0u;
        if constexpr (HIST) {
            for (int w = lane; w <= n; w += 64) lh[w] = 0;
        }
        u32 lmin = BIG;
        const u64 cnt = run_chunk<P, W, HIST>(sd, k, sd.j - 1, rows, binom, first, last, lmin, lh, woff);
        // wave min
        for (int off = 32; off >= 1; off >>= 1) lmin = min(lmin, (u32)__shfl_xor((int)lmin, off));
        if (lane == 0) {
            if (lmin != BIG) atomicMin(&cs->res.stage_min[s], (int)(lmin + woff));
            atomicAdd((unsigned long long *)&cs->res.stage_count[s], (unsigned long long)cnt);
        }
        if constexpr (HIST) {
            for (int w = lane; w <= n; w += 64) {
                const u32 c = lh[w];
                if (c) atomicAdd((unsigned long long *)&hist[(size_t)s * (BZ_MAX_N + 1) + w], (unsigned long long)c);
            }
        }
        __threadfence();
        if (lane == 0) {
            __hip_atomic_fetch_add(&cs->stage_done[s], 1ull, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
            run_checker(cs);
        }
    }
}

// =====================================================================
// Sliced vector arithmetic (tests and the arithmetic microbenchmark)
// =====================================================================
template <int P>
__global__ void pack_kernel(int enc, int nvec, int nsym, const uint8_t *__restrict__ sym, u32 *__restrict__ planes) {
    constexpr int R = (P == 3) ? 2 : 3;
    const int words = (nsym + 31) / 32;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)nvec * words) return;
    const int v = (int)(idx / words), w = (int)(idx % words);
    u32 pl[3] = {0, 0, 0};
    for (int t = 0; t < 32; t++) {
        const int c = w * 32 + t;
        if (c >= nsym) break;
        int x = sym[(size_t)v * nsym + c];
        if (enc == BZ_ENC_KAT) x = (x == 0) ? 3 : (x == 1) ? 2 : 1;  // 0=(1,1) 1=(0,1) 2=(1,0)
        for (int b = 0; b < R; b++) pl[b] |= (u32)((x >> b) & 1) << t;
    }
    for (int b = 0; b < R; b++) planes[((size_t)v * R + b) * words + w] = pl[b];
}

template <int P>
__global__ void unpack_kernel(int enc, int nvec, int nsym, const u32 *__restrict__ planes, uint8_t *__restrict__ sym) {
    constexpr int R = (P == 3) ? 2 : 3;
    const int words = (nsym + 31) / 32;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)nvec * nsym) return;
    const int v = (int)(idx / nsym), c = (int)(idx % nsym);
    int x = 0;
    for (int b = 0; b < R; b++) x |= (int)((planes[((size_t)v * R + b) * words + c / 32] >> (c % 32)) & 1) << b;
    if (enc == BZ_ENC_KAT) x = (x == 3) ? 0 : (x == 2) ? 1 : (x == 1) ? 2 : 255;
    else if (x >= P) x = 255;
    sym[idx] = (uint8_t)x;
}

// Algorithm 2 (Kawahara et al.) in its own encoding, for comparison only
__device__ __forceinline__ void kat_add(u32 a0, u32 a1, u32 b0, u32 b1, u32 &s0, u32 &s1) {
    const u32 t0 = a0 ^ b0, t1 = a1 ^ b1;
    const u32 u0 = t0 ^ a1, u1 = t1 ^ a0;
    s0 = t1 | u0;
    s1 = t0 | u1;
}

template <int P>
__global__ void op_kernel(int op, int nvec, int words, const u32 *__restrict__ A, const u32 *__restrict__ B,
                          u32 *__restrict__ O, int reps) {
    constexpr int R = (P == 3) ? 2 : 3;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)nvec * words) return;
    const int v = (int)(idx / words), w = (int)(idx % words);
    u32 a[3] = {0, 0, 0}, b[3] = {0, 0, 0}, o[3] = {0, 0, 0};
    for (int i = 0; i < R; i++) {
        a[i] = A[((size_t)v * R + i) * words + w];
        b[i] = B ? B[((size_t)v * R + i) * words + w] : 0u;
    }
    for (int rep = 0; rep < reps; rep++) {
        // opaque copies: every repetition recomputes the operation
        u32 x[3] = {a[0], a[1], a[2]}, y[3] = {b[0], b[1], b[2]};
        for (int i = 0; i < 3; i++) {
            asm volatile("" : "+v"(x[i]));
            asm volatile("" : "+v"(y[i]));
        }
        if constexpr (P == 3) {
            switch (op) {
            case BZ_OP_ADD: f3_add(x[0], x[1], y[0], y[1], o[0], o[1]); break;
            case BZ_OP_SUB: { u32 n0, n1; f3_neg(y[0], y[1], n0, n1); f3_add(x[0], x[1], n0, n1, o[0], o[1]); } break;
            case BZ_OP_DOUBLE: f3_neg(x[0], x[1], o[0], o[1]); break;
            case BZ_OP_ISO_ADD: o[0] = f3_iso_add(x[0], x[1], y[0], y[1]); o[1] = 0; break;
            case BZ_OP_ISO_SUB: o[0] = f3_iso_sub(x[0], x[1], y[0], y[1]); o[1] = 0; break;
            default: kat_add(x[0], x[1], y[0], y[1], o[0], o[1]); break;
            }
        } else {
            switch (op) {
            case BZ_OP_ADD: f7_add(x[0], x[1], x[2], y[0], y[1], y[2], o[0], o[1], o[2]); break;
            case BZ_OP_SUB: {
                u32 n0, n1, n2;
                f7_neg(y[0], y[1], y[2], n0, n1, n2);
                f7_add(x[0], x[1], x[2], n0, n1, n2, o[0], o[1], o[2]);
            } break;
            case BZ_OP_DOUBLE: f7_double(x[0], x[1], x[2], o[0], o[1], o[2]); break;
            case BZ_OP_ISO_ADD: o[0] = f7_iso_add(x[0], x[1], x[2], y[0], y[1], y[2]); o[1] = o[2] = 0; break;
            default: o[0] = f7_iso_sub(x[0], x[1], x[2], y[0], y[1], y[2]); o[1] = o[2] = 0; break;
            }
        }
        for (int i = 0; i < R; i++) asm volatile("" ::"v"(o[i]));
    }
    for (int i = 0; i < R; i++) O[((size_t)v * R + i) * words + w] = o[i];
}

}  // namespace bz
