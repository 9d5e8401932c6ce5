// bz_kernels.hpp -- gfx950 kernels of the Brouwer-Zimmermann path.
//
//   decompose_kernel  one wavefront per code: validates G, packs it into bit
//                     planes, computes the information-set decomposition
//                     Gamma_1..Gamma_m by Gauss-Jordan on bit-sliced rows (one
//                     row per lane), packs each Gamma_j for the enumeration
//                     (with its table of pair sums, see pair_units), and
//                     writes the stage schedule and the initial completion state.
//   enum_kernel       persistent: every workgroup walks the stages in order and
//                     takes its share of each stage's tiles; a lane builds the
//                     exact prefix sums of its item in registers (the two
//                     highest rows from the pair table when there is one),
//                     finishes every combination with the isometric addition,
//                     takes the weight by popcount and min-reduces it.  The workgroup that
//                     completes a stage last applies the L >= U test; workgroups
//                     that already moved on to later stages stop when it holds.
//
// Paper: Hernando & Quintana-Orti, arXiv 2603.29942 (Sec. 2-4, Algorithm 6).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "bz_arith.hpp"
#include "bz_mlp.hpp"
#include "bz_state.hpp"

namespace bz {

constexpr u32 BIG = 0x7fffffffu;
constexpr int BIN_I = 17;  // binomials C(c, i) with i < BIN_I are kept in LDS

__device__ __forceinline__ u32 uni(u32 x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ u64 uni64(u64 x) {
    const u32 lo = __builtin_amdgcn_readfirstlane((u32)x);
    const u32 hi = __builtin_amdgcn_readfirstlane((u32)(x >> 32));
    return ((u64)hi << 32) | lo;
}

// Run state shared between workgroups.  No release/acquire fences are used
// (an agent-scope fence writes back or invalidates a whole L2, which costs
// every wave on the XCD): a workgroup's published minimum and count are
// atomics that have completed (vmcnt drained) before its done-increment is
// issued, and the checker reads counters and minima with read-modify-write
// atomics, which are performed at the single coherence point of their
// address.  Waiting workgroups poll the control word with plain atomic loads.
template <typename T>
__device__ __forceinline__ T ld_poll(T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T rd_atomic(T *p) {
    return __hip_atomic_fetch_or(p, (T)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void drain_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// word q of a small register array, q wave-uniform (no dynamic register indexing)
template <int N>
__device__ __forceinline__ u32 pick(const u32 (&a)[N], int q) {
    u32 v = a[0];
#pragma unroll
    for (int i = 1; i < N; i++) v = (q == i) ? a[i] : v;
    return v;
}

// Launch arguments of the enumeration kernel (known to the host up front).
struct EnumArgs {
    int32_t k, n, flags, lookahead;
    u64 timeout_ticks;
    // optional: when a check ends the run (or checks the last stage), the
    // checking wavefront copies the result block to res_out (mapped host
    // memory) and then stores epoch to *flag_out
    CodeResult *res_out;
    uint32_t *flag_out;
    uint32_t epoch;
    uint32_t pair_stride;  // 16-byte units between the pair tables of two sets (with a table)
};

// A code's result block to mapped host memory by one whole wavefront:
// agent-scope atomic loads (the minima and counts are atomics performed at the
// coherence point), plain stores, a system-scope release, then lane 0 stores
// `value` to the flag the host waits on.  res_out may be NULL (flag only).
__device__ __forceinline__ void hand_out_result(const CodeState *cs, CodeResult *res_out, uint32_t *flag,
                                                uint32_t value) {
    const int lane = __lane_id();
    if (res_out) {
        // what the host reads of the block: the header, ranks[0, m) and the
        // stage minima and counts of the n_table stages, as 32-bit words;
        // the loads of 256 words are issued before their stores
        static_assert(sizeof(CodeResult) % sizeof(u32) == 0, "the result block in 32-bit words");
        constexpr int RK = (int)(offsetof(CodeResult, ranks) / 4), SM = (int)(offsetof(CodeResult, stage_min) / 4),
                      SC = (int)(offsetof(CodeResult, stage_count) / 4);
        const u32 *src = reinterpret_cast<const u32 *>(&cs->res);
        u32 *dst = reinterpret_cast<u32 *>(res_out);
        const int m = min(max(uni(__hip_atomic_load(&cs->res.m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)), 0), BZ_MAX_M);
        const int ns = min(max(uni(__hip_atomic_load(&cs->res.n_table, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)), 0),
                           BZ_MAX_STAGES);
        const int n1 = RK + m, n2 = n1 + ns, total = n2 + 2 * ns;
        auto word = [&](int t) { return t < n1 ? t : (t < n2 ? SM + (t - n1) : SC + (t - n2)); };
        for (int t0 = 0; t0 < total; t0 += 4 * 64) {
            u32 v[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int t = t0 + lane + 64 * r;
                v[r] = t < total ? __hip_atomic_load(const_cast<u32 *>(src + word(t)), __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                                 : 0u;
            }
#pragma unroll
            for (int r = 0; r < 4; r++) asm volatile("" ::"v"(v[r]));
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int t = t0 + lane + 64 * r;
                if (t < total) dst[word(t)] = v[r];
            }
        }
        __atomic_thread_fence(__ATOMIC_RELEASE);  // system scope: the stores before the flag
    }
    if (lane == 0) __hip_atomic_store(flag, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

struct RunArgs {
    int32_t n, k, flags, U0;
    u64 max_codewords;
    uint32_t grid;       // workgroups of the enumeration launch
    uint32_t sweep_ops;  // VALU operations per lane and task (sizes the blocks of rows s)
    u64 timeout_ticks;   // wall_clock64() ticks a workgroup may wait for earlier stages
    const RoundTable *rounds;  // the rounds' task counts for this shape, or NULL: counted here
    SpecBuf *spec;             // the second information set computed ahead, or NULL
    uint32_t epoch, pad;       // this call's value of spec->flag
    // the pair table of set j at pairs + j * pair_stride (16-byte units), for
    // pair_w words per plane; NULL: no tables (the enumeration then builds
    // its prefixes itself)
    uint4 *pairs = nullptr;
    uint32_t pair_stride = 0;
    int32_t pair_w = 0;
    int32_t pair_t0 = 0;  // 1: a workgroup of its own builds the first set's table (ROLE_TABLE0)
};

// Workgroups of a decomposition launch: the one that decomposes the code
// (MAIN); on the plain path also one that computes the second information set
// ahead (AHEAD, see SpecBuf) and builds its pair table in a slot of its own,
// and one that repeats the first set's elimination only to build its pair
// table (TABLE0), so that neither table lengthens the main workgroup's path.
enum { ROLE_MAIN = 0, ROLE_AHEAD = 1, ROLE_TABLE0 = 2 };

// q-groups of a stage with g >= 3 computed by the 64 lanes of a wavefront
// (lane = q - (g-3)); the same values as fill_qtable.  Returns the number of
// tasks (wave-uniform); with tab != nullptr the lanes also store their entry.
// The binomials C(q, g-3) come from the workgroup's LDS copy when g-3 < BIN_I
// (C(c, i) at sbin[c * BIN_I + i]), else from the global table.
__device__ __forceinline__ u64 wave_qtable(int p, int k, int g, u64 M, uint32_t cap, uint32_t vcap,
                                           const u64 *sbin, const u64 *__restrict__ gbin, QEntry *tab) {
    const int lane = __lane_id();
    const int q = g - 3 + lane;
    const bool in = q <= k - 3;
    u64 bases = 0, val = 0;
    uint32_t nb = 0, vd = 0;
    if (in) {
        // the values of qgroup
        const u64 c = (g - 3 < BIN_I) ? sbin[q * BIN_I + (g - 3)] : gbin[q * 65 + (g - 3)];
        bases = sat_mul(c, M);
        nb = qgroup_blocks(k, cap, q);
        vd = qgroup_digits(p, k, g, vcap, q, bases);
        val = qgroup_tasks(p, bases, nb, vd);  // <= 2^58 * 62: no overflow
    }
    // inclusive scan of val over the lanes (saturating)
    u64 inc = val;
    for (int off = 1; off < 64; off <<= 1) {
        const u64 o = __shfl_up(inc, off);
        if (lane >= off) inc = sat_add(inc, o);
    }
    if (tab && in) {
        QEntry &e = tab[lane];
        e.first = inc - val;
        e.bases = bases;
        e.nb = nb;
        e.vd = vd;
    }
    return uni64(__shfl(inc, 63));
}

// =====================================================================
// Decomposition: one wavefront per code, lane i holds row i.
// =====================================================================
// LDS of one decomposition (a kernel declares it once and passes it down, so
// that one kernel can hold several instantiations of decompose_code)
struct DecompLDS {
    u64 binom[(BZ_MAX_K + 1) * 65];  // C(c, i) at [c * 65 + i], rows c <= k
    int32_t sranks[BZ_MAX_M];
    u64 s_cw[BZ_MAX_K], s_tasks[BZ_MAX_K];
    u64 s_tbefore[BZ_MAX_K];  // tiles of the rounds before round g, at [g - 1]
    uint32_t s_vcap[BZ_MAX_K];  // run budget of round g (0: no runs), at [g - 1]
    uint32_t s_combos[BZ_MAX_K];
    uint32_t s_nb[BZ_MAX_K];  // blocks of rows s of the q-group with top row q, at [q]
    uint32_t s_dt[BZ_MAX_K];  // digits_by_steps of the q-group with top row q, at [q]
    uint4 prow[BZ_MAX_K * 4];  // the packed rows of the set whose pair table is built, row i word w at [i * 4 + w]
};

// The pair table of one information set (see pair_units) from its packed rows
// in LDS, lane t taking the pairs t, t + 64, ...  Plain stores: the
// enumeration reads the table in a later launch.
template <int P>
__device__ void build_pair_table(uint4 *__restrict__ ptab, int k, int W, const uint4 *prow) {
    const int lane = threadIdx.x;
    const int np = k * (k - 1) / 2;
    // (s, rem): pair e is (s, s + 1 + rem); advanced by 64 pairs per step
    int s = 0, rem = 0;
    pair_advance(k, s, rem, lane);
    for (int e = lane; e < np; e += 64) {
        const int L = s + 1 + rem;
        for (int w = 0; w < W; w++) {
            const uint4 a = prow[s * 4 + w], b = prow[L * 4 + w];
            if constexpr (P == 3) {
                u32 t0, t1, u0, u1;
                f3_add(a.x, a.y, b.x, b.y, t0, t1);  // R_s + R_L
                f3_add(a.x, a.y, b.y, b.x, u0, u1);  // R_s - R_L (= R_s + 2 R_L: planes swapped)
                ptab[(size_t)e * W + w] = make_uint4(t0, t1, u0, u1);
            } else {
                const u32 bl[3] = {b.x, b.y, b.z};
#pragma unroll
                for (int c = 1; c < 7; c++) {
                    u32 sc[3], t[3];
                    scale<7>(c, bl, sc);
                    f7_add(a.x, a.y, a.z, sc[0], sc[1], sc[2], t[0], t[1], t[2]);
                    ptab[((size_t)e * 6 + (c - 1)) * W + w] = make_uint4(t[0], t[1], t[2], t[0] | t[1] | t[2]);
                }
            }
        }
        pair_advance(k, s, rem, 64);
    }
}

// One Gauss-Jordan step on the rows held one per lane: row pl (pivot value
// pv in the pivot column) becomes pv^-1 times itself, every other row i
// becomes row_i - v_i pv^-1 row_pl (v_i = its entry in the pivot column).
// Branch-free per lane: a row takes h times the raw pivot row, h = -v pv^-1
// off the pivot lane; the pivot lane's row is replaced by pv^-1 times the
// pivot row (F_7) or adds pv^-1 - 1 times itself (F_3).  h * row is a
// rotation and a negation of its planes (F_3: 2 = -1 swaps the planes; F_7:
// every nonzero h is +-2^e, times 2 rotates the three planes, negation is the
// complement on the nonzero positions, Sec. 4.2).
template <int P, int WF>
__device__ __forceinline__ void eliminate(u32 (&x)[3][4], int v, int pl, int pv) {
    const int lane = __lane_id();
    const bool me = lane == pl;
    if constexpr (P == 3) {
        // every row adds h times the pivot row: h = pv^-1 - 1 = pv - 1 on the
        // pivot lane (its own row, which so becomes pv^-1 times itself) and
        // -v pv^-1 = -v pv elsewhere, i.e. 0 for v = 0, 2 for v = pv, else 1.
        // h = 0: unchanged; h = 2: the planes swapped.
        const bool sw = !me && v == pv;
        const u32 live = (me ? pv == 2 : v != 0) ? ~0u : 0u;
#pragma unroll
        for (int w = 0; w < WF; w++) {
            const u32 a0 = __builtin_amdgcn_readlane(x[0][w], pl), a1 = __builtin_amdgcn_readlane(x[1][w], pl);
            const u32 s0 = (sw ? a1 : a0) & live, s1 = (sw ? a0 : a1) & live;
            f3_add(x[0][w], x[1][w], s0, s1, x[0][w], x[1][w]);
        }
    } else {
        const u32 keep = me ? 0u : ~0u;              // pivot lane: replaced, others: added to
        const u32 live = (me || v != 0) ? ~0u : 0u;  // rows with v = 0 are unchanged
        // h = (-1)^neg 2^e; tables over v = 0..6 packed in constants:
        // e(v) two bits at 2v, neg(v) one bit at v (1, 2, 4 = +2^e; 6, 5, 3 = -2^e)
        constexpr u32 ETAB = 0x690u, NTAB = 0x68u;
        const int e_pv = (int)((ETAB >> (2 * pv)) & 3u), n_pv = (int)((NTAB >> pv) & 1u);
        const int e_inv = (3 - e_pv) % 3, n_inv = n_pv;  // pv^-1 = (-1)^n 2^-e
        const int e_v = (int)((ETAB >> (2 * v)) & 3u), n_v = (int)((NTAB >> v) & 1u);
        int e = me ? e_inv : e_v + e_inv;
        if (e >= 3) e -= 3;
        const u32 negm = (me ? n_inv : (n_v ^ n_inv ^ 1)) ? ~0u : 0u;
#pragma unroll
        for (int w = 0; w < WF; w++) {
            const u32 a0 = __builtin_amdgcn_readlane(x[0][w], pl), a1 = __builtin_amdgcn_readlane(x[1][w], pl),
                      a2 = __builtin_amdgcn_readlane(x[2][w], pl);
            // times 2^e: (a0, a1, a2) -> (a2, a0, a1) per factor 2
            u32 r0 = e == 0 ? a0 : (e == 1 ? a2 : a1);
            u32 r1 = e == 0 ? a1 : (e == 1 ? a0 : a2);
            u32 r2 = e == 0 ? a2 : (e == 1 ? a1 : a0);
            const u32 flip = (a0 | a1 | a2) & negm;
            r0 = (r0 ^ flip) & live;
            r1 = (r1 ^ flip) & live;
            r2 = (r2 ^ flip) & live;
            f7_add(x[0][w] & keep, x[1][w] & keep, x[2][w] & keep, r0, r1, r2, x[0][w], x[1][w], x[2][w]);
        }
    }
}

// This lane's entries of the per-shape round table (the plain path), read by
// the caller at the start of the launch so that the loads complete during
// the elimination; have = false: the rounds are counted instead.
struct RoundPrefetch {
    bool have = false;
    u64 tasks = 0;
    uint32_t vcap = 0;
    int cut = 0;
};

// One code on one wavefront (threads 0..63 of the workgroup).
// role ROLE_AHEAD: the elimination of one set with the columns 0 .. k-1 taken
// as used, packed into args.spec, then (with tables) its pair table in slot
// pair_sets(n, k), and nothing else.  ROLE_TABLE0: the first set's
// elimination and its pair table in slot 0, and nothing else.
template <int P, int WF>
__device__ void decompose_code(const uint8_t *__restrict__ G, CodeState *cs, u32 *__restrict__ rows,
                               const RunArgs args, DecompLDS &lds, int role = ROLE_MAIN,
                               RoundPrefetch pre = RoundPrefetch()) {
    const bool ahead = role == ROLE_AHEAD, main_wg = role == ROLE_MAIN;
    constexpr int R = (P == 3) ? 2 : 3;
    u64 *binom = lds.binom;
    int32_t *sranks = lds.sranks;
    const int lane = threadIdx.x;
    // the arguments arrive in vector registers (a call, not inlined): pin them
    // to scalars so that everything derived from them is wave-uniform
    const int n = uni(args.n), k = uni(args.k), flags = uni(args.flags);
    CodeResult &res = cs->res;
    const bool tracing = main_wg && (flags & FLAG_TRACE) != 0;
    const u64 t_start = tracing ? (u64)wall_clock64() : 0;
    SpecBuf *spec = args.spec;
    uint4 *const pairs = args.pairs;
    const int pair_w = uni(args.pair_w);
    const uint32_t pair_stride = uni(args.pair_stride);
    const bool t0_elsewhere = uni(args.pair_t0) != 0;
    const bool have_rt = pre.have;
    const u64 rt_tasks = pre.tasks;
    const uint32_t rt_vcap = pre.vcap;
    const int rt_cut = pre.cut;
    if (lane == 0 && main_wg) {
        cs->p = P;
        cs->n = n;
        cs->k = k;
        cs->flags = flags;
        cs->U0 = args.U0;
        cs->pair_slot1 = 1;
        cs->max_codewords = args.max_codewords;
    }

    // -- one round of independent loads: lane i < k reads row i of G (k x n
    //    bytes, row-major) as the aligned 32-bit words that cover it (reads
    //    stay inside the aligned words that hold bytes of G)
    constexpr int NW = 8 * WF + 1;  // covers 32 WF bytes at any alignment
    u32 raw[NW];
    int sh;
    {
        const uintptr_t g0 = reinterpret_cast<uintptr_t>(G);
        const uintptr_t addr = g0 + (uintptr_t)(lane < k ? lane : 0) * (uintptr_t)n;
        const u32 *src = reinterpret_cast<const u32 *>(addr & ~(uintptr_t)3);
        const u32 *last = reinterpret_cast<const u32 *>((g0 + (uintptr_t)k * (uintptr_t)n - 1) & ~(uintptr_t)3);
        sh = (int)(addr & 3);
#pragma unroll
        for (int t = 0; t < NW; t++) raw[t] = *(src + t <= last ? src + t : last);
    }
    // binomials for the schedule by Pascal's rule while the loads are in
    // flight, lane i holding C(c, i) (exact: every C(c, i) with c <= 64 fits 64 bits)
    // (the left neighbour by a wave-wide DPP shift; lane 0 receives 0)
    {
        u64 v = (lane == 0) ? 1u : 0u;
        for (int c = 0; c <= k; c++) {
            binom[c * 65 + lane] = v;
            if (lane == 0) binom[c * 65 + 64] = (c == 64) ? 1u : 0u;
            const u32 llo = __builtin_amdgcn_update_dpp(0u, (u32)v, 0x138, 0xf, 0xf, false);  // wave_shr:1
            const u32 lhi = __builtin_amdgcn_update_dpp(0u, (u32)(v >> 32), 0x138, 0xf, 0xf, false);
            v += ((u64)lhi << 32) | llo;
        }
    }
    // the row's bytes, realigned, into bit planes: bit b of the symbol in
    // column c goes to bit c % 32 of x[b][c / 32]; columns >= n are cleared
    // below, symbols >= p flag the code as invalid
    u32 colmask[4];
#pragma unroll
    for (int w = 0; w < 4; w++) {
        const int lo = w * 32;
        colmask[w] = (n >= lo + 32) ? 0xffffffffu : (n > lo ? ((1u << (n - lo)) - 1u) : 0u);
    }
    u32 x[3][4];
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
        for (int w = 0; w < 4; w++) x[b][w] = 0;
    bool bad = false;
    {
        constexpr u32 K = (0x80u - (u32)P) * 0x01010101u;  // byte + K has bit 7 set iff byte >= P (byte < 128)
#pragma unroll
        for (int t = 0; t < 8 * WF; t++) {
            const u32 wd = __builtin_amdgcn_alignbyte(raw[t + 1], raw[t], (u32)sh);  // bytes 4t .. 4t+3
            const int valid = n - 4 * t;  // bytes of this word inside the row (uniform)
            const u32 vm = valid >= 4 ? 0x80808080u : valid > 0 ? (0x80808080u >> (8 * (4 - valid))) : 0u;
            bad |= ((wd | (wd + K)) & vm) != 0;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int c = 4 * t + q;
#pragma unroll
                for (int b = 0; b < R; b++)
                    x[b][c >> 5] |= ((wd >> (8 * q + b)) & 1u) << (c & 31);
            }
        }
        if (lane >= k) bad = false;
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
            for (int w = 0; w < 4; w++) x[b][w] = (lane < k) ? (x[b][w] & colmask[w]) : 0u;
    }
    __syncthreads();
    const u64 t_loaded = tracing ? (u64)wall_clock64() : 0;

    int status = BZ_OK;
    if (__any(bad)) status = BZ_ERR_VALUE;

    int m = 0;
    u32 used[4] = {0, 0, 0, 0};
    const bool skip = (flags & FLAG_SKIP) != 0;
    const int W = skip ? (n - k + 31) / 32 : WF;
    // the columns 0 .. k-1
    u32 firstk[4];
#pragma unroll
    for (int w = 0; w < 4; w++) {
        const int lo = w * 32;
        firstk[w] = (k >= lo + 32) ? 0xffffffffu : (k > lo ? ((1u << (k - lo)) - 1u) : 0u);
    }
    if (ahead) {
#pragma unroll
        for (int w = 0; w < 4; w++) used[w] = firstk[w];
    }
    bool first_is_firstk = false;  // the first set's pivots are the columns 0 .. k-1
    bool handed = false;           // the second set came from the workgroup ahead

    while (status == BZ_OK) {
        u32 unused[4];
        bool anyu = false;
#pragma unroll
        for (int w = 0; w < 4; w++) {
            unused[w] = colmask[w] & ~used[w];
            anyu |= unused[w] != 0;
        }
        if (!anyu) break;
        if (main_wg && spec != nullptr && m == 1 && first_is_firstk) {
            // the second set from the workgroup that computed it ahead, when it
            // has finished (a bounded wait; else it is computed here)
            u32 f = 0;
            for (int it = 0; it < 1024; it++) {
                f = uni(__hip_atomic_load(&spec->flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
                if (f == args.epoch) break;
                __builtin_amdgcn_s_sleep(1);
            }
            // every load of the hand-over issued together (one wait): its
            // status, size and pivot columns, and the rows as plain 16-byte loads
            // (the acquire of the flag orders them after the other workgroup's
            // stores, its release)
            u32 okv = 0, kjv = 0, pmv[4] = {0, 0, 0, 0};
            uint4 v[ROW_WORDS / 4];
            if (f == args.epoch) {
                okv = __hip_atomic_load(&spec->ok, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                kjv = __hip_atomic_load(&spec->kj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int w = 0; w < 4; w++)
                    pmv[w] = __hip_atomic_load(&spec->pivmask[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint4 *srow = reinterpret_cast<const uint4 *>(spec->rows + (size_t)(lane < k ? lane : 0) * ROW_WORDS);
#pragma unroll
                for (int w = 0; w < ROW_WORDS / 4; w++) v[w] = srow[w];
#pragma unroll
                for (int w = 0; w < ROW_WORDS / 4; w++)
                    asm volatile("" ::"v"(v[w].x), "v"(v[w].y), "v"(v[w].z), "v"(v[w].w));
            }
            if (f == args.epoch && uni(okv)) {
                const int kj2 = uni((int)kjv);
                if (lane < k) {
                    uint4 *drow = reinterpret_cast<uint4 *>(rows + (size_t)(BZ_MAX_K + lane) * ROW_WORDS);
#pragma unroll
                    for (int w = 0; w < ROW_WORDS / 4; w++) drow[w] = v[w];
                }
                // its pair table is built by that workgroup, in slot pair_sets(n, k)
                if (lane == 0 && pairs != nullptr) cs->pair_slot1 = pair_sets(n, k);
#pragma unroll
                for (int w = 0; w < 4; w++) used[w] |= uni(pmv[w]) & unused[w];
                if (lane == 0) sranks[1] = kj2;
                m = 2;
                handed = true;
                if (kj2 < k || m == BZ_MAX_M) break;
                continue;
            }
        }
        // Gauss-Jordan with the unused columns first, then the used ones, each
        // ascending; the pivot of a column is the lowest row that is not yet a
        // pivot row and has a nonzero entry there.  piv_lane = pivot index of
        // this lane's row; free_rows (wave-uniform) = rows not yet pivots.
        int piv_lane = -1, npiv = 0, kj = 0;
        u64 free_rows = (k >= 64) ? ~0ull : ((1ull << k) - 1ull);
        u32 pivmask[4] = {0, 0, 0, 0};
        for (int pass = 0; pass < 2 && npiv < k; pass++) {
#pragma unroll
            for (int w = 0; w < WF; w++) {
                u32 bits = uni(pass == 0 ? unused[w] : (colmask[w] & used[w]));
                while (bits && npiv < k) {
                    const int t = __builtin_ctz(bits);
                    bits &= bits - 1;
                    int v = 0;
#pragma unroll
                    for (int b = 0; b < R; b++) v |= (int)((x[b][w] >> t) & 1u) << b;
                    // (the wave-uniform loop state is pinned to scalar registers)
                    const u64 cm = uni64(__ballot(v != 0) & free_rows);
                    if (cm == 0) continue;
                    const int pl = uni(__builtin_ctzll(cm));
                    free_rows = uni64(free_rows & ~(1ull << pl));
                    const int pv = __builtin_amdgcn_readlane(v, pl);
                    eliminate<P, WF>(x, v, pl, pv);
                    piv_lane = (lane == pl) ? npiv : piv_lane;
                    npiv = uni(npiv + 1);
                    if (pass == 0) kj = uni(kj + 1);
                    pivmask[w] = uni(pivmask[w] | (1u << t));
                }
            }
        }
        if (npiv < k) {
            status = BZ_ERR_RANK;
            break;
        }
        if (kj == 0) break;
        if (m == 0) first_is_firstk = kj == k && pivmask[0] == firstk[0] && pivmask[1] == firstk[1] &&
                                      pivmask[2] == firstk[2] && pivmask[3] == firstk[3];
        // -- pack Gamma_m: row piv_lane of matrix m; slot 3 of each word = OR of planes.
        //    Identity skip: the n-k non-pivot columns of every row compressed, in
        //    order, into columns 0 .. n-k-1 (one column map for all rows; only
        //    weights are used, so any fixed map would do).  The compress plans
        //    and bit positions depend on the pivot columns only (wave-uniform).
        Compress32 plan[WF];
        u32 npm[WF];
        int at[WF];
        if (skip) {
            int pos = 0;
#pragma unroll
            for (int w = 0; w < WF; w++) {
                npm[w] = uni(colmask[w] & ~pivmask[w]);
                plan[w] = compress_plan(npm[w]);
                at[w] = pos;
                pos += __builtin_popcount(npm[w]);
            }
        }
        if (lane < k) {
            u32 *dst = ahead ? spec->rows + (size_t)piv_lane * ROW_WORDS
                             : rows + (size_t)(m * BZ_MAX_K + piv_lane) * ROW_WORDS;
            u32 out[3][4];
#pragma unroll
            for (int b = 0; b < 3; b++)
#pragma unroll
                for (int w = 0; w < 4; w++) out[b][w] = 0;
            if (skip) {
#pragma unroll
                for (int b = 0; b < R; b++) {
                    u64 lo = 0, hi = 0;
#pragma unroll
                    for (int w = 0; w < WF; w++) {
                        const u64 c = compress_apply(x[b][w], npm[w], plan[w]);
                        if (at[w] < 64) {
                            lo |= c << at[w];
                            if (at[w] > 32) hi |= c >> (64 - at[w]);
                        } else {
                            hi |= c << (at[w] - 64);
                        }
                    }
                    out[b][0] = (u32)lo;
                    out[b][1] = (u32)(lo >> 32);
                    out[b][2] = (u32)hi;
                    out[b][3] = (u32)(hi >> 32);
                }
            } else {
#pragma unroll
                for (int b = 0; b < 3; b++)
#pragma unroll
                    for (int w = 0; w < 4; w++) out[b][w] = (w < WF) ? x[b][w] : 0u;
            }
            if (role != ROLE_TABLE0) {
#pragma unroll
                for (int w = 0; w < 4; w++) {
                    dst[w * 4 + 0] = out[0][w];
                    dst[w * 4 + 1] = out[1][w];
                    dst[w * 4 + 2] = out[2][w];
                    dst[w * 4 + 3] = out[0][w] | out[1][w] | out[2][w];
                }
            }
            if (pairs != nullptr) {
#pragma unroll
                for (int w = 0; w < 4; w++)
                    lds.prow[piv_lane * 4 + w] =
                        make_uint4(out[0][w], out[1][w], out[2][w], out[0][w] | out[1][w] | out[2][w]);
            }
        }
        if (role == ROLE_TABLE0) {
            if (pairs != nullptr) {
                __syncthreads();
                build_pair_table<P>(pairs, k, pair_w, lds.prow);
            }
            return;
        }
        // (m < pair_sets(n, k) always holds, see pair_sets)
        if (main_wg && pairs != nullptr && m < pair_sets(n, k) && !(m == 0 && t0_elsewhere)) {
            __syncthreads();
            build_pair_table<P>(pairs + (size_t)m * pair_stride, k, pair_w, lds.prow);
            __syncthreads();
        }
        if (ahead) {
            // publish: the rows and the set's description, then the flag
            if (lane == 0) {
#pragma unroll
                for (int w = 0; w < 4; w++) spec->pivmask[w] = pivmask[w] & unused[w];
                spec->kj = kj;
                spec->ok = 1;
            }
            __threadfence();
            if (lane == 0) __hip_atomic_store(&spec->flag, args.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (pairs != nullptr) {
                __syncthreads();
                build_pair_table<P>(pairs + (size_t)pair_sets(n, k) * pair_stride, k, pair_w, lds.prow);
            }
            return;
        }
        if (lane == 0) sranks[m] = kj;
        m++;
#pragma unroll
        for (int w = 0; w < 4; w++) used[w] |= pivmask[w] & unused[w];
        if (kj < k || m == BZ_MAX_M) break;
    }
    if (role == ROLE_TABLE0) return;  // no first set (an invalid symbol, rank < k)
    if (ahead) {
        // no second set to hand over (an invalid symbol, rank < k, no unused column)
        if (lane == 0) spec->ok = 0;
        __threadfence();
        if (lane == 0) __hip_atomic_store(&spec->flag, args.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    __syncthreads();

    const u64 t_reduced = tracing ? (u64)wall_clock64() : 0;
    // -- schedule (the stage order of Alg. 6): one round g per lane, a
    //    saturating scan for the codewords before each round, then one stage per
    //    lane; the same table as build_schedule
    u64 *s_cw = lds.s_cw, *s_tasks = lds.s_tasks;
    uint32_t *s_combos = lds.s_combos;
    int ns = 0, complete = 1;
    if (status == BZ_OK && ((flags & FLAG_NO_TERM) != 0 || args.U0 > 1)) {
        const int g = lane + 1;
        const bool in = g <= k;
        const u64 cw = in ? round_codewords(P, k, g, binom) : 0;
        const u64 combos = round_combos(P, g);
        const u64 mine = sat_mul(cw, (u64)m);
        u64 inc = mine;
        for (int off = 1; off < 64; off <<= 1) {
            const u64 o = __shfl_up(inc, off);
            if (lane >= off) inc = sat_add(inc, o);
        }
        u64 before = __shfl_up(inc, 1);  // codewords of the rounds before g
        if (lane == 0) before = 0;
        const int js = in ? round_stages(m, before, cw, combos, args.max_codewords) : m;
        const u64 short_rounds = __ballot(in && js < m);
        if (short_rounds) {
            const int g0 = __builtin_ctzll(short_rounds);
            ns = g0 * m + __shfl(js, g0);
            complete = 0;
        } else {
            ns = k * m;
        }
        if (in) {
            s_cw[lane] = cw;
            s_combos[lane] = (uint32_t)combos;
            s_tasks[lane] = (g <= SUBSET_G) ? small_stage_tasks(k, g) : 0;
            lds.s_vcap[lane] = 0;
        }
        __syncthreads();
        // task counts of the rounds g > SUBSET_G that the table reaches, one
        // round per lane: tasks(g) = sum over q of ceil(bases(q, g) / 64) nb(q),
        // the blocks nb(q) of a q-group being the same in every round (the sum
        // of fill_qtable)
        const int last_g = (ns + m - 1) / m;
        const uint32_t cap = sweep_cap_for(P, W, args.sweep_ops);
        const uint32_t budget = run_budget(P, cap);
        if (!have_rt && lane <= k - 3) {
            lds.s_nb[lane] = qgroup_blocks(k, cap, lane);
            lds.s_dt[lane] = digits_by_steps(P, k, lane, budget);
        }
        __syncthreads();
        const bool counted = in && g > SUBSET_G && g <= last_g;
        u64 tg = 0, tgv = 0;  // without and with runs of bases
        if (have_rt) {
            // the table of this shape (fill_round_table)
            if (counted) {
                s_tasks[lane] = rt_tasks;
                lds.s_vcap[lane] = rt_vcap;
            }
            tg = (counted && g >= uni(rt_cut)) ? (1ull << 62) : 0;  // the cut below, from cut_g
        } else if (counted) {
            // q runs over a wave-uniform range (rows q < g-3 add nothing) so
            // that the unrolled LDS reads overlap
            const int q0 = uni(SUBSET_G - 2);  // the smallest g - 3 of a counted round
#pragma unroll 4
            for (int q = q0; q <= k - 3; q++) {
                if (q < g - 3) continue;
                // (ceil64 <= 2^58 and nb <= 62: the product cannot overflow)
                const u64 bases = sat_mul32(binom[q * 65 + (g - 3)], (uint32_t)combos);
                const uint32_t nb = lds.s_nb[q];
                tg = sat_add(tg, qgroup_tasks(P, bases, nb, 0));
                tgv = sat_add(tgv, qgroup_tasks(P, bases, nb, digits_of(P, g, lds.s_dt[q], bases)));
            }
            // the round takes runs of bases where they pay (qgroup_digits with
            // the run budget, as a table of digits_by_steps)
            const bool runs = runs_pay(tgv, args.grid);
            s_tasks[lane] = runs ? tgv : tg;
            lds.s_vcap[lane] = runs ? budget : 0u;
        }
        // the first round with 2^62 tasks or more cuts the table before it
        const u64 over = __ballot(counted && tg >= (1ull << 62));
        if (over) {
            ns = min(ns, __builtin_ctzll(over) * m);
            complete = 0;
        }
        if (ns > BZ_MAX_STAGES) {
            ns = BZ_MAX_STAGES;
            complete = 0;
        }
        __syncthreads();
        // tiles of the rounds before each round (exclusive saturating scan)
        {
            const u64 mine_t = in ? (s_tasks[lane] + WAVES_PER_GROUP - 1) / WAVES_PER_GROUP : 0;
            u64 it = mine_t;
            for (int off = 1; off < 64; off <<= 1) {
                const u64 o = __shfl_up(it, off);
                if (lane >= off) it = sat_add(it, o);
            }
            u64 tb = __shfl_up(it, 1);
            if (lane == 0) tb = 0;
            if (in) lds.s_tbefore[lane] = tb;
        }
        __syncthreads();
    }
    {
        const uint32_t cap = sweep_cap_for(P, W, args.sweep_ops);
        for (int s = lane; s < ns; s += 64) {
            const int g = s / m + 1, j = s % m + 1;
            int L = 0;
            for (int i = 1; i <= m; i++) L += bound_c(i <= j ? g : g - 1, k, sranks[i - 1]);
            StageDesc d;
            d.g = g;
            d.j = j;
            d.L = L;
            d.check = (flags & FLAG_NO_TERM) ? 0 : ((flags & FLAG_ROUND) ? (j == m) : 1);
            d.tasks = s_tasks[g - 1];
            d.tiles = (d.tasks + WAVES_PER_GROUP - 1) / WAVES_PER_GROUP;
            d.codewords = s_cw[g - 1];
            d.coef_combos = s_combos[g - 1];
            d.parts = (uint32_t)(d.tiles < (u64)args.grid ? d.tiles : (u64)args.grid);
            d.sweep_cap = cap;
            d.vcap = lds.s_vcap[g - 1];
            d.pad = 0;
            const u64 off = deal_offset(m, lds.s_tbefore[g - 1], j, d.tiles);
            d.nowait = off < (u64)args.grid;
            d.rot = deal_rot(off, args.grid);
            cs->stages[s] = d;
            res.stage_min[s] = (int)BIG;
            res.stage_count[s] = 0;
            cs->stage_done[s] = 0;
            if (tracing) {
                cs->trace[2 + s][0] = ~0ull;
                cs->trace[2 + s][1] = 0;
                cs->trace[2 + s][2] = 0;
                cs->trace[2 + s][3] = 0;
            }
        }
    }
    if (tracing && lane == 0) {
        cs->trace[0][0] = t_start;
        cs->trace[0][1] = t_loaded;
        cs->trace[0][2] = t_reduced;
        cs->trace[0][3] = (u64)wall_clock64();
        cs->trace[1][0] = ~0ull;
        cs->trace[1][1] = 0;
    }
    for (int j = lane; j < m; j += 64) res.ranks[j] = sranks[j];
    if (lane == 0) {
        res.status = status;
        res.m = m;
        res.W = W;
        res.info = (handed ? BZ_INFO_AHEAD : 0) | (pairs != nullptr ? BZ_INFO_PAIRS : 0);
        res.t_end = 0;
        res.ctl = ctl_make(0, -1, args.U0);
        res.n_table = ns;
        res.table_complete = complete;
    }
    if (lane < WAKE_COPIES) cs->wake[lane][0] = wake_make(0, -1);
    if (lane < (int)POOL_SLICES) cs->pool_next[lane][0] = 0;
}

template <int P, int WF>
__global__ __launch_bounds__(64) void decompose_kernel(const uint8_t *__restrict__ G, CodeState *cs,
                                                       u32 *__restrict__ rows, RunArgs args) {
    __shared__ DecompLDS lds;
    RoundPrefetch pre;
    if (args.rounds != nullptr && blockIdx.x == 0) {
        const int lane = __lane_id();
        pre.have = true;
        pre.tasks = args.rounds->tasks[lane];
        pre.vcap = args.rounds->vcap[lane];
        pre.cut = args.rounds->cut_g;
    }
    // workgroup 1: the second information set ahead (with args.spec), else
    // the first set's pair table; workgroup 2: the first set's pair table
    const int role = blockIdx.x == 0 ? ROLE_MAIN : (blockIdx.x == 1 && args.spec != nullptr) ? ROLE_AHEAD : ROLE_TABLE0;
    decompose_code<P, WF>(G, cs, rows, args, lds, role, pre);
}

// =====================================================================
// Enumeration
// =====================================================================

template <int W>
struct Row {
    u32 p[3][W];  // planes
    u32 any[W];   // OR of the planes
};

template <int P, int W>
__device__ __forceinline__ Row<W> load_row(const u32 *__restrict__ rows, int j, int i) {
    const uint4 *src = reinterpret_cast<const uint4 *>(rows + (size_t)(j * BZ_MAX_K + i) * ROW_WORDS);
    Row<W> r;
#pragma unroll
    for (int w = 0; w < W; w++) {
        const uint4 v = src[w];
        r.p[0][w] = v.x;
        r.p[1][w] = v.y;
        r.p[2][w] = (P == 3) ? 0u : v.z;
        r.any[w] = v.w;
    }
    return r;
}

// A row at a lane-specific index (decoding a base, the rows of a subset): from
// the workgroup's LDS copy of the first LROW_SETS matrices when it has one
// (lrows != nullptr), else from memory.  Wave-uniform rows keep coming from
// memory through scalar loads.
constexpr int LROW_SETS = 2;
template <int P, int W>
__device__ __forceinline__ Row<W> load_row_lane(const u32 *__restrict__ rows, const uint4 *lrows, int j, int i) {
    if (lrows != nullptr && j < LROW_SETS) {
        const uint4 *src = lrows + (j * BZ_MAX_K + i) * W;
        Row<W> r;
#pragma unroll
        for (int w = 0; w < W; w++) {
            const uint4 v = src[w];
            r.p[0][w] = v.x;
            r.p[1][w] = v.y;
            r.p[2][w] = (P == 3) ? 0u : v.z;
            r.any[w] = v.w;
        }
        return r;
    }
    return load_row<P, W>(rows, j, i);
}

// x = x + h * r (exact, Algorithm 3 / 4 after the scaling of Sec. 4.2)
// An empty asm that takes the (wave-uniform) words of a row as scalar
// operands: the loads of a group of rows are all issued before it, so they are
// not sunk one by one into the conditional blocks that use them.
template <int P, int W>
__device__ __forceinline__ void pin_row(const Row<W> &r) {
#pragma unroll
    for (int w = 0; w < W; w++) {
        asm volatile("" ::"s"(r.p[0][w]), "s"(r.p[1][w]));
        if constexpr (P == 7) asm volatile("" ::"s"(r.p[2][w]), "s"(r.any[w]));
    }
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

template <int P, int W, bool HIST>
__device__ __forceinline__ void count_hist(u32 *lh, u32 wt) {
    if constexpr (HIST) atomicAdd(&lh[wt], 1u);
}

// Weights of the combinations prefix + h * row for the p-1 prefixes of one
// lane and every multiplier h: F_3 needs v + w and v - w (Sec. 4.2); F_7 needs
// v +- 2^e w, e = 0, 1, 2, the scaling being a rotation of the planes.
// Isometric additions (Sec. 4.3) give the nonzero masks, popcount the weights.
template <int P, int W, int NA, bool HIST>
__device__ __forceinline__ void complete_all(const u32 (&Pv)[NA][3][W], const u32 (&anyP)[NA][W],
                                             const Row<W> &R, u32 &lmin, u32 *lh, u32 woff, u32 cap) {
#pragma unroll
    for (int a = 0; a < NA; a++) {
        if constexpr (P == 3) {
            u32 wa = 0, ws = 0;
#pragma unroll
            for (int w = 0; w < W; w++) {
                wa += __builtin_popcount(f3_iso_add(Pv[a][0][w], Pv[a][1][w], R.p[0][w], R.p[1][w]));
                ws += __builtin_popcount(f3_iso_sub(Pv[a][0][w], Pv[a][1][w], R.p[0][w], R.p[1][w]));
            }
            lmin = min(lmin, min(wa, ws));
            if constexpr (HIST) {
                count_hist<P, W, HIST>(lh, min(wa + woff, cap));
                count_hist<P, W, HIST>(lh, min(ws + woff, cap));
            }
        } else {
            u32 anyPR[W];
#pragma unroll
            for (int w = 0; w < W; w++) anyPR[w] = anyP[a][w] | R.any[w];
#pragma unroll
            for (int e = 0; e < 3; e++) {
                u32 wa = 0, ws = 0;
#pragma unroll
                for (int w = 0; w < W; w++) {
                    // rotation by e: S_i = R_{i-e} (multiplication by 2^e)
                    const u32 s0 = R.p[(3 - e) % 3][w], s1 = R.p[(4 - e) % 3][w], s2 = R.p[(5 - e) % 3][w];
                    const u32 x0 = Pv[a][0][w] ^ s0, x1 = Pv[a][1][w] ^ s1, x2 = Pv[a][2][w] ^ s2;
                    ws += __builtin_popcount(x0 | x1 | x2);                // prefix - 2^e row
                    wa += __builtin_popcount(~(x0 & x1 & x2) & anyPR[w]);  // prefix + 2^e row
                }
                lmin = min(lmin, min(wa, ws));
                if constexpr (HIST) {
                    count_hist<P, W, HIST>(lh, min(wa + woff, cap));
                    count_hist<P, W, HIST>(lh, min(ws + woff, cap));
                }
            }
        }
    }
}

// Prefixes Q + h * Rs for the NA coefficients h = 1..NA of row s, then every
// last row L = s+1..k-1 for all of them.  Returns the last rows combined
// (each gives NA (p-1) combinations per lane).
template <int P, int W, int NA, bool HIST>
__device__ __forceinline__ int extend_and_sweep(const u32 *__restrict__ rows, int j, int s, int k,
                                                const u32 (&Q)[3][W], const Row<W> &Rs, u32 &lmin, u32 *lh,
                                                u32 woff, u32 cap) {
    u32 Pv[NA][3][W], anyP[NA][W];
#pragma unroll
    for (int a = 0; a < NA; a++) {
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
            for (int w = 0; w < W; w++) Pv[a][b][w] = Q[b][w];
        add_scaled<P, W>(Pv[a], Rs.p, a + 1);
#pragma unroll
        for (int w = 0; w < W; w++) anyP[a][w] = Pv[a][0][w] | Pv[a][1][w] | Pv[a][2][w];
    }
    // UR rows per step, all loads issued before the first is used, so one wait
    // covers UR rows (rows past k-1 repeat row k-1 and are not combined)
    constexpr int UR = (W <= 2) ? 4 : 2;
    return sweep_last_rows<UR>(uni(s), k, [&](int L, int nr) {
        Row<W> R[UR];
#pragma unroll
        for (int u = 0; u < UR; u++) R[u] = load_row<P, W>(rows, j, min(L + u, k - 1));
#pragma unroll
        for (int u = 0; u < UR; u++) pin_row<P, W>(R[u]);
#pragma unroll
        for (int u = 0; u < UR; u++)
            if (u < nr) complete_all<P, W, NA, HIST>(Pv, anyP, R[u], lmin, lh, woff, cap);
    });
}

// One unit of a pair table (see pair_units): W words of 16 bytes at a
// wave-uniform index, held as a Row (F_3: planes 0, 1 of R_s + R_L in p[0],
// p[1] and of R_s - R_L in p[2], any).
// (through the constant address space: the table is read-only while the
// enumeration runs, so the wave-uniform loads are scalar loads)
typedef const __attribute__((address_space(4))) u32 *const_u32_ptr;
template <int W>
__device__ __forceinline__ Row<W> load_unit(const uint4 *__restrict__ ptab, int u) {
    const_u32_ptr src = (const_u32_ptr)(ptab + (size_t)u * W);
    Row<W> r;
#pragma unroll
    for (int w = 0; w < W; w++) {
        r.p[0][w] = src[4 * w];
        r.p[1][w] = src[4 * w + 1];
        r.p[2][w] = src[4 * w + 2];
        r.any[w] = src[4 * w + 3];
    }
    return r;
}

template <int W>
__device__ __forceinline__ void pin_unit(const Row<W> &r) {
#pragma unroll
    for (int w = 0; w < W; w++) asm volatile("" ::"s"(r.p[0][w]), "s"(r.p[1][w]), "s"(r.p[2][w]), "s"(r.any[w]));
}

// The combinations of an exact sum Q (its planes in Pv[0], nonzero mask in
// anyQ[0]) and one unit T of a pair table, through isometric additions and
// subtractions only: F_3 Q +- (R_s + R_L) and Q +- (R_s - R_L) (4); F_7
// Q + h T_c, h = +-2^e (complete_all with one prefix; 6).
template <int P, int W, bool HIST>
__device__ __forceinline__ void complete_unit(const u32 (&Pv)[1][3][W], const u32 (&anyQ)[1][W], const Row<W> &T,
                                              u32 &lmin, u32 *lh, u32 woff, u32 cap) {
    if constexpr (P == 3) {
        u32 wa = 0, ws = 0, wb = 0, wt = 0;
#pragma unroll
        for (int w = 0; w < W; w++) {
            wa += __builtin_popcount(f3_iso_add(Pv[0][0][w], Pv[0][1][w], T.p[0][w], T.p[1][w]));
            ws += __builtin_popcount(f3_iso_sub(Pv[0][0][w], Pv[0][1][w], T.p[0][w], T.p[1][w]));
            wb += __builtin_popcount(f3_iso_add(Pv[0][0][w], Pv[0][1][w], T.p[2][w], T.any[w]));
            wt += __builtin_popcount(f3_iso_sub(Pv[0][0][w], Pv[0][1][w], T.p[2][w], T.any[w]));
        }
        lmin = min(lmin, min(min(wa, ws), min(wb, wt)));
        if constexpr (HIST) {
            count_hist<P, W, HIST>(lh, min(wa + woff, cap));
            count_hist<P, W, HIST>(lh, min(ws + woff, cap));
            count_hist<P, W, HIST>(lh, min(wb + woff, cap));
            count_hist<P, W, HIST>(lh, min(wt + woff, cap));
        }
    } else {
        complete_all<P, W, 1, HIST>(Pv, anyQ, T, lmin, lh, woff, cap);
    }
}

// Every combination Q + h_s R_s + h_L R_L of the pairs [e0, e1) of a pair
// table with the lane's exact base Q, (p-1)^2 per pair: complete_unit for
// every unit of those pairs, UR units per step with their loads issued before
// the first is used; the last step's loads may run past the pairs' range into
// the next set's table or the buffer's PAIR_PAD_UNITS.  GROUPS: whole steps
// are one basic block each, so that the units' instructions interleave (the
// batched kernel: +0.9%; the plain kernel, bound by latency, ran 1% slower
// with the longer code).
template <int P, int W, bool HIST, bool GROUPS = false>
__device__ __forceinline__ void sweep_pairs(const uint4 *__restrict__ ptab, int e0, int e1, const u32 (&Q)[3][W],
                                            u32 &lmin, u32 *lh, u32 woff, u32 cap) {
    constexpr int UN = (P == 3) ? 1 : P - 1;
    constexpr int UR = (W <= 2) ? 4 : 2;
    u32 Pv[1][3][W], anyQ[1][W];
#pragma unroll
    for (int w = 0; w < W; w++) {
#pragma unroll
        for (int b = 0; b < 3; b++) Pv[0][b][w] = Q[b][w];
        anyQ[0][w] = Q[0][w] | Q[1][w] | Q[2][w];
    }
    const int u1 = uni(e1 * UN);
    int u = uni(e0 * UN);
    for (; GROUPS && u + UR <= u1; u += UR) {
        Row<W> T[UR];
#pragma unroll
        for (int i = 0; i < UR; i++) T[i] = load_unit<W>(ptab, u + i);
#pragma unroll
        for (int i = 0; i < UR; i++) pin_unit<W>(T[i]);
#pragma unroll
        for (int i = 0; i < UR; i++) complete_unit<P, W, HIST>(Pv, anyQ, T[i], lmin, lh, woff, cap);
    }
    for (; u < u1; u += UR) {
        Row<W> T[UR];
#pragma unroll
        for (int i = 0; i < UR; i++) T[i] = load_unit<W>(ptab, u + i);
#pragma unroll
        for (int i = 0; i < UR; i++) pin_unit<W>(T[i]);
#pragma unroll
        for (int i = 0; i < UR; i++) {
            if (u + i >= u1) break;
            complete_unit<P, W, HIST>(Pv, anyQ, T[i], lmin, lh, woff, cap);
        }
    }
}

// F_7: sweep_pairs for the NA exact sums of a run of bases at once (their
// planes in Pv, nonzero masks in anyP): each unit, loaded once, serves all of
// them (complete_all with NA prefixes), so the run's loads, loop control and
// waits are paid once instead of NA times.
template <int P, int W, bool HIST, int NA>
__device__ __forceinline__ void sweep_pairs_multi(const uint4 *__restrict__ ptab, int e0, int e1,
                                                  const u32 (&Pv)[NA][3][W], const u32 (&anyP)[NA][W], u32 &lmin,
                                                  u32 *lh, u32 woff, u32 cap) {
    static_assert(P == 7, "F_7 units");
    constexpr int UN = P - 1, UR = 4;
    const int u1 = uni(e1 * UN);
    int u = uni(e0 * UN);
    for (; u + UR <= u1; u += UR) {
        Row<W> T[UR];
#pragma unroll
        for (int i = 0; i < UR; i++) T[i] = load_unit<W>(ptab, u + i);
#pragma unroll
        for (int i = 0; i < UR; i++) pin_unit<W>(T[i]);
#pragma unroll
        for (int i = 0; i < UR; i++) complete_all<P, W, NA, HIST>(Pv, anyP, T[i], lmin, lh, woff, cap);
    }
    for (; u < u1; u++) {
        const Row<W> T = load_unit<W>(ptab, u);
        pin_unit<W>(T);
        complete_all<P, W, NA, HIST>(Pv, anyP, T, lmin, lh, woff, cap);
    }
}

// C(c, i) for c < crows and i < BIN_I into LDS: every load of a thread is
// issued before its first store (a loop that stores each value before the next
// load waits for one memory round trip per element).  blockDim.x = 256.
__device__ __forceinline__ void stage_binomials(u64 *sbin, const u64 *__restrict__ gbin, int crows) {
    constexpr int NMAX = BZ_MAX_K * BIN_I, PER = (NMAX + 255) / 256;
    const int N = min(crows, BZ_MAX_K) * BIN_I;
    u64 v[PER];
#pragma unroll
    for (int r = 0; r < PER; r++) {
        const int i = threadIdx.x + r * 256;
        v[r] = i < N ? gbin[(i / BIN_I) * 65 + i % BIN_I] : 0;
    }
#pragma unroll
    for (int r = 0; r < PER; r++) {
        const int i = threadIdx.x + r * 256;
        if (i < N) sbin[i] = v[r];
    }
}

// binomial C(c, i): LDS for small i, global memory otherwise
__device__ __forceinline__ u64 binom_at(const u64 *sbin, const u64 *__restrict__ gbin, int c, int i) {
    return (i < BIN_I) ? sbin[c * BIN_I + i] : gbin[c * 65 + i];
}

// Prefixes Q + a R for a = a0 .. a0+NA-1 and their nonzero masks, then every
// multiple of the last row T through complete_all.
template <int P, int W, int NA, bool HIST>
__device__ __forceinline__ void prefixes_then_complete(const u32 (&Q)[3][W], const Row<W> &R, int a0, const Row<W> &T,
                                                       u32 &lmin, u32 *lh, u32 woff, u32 cap) {
    u32 Pv[NA][3][W], anyP[NA][W];
#pragma unroll
    for (int a = 0; a < NA; a++) {
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
            for (int w = 0; w < W; w++) Pv[a][b][w] = Q[b][w];
        add_scaled<P, W>(Pv[a], R.p, a0 + a);
#pragma unroll
        for (int w = 0; w < W; w++) anyP[a][w] = Pv[a][0][w] | Pv[a][1][w] | Pv[a][2][w];
    }
    complete_all<P, W, NA, HIST>(Pv, anyP, T, lmin, lh, woff, cap);
}

// G = 3 (and 4 when SUBSET_G is 4): the lane's subset rows r[0] < ... <
// r[G-1]; r[0] has coefficient 1, the middle rows every multiplier (exact
// prefixes, one at a time to keep the registers in check), the top row every
// multiplier through complete_all.
// Adds the combinations completed to the lane's count ncomb.
template <int P, int W, int G, bool HIST>
__device__ __forceinline__ void run_subset(const u32 *__restrict__ rows, const uint4 *lrows, int j,
                                           const int (&r)[G], u32 &lmin, u32 &ncomb, u32 *lh, u32 woff, u32 cap) {
    constexpr int NA = 1;  // one prefix at a time (registers)
    const Row<W> R0 = load_row_lane<P, W>(rows, lrows, j, r[0]);
    const Row<W> R1 = load_row_lane<P, W>(rows, lrows, j, r[1]);
    const Row<W> R2 = load_row_lane<P, W>(rows, lrows, j, r[2]);
    if constexpr (G == 3) {
        for (int a0 = 1; a0 < P; a0 += NA) {
            prefixes_then_complete<P, W, NA, HIST>(R0.p, R1, a0, R2, lmin, lh, woff, cap);
            ncomb += NA * (P - 1);
        }
    } else {
        const Row<W> R3 = load_row_lane<P, W>(rows, lrows, j, r[3]);
        for (int h = 1; h < P; h++) {
            u32 Q[3][W];
#pragma unroll
            for (int b = 0; b < 3; b++)
#pragma unroll
                for (int w = 0; w < W; w++) Q[b][w] = R0.p[b][w];
            add_scaled<P, W>(Q, R1.p, h);
            for (int a0 = 1; a0 < P; a0 += NA) {
                prefixes_then_complete<P, W, NA, HIST>(Q, R2, a0, R3, lmin, lh, woff, cap);
                ncomb += NA * (P - 1);
            }
        }
    }
}

// g <= SUBSET_G: one item per lane (a row, a pair of rows, a triple; colex
// rank task * 64 + lane).  Adds the combinations the lane evaluated to lcnt.
template <int P, int W, bool HIST>
__device__ void run_small_task(int g, int k, int j, const u32 *__restrict__ rows, const uint4 *lrows,
                               const u64 *sbin, const u64 *__restrict__ gbin, u64 task, u32 &lmin, u64 &lcnt,
                               u32 *lh, u32 woff, u32 cap) {
    const int lane = __lane_id();
    const u64 item = task * 64 + (u64)lane;
    if (g == 1) {
        const bool valid = item < (u64)k;
        if (valid) {
            const Row<W> r = load_row<P, W>(rows, j, (int)item);
            u32 wt = 0;
#pragma unroll
            for (int w = 0; w < W; w++) wt += __builtin_popcount(r.any[w]);
            lmin = min(lmin, wt);
            if constexpr (HIST) count_hist<P, W, HIST>(lh, min(wt + woff, cap));
            lcnt += 1;
        }
        return;
    }
    if (g == 2) {
        // a pair s < L; row s has coefficient 1, row L every multiplier
        const bool pv = item < (u64)(k * (k - 1) / 2);
        if (pv) {
            int s, L;
            pair_of((int)item, k, &s, &L);
            const Row<W> Rs = load_row<P, W>(rows, j, s);
            const Row<W> RL = load_row<P, W>(rows, j, L);
            u32 Pv[1][3][W], A1[1][W];
#pragma unroll
            for (int b = 0; b < 3; b++)
#pragma unroll
                for (int w = 0; w < W; w++) Pv[0][b][w] = Rs.p[b][w];
#pragma unroll
            for (int w = 0; w < W; w++) A1[0][w] = Rs.any[w];
            complete_all<P, W, 1, HIST>(Pv, A1, RL, lmin, lh, woff, cap);
            lcnt += P - 1;
        }
        return;
    }
    auto bin = [&](int c, int i) { return binom_at(sbin, gbin, c, i); };
    const bool valid = item < binom_sat(k, g);
    u32 ncomb = 0;
    if (g == 3) {
        if (valid) {
            int r[3];
            decode_subset<3>(item, k, bin, r);
            run_subset<P, W, 3, HIST>(rows, lrows, j, r, lmin, ncomb, lh, woff, cap);
        }
    } else if constexpr (SUBSET_G >= 4) {
        if (valid) {
            int r[4];
            decode_subset<4>(item, k, bin, r);
            run_subset<P, W, 4, HIST>(rows, lrows, j, r, lmin, ncomb, lh, woff, cap);
        }
    }
    lcnt += ncomb;
}

// g > SUBSET_G: one task = (q, chunk of 64 lanes, block of rows s); see
// StageDesc.  A lane takes the r = (p-1)^vd consecutive bases (r bi, ...,
// r bi + r - 1): they differ in the coefficients of the first vd rows in
// decoding order, the top row q first.  The lane decodes the first of them
// and walks the others: F_3 in Gray-code order, one row added (coefficient
// 1 -> 2) or subtracted (2 -> 1) per step; F_7 (vd = 1) through the
// coefficients 1 .. 6 of row q, one addition of row q per step.  Adds the
// combinations the lane evaluated (the rows its sweeps combined) to lcnt.
// TABLE_ONLY: every caller passes a pair table, and the path without one is
// not compiled (it would hold the p-1 prefixes in registers).  GROUPS: see
// sweep_pairs.
template <int P, int W, bool HIST, bool TABLE_ONLY = false, bool GROUPS = false>
__device__ void run_base_task(const StageDesc &sd, int k, int j, const u32 *__restrict__ rows, const uint4 *lrows,
                              const uint4 *__restrict__ ptab, const u64 *sbin, const u64 *__restrict__ gbin,
                              const QEntry *qtab, int nq, u64 task, u32 &lmin, u64 &lcnt, u32 *lh, u32 woff,
                              u32 cap) {
    const int lane = __lane_id();
    const int g = uni(sd.g);
    const u64 M = uni(sd.coef_combos);
    const int qi = uni(qtable_find(qtab, nq, task));
    const int q = g - 3 + qi;
    // the q-group's entry as wave-uniform (scalar) values
    const u64 e_first = uni64(qtab[qi].first), e_bases = uni64(qtab[qi].bases);
    const uint32_t e_nb = uni(qtab[qi].nb);
    const int vd = uni(qtab[qi].vd);
    const u64 local = task - e_first;
    const u64 chunk = local / e_nb;
    const int block = (int)(local - chunk * e_nb);
    const int s_lo = q + 1 + uni(qgroup_block_start(k, q, e_nb, (uint32_t)block));
    const int s_hi = q + 1 + uni(qgroup_block_start(k, q, e_nb, (uint32_t)block + 1));
    const u64 bi = (chunk * 64 + (u64)lane) * (u64)run_len(P, (uint32_t)vd);
    const bool valid = bi < e_bases;  // the bases of a lane's run are valid together (its length divides bases)
    u32 Q[3][W];
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
        for (int w = 0; w < W; w++) Q[b][w] = 0;
    // combinations this lane completes: p-1 coefficients of row s times p-1
    // multipliers of every last row its sweeps combine
    constexpr u32 PER_ROW = (u32)((P - 1) * (P - 1));
    u32 ncomb = 0;
    // every row s of the block and every last row L > s for the lane's base Q:
    // from the set's pair table when it has one, else through the exact
    // prefixes Q + h R_s
    auto sweep_block = [&]() {
        if (TABLE_ONLY || ptab != nullptr) {
            const int e0 = uni((int)pair_first(s_lo, k)), e1 = uni((int)pair_first(s_hi, k));
            if (valid) {
                sweep_pairs<P, W, HIST, GROUPS>(ptab, e0, e1, Q, lmin, lh, woff, cap);
                ncomb += PER_ROW * (u32)(e1 - e0);
            }
            return;
        }
        if constexpr (!TABLE_ONLY) {
            for (int s = s_lo; s < s_hi; s++) {
                const Row<W> Rs = load_row<P, W>(rows, j, uni(s));
                if (valid)
                    ncomb += PER_ROW * (u32)extend_and_sweep<P, W, P - 1, HIST>(rows, j, s, k, Q, Rs, lmin, lh, woff,
                                                                                cap);
            }
        }
    };
    if (vd == 0) {
        // one base per lane
        if (valid) {
            decode_base<P>(g, q, M, bi, [&](int c, int i) { return binom_at(sbin, gbin, c, i); },
                           [&](int row, int coef) {
                               const Row<W> r = load_row_lane<P, W>(rows, lrows, j, row);
                               add_scaled<P, W>(Q, r.p, coef);
                           });
        }
        sweep_block();
        lcnt += ncomb;
        return;
    }
    if constexpr (P == 7) {
        // a run of 6 bases per lane: the first has coefficient 1 on row q (its
        // digit 0 is 0, the run being aligned), the next ones 2, ..., 6, each
        // one addition of row q (wave-uniform) away from the previous
        if (valid) {
            decode_base<P>(g, q, M, bi, [&](int c, int i) { return binom_at(sbin, gbin, c, i); },
                           [&](int row, int coef) {
                               const Row<W> r = load_row_lane<P, W>(rows, lrows, j, row);
                               add_scaled<P, W>(Q, r.p, coef);
                           });
        }
        const Row<W> Rq = load_row<P, W>(rows, j, q);
        if constexpr (TABLE_ONLY && W == 1) {
            // the six sums of the run at once (sweep_pairs_multi)
            u32 Pv[P - 1][3][W], anyP[P - 1][W];
#pragma unroll
            for (int v = 0; v < P - 1; v++) {
                if (v > 0) add_scaled<P, W>(Q, Rq.p, 1);
#pragma unroll
                for (int w = 0; w < W; w++) {
#pragma unroll
                    for (int b = 0; b < 3; b++) Pv[v][b][w] = Q[b][w];
                    anyP[v][w] = Q[0][w] | Q[1][w] | Q[2][w];
                }
            }
            const int e0 = uni((int)pair_first(s_lo, k)), e1 = uni((int)pair_first(s_hi, k));
            if (valid) {
                sweep_pairs_multi<P, W, HIST, P - 1>(ptab, e0, e1, Pv, anyP, lmin, lh, woff, cap);
                ncomb += (P - 1) * PER_ROW * (u32)(e1 - e0);
            }
        } else {
            for (int v = 0; v < P - 1; v++) {
                if (v > 0 && valid) add_scaled<P, W>(Q, Rq.p, 1);
                sweep_block();
            }
        }
    }
    if constexpr (P == 3) {
        // a run of 2^vd bases per lane; the rows of digits 1 and 2 are held
        // (lane-specific), row q (digit 0) is loaded again (wave-uniform)
        Row<W> Rd1, Rd2;
        if (valid) {
            int vi = 0;
            decode_base<P>(g, q, M, bi, [&](int c, int i) { return binom_at(sbin, gbin, c, i); },
                           [&](int row, int coef) {
                               const Row<W> r = load_row_lane<P, W>(rows, lrows, j, row);
                               add_scaled<P, W>(Q, r.p, coef);
                               if (vi == 1) Rd1 = r;
                               if (vi == 2) Rd2 = r;
                               vi++;
                           });
        }
        const int nv = 1 << vd;
        uint32_t cur = 0;  // bit t: digit t's row has coefficient 2 (wave-uniform)
        for (int v = 0; v < nv; v++) {
            if (v > 0) {
                const int t = __builtin_ctz((uint32_t)v);
                const int h = ((cur >> t) & 1u) ? 2 : 1;  // 1 -> 2: + row; 2 -> 1: - row = + 2 row
                cur ^= 1u << t;
                if (t == 0) {
                    const Row<W> Rq = load_row<P, W>(rows, j, q);
                    if (valid) add_scaled<P, W>(Q, Rq.p, h);
                } else if (t == 1) {
                    if (valid) add_scaled<P, W>(Q, Rd1.p, h);
                } else {
                    if (valid) add_scaled<P, W>(Q, Rd2.p, h);
                }
            }
            sweep_block();
        }
    }
    lcnt += ncomb;
}

// Stage-completion check, run by one whole wavefront: lane i looks at stage
// c + i, c being the first unchecked stage.  The stages c, c+1, ... whose
// workgroups are all done are checked in order (U takes their minima, a
// prefix minimum over the lanes) and the first with L_{g,j} >= U ends the
// run; one compare-and-swap publishes the new state.
__device__ void run_checker(CodeState *cs, const StageDesc *sdesc, int ns, const EnumArgs &ea) {
    const int lane = __lane_id();
    for (int guard = 0; guard <= 2 * BZ_MAX_STAGES; guard++) {
        u64 st = 0;
        if (lane == 0) st = rd_atomic(&cs->res.ctl);
        st = uni64(st);
        const int c = ctl_checked(st);
        if (c >= ns || ctl_term(st) >= 0) return;
        const int s = c + lane;
        // every participant's minimum was performed before its increment of done
        const bool done = s < ns && rd_atomic(&cs->stage_done[s]) == sdesc[s].parts;
        const u64 notdone = __ballot(!done);
        const int nd = notdone ? __builtin_ctzll(notdone) : 64;  // stages c .. c+nd-1 are done
        if (nd == 0) return;
        int u = (int)ctl_U(st);
        if (lane < nd) u = min(u, rd_atomic(&cs->res.stage_min[s]));
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(u, off);
            if (lane >= off) u = min(u, o);
        }
        const u64 stops = __ballot(lane < nd && sdesc[s].check && sdesc[s].L >= u);
        const int i = stops ? __builtin_ctzll(stops) : nd - 1;
        const int ui = __shfl(u, i);
        const u64 nw = stops ? ctl_make(c + i, c + i, ui) : ctl_make(c + nd, -1, ui);
        int ok = 0;
        if (lane == 0)
            ok = __hip_atomic_compare_exchange_strong(&cs->res.ctl, &st, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
        ok = __shfl(ok, 0);
        if (ok && lane < WAKE_COPIES)
            __hip_atomic_fetch_max(&cs->wake[lane][0], wake_make(ctl_checked(nw), ctl_term(nw)), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        // the run's result is final: the terminating stage is found, or every stage is checked
        if (ok && ea.res_out && (stops || c + nd >= ns)) hand_out_result(cs, ea.res_out, ea.flag_out, ea.epoch);
        // done: the run ended, or every done stage is checked; another checker
        // moved the state first: look again
        if (ok && (stops || nd < 64)) return;
    }
}

// TAB: the launch has pair tables (the base rounds take their two highest
// rows from them; no prefix path is compiled), or has none.
template <int P, int W, bool HIST, bool TAB>
__global__ __launch_bounds__(256) void enum_kernel(CodeState *cs, const u32 *__restrict__ rows,
                                                   const uint4 *__restrict__ pairs, const u64 *__restrict__ gbin,
                                                   u64 *__restrict__ hist, EnumArgs ea) {
    const int lookahead = ea.lookahead;
    const u64 timeout_ticks = ea.timeout_ticks;
    const int pslot1 = TAB ? uni(cs->pair_slot1) : 1;  // slot of set 1's pair table
    __shared__ u64 sbin[BZ_MAX_K * BIN_I];
    __shared__ StageDesc sdesc[BZ_MAX_STAGES];
    __shared__ QEntry qtab[BZ_MAX_K];
    __shared__ u32 lhist[HIST ? WAVES_PER_GROUP * (BZ_MAX_N + 1) : 1];
    __shared__ u32 red_min[WAVES_PER_GROUP];
    __shared__ u64 red_cnt[WAVES_PER_GROUP];
    __shared__ int s_term;
    __shared__ int s_crit;
    __shared__ u64 s_claim[2];
    __shared__ int s_cterm[2];
    // F_3: the rows of the first matrices, for the loads at lane-specific rows
    // (measured: 2-3% faster F_3 codes; F_7 codes slightly slower)
    __shared__ uint4 lrow_buf[P == 3 ? LROW_SETS * BZ_MAX_K * W : 1];
    const int lane = __lane_id();
    const int wid = threadIdx.x >> 6;
    const uint32_t grid = gridDim.x, b = blockIdx.x;
    const int k = ea.k, n = ea.n;
    const bool tracing = (ea.flags & FLAG_TRACE) != 0;
    // workgroup times from every TRACE_EVERY-th workgroup only: the real-time
    // counter is one unit for the whole device, and a thousand workgroups
    // reading it at the same moment (all leave a wait together) queue for tens
    // of microseconds, which would show up as a false spread of start times
    constexpr uint32_t TRACE_EVERY = 7;
    const bool tr_wg = tracing && blockIdx.x % TRACE_EVERY == 0;
    if (tr_wg && threadIdx.x == 0) atomicMin((unsigned long long *)&cs->trace[1][0], (unsigned long long)wall_clock64());
    // one round of independent loads: the decomposition's status and table
    // size, one stage descriptor per thread (ns <= BZ_MAX_STAGES = blockDim.x)
    // and the binomials
    static_assert(BZ_MAX_STAGES == 256, "one stage descriptor per thread");
    const int status0 = cs->res.status, ns0 = cs->res.n_table;
    constexpr int EARLY = 32;  // descriptors loaded before the table size is known
    if (threadIdx.x < EARLY) sdesc[threadIdx.x] = cs->stages[threadIdx.x];
    if constexpr (P == 3) {
        // the rows of the first LROW_SETS matrices (the row buffer holds every
        // set, so the sets past m read unused rows): loads issued before any store
        constexpr int NR = LROW_SETS * BZ_MAX_K * W, PER = (NR + 255) / 256;
        uint4 v[PER];
#pragma unroll
        for (int r = 0; r < PER; r++) {
            const int t = (int)threadIdx.x + r * 256;
            const int jj = t / (BZ_MAX_K * W), rem = t - jj * (BZ_MAX_K * W), i = rem / W, w = rem - i * W;
            if (t < NR) v[r] = reinterpret_cast<const uint4 *>(rows + (size_t)(jj * BZ_MAX_K + i) * ROW_WORDS)[w];
        }
#pragma unroll
        for (int r = 0; r < PER; r++) {
            const int t = (int)threadIdx.x + r * 256;
            if (t < NR) lrow_buf[t] = v[r];
        }
    }
    stage_binomials(sbin, gbin, k);  // the rows c < k: every binomial the stages read
    if (threadIdx.x >= EARLY && (int)threadIdx.x < ns0) sdesc[threadIdx.x] = cs->stages[threadIdx.x];
    __syncthreads();
    if (uni(status0) != BZ_OK) return;
    const int ns = uni(ns0);
    const bool skip = (ea.flags & FLAG_SKIP) != 0;
    u64 *wake = &cs->wake[b % WAKE_COPIES][0];
    u32 *lh = HIST ? &lhist[wid * (BZ_MAX_N + 1)] : nullptr;
    const u32 cap = (u32)n;
    const uint4 *lrows = nullptr;
    if constexpr (P == 3) lrows = lrow_buf;  // (filled before the first barrier)
    // the pool (see pool_stages): its stages complete when all their tiles
    // are done, so their part count in this workgroup's copy is the tile count
    u64 pool_tiles;
    const int sp = uni(pool_stages(sdesc, ns, grid, &pool_tiles));
    pool_tiles = uni64(pool_tiles);
    if ((int)threadIdx.x < sp) sdesc[threadIdx.x].parts = (uint32_t)sdesc[threadIdx.x].tiles;
    __syncthreads();

    // one tile of stage s: wavefront wid runs task tile * 4 + wid
    auto run_tile = [&](const StageDesc &sd, int s, u64 tile, u32 &lmin, u64 &lcnt) {
        const int sg = uni(sd.g);
        const u64 tasks = uni64(sd.tasks);
        const u64 task = tile * WAVES_PER_GROUP + (u64)wid;
        if (task >= tasks) return;  // a missing task only happens in the last tile
        const u32 woff = skip ? (u32)sg : 0u;
        if constexpr (HIST) {
            for (int w = lane; w <= n; w += 64) lh[w] = 0;
        }
        if (sg > SUBSET_G) {
            const int sj = uni(sd.j - 1);
            const uint4 *ptab = TAB ? pairs + (size_t)(sj == 1 ? pslot1 : sj) * ea.pair_stride : nullptr;
            run_base_task<P, W, HIST, TAB>(sd, k, sj, rows, lrows, ptab, sbin, gbin, qtab, k - 2 - (sg - 3), task,
                                           lmin, lcnt, lh, woff, cap);
        }
        else
            run_small_task<P, W, HIST>(sg, k, uni(sd.j - 1), rows, lrows, sbin, gbin, task, lmin, lcnt, lh, woff, cap);
        if constexpr (HIST) {
            for (int w = lane; w <= n; w += 64) {
                const u32 c = lh[w];
                if (c) atomicAdd((unsigned long long *)&hist[(size_t)s * (BZ_MAX_N + 1) + w], (unsigned long long)c);
            }
        }
    };
    // this workgroup's results for stage s: a workgroup reduction, then one set
    // of atomics; `add` counts towards the stage's parts (the workgroup that
    // completes them checks the stage and every done stage after it)
    // next >= 0: wavefront 1 builds the q-groups of stage next meanwhile (the
    // workgroup moves on to it)
    auto flush_stage = [&](int s, u32 lmin, u64 lcnt, uint32_t add, int next) {
        const StageDesc &sd = sdesc[s];
        const u32 woff = skip ? (u32)uni(sd.g) : 0u;
        for (int off = 32; off >= 1; off >>= 1) {
            lmin = min(lmin, (u32)__shfl_xor((int)lmin, off));
            lcnt += __shfl_xor(lcnt, off);
        }
        if (lane == 0) {
            red_min[wid] = lmin;
            red_cnt[wid] = lcnt;
        }
        if constexpr (HIST) drain_vmem();  // this wave's histogram atomics are performed
        __syncthreads();
        if (wid == 0) {
            uint32_t done = 0;
            if (lane == 0) {
                u32 bm = red_min[0];
                u64 bc = red_cnt[0];
                for (int w = 1; w < WAVES_PER_GROUP; w++) {
                    bm = min(bm, red_min[w]);
                    bc += red_cnt[w];
                }
                if (bm != BIG) atomicMin(&cs->res.stage_min[s], (int)(bm + woff));
                atomicAdd((unsigned long long *)&cs->res.stage_count[s], (unsigned long long)bc);
                drain_vmem();  // minimum and count performed before done counts this workgroup
                done = __hip_atomic_fetch_add(&cs->stage_done[s], add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + add;
                if (tr_wg || (tracing && done == sd.parts))  // the last one always
                    atomicMax((unsigned long long *)&cs->trace[2 + s][1], (unsigned long long)wall_clock64());
            }
            if (uni(done) == sd.parts) {
                run_checker(cs, sdesc, ns, ea);
                if (tracing && lane == 0)
                    atomicMax((unsigned long long *)&cs->trace[2 + s][2], (unsigned long long)wall_clock64());
            }
        } else if (wid == 1 && next >= 0 && sdesc[next].g > SUBSET_G) {
            const StageDesc &nd = sdesc[next];
            wave_qtable(P, k, nd.g, nd.coef_combos, nd.sweep_cap, nd.vcap, sbin, gbin, qtab);
        }
        __syncthreads();  // qtab and red_* are rewritten next
    };

    if (sp > 0) {
        // the pool: workgroup b runs pool tile b first, then claims the
        // others (grid and up) from its slice, each claim issued before the
        // tile in hand runs so that its latency is hidden, until the slice is
        // empty or the run has ended before the claimed tile's stage.  Claims
        // of one slice come in increasing order, so a workgroup's stages only
        // move forward; it reports a stage when it moves past it.
        const uint32_t C = pool_slices(grid), slice = b % C;
        uint32_t *ctr = &cs->pool_next[slice][0];
        int ps = -1;          // the stage whose results this workgroup holds
        u64 pbase = 0;        // its first pool tile
        uint32_t pheld = 0;   // its tiles done here
        u32 lmin = BIG;
        u64 lcnt = 0;
        u64 u = (u64)b < pool_tiles ? (u64)b : ~0ull;
        int t2 = -1;
        for (uint32_t it = 0;; it++) {
            // the next claim and the progress word, read while the tile runs
            uint32_t ci = 0;
            u64 wk = 0;
            if (threadIdx.x == 0 && u != ~0ull) {
                ci = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                wk = ld_poll(wake);
            }
            int sn = ps < 0 ? 0 : ps;
            bool end = u == ~0ull;
            if (!end) {
                sn = uni(pool_stage_of(sdesc, sp, sn, u, grid));
                // the run ended before this stage (the claim just made is of a
                // later stage still, and is dropped)
                end = t2 >= 0 && sn > t2;
            }
            if (ps >= 0 && (end || sn != ps)) {
                flush_stage(ps, lmin, lcnt, pheld, end ? -1 : sn);  // (with the q-groups of sn)
                lmin = BIG;
                lcnt = 0;
                pheld = 0;
            } else if (!end && sn != ps) {
                // the first stage of this workgroup
                const StageDesc &sd = sdesc[sn];
                if (wid == 0 && sd.g > SUBSET_G)
                    wave_qtable(P, k, sd.g, sd.coef_combos, sd.sweep_cap, sd.vcap, sbin, gbin, qtab);
                __syncthreads();
            }
            if (end) break;
            if (sn != ps) {
                ps = sn;
                pbase = nowait_offset(uni(sdesc[sn].rot), grid);
                if (tr_wg && threadIdx.x == 0) {
                    const unsigned long long now = (unsigned long long)wall_clock64();
                    atomicMin((unsigned long long *)&cs->trace[2 + sn][0], now);
                    atomicMax((unsigned long long *)&cs->trace[2 + sn][3], now);
                }
            }
            run_tile(sdesc[ps], ps, u - pbase, lmin, lcnt);
            pheld++;
            if (threadIdx.x == 0) {
                const u64 nu = (u64)grid + pool_tile(slice, ci, C);
                s_claim[it & 1] = nu < pool_tiles ? nu : ~0ull;
                s_cterm[it & 1] = wake_term(wk);
            }
            __syncthreads();  // (double buffers: the pair written two rounds ago was read before the last barrier)
            u = uni64(s_claim[it & 1]);
            t2 = uni(s_cterm[it & 1]);
        }
    }

    for (int s = sp; s < ns; s++) {
        const StageDesc &sd = sdesc[s];
        if (tile_of(0, b, grid, sd.rot) >= sd.tiles) continue;  // no tile of this stage here
        int term0 = 0;
        if (threadIdx.x == 0) {
            // a stage that is not nowait waits until every stage before
            // s - lookahead is checked, or the run ended
            // the clock and the status word are read every 256 polls only: the
            // real-time counter is one shared unit, slow when a thousand waves read it
            // (a nowait stage reads nothing: it starts at once, and work it
            // does after the run has ended is never read)
            u64 t0 = 0;
            int term = -1;
            u64 st = wake_make(-1, -1);
            for (uint32_t it = 0; !sd.nowait; it++) {
                st = ld_poll(wake);
                term = wake_term(st);
                if (term >= 0 || wake_checked(st) >= s - lookahead) break;
                if ((it & 255u) == 255u) {
                    if (ld_poll(&cs->res.status) != BZ_OK) {
                        term = -2;
                        break;
                    }
                    const u64 now = (u64)wall_clock64();
                    if (t0 == 0) {
                        t0 = now;
                    } else if (now - t0 > timeout_ticks) {
                        __hip_atomic_store(&cs->res.status, (int)BZ_ERR_DEVICE, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        term = -2;
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(8);
            }
            s_term = term;
            term0 = term;
            if (tr_wg) {
                const unsigned long long now = (unsigned long long)wall_clock64();
                atomicMin((unsigned long long *)&cs->trace[2 + s][0], now);
                atomicMax((unsigned long long *)&cs->trace[2 + s][3], now);
            }
            s_crit = wake_checked(st) >= s;  // the earliest unchecked stage: no later stage can wait on it
        }
        if (wid == 0 && sd.g > SUBSET_G) {
            // the q-groups of the stage, unless the run ended (thread 0 is lane 0 of wave 0)
            const int tw = __builtin_amdgcn_readfirstlane(term0);
            if (!(tw == -2 || (tw >= 0 && s > tw))) wave_qtable(P, k, sd.g, sd.coef_combos, sd.sweep_cap, sd.vcap, sbin, gbin, qtab);
        }
        __syncthreads();
        const int term = s_term;
        const bool crit = s_crit != 0;
        __syncthreads();  // every thread has read s_term: one decision for the whole workgroup
        if (term == -2 || (term >= 0 && s > term)) break;
        // work on the earliest unchecked stage runs at a higher wave priority than run-ahead work
        if (crit) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(0);
        u32 lmin = BIG;
        u64 lcnt = 0;  // combinations this lane evaluated in the stage
        for (u64 r = 0;; r++) {
            const u64 tile = tile_of(r, b, grid, sd.rot);
            if (tile >= sd.tiles) break;  // a missing tile only happens in the last round
            if (r > 0) {
                // a later stage after termination is abandoned (its results are never read)
                const int t2 = uni(lane == 0 ? wake_term(ld_poll(wake)) : 0);
                if (t2 >= 0 && s > t2) break;
            }
            run_tile(sd, s, tile, lmin, lcnt);
        }
        flush_stage(s, lmin, lcnt, 1u, -1);
    }
    if (tr_wg && threadIdx.x == 0) atomicMax((unsigned long long *)&cs->trace[1][1], (unsigned long long)wall_clock64());
}

// =====================================================================
// Batches: many codes of different p, n, k in one decomposition launch and
// one persistent enumeration launch
// =====================================================================

// One workgroup (one wavefront) per code (or per listed slot).  Also
// publishes the code's first claim word and counts it in
// BatchState::remaining.
__global__ __launch_bounds__(64) void decompose_batch_kernel(const uint8_t *__restrict__ G,
                                                             const BatchCode *__restrict__ codes, CodeState *css,
                                                             u64 *claims, u32 *__restrict__ rows,
                                                             uint4 *__restrict__ pairs, uint32_t grid,
                                                             BatchState *bs, const int32_t *__restrict__ slots,
                                                             uint32_t *done_flags, CodeResult *res_map) {
    __shared__ DecompLDS lds;
    if (threadIdx.x == 0) atomicMin((unsigned long long *)&bs->t0, (unsigned long long)wall_clock64());
    const int c = slots ? slots[blockIdx.x] : (int)blockIdx.x;  // a list of slots, or every code
    const BatchCode bc = codes[c];
    CodeState *cs = css + c;
    RunArgs a;
    a.n = bc.n;
    a.k = bc.k;
    a.flags = bc.flags;
    a.U0 = bc.U0;
    a.max_codewords = bc.max_codewords;
    a.grid = grid;
    a.sweep_ops = bc.sweep_ops;
    a.timeout_ticks = 0;
    a.rounds = nullptr;  // codes of every shape: the rounds are counted here
    a.spec = nullptr;
    a.epoch = 0;
    a.pad = 0;
    a.pairs = pairs + bc.pair_offset;  // every code of a batch or a serving slot has its tables
    a.pair_stride = bc.pair_stride;
    a.pair_w = bc.W;
    const uint8_t *g = G + bc.g_offset;
    u32 *r = rows + bc.row_offset;
    if (bc.p == 3) {
        switch (bc.WF) {
        case 1: decompose_code<3, 1>(g, cs, r, a, lds); break;
        case 2: decompose_code<3, 2>(g, cs, r, a, lds); break;
        case 3: decompose_code<3, 3>(g, cs, r, a, lds); break;
        default: decompose_code<3, 4>(g, cs, r, a, lds); break;
        }
    } else {
        switch (bc.WF) {
        case 1: decompose_code<7, 1>(g, cs, r, a, lds); break;
        case 2: decompose_code<7, 2>(g, cs, r, a, lds); break;
        case 3: decompose_code<7, 3>(g, cs, r, a, lds); break;
        default: decompose_code<7, 4>(g, cs, r, a, lds); break;
        }
    }
    int work = 0;
    if (threadIdx.x == 0) {
        // lane 0 wrote the status, the table size and stage 0 itself
        work = cs->res.status == BZ_OK && cs->res.n_table > 0;
        claims[c] = work ? claim_make(0, cs->stages[0].parts) : 0ull;
        if (work) atomicAdd(&bs->remaining, 1u);
        else cs->res.t_end = (u64)wall_clock64();  // nothing to enumerate: ends here
    }
    // serving: a code with nothing to enumerate is done at once; its result
    // block (written by this wavefront with plain stores) goes to the device's
    // memory first so that the hand-out's coherent loads see it
    if (!uni(work) && done_flags) {
        __threadfence();
        hand_out_result(cs, res_map ? res_map + c : nullptr, done_flags + c, 1u);
    }
}

// Serving: the predictor's inputs for the listed slots, from their
// decomposition (field, length, dimension, rank deficit of the last
// information set), normalised as the network was trained.
__global__ void features_kernel(const CodeState *__restrict__ css, const int32_t *__restrict__ slots, int n,
                                float *__restrict__ feat) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const CodeState &cs = css[slots[i]];
    const int m = cs.res.m;
    const int km = m > 0 ? cs.res.ranks[m - 1] : cs.k;
    mlp_features(cs.p, cs.n, cs.k, cs.k - km, feat + i * 4);
}

// The tiles of one part of a stage: tile_of(r, part, parts, rot) for r = 0, 1, ...
// The lane's combinations are added to lcnt.
template <int P, int W>
__device__ void run_part(const StageDesc &sd, int s, uint32_t part, int k, const u32 *__restrict__ rows,
                         const uint4 *__restrict__ ptab, const u64 *sbin, const u64 *__restrict__ gbin,
                         const QEntry *qtab, u32 woff, u32 cap, u32 &lmin, u64 &lcnt) {
    const int wid = threadIdx.x >> 6;
    const int g = uni(sd.g), j = uni(sd.j - 1), nq = k - 2 - (g - 3);
    const u64 tiles = uni64(sd.tiles), tasks = uni64(sd.tasks);
    const uint32_t parts = uni(sd.parts);
    for (u64 r = 0;; r++) {
        const u64 tile = tile_of(r, part, parts, sd.rot);
        if (tile >= tiles) break;
        const u64 task = tile * WAVES_PER_GROUP + (u64)wid;
        if (task >= tasks) continue;
        if (g > SUBSET_G)
            run_base_task<P, W, false, true, true>(sd, k, j, rows, nullptr, ptab, sbin, gbin, qtab, nq, task, lmin, lcnt, nullptr, woff,
                                      cap);
        else
            run_small_task<P, W, false>(g, k, j, rows, nullptr, sbin, gbin, task, lmin, lcnt, nullptr, woff, cap);
    }
}

// After the last part of stage s of a code: U takes the stage minimum, the
// L >= U test (Alg. 6) ends the code or publishes the next stage's claim word.
// Run by one whole wavefront; lane 0 applies the check.  done_flag (serving)
// is raised when the code ends, after its result block went to res_out.
__device__ void batch_check(CodeState *cs, u64 *claim, int s, const StageDesc &sd, BatchState *bs,
                            uint32_t *done_flag, CodeResult *res_out) {
    int last = 0;
    if (__lane_id() == 0) {
        const u64 st = rd_atomic(&cs->res.ctl);
        const int U = min((int)ctl_U(st), rd_atomic(&cs->res.stage_min[s]));
        const int ns = cs->res.n_table;
        const bool stop = sd.check && sd.L >= U;
        last = stop || s + 1 >= ns;
        if (last) __hip_atomic_store(&cs->res.t_end, (u64)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_exchange(&cs->res.ctl, stop ? ctl_make(s, s, U) : ctl_make(s + 1, -1, U), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
        drain_vmem();  // U is in place before the next stage can be claimed and checked
        __hip_atomic_exchange(claim, last ? 0ull : claim_make(s + 1, cs->stages[s + 1].parts),
                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (last) __hip_atomic_fetch_sub(&bs->remaining, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // serving: hand the result block and the done flag to the host (mapped memory)
    if (uni(last) && done_flag) hand_out_result(cs, res_out, done_flag, 1u);
}

// Persistent: every workgroup repeatedly claims one part of the
// current stage of some code (wave 0 scans 64 codes per step for an open claim
// word, starting after the code it took last), runs it, reports minimum and
// count, and the workgroup that finishes a stage's last part checks it.  Exits
// when no code has stages left.  Codes of every (p, W <= WMAX) share the launch.
// Serving adds three optional arrays: order (codes scanned in this priority
// order, always from the front), yield (mapped host flag: once set, workgroups
// stop claiming and exit after their current part; every code keeps its
// progress in its claim word for the next launch) and done_flags (mapped host
// flags raised as codes end).
template <int WMAX>
__global__ __launch_bounds__(256) void enum_batch_kernel(CodeState *css, u64 *claims,
                                                         const BatchCode *__restrict__ codes,
                                                         int ncodes, const u32 *__restrict__ rows,
                                                         const uint4 *__restrict__ pairs,
                                                         const u64 *__restrict__ gbin, BatchState *bs,
                                                         u64 timeout_ticks, const int32_t *__restrict__ order,
                                                         const uint32_t *yield, uint32_t *done_flags,
                                                         CodeResult *res_map) {
    __shared__ u64 sbin[BZ_MAX_K * BIN_I];
    __shared__ QEntry qtab[BZ_MAX_K];
    __shared__ u32 red_min[WAVES_PER_GROUP];
    __shared__ u64 red_cnt[WAVES_PER_GROUP];
    __shared__ int s_code, s_stage;
    __shared__ uint32_t s_part;
    const int lane = __lane_id();
    const int wid = threadIdx.x >> 6;
    stage_binomials(sbin, gbin, BZ_MAX_K);
    uint32_t scan = (uint32_t)((u64)blockIdx.x * (u64)ncodes / gridDim.x);
    __syncthreads();
    for (;;) {
        if (wid == 0) {
            int code = -1, stage = 0;
            uint32_t part = 0;
            u64 t0 = 0;
            for (uint32_t it = 0;; it++) {
                int rem = 0, bst = 0, yl = 0;
                if (lane == 0) {
                    rem = (int)ld_poll(&bs->remaining);
                    bst = ld_poll(&bs->status);
                    // host memory: read when a scan starts, then every 16th idle step
                    if (yield && (it & 15u) == 0u)
                        yl = (int)__hip_atomic_load(yield, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                if (uni(rem) == 0 || uni(bst) != BZ_OK || uni(yl) != 0) break;
                bool got = false;
                for (int base = 0; base < ncodes && !got; base += 64) {
                    const bool in = base + lane < ncodes;
                    const int c = order ? (in ? order[base + lane] : 0)
                                        : (int)((scan + (uint32_t)(base + lane)) % (uint32_t)ncodes);
                    bool open = false;
                    if (in) {
                        const u64 cw = ld_poll(&claims[c]);
                        open = claim_stage(cw) >= 0 && claim_next(cw) < claim_parts(cw);
                    }
                    u64 cands = __ballot(open);
                    while (cands) {
                        const int l = __builtin_ctzll(cands);
                        cands &= cands - 1;
                        const int cc = __shfl(c, l);
                        u64 old = 0;
                        if (lane == 0)
                            old = __hip_atomic_fetch_add(&claims[cc], 1ull, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                        old = uni64(old);
                        if (claim_stage(old) >= 0 && claim_next(old) < claim_parts(old)) {
                            code = cc;
                            stage = claim_stage(old);
                            part = claim_next(old);
                            got = true;
                            break;
                        }
                    }
                }
                if (got) break;
                if ((it & 255u) == 255u) {
                    u64 now = 0;
                    if (lane == 0) now = (u64)wall_clock64();
                    now = uni64(now);
                    if (t0 == 0) {
                        t0 = now;
                    } else if (now - t0 > timeout_ticks) {
                        if (lane == 0)
                            __hip_atomic_store(&bs->status, (int)BZ_ERR_DEVICE, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(8);
            }
            if (code >= 0) scan = (uint32_t)code + 1u;
            if (lane == 0) {
                s_code = code;
                s_stage = stage;
                s_part = part;
            }
        }
        __syncthreads();
        const int code = s_code;
        if (code < 0) break;
        const int s = s_stage;
        const uint32_t part = s_part;
        CodeState *cs = css + code;
        const int p = uni(codes[code].p), W = uni(codes[code].W), k = uni(codes[code].k);
        const int n = uni(codes[code].n);
        const u64 row_off = uni64(codes[code].row_offset);
        const StageDesc sd = cs->stages[s];
        if (wid == 0 && sd.g > SUBSET_G) wave_qtable(p, k, sd.g, sd.coef_combos, sd.sweep_cap, sd.vcap, sbin, gbin, qtab);
        __syncthreads();
        const u32 woff = (uni(codes[code].flags) & FLAG_SKIP) ? (u32)sd.g : 0u;
        const u32 cap = (u32)n;
        const u32 *r = rows + row_off;
        // (every code of a batch or a serving slot has its pair tables)
        const uint4 *pt = pairs + uni64(codes[code].pair_offset) + (size_t)uni(sd.j - 1) * uni(codes[code].pair_stride);
        u32 lmin = BIG;
        u64 lcnt = 0;
        if (p == 3) {
            if (W == 1) run_part<3, 1>(sd, s, part, k, r, pt, sbin, gbin, qtab, woff, cap, lmin, lcnt);
            if constexpr (WMAX >= 2) if (W == 2) run_part<3, 2>(sd, s, part, k, r, pt, sbin, gbin, qtab, woff, cap, lmin, lcnt);
            if constexpr (WMAX >= 3) if (W == 3) run_part<3, 3>(sd, s, part, k, r, pt, sbin, gbin, qtab, woff, cap, lmin, lcnt);
            if constexpr (WMAX >= 4) if (W == 4) run_part<3, 4>(sd, s, part, k, r, pt, sbin, gbin, qtab, woff, cap, lmin, lcnt);
        } else {
            if (W == 1) run_part<7, 1>(sd, s, part, k, r, pt, sbin, gbin, qtab, woff, cap, lmin, lcnt);
            if constexpr (WMAX >= 2) if (W == 2) run_part<7, 2>(sd, s, part, k, r, pt, sbin, gbin, qtab, woff, cap, lmin, lcnt);
            if constexpr (WMAX >= 3) if (W == 3) run_part<7, 3>(sd, s, part, k, r, pt, sbin, gbin, qtab, woff, cap, lmin, lcnt);
            if constexpr (WMAX >= 4) if (W == 4) run_part<7, 4>(sd, s, part, k, r, pt, sbin, gbin, qtab, woff, cap, lmin, lcnt);
        }
        for (int off = 32; off >= 1; off >>= 1) {
            lmin = min(lmin, (u32)__shfl_xor((int)lmin, off));
            lcnt += __shfl_xor(lcnt, off);
        }
        if (lane == 0) {
            red_min[wid] = lmin;
            red_cnt[wid] = lcnt;
        }
        __syncthreads();
        if (wid == 0) {
            uint32_t done = 0;
            if (lane == 0) {
                u32 bm = red_min[0];
                u64 bc = red_cnt[0];
                for (int w = 1; w < WAVES_PER_GROUP; w++) {
                    bm = min(bm, red_min[w]);
                    bc += red_cnt[w];
                }
                if (bm != BIG) atomicMin(&cs->res.stage_min[s], (int)(bm + woff));
                atomicAdd((unsigned long long *)&cs->res.stage_count[s], (unsigned long long)bc);
                drain_vmem();  // minimum and count performed before done counts this part
                done = __hip_atomic_fetch_add(&cs->stage_done[s], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
            }
            if (uni(done) == sd.parts)
                batch_check(cs, claims + code, s, sd, bs, done_flags ? done_flags + code : nullptr,
                            res_map ? res_map + code : nullptr);
        }
        __syncthreads();  // qtab, red_* and s_* are rewritten by the next claim
    }
}

// =====================================================================
// VALU issue-rate probe (the roofline's peak rates)
// =====================================================================
// Eight independent chains of one VALU instruction per thread, `iters` times
// eight instructions per thread, and one store per thread: the rate at which
// the chip issues that instruction.  OP: 0 v_xor_b32, 1 v_add_u32,
// 2 v_bitop3_b32, 3 v_bcnt_u32_b32, 4 v_min_u32, 5 v_fma_f32.
template <int OP>
__global__ __launch_bounds__(256) void valu_rate_kernel(u32 *out, int iters, u32 seed) {
    const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
    u32 a[8];
#pragma unroll
    for (int i = 0; i < 8; i++) a[i] = t + (u32)i + seed;
    const u32 b = seed * 3u + 1u, c = seed ^ 0x5555u;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int i = 0; i < 8; i++) {
            if constexpr (OP == 0) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[i]) : "v"(b));
            else if constexpr (OP == 1) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[i]) : "v"(b));
            else if constexpr (OP == 2)
                asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[i]) : "v"(b), "v"(c));
            else if constexpr (OP == 3) asm volatile("v_bcnt_u32_b32 %0, %1, %0" : "+v"(a[i]) : "v"(b));
            else if constexpr (OP == 4) asm volatile("v_min_u32 %0, %0, %1" : "+v"(a[i]) : "v"(b));
            else asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[i]) : "v"(b), "v"(c));
        }
    }
    u32 x = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) x ^= a[i];
    out[t] = x;
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

// One application of op to x (in place) with operand y.
template <int P, int OP>
__device__ __forceinline__ void apply_op(u32 (&x)[3], const u32 (&y)[3]) {
    if constexpr (P == 3) {
        if constexpr (OP == BZ_OP_ADD) f3_add(x[0], x[1], y[0], y[1], x[0], x[1]);
        else if constexpr (OP == BZ_OP_SUB) {
            u32 n0, n1;
            f3_neg(y[0], y[1], n0, n1);
            f3_add(x[0], x[1], n0, n1, x[0], x[1]);
        } else if constexpr (OP == BZ_OP_DOUBLE) f3_neg(x[0], x[1], x[0], x[1]);
        else if constexpr (OP == BZ_OP_ISO_ADD) { x[0] = f3_iso_add(x[0], x[1], y[0], y[1]); x[1] = 0; }
        else if constexpr (OP == BZ_OP_ISO_SUB) { x[0] = f3_iso_sub(x[0], x[1], y[0], y[1]); x[1] = 0; }
        else kat_add(x[0], x[1], y[0], y[1], x[0], x[1]);
    } else {
        if constexpr (OP == BZ_OP_ADD) f7_add(x[0], x[1], x[2], y[0], y[1], y[2], x[0], x[1], x[2]);
        else if constexpr (OP == BZ_OP_SUB) {
            u32 n0, n1, n2;
            f7_neg(y[0], y[1], y[2], n0, n1, n2);
            f7_add(x[0], x[1], x[2], n0, n1, n2, x[0], x[1], x[2]);
        } else if constexpr (OP == BZ_OP_DOUBLE) f7_double(x[0], x[1], x[2], x[0], x[1], x[2]);
        else if constexpr (OP == BZ_OP_ISO_ADD) { x[0] = f7_iso_add(x[0], x[1], x[2], y[0], y[1], y[2]); x[1] = x[2] = 0; }
        else { x[0] = f7_iso_sub(x[0], x[1], x[2], y[0], y[1], y[2]); x[1] = x[2] = 0; }
    }
}

// out = op applied reps times to a with operand b (x <- op(x, b), x = a first):
// a + reps*b, a - reps*b, 2^reps a; the isometric masks take reps = 1.  One
// thread per (vector, word); the chain stays in registers, so reps > 1 times
// the arithmetic itself and reps = 1 one streaming pass over HBM.
template <int P, int OP>
__global__ void op_kernel(int nvec, int words, const u32 *__restrict__ A, const u32 *__restrict__ B,
                          u32 *__restrict__ O, int reps) {
    constexpr int R = (P == 3) ? 2 : 3;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)nvec * words) return;
    const int v = (int)(idx / words), w = (int)(idx % words);
    u32 x[3] = {0, 0, 0}, y[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < R; i++) {
        x[i] = A[((size_t)v * R + i) * words + w];
        y[i] = B ? B[((size_t)v * R + i) * words + w] : 0u;
    }
    for (int rep = 0; rep < reps; rep++) apply_op<P, OP>(x, y);
#pragma unroll
    for (int i = 0; i < R; i++) O[((size_t)v * R + i) * words + w] = x[i];
}

}  // namespace bz
