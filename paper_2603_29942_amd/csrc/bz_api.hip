// bz_api.hip -- host side of the C ABI declared in include/bz.h.
//
// Per device, one context holds the library stream, the device workspace
// (code state, packed Gamma_j rows, binomial table, histograms) and a pinned
// host buffer for the results; it is created on first use and kept until the
// process ends.  A call validates its arguments, launches the decomposition
// and the persistent enumeration kernel back to back on the stream, copies the
// compact result block back and rebuilds the stage trace from it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <vector>

#include "bz_kernels.hpp"
#include "bz_mlp.hpp"

using namespace bz;

// The device state of bz_min_distance_noalloc (see there).  In host code this
// name only stands for the array: its device address comes from
// hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[BZ_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEV = 16;

struct DevCtx {
    bool ready = false;
    int cu = 0;
    u64 ticks_per_s = 0;
    hipStream_t stream = nullptr;
    uint8_t *g_buf = nullptr;
    CodeState *cs = nullptr;
    u32 *rows = nullptr;
    uint4 *pairs = nullptr;  // the pair tables of the sets (pair_table_units per set)
    u64 *binom = nullptr;
    u64 *hist = nullptr;
    CodeResult *host_res = nullptr;
    // mapped host memory the final check writes the result block to, and the
    // flag it raises after it (the call's epoch); device addresses of both
    CodeResult *res_map = nullptr, *res_map_dev = nullptr;
    uint32_t *flag_map = nullptr, *flag_map_dev = nullptr;
    uint32_t epoch = 0;
    u64 *host_hist = nullptr;
    u64 (*host_trace)[4] = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    // batch workspace, grown on demand and kept
    size_t b_codes_cap = 0, b_rows_cap = 0, b_g_cap = 0, b_pairs_cap = 0;
    CodeState *b_cs = nullptr;
    u64 *b_claims = nullptr;  // the codes' claim words, contiguous
    BatchCode *b_codes = nullptr;
    u32 *b_rows = nullptr;
    uint4 *b_pairs = nullptr;
    uint8_t *b_g = nullptr;
    BatchState *b_state = nullptr;
    CodeResult *b_host_res = nullptr;
    BatchState *b_host_state = nullptr;
    // the rounds' task counts per shape (p, k, W, grid, task size), on the
    // device, built once on first use (fill_round_table)
    std::map<u64, RoundTable *> rounds;  // key: (p, k, W, grid, task size) in 64 bits
    // the second information set computed ahead by a second workgroup of the
    // decomposition launch, and the value its flag takes in this call
    SpecBuf *spec = nullptr;
    uint32_t spec_epoch = 0;
    // ordering of plain calls across streams: done_ev is recorded after the
    // enumeration launch of the last plain call, on last_stream (its late
    // workgroups may still update the workspace after the call returned)
    hipEvent_t done_ev = nullptr;
    hipStream_t last_stream = nullptr;
    bool have_last = false;
    // servers running on this device (their rounds yield to plain calls),
    // guarded by srv_mu; plain_active = 1 while a plain call runs, and no
    // server starts a round meanwhile
    std::vector<bz_server *> servers;
    std::mutex srv_mu;
    std::atomic<int> plain_active{0};
    std::mutex mu;  // serialises the plain calls (and everything else) on the device
};

DevCtx g_ctx[MAX_DEV];
std::mutex g_init_mu;

// binomial coefficients C(c, i), c, i <= 64 (exact in 64 bits)
const u64 *host_binom() {
    static u64 tab[65 * 65];
    static std::once_flag once;
    std::call_once(once, [] { fill_binomials(tab); });
    return tab;
}

#define HIP_OK(expr)                              \
    do {                                          \
        if ((expr) != hipSuccess) return BZ_ERR_DEVICE; \
    } while (0)

// 16-byte units of the pair tables of one code: every set it can produce
// (slots 0 .. pair_sets - 1), plus, on the plain path, the slot pair_sets
// that the workgroup computing the second set ahead builds its table in
u64 code_pair_units(int p, int n, int k, int W, bool ahead_slot) {
    return (u64)(pair_sets(n, k) + (ahead_slot ? 1 : 0)) * pair_table_units(p, k, W);
}

// the largest code_pair_units of any code with n <= max_n (p = 7 has the
// larger tables; W as the enumeration takes it: with the identity skip when
// skip is 1, without it when 0, either when -1)
u64 max_pair_units(int max_n, int skip, bool ahead_slot) {
    u64 best = 0;
    for (int n = 1; n <= max_n; n++)
        for (int k = 1; k <= n && k <= BZ_MAX_K; k++) {
            const int WF = (n + 31) / 32, Ws = (n - k + 31) / 32 < 1 ? 1 : (n - k + 31) / 32;
            for (int W : {WF, Ws}) {
                if ((skip == 1 && W != Ws) || (skip == 0 && W != WF)) continue;
                const u64 u = code_pair_units(7, n, k, W, ahead_slot);
                if (u > best) best = u;
            }
        }
    return best;
}

int init_ctx(int dev) {
    DevCtx &c = g_ctx[dev];
    if (c.ready) return BZ_OK;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || dev >= ndev) return BZ_ERR_DEVICE;
    HIP_OK(hipSetDevice(dev));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BZ_ERR_DEVICE;
    c.cu = prop.multiProcessorCount;
    int rate_khz = 0;
    HIP_OK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    c.ticks_per_s = (u64)(rate_khz > 0 ? rate_khz : 100000) * 1000ull;
    // a blocking stream: work queued earlier on the null stream (where callers such as
    // torch place their copies by default) completes before the library reads its inputs
    HIP_OK(hipStreamCreateWithFlags(&c.stream, hipStreamDefault));
    if (hipMalloc(&c.g_buf, (size_t)BZ_MAX_K * BZ_MAX_N) != hipSuccess) return BZ_ERR_NOMEM;
    if (hipMalloc(&c.cs, sizeof(CodeState)) != hipSuccess) return BZ_ERR_NOMEM;
    if (hipMalloc(&c.rows, sizeof(u32) * BZ_MAX_M * BZ_MAX_K * ROW_WORDS) != hipSuccess) return BZ_ERR_NOMEM;
    if (hipMalloc(&c.pairs, sizeof(uint4) * (max_pair_units(BZ_MAX_N, -1, true) + PAIR_PAD_UNITS)) != hipSuccess)
        return BZ_ERR_NOMEM;
    if (hipMalloc(&c.binom, sizeof(u64) * 65 * 65) != hipSuccess) return BZ_ERR_NOMEM;
    if (hipMalloc(&c.hist, sizeof(u64) * BZ_MAX_STAGES * (BZ_MAX_N + 1)) != hipSuccess) return BZ_ERR_NOMEM;
    if (hipMalloc(&c.spec, sizeof(SpecBuf)) != hipSuccess) return BZ_ERR_NOMEM;
    HIP_OK(hipMemset(c.spec, 0, sizeof(SpecBuf)));
    if (hipHostMalloc(&c.host_res, sizeof(CodeResult), hipHostMallocDefault) != hipSuccess) return BZ_ERR_NOMEM;
    if (hipHostMalloc(&c.host_hist, sizeof(u64) * BZ_MAX_STAGES * (BZ_MAX_N + 1), hipHostMallocDefault) !=
        hipSuccess)
        return BZ_ERR_NOMEM;
    if (hipHostMalloc(&c.host_trace, sizeof(CodeState::trace), hipHostMallocDefault) != hipSuccess)
        return BZ_ERR_NOMEM;
    if (hipHostMalloc(&c.res_map, sizeof(CodeResult), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(&c.flag_map, sizeof(uint32_t), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return BZ_ERR_NOMEM;
    *c.flag_map = 0;
    HIP_OK(hipHostGetDevicePointer((void **)&c.res_map_dev, c.res_map, 0));
    HIP_OK(hipHostGetDevicePointer((void **)&c.flag_map_dev, c.flag_map, 0));
    HIP_OK(hipMemcpy(c.binom, host_binom(), sizeof(u64) * 65 * 65, hipMemcpyHostToDevice));
    // timing only: no system-scope fence at the records (the results are read after a
    // stream synchronisation anyway), which otherwise writes back and invalidates caches
    for (auto &e : c.ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    HIP_OK(hipEventCreateWithFlags(&c.done_ev, hipEventDisableTiming));
    c.have_last = false;
    c.ready = true;
    return BZ_OK;
}

// Frees what init_ctx and later calls set up for the device (the caller holds
// c.mu, the device is current and no server is registered).
void release_ctx(DevCtx &c) {
    // teardown: errors are not actionable here
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    if (c.have_last && c.done_ev) (void)hipEventSynchronize(c.done_ev);
    for (auto &kv : c.rounds) (void)hipFree(kv.second);
    c.rounds.clear();
    for (void *p : {(void *)c.g_buf, (void *)c.cs, (void *)c.rows, (void *)c.pairs, (void *)c.binom, (void *)c.hist,
                    (void *)c.spec, (void *)c.b_cs, (void *)c.b_claims, (void *)c.b_codes, (void *)c.b_rows,
                    (void *)c.b_pairs, (void *)c.b_g, (void *)c.b_state})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)c.host_res, (void *)c.host_hist, (void *)c.host_trace, (void *)c.res_map,
                    (void *)c.flag_map, (void *)c.b_host_res, (void *)c.b_host_state})
        if (p) (void)hipHostFree(p);
    for (auto &e : c.ev)
        if (e) (void)hipEventDestroy(e);
    if (c.done_ev) (void)hipEventDestroy(c.done_ev);
    if (c.stream) (void)hipStreamDestroy(c.stream);
    c.g_buf = nullptr;
    c.cs = nullptr;
    c.rows = nullptr;
    c.pairs = nullptr;
    c.binom = nullptr;
    c.hist = nullptr;
    c.spec = nullptr;
    c.b_cs = nullptr;
    c.b_claims = nullptr;
    c.b_codes = nullptr;
    c.b_rows = nullptr;
    c.b_pairs = nullptr;
    c.b_g = nullptr;
    c.b_state = nullptr;
    c.host_res = nullptr;
    c.host_hist = nullptr;
    c.host_trace = nullptr;
    c.res_map = c.res_map_dev = nullptr;
    c.flag_map = c.flag_map_dev = nullptr;
    c.b_host_res = nullptr;
    c.b_host_state = nullptr;
    c.b_codes_cap = c.b_rows_cap = c.b_g_cap = c.b_pairs_cap = 0;
    for (auto &e : c.ev) e = nullptr;
    c.done_ev = nullptr;
    c.stream = nullptr;
    c.last_stream = nullptr;
    c.have_last = false;
    c.ready = false;
}

int get_ctx(int dev, DevCtx **out) {
    if (dev < 0 || dev >= MAX_DEV) return BZ_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_init_mu);
    int st = init_ctx(dev);
    if (st != BZ_OK) return st;
    *out = &g_ctx[dev];
    return BZ_OK;
}

__global__ void zero_u64(u64 *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---- kernel dispatch over (P, words)
template <int P>
hipError_t launch_decompose(int WF, const uint8_t *G, CodeState *cs, u32 *rows, RunArgs a,
                            hipStream_t s) {
    // workgroup 1 computes the second information set ahead; one more builds
    // the first set's pair table (see ROLE_TABLE0)
    const int nb = 1 + (a.spec ? 1 : 0) + (a.pairs && a.pair_t0 ? 1 : 0);
    switch (WF) {
    case 1: decompose_kernel<P, 1><<<nb, 64, 0, s>>>(G, cs, rows, a); break;
    case 2: decompose_kernel<P, 2><<<nb, 64, 0, s>>>(G, cs, rows, a); break;
    case 3: decompose_kernel<P, 3><<<nb, 64, 0, s>>>(G, cs, rows, a); break;
    default: decompose_kernel<P, 4><<<nb, 64, 0, s>>>(G, cs, rows, a); break;
    }
    return hipGetLastError();
}

// The enumeration kernel's grid (see enum_grid) is clamped to its occupancy,
// so on an otherwise idle device every workgroup is resident at once, which
// its waits for earlier stages rely on (plain calls hold the device's server
// rounds off while they run).
template <int P, int W, bool H>
hipError_t launch_enum_one(int grid, CodeState *cs, const u32 *rows, const uint4 *pairs, const u64 *binom, u64 *hist,
                           EnumArgs ea, hipStream_t s) {
    // with pair tables the instantiation that has no prefix path, else the one without tables
    if (pairs != nullptr) enum_kernel<P, W, H, true><<<grid, 256, 0, s>>>(cs, rows, pairs, binom, hist, ea);
    else enum_kernel<P, W, H, false><<<grid, 256, 0, s>>>(cs, rows, nullptr, binom, hist, ea);
    return hipGetLastError();
}

template <int P, bool H>
hipError_t launch_enum_h(int W, int grid, CodeState *cs, const u32 *rows, const uint4 *pairs, const u64 *binom,
                         u64 *hist, EnumArgs ea, hipStream_t s) {
    switch (W) {
    case 1: return launch_enum_one<P, 1, H>(grid, cs, rows, pairs, binom, hist, ea, s);
    case 2: return launch_enum_one<P, 2, H>(grid, cs, rows, pairs, binom, hist, ea, s);
    case 3: return launch_enum_one<P, 3, H>(grid, cs, rows, pairs, binom, hist, ea, s);
    default: return launch_enum_one<P, 4, H>(grid, cs, rows, pairs, binom, hist, ea, s);
    }
}

template <int P>
hipError_t launch_enum(bool hist_mode, int W, int grid, CodeState *cs, const u32 *rows, const uint4 *pairs,
                       const u64 *binom, u64 *hist, EnumArgs ea, hipStream_t s) {
    return hist_mode ? launch_enum_h<P, true>(W, grid, cs, rows, pairs, binom, hist, ea, s)
                     : launch_enum_h<P, false>(W, grid, cs, rows, pairs, binom, hist, ea, s);
}

// Largest grid the enumeration kernel may get for (p, W, histograms, pair
// tables): the schedule is dealt to exactly this many workgroups.
template <int P, int W, bool H, bool T>
int grid_for(int cu, int bpc) {
    static int max_bpc = -1;
    if (max_bpc < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, enum_kernel<P, W, H, T>, 256, 0) != hipSuccess || nb < 1)
            return -1;
        max_bpc = nb;
    }
    return cu * (bpc < max_bpc ? bpc : max_bpc);
}

template <int P, bool H, bool T>
int grid_for_w(int W, int cu, int bpc) {
    switch (W) {
    case 1: return grid_for<P, 1, H, T>(cu, bpc);
    case 2: return grid_for<P, 2, H, T>(cu, bpc);
    case 3: return grid_for<P, 3, H, T>(cu, bpc);
    default: return grid_for<P, 4, H, T>(cu, bpc);
    }
}

template <int P, bool T>
int enum_grid_t(bool hist, int W, int cu, int bpc) {
    return hist ? grid_for_w<P, true, T>(W, cu, bpc) : grid_for_w<P, false, T>(W, cu, bpc);
}

int enum_grid(int p, bool hist, bool tables, int W, int cu, int bpc) {
    if (p == 3) return tables ? enum_grid_t<3, true>(hist, W, cu, bpc) : enum_grid_t<3, false>(hist, W, cu, bpc);
    return tables ? enum_grid_t<7, true>(hist, W, cu, bpc) : enum_grid_t<7, false>(hist, W, cu, bpc);
}

// A plain call needs every workgroup of its persistent launch resident: it
// holds the device's servers off while it runs (defined after bz_server).
void servers_hold(DevCtx &c);
void servers_release(DevCtx &c);
struct PlainGuard {
    DevCtx *c;
    explicit PlainGuard(DevCtx *c_) : c(c_) { servers_hold(*c); }
    ~PlainGuard() { servers_release(*c); }
    PlainGuard(const PlainGuard &) = delete;
    PlainGuard &operator=(const PlainGuard &) = delete;
};

int check_args(int p, int n, int k, const void *G, const void *out) {
    if (p != 3 && p != 7) return BZ_ERR_ARG;
    if (n < 1 || n > BZ_MAX_N || k < 1 || k > BZ_MAX_K || k > n) return BZ_ERR_ARG;
    if (!G || !out) return BZ_ERR_ARG;
    return BZ_OK;
}

// Rebuild the trace from the per-stage minima and counts; returns the status.
int finish(int p, int n, int k, int flags, u64 max_cw, const CodeResult &r, bz_result *out,
           uint32_t sweep_ops = DEFAULT_SWEEP_OPS) {
    std::memset(out, 0, sizeof *out);
    out->m = r.m;
    out->info = r.info;
    for (int j = 0; j < r.m && j < BZ_MAX_M; j++) out->ranks[j] = r.ranks[j];
    if (r.status != BZ_OK) return r.status;
    StageDesc st[BZ_MAX_STAGES];
    int complete = 1;
    int ns = 0;
    const int U0 = n - k + 1;
    if ((flags & FLAG_NO_TERM) || U0 > 1) {
        // the stage list without the task counts first (they only matter where a
        // round would reach 2^62 tasks); with them when the stage counts differ
        const u64 lim = max_cw ? max_cw : DEFAULT_LIMIT;
        ns = build_schedule(p, k, r.m, r.ranks, flags, lim, 1, r.W, host_binom(), st, &complete, false, sweep_ops);
        if (ns != r.n_table)
            ns = build_schedule(p, k, r.m, r.ranks, flags, lim, 1, r.W, host_binom(), st, &complete, true, sweep_ops);
    }
    if (ns != r.n_table) return BZ_ERR_DEVICE;
    int U = U0, term = -1;
    out->terminated_by = 2;
    for (int s = 0; s < ns; s++) {
        bz_stage &o = out->stages[s];
        o.g = st[s].g;
        o.j = st[s].j;
        o.codewords = r.stage_count[s];
        o.stage_min = r.stage_min[s];
        U = std::min(U, r.stage_min[s]);
        o.upper_after = U;
        o.lower_after = st[s].L;
        out->codewords_total += o.codewords;
        out->n_stages = s + 1;
        out->terminated_by = 1;
        if (st[s].check && st[s].L >= U) {
            term = s;
            out->terminated_by = 0;
            break;
        }
    }
    if (term != ctl_term(r.ctl)) return BZ_ERR_DEVICE;  // device and host disagree on the schedule
    out->d = U;
    if (term < 0 && !r.table_complete) {
        out->terminated_by = 1;
        return BZ_ERR_LIMIT;
    }
    return BZ_OK;
}

template <int P>
void launch_op(int op, int blocks, hipStream_t s, int nvec, int words, const u32 *a, const u32 *b, u32 *out,
               int reps) {
    switch (op) {
    case BZ_OP_ADD: op_kernel<P, BZ_OP_ADD><<<blocks, 256, 0, s>>>(nvec, words, a, b, out, reps); break;
    case BZ_OP_SUB: op_kernel<P, BZ_OP_SUB><<<blocks, 256, 0, s>>>(nvec, words, a, b, out, reps); break;
    case BZ_OP_DOUBLE: op_kernel<P, BZ_OP_DOUBLE><<<blocks, 256, 0, s>>>(nvec, words, a, b, out, reps); break;
    case BZ_OP_ISO_ADD: op_kernel<P, BZ_OP_ISO_ADD><<<blocks, 256, 0, s>>>(nvec, words, a, b, out, reps); break;
    case BZ_OP_ISO_SUB: op_kernel<P, BZ_OP_ISO_SUB><<<blocks, 256, 0, s>>>(nvec, words, a, b, out, reps); break;
    default: op_kernel<P, BZ_OP_KAT_ADD><<<blocks, 256, 0, s>>>(nvec, words, a, b, out, reps); break;
    }
}

// ---- batches
template <int WMAX>
int batch_grid_w(int cu, int bpc) {
    static int max_bpc = -1;
    if (max_bpc < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, enum_batch_kernel<WMAX>, 256, 0) != hipSuccess ||
            nb < 1)
            return -1;
        max_bpc = nb;
    }
    return cu * (bpc < max_bpc ? bpc : max_bpc);
}

int batch_grid(int wmax, int cu, int bpc) {
    return wmax <= 2 ? batch_grid_w<2>(cu, bpc) : batch_grid_w<4>(cu, bpc);
}

// rows of one code: at most min(BZ_MAX_M, n - k + 1) information sets (each
// after the first takes at least one new column), 64 row slots each
u64 batch_row_words(int n, int k) {
    const int m = n - k + 1 < BZ_MAX_M ? n - k + 1 : BZ_MAX_M;
    return (u64)m * 64 * ROW_WORDS;
}

int grow_batch(DevCtx &c, size_t ncodes, size_t row_words, size_t pair_units, size_t g_bytes) {
    if (ncodes > c.b_codes_cap) {
        // (errors of the frees are not actionable here; every pointer is reset so
        // that a failed allocation below leaves nothing to free twice)
        if (c.b_cs) (void)hipFree(c.b_cs);
        if (c.b_claims) (void)hipFree(c.b_claims);
        if (c.b_codes) (void)hipFree(c.b_codes);
        if (c.b_host_res) (void)hipHostFree(c.b_host_res);
        c.b_cs = nullptr;
        c.b_claims = nullptr;
        c.b_codes = nullptr;
        c.b_host_res = nullptr;
        c.b_codes_cap = 0;
        if (hipMalloc(&c.b_cs, sizeof(CodeState) * ncodes) != hipSuccess) return BZ_ERR_NOMEM;
        if (hipMalloc(&c.b_claims, sizeof(u64) * ncodes) != hipSuccess) return BZ_ERR_NOMEM;
        if (hipMalloc(&c.b_codes, sizeof(BatchCode) * ncodes) != hipSuccess) return BZ_ERR_NOMEM;
        if (hipHostMalloc(&c.b_host_res, sizeof(CodeResult) * ncodes, hipHostMallocDefault) != hipSuccess)
            return BZ_ERR_NOMEM;
        c.b_codes_cap = ncodes;
    }
    if (row_words > c.b_rows_cap) {
        if (c.b_rows) (void)hipFree(c.b_rows);
        c.b_rows = nullptr;
        c.b_rows_cap = 0;
        if (hipMalloc(&c.b_rows, sizeof(u32) * row_words) != hipSuccess) return BZ_ERR_NOMEM;
        c.b_rows_cap = row_words;
    }
    if (pair_units > c.b_pairs_cap) {
        if (c.b_pairs) (void)hipFree(c.b_pairs);
        c.b_pairs = nullptr;
        c.b_pairs_cap = 0;
        if (hipMalloc(&c.b_pairs, sizeof(uint4) * (pair_units + PAIR_PAD_UNITS)) != hipSuccess) return BZ_ERR_NOMEM;
        c.b_pairs_cap = pair_units;
    }
    if (g_bytes > c.b_g_cap) {
        if (c.b_g) (void)hipFree(c.b_g);
        c.b_g = nullptr;
        c.b_g_cap = 0;
        if (hipMalloc(&c.b_g, g_bytes) != hipSuccess) return BZ_ERR_NOMEM;
        c.b_g_cap = g_bytes;
    }
    if (!c.b_state) {
        if (hipMalloc(&c.b_state, sizeof(BatchState)) != hipSuccess) return BZ_ERR_NOMEM;
        if (hipHostMalloc(&c.b_host_state, sizeof(BatchState), hipHostMallocDefault) != hipSuccess)
            return BZ_ERR_NOMEM;
    }
    return BZ_OK;
}

__global__ void zero_batch_state(BatchState *bs) {
    bs->remaining = 0;
    bs->status = BZ_OK;
    bs->t0 = ~0ull;
}

}  // namespace

extern "C" {

void bz_default_options(bz_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->check = BZ_CHECK_STAGE;
    o->identity_skip = 1;
}

const char *bz_status_str(int s) {
    switch (s) {
    case BZ_OK: return "ok";
    case BZ_ERR_ARG: return "invalid argument";
    case BZ_ERR_VALUE: return "generator entry >= p";
    case BZ_ERR_RANK: return "generator matrix has rank < k";
    case BZ_ERR_DEVICE: return "HIP device error or no gfx950 device";
    case BZ_ERR_NOMEM: return "out of memory";
    case BZ_ERR_LIMIT: return "work limit reached";
    default: return "unknown status";
    }
}

int bz_min_distance_ex(int p, int n, int k, const uint8_t *G, int G_is_device, const bz_options *opt,
                       bz_result *out) {
    int st = check_args(p, n, k, G, out);
    if (st != BZ_OK) return st;
    bz_options o;
    if (opt) o = *opt;
    else bz_default_options(&o);
    if (o.check != BZ_CHECK_STAGE && o.check != BZ_CHECK_ROUND) return BZ_ERR_ARG;
    if (o.histograms && !o.hist_out) return BZ_ERR_ARG;
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 64 || o.cooperative) return BZ_ERR_ARG;
    if (o.pair_tables < -1 || o.pair_tables > 1) return BZ_ERR_ARG;
    DevCtx *c = nullptr;
    st = get_ctx(o.device, &c);
    if (st != BZ_OK) return st;
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_OK(hipSetDevice(o.device));
    hipStream_t s = o.hip_stream ? (hipStream_t)o.hip_stream : c->stream;
    PlainGuard guard(c);
    // the previous plain call's late workgroups may still update the workspace
    // (it returned at the final check): on another stream, wait for them
    if (c->have_last && c->last_stream != s) HIP_OK(hipStreamWaitEvent(s, c->done_ev, 0));

    const int flags = (o.check == BZ_CHECK_ROUND ? FLAG_ROUND : 0) | (o.no_termination ? FLAG_NO_TERM : 0) |
                      (o.identity_skip ? FLAG_SKIP : 0) | (o.histograms ? FLAG_HIST : 0) |
                      (o.trace_out ? FLAG_TRACE : 0);
    const u64 max_cw = o.max_codewords ? o.max_codewords : DEFAULT_LIMIT;
    const int WF = (n + 31) / 32;
    int W = o.identity_skip ? (n - k + 31) / 32 : WF;
    if (W < 1) W = 1;
    // default: as many workgroups as fit (finer deals of the large stages)
    const int bpc = o.blocks_per_cu ? o.blocks_per_cu : 64;
    // pair tables by default for F_7 only: the plain F_3 runs measured no
    // faster with them (their enumeration is bound by latency, not by the
    // prefixes)
    const bool tables = o.pair_tables > 0 || (o.pair_tables == 0 && p == 7);
    const int grid = enum_grid(p, o.histograms != 0, tables, W, c->cu, bpc);
    if (grid < 1) return BZ_ERR_DEVICE;
    const u64 timeout = c->ticks_per_s * (u64)(o.wait_timeout_s > 0 ? o.wait_timeout_s : 120);

    const uint8_t *Gd = G;
    if (!G_is_device) {
        HIP_OK(hipMemcpyAsync(c->g_buf, G, (size_t)k * n, hipMemcpyHostToDevice, s));
        Gd = c->g_buf;
    }
    if (o.histograms) {
        zero_u64<<<256, 256, 0, s>>>(c->hist, (size_t)BZ_MAX_STAGES * (BZ_MAX_N + 1));
        HIP_OK(hipGetLastError());
    }
    RunArgs a;
    a.n = n;
    a.k = k;
    a.flags = flags;
    a.U0 = n - k + 1;
    a.max_codewords = max_cw;
    a.grid = (uint32_t)grid;
    a.sweep_ops = plain_sweep_ops(p);
    a.timeout_ticks = timeout;
    {
        // (p, k, W, grid, task size) packed: 3 + 7 + 3 + 19 + 32 bits
        const u64 key = ((u64)p << 61) | ((u64)k << 54) | ((u64)W << 51) | ((u64)(grid & 0x7ffff) << 32) |
                        (u64)a.sweep_ops;
        auto it = c->rounds.find(key);
        if (it == c->rounds.end()) {
            RoundTable t;
            fill_round_table(p, k, W, (uint32_t)grid, a.sweep_ops, host_binom(), &t);
            RoundTable *d = nullptr;
            HIP_OK(hipMalloc(&d, sizeof(RoundTable)));
            if (hipMemcpy(d, &t, sizeof(RoundTable), hipMemcpyHostToDevice) != hipSuccess) {
                (void)hipFree(d);
                return BZ_ERR_DEVICE;
            }
            it = c->rounds.emplace(key, d).first;
        }
        a.rounds = it->second;
    }
    if (++c->spec_epoch == 0) c->spec_epoch = 1;
    a.spec = o.no_ahead ? nullptr : c->spec;
    a.epoch = c->spec_epoch;
    a.pad = 0;
    a.pairs = tables ? c->pairs : nullptr;
    a.pair_stride = (uint32_t)pair_table_units(p, k, W);
    a.pair_w = W;
    a.pair_t0 = 1;  // a workgroup of the decomposition launch of its own builds set 0's table
    if (o.timing) HIP_OK(hipEventRecord(c->ev[0], s));
    HIP_OK(p == 3 ? launch_decompose<3>(WF, Gd, c->cs, c->rows, a, s)
                  : launch_decompose<7>(WF, Gd, c->cs, c->rows, a, s));
    if (o.timing) HIP_OK(hipEventRecord(c->ev[1], s));
    EnumArgs ea;
    ea.k = k;
    ea.n = n;
    ea.flags = flags;
    ea.lookahead = LOOKAHEAD;
    ea.timeout_ticks = timeout;
    // without histograms or a trace, the check that ends the run hands the
    // result block to the host itself (mapped memory and a flag): no copy
    // launch and no wait for the last workgroups to retire
    const bool mapped = !o.histograms && !o.trace_out;
    ea.res_out = nullptr;
    ea.flag_out = nullptr;
    ea.epoch = 0;
    ea.pair_stride = a.pair_stride;
    if (mapped) {
        if (++c->epoch == 0) c->epoch = 1;
        ea.res_out = c->res_map_dev;
        ea.flag_out = c->flag_map_dev;
        ea.epoch = c->epoch;
    }
    HIP_OK(p == 3 ? launch_enum<3>(o.histograms != 0, W, grid, c->cs, c->rows, a.pairs, c->binom, c->hist, ea, s)
                  : launch_enum<7>(o.histograms != 0, W, grid, c->cs, c->rows, a.pairs, c->binom, c->hist, ea, s));
    if (o.timing) HIP_OK(hipEventRecord(c->ev[2], s));
    HIP_OK(hipEventRecord(c->done_ev, s));
    c->last_stream = s;
    c->have_last = true;
    bool have = false;
    if (mapped) {
        // the flag, or the end of the launch without it (no stage, a failed
        // decomposition, a device-side wait timeout: the block is then read
        // the ordinary way below); the stream is asked now and then so that a
        // device error cannot leave the caller spinning
        for (u64 it = 1;; it++) {
            if (__atomic_load_n(c->flag_map, __ATOMIC_ACQUIRE) == ea.epoch) {
                have = true;
                break;
            }
            if ((it & 1023u) == 0) {
                const hipError_t q = hipStreamQuery(s);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) return BZ_ERR_DEVICE;
                have = __atomic_load_n(c->flag_map, __ATOMIC_ACQUIRE) == ea.epoch;
                break;
            }
        }
        if (have) {
            std::memcpy(c->host_res, c->res_map, sizeof(CodeResult));
            if (o.timing) HIP_OK(hipEventSynchronize(c->ev[2]));
        }
    }
    if (!have) {
        HIP_OK(hipMemcpyAsync(c->host_res, &c->cs->res, sizeof(CodeResult), hipMemcpyDeviceToHost, s));
        if (o.histograms)
            HIP_OK(hipMemcpyAsync(c->host_hist, c->hist, sizeof(u64) * BZ_MAX_STAGES * (BZ_MAX_N + 1),
                                  hipMemcpyDeviceToHost, s));
        if (o.trace_out)
            HIP_OK(hipMemcpyAsync(c->host_trace, c->cs->trace, sizeof(c->cs->trace), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    st = finish(p, n, k, flags, max_cw, *c->host_res, out, plain_sweep_ops(p));
    if (o.timing) {
        HIP_OK(hipEventElapsedTime(&out->decompose_ms, c->ev[0], c->ev[1]));
        HIP_OK(hipEventElapsedTime(&out->enum_ms, c->ev[1], c->ev[2]));
    }
    if (o.trace_out) {
        // ticks -> ns from the decomposition start; keep the stage rows the run reached
        const u64 t0 = c->host_trace[0][0];
        auto ns = [&](u64 t) -> u64 {
            if (t == 0 || t == ~0ull) return 0;
            return (u64)((double)(t - t0) * 1e9 / (double)c->ticks_per_s);
        };
        for (int r = 0; r < BZ_MAX_STAGES + 2; r++)
            for (int i = 0; i < 4; i++) o.trace_out[r * 4 + i] = 0;
        for (int i = 0; i < 4; i++) o.trace_out[i] = ns(c->host_trace[0][i]);
        o.trace_out[4] = ns(c->host_trace[1][0]);
        o.trace_out[5] = ns(c->host_trace[1][1]);
        const int nt = c->host_res->n_table;
        for (int sidx = 0; sidx < nt; sidx++)
            for (int i = 0; i < 4; i++) o.trace_out[(2 + sidx) * 4 + i] = ns(c->host_trace[2 + sidx][i]);
    }
    if (o.histograms && (st == BZ_OK || st == BZ_ERR_LIMIT)) {
        for (int sidx = 0; sidx < out->n_stages; sidx++)
            for (int w = 0; w <= n; w++)
                o.hist_out[(size_t)sidx * (n + 1) + w] = c->host_hist[(size_t)sidx * (BZ_MAX_N + 1) + w];
    }
    return st;
}

int bz_min_distance(int p, int n, int k, const uint8_t *G, bz_result *out) {
    return bz_min_distance_ex(p, n, k, G, 0, nullptr, out);
}

// ---------------------------------------------------------------- sliced ops
void bz_default_batch_options(bz_batch_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->check = BZ_CHECK_STAGE;
    o->identity_skip = 1;
}

int bz_min_distance_batch(int ncodes, const bz_code *codes, const uint8_t *G, uint64_t g_bytes, int G_is_device,
                          bz_batch_options *opt, bz_result *out, int32_t *status_out) {
    if (ncodes < 0 || ncodes > BZ_MAX_BATCH || (ncodes > 0 && (!codes || !G || !out || !status_out)))
        return BZ_ERR_ARG;
    bz_batch_options o;
    if (opt) o = *opt;
    else bz_default_batch_options(&o);
    if (o.check != BZ_CHECK_STAGE && o.check != BZ_CHECK_ROUND) return BZ_ERR_ARG;
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 64 || o.cooperative) return BZ_ERR_ARG;
    if (ncodes == 0) return BZ_OK;
    const int flags = (o.check == BZ_CHECK_ROUND ? FLAG_ROUND : 0) | (o.no_termination ? FLAG_NO_TERM : 0) |
                      (o.identity_skip ? FLAG_SKIP : 0);
    const u64 max_cw = o.max_codewords ? o.max_codewords : DEFAULT_LIMIT;
    // validate every code and lay out its rows
    std::vector<BatchCode> bc((size_t)ncodes);
    u64 row_words = 0, pair_units = 0;
    int wmax = 1;
    for (int i = 0; i < ncodes; i++) {
        const bz_code &cd = codes[i];
        if (check_args(cd.p, cd.n, cd.k, G, out) != BZ_OK || cd.sweep_ops < 0) return BZ_ERR_ARG;
        if (cd.g_offset > g_bytes || (u64)cd.k * (u64)cd.n > g_bytes - cd.g_offset) return BZ_ERR_ARG;
        BatchCode &b = bc[(size_t)i];
        b.g_offset = cd.g_offset;
        b.row_offset = row_words;
        b.max_codewords = max_cw;
        b.p = cd.p;
        b.n = cd.n;
        b.k = cd.k;
        b.flags = flags;
        b.U0 = cd.n - cd.k + 1;
        b.WF = (cd.n + 31) / 32;
        b.W = o.identity_skip ? (cd.n - cd.k + 31) / 32 : b.WF;
        if (b.W < 1) b.W = 1;
        b.sweep_ops = cd.sweep_ops > 0 ? (uint32_t)cd.sweep_ops : DEFAULT_SWEEP_OPS;
        b.pair_stride = (uint32_t)pair_table_units(cd.p, cd.k, b.W);
        b.pair_offset = pair_units;
        if (b.W > wmax) wmax = b.W;
        row_words += batch_row_words(cd.n, cd.k);
        pair_units += code_pair_units(cd.p, cd.n, cd.k, b.W, false);
    }
    DevCtx *c = nullptr;
    int st = get_ctx(o.device, &c);
    if (st != BZ_OK) return st;
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_OK(hipSetDevice(o.device));
    hipStream_t s = o.hip_stream ? (hipStream_t)o.hip_stream : c->stream;
    st = grow_batch(*c, (size_t)ncodes, (size_t)row_words, (size_t)pair_units, G_is_device ? 0 : (size_t)g_bytes);
    if (st != BZ_OK) return st;
    const int bpc = o.blocks_per_cu ? o.blocks_per_cu : 64;  // default: as many as fit
    const int grid = batch_grid(wmax, c->cu, bpc);
    if (grid < 1) return BZ_ERR_DEVICE;
    const u64 timeout = c->ticks_per_s * (u64)(o.wait_timeout_s > 0 ? o.wait_timeout_s : 120);
    const uint8_t *Gd = G;
    if (!G_is_device) {
        HIP_OK(hipMemcpyAsync(c->b_g, G, (size_t)g_bytes, hipMemcpyHostToDevice, s));
        Gd = c->b_g;
    }
    HIP_OK(hipMemcpyAsync(c->b_codes, bc.data(), sizeof(BatchCode) * (size_t)ncodes, hipMemcpyHostToDevice, s));
    zero_batch_state<<<1, 1, 0, s>>>(c->b_state);
    HIP_OK(hipGetLastError());
    if (o.timing) HIP_OK(hipEventRecord(c->ev[0], s));
    decompose_batch_kernel<<<ncodes, 64, 0, s>>>(Gd, c->b_codes, c->b_cs, c->b_claims, c->b_rows, c->b_pairs,
                                                (uint32_t)grid, c->b_state, nullptr, nullptr, nullptr);
    HIP_OK(hipGetLastError());
    if (o.timing) HIP_OK(hipEventRecord(c->ev[1], s));
    {
        CodeState *css = c->b_cs;
        u64 *clm = c->b_claims;
        const BatchCode *cds = c->b_codes;
        int nc = ncodes;
        const u32 *rows = c->b_rows;
        const uint4 *prs = c->b_pairs;
        const u64 *bin = c->binom;
        BatchState *bs = c->b_state;
        u64 to = timeout;
        const int32_t *order = nullptr;
        const uint32_t *yield = nullptr;
        uint32_t *done = nullptr;
        CodeResult *resm = nullptr;
        void *args[] = {&css, &clm, &cds, &nc, &rows, &prs, &bin, &bs, &to, &order, &yield, &done, &resm};
        const void *fn = wmax <= 2 ? (const void *)enum_batch_kernel<2> : (const void *)enum_batch_kernel<4>;
        HIP_OK(hipLaunchKernel(fn, dim3(grid), dim3(256), args, 0, s));
    }
    if (o.timing) HIP_OK(hipEventRecord(c->ev[2], s));
    HIP_OK(hipMemcpy2DAsync(c->b_host_res, sizeof(CodeResult), &c->b_cs->res, sizeof(CodeState),
                            sizeof(CodeResult), (size_t)ncodes, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(c->b_host_state, c->b_state, sizeof(BatchState), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (c->b_host_state->status != BZ_OK) return BZ_ERR_DEVICE;
    for (int i = 0; i < ncodes; i++) {
        const bz_code &cd = codes[i];
        status_out[i] = finish(cd.p, cd.n, cd.k, flags, max_cw, c->b_host_res[i], &out[i], bc[(size_t)i].sweep_ops);
    }
    if (o.code_ms_out) {
        const u64 t0 = c->b_host_state->t0;
        for (int i = 0; i < ncodes; i++) {
            const u64 t1 = c->b_host_res[i].t_end;
            o.code_ms_out[i] = t1 > t0 ? (float)((double)(t1 - t0) * 1e3 / (double)c->ticks_per_s) : 0.0f;
        }
    }
    if (o.timing) {
        HIP_OK(hipEventElapsedTime(&o.decompose_ms, c->ev[0], c->ev[1]));
        HIP_OK(hipEventElapsedTime(&o.enum_ms, c->ev[1], c->ev[2]));
        if (opt) {
            opt->decompose_ms = o.decompose_ms;
            opt->enum_ms = o.enum_ms;
        }
    }
    return BZ_OK;
}

int bz_mlp_forward(const float *params, const float *x, int n, float *y, float *cache, void *stream) {
    if (!params || n < 0 || (n > 0 && (!x || !y))) return BZ_ERR_ARG;
    if (n == 0) return BZ_OK;
    mlp_forward_kernel<<<(n + 255) / 256, 256, 0, (hipStream_t)stream>>>(params, x, n, y, cache);
    return hipGetLastError() == hipSuccess ? BZ_OK : BZ_ERR_DEVICE;
}

int bz_mlp_backward(const float *params, const float *x, const float *target, int n, const float *y,
                    const float *cache, float *dz, float *grad, float *loss, void *stream) {
    if (!params || !x || !target || n < 1 || !y || !cache || !dz || !grad) return BZ_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    mlp_delta_kernel<<<(n + 255) / 256, 256, 0, s>>>(params, target, n, y, cache, dz);
    mlp_grad_kernel<<<(MLP_NPARAM + 255) / 256, 256, 0, s>>>(x, n, cache, dz, grad);
    if (loss) mlp_loss_kernel<<<1, 64, 0, s>>>(y, target, n, loss);
    return hipGetLastError() == hipSuccess ? BZ_OK : BZ_ERR_DEVICE;
}

int bz_mlp_adam(float *params, const float *grad, float *m, float *v, int step, float lr, float beta1, float beta2,
                float eps, void *stream) {
    if (!params || !grad || !m || !v || step < 1) return BZ_ERR_ARG;
    mlp_adam_kernel<<<(MLP_NPARAM + 255) / 256, 256, 0, (hipStream_t)stream>>>(params, grad, m, v, step, lr, beta1,
                                                                              beta2, eps);
    return hipGetLastError() == hipSuccess ? BZ_OK : BZ_ERR_DEVICE;
}

int bz_valu_rate(int op, int iters, int blocks_per_cu, uint32_t *out, float *ms, double *lane_ops, void *stream) {
    if (op < 0 || op > 5 || iters < 1 || blocks_per_cu < 1 || blocks_per_cu > 8 || !out || !ms || !lane_ops)
        return BZ_ERR_ARG;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    const int blocks = prop.multiProcessorCount * blocks_per_cu;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return BZ_ERR_DEVICE;
    }
    hipError_t err = hipEventRecord(e0, s);
    switch (op) {
    case 0: valu_rate_kernel<0><<<blocks, 256, 0, s>>>(out, iters, 1u); break;
    case 1: valu_rate_kernel<1><<<blocks, 256, 0, s>>>(out, iters, 1u); break;
    case 2: valu_rate_kernel<2><<<blocks, 256, 0, s>>>(out, iters, 1u); break;
    case 3: valu_rate_kernel<3><<<blocks, 256, 0, s>>>(out, iters, 1u); break;
    case 4: valu_rate_kernel<4><<<blocks, 256, 0, s>>>(out, iters, 1u); break;
    default: valu_rate_kernel<5><<<blocks, 256, 0, s>>>(out, iters, 1u); break;
    }
    if (err == hipSuccess) err = hipGetLastError();
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *lane_ops = (double)blocks * 256.0 * (double)iters * 8.0;
    return err == hipSuccess ? BZ_OK : BZ_ERR_DEVICE;
}

int bz_sliced_pack(int p, int enc, int nvec, int nsym, const uint8_t *sym, uint32_t *planes, void *stream) {
    if ((p != 3 && p != 7) || nvec < 0 || nsym < 1 || !sym || !planes) return BZ_ERR_ARG;
    if (enc != BZ_ENC_NATURAL && !(enc == BZ_ENC_KAT && p == 3)) return BZ_ERR_ARG;
    const long long total = (long long)nvec * ((nsym + 31) / 32);
    if (total == 0) return BZ_OK;
    const int blocks = (int)((total + 255) / 256);
    if (p == 3) pack_kernel<3><<<blocks, 256, 0, (hipStream_t)stream>>>(enc, nvec, nsym, sym, planes);
    else pack_kernel<7><<<blocks, 256, 0, (hipStream_t)stream>>>(enc, nvec, nsym, sym, planes);
    return hipGetLastError() == hipSuccess ? BZ_OK : BZ_ERR_DEVICE;
}

int bz_sliced_unpack(int p, int enc, int nvec, int nsym, const uint32_t *planes, uint8_t *sym, void *stream) {
    if ((p != 3 && p != 7) || nvec < 0 || nsym < 1 || !sym || !planes) return BZ_ERR_ARG;
    if (enc != BZ_ENC_NATURAL && !(enc == BZ_ENC_KAT && p == 3)) return BZ_ERR_ARG;
    const long long total = (long long)nvec * nsym;
    if (total == 0) return BZ_OK;
    const int blocks = (int)((total + 255) / 256);
    if (p == 3) unpack_kernel<3><<<blocks, 256, 0, (hipStream_t)stream>>>(enc, nvec, nsym, planes, sym);
    else unpack_kernel<7><<<blocks, 256, 0, (hipStream_t)stream>>>(enc, nvec, nsym, planes, sym);
    return hipGetLastError() == hipSuccess ? BZ_OK : BZ_ERR_DEVICE;
}

int bz_sliced_op(int p, int op, int nvec, int nsym, const uint32_t *a, const uint32_t *b, uint32_t *out,
                 int reps, void *stream) {
    if ((p != 3 && p != 7) || nvec < 0 || nsym < 1 || !a || !out || reps < 1) return BZ_ERR_ARG;
    if (op < BZ_OP_ADD || op > BZ_OP_KAT_ADD || (op == BZ_OP_KAT_ADD && p != 3)) return BZ_ERR_ARG;
    if (op != BZ_OP_DOUBLE && !b) return BZ_ERR_ARG;
    if ((op == BZ_OP_ISO_ADD || op == BZ_OP_ISO_SUB) && reps != 1) return BZ_ERR_ARG;
    const int words = (nsym + 31) / 32;
    const long long total = (long long)nvec * words;
    if (total == 0) return BZ_OK;
    if (total > (1ll << 40)) return BZ_ERR_ARG;
    const int blocks = (int)((total + 255) / 256);
    if (p == 3) launch_op<3>(op, blocks, (hipStream_t)stream, nvec, words, a, b, out, reps);
    else launch_op<7>(op, blocks, (hipStream_t)stream, nvec, words, a, b, out, reps);
    return hipGetLastError() == hipSuccess ? BZ_OK : BZ_ERR_DEVICE;
}

}  // extern "C"

// =====================================================================
// The entry point that allocates nothing
// =====================================================================
//
// Its device state (the code state, the packed rows of up to BZ_MAX_M
// information sets, the set computed ahead and the binomial table) lives in
// one static device array, `scratch`, of which every GPU holds its own copy.
// Host code never uses the array's name as an address: the first call on a
// device looks up that device's copy with hipGetSymbolAddress and keeps the
// pointer.  The decomposition counts the rounds' tasks itself (no per-shape
// table, which would be device memory of its own), and the result block is
// copied back into the call's own stack frame.

namespace {

struct NoAllocScratch {
    CodeState cs;
    SpecBuf spec;
    u64 binom[65 * 65];
    u32 rows[BZ_MAX_M * BZ_MAX_K * ROW_WORDS];
};
static_assert(sizeof(NoAllocScratch) <= BZ_NOALLOC_SCRATCH_BYTES, "the no-allocation workspace fits its array");

struct NoAllocDev {
    bool ready = false;
    NoAllocScratch *ws = nullptr;  // this device's copy of `scratch`
    int cu = 0;
    u64 ticks_per_s = 0;
    uint32_t epoch = 0;  // the value of ws->spec.flag in the latest call
};
NoAllocDev g_na[MAX_DEV];

// C(a, b), a, b <= 64, by Pascal's rule one row at a time (thread b owns column b).
__global__ void binom_fill_kernel(u64 *tab) {
    __shared__ u64 row[65];
    const int b = threadIdx.x;
    u64 v = (b == 0) ? 1u : 0u;
    for (int a = 0; a <= 64; a++) {
        if (a > 0) v = (b > 0 ? row[b - 1] : 0u) + row[b];
        tab[a * 65 + b] = v;
        __syncthreads();
        row[b] = v;
        __syncthreads();
    }
}

__global__ void spec_reset_kernel(SpecBuf *sp) {
    sp->flag = 0;
    sp->ok = 0;
}

// Once per device, with the device current (the caller holds the device's lock).
int noalloc_setup(int dev, NoAllocDev &na, hipStream_t s) {
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BZ_ERR_DEVICE;
    int rate_khz = 0;
    HIP_OK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return BZ_ERR_DEVICE;
    NoAllocScratch *ws = static_cast<NoAllocScratch *>(ptr);
    binom_fill_kernel<<<1, 65, 0, s>>>(ws->binom);
    HIP_OK(hipGetLastError());
    spec_reset_kernel<<<1, 1, 0, s>>>(&ws->spec);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    na.ws = ws;
    na.cu = prop.multiProcessorCount;
    na.ticks_per_s = (u64)(rate_khz > 0 ? rate_khz : 100000) * 1000ull;
    na.epoch = 0;
    na.ready = true;
    return BZ_OK;
}

}  // namespace

extern "C" int bz_min_distance_noalloc(int p, int n, int k, const uint8_t *G, const bz_options *opt,
                                       bz_result *out) {
    int st = check_args(p, n, k, G, out);
    if (st != BZ_OK) return st;
    bz_options o;
    if (opt) o = *opt;
    else bz_default_options(&o);
    if (o.check != BZ_CHECK_STAGE && o.check != BZ_CHECK_ROUND) return BZ_ERR_ARG;
    if (o.histograms || o.trace_out || o.timing || o.cooperative) return BZ_ERR_ARG;
    if (o.pair_tables < -1 || o.pair_tables > 1) return BZ_ERR_ARG;
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 64 || o.device < 0 || o.device >= MAX_DEV) return BZ_ERR_ARG;
    DevCtx &c = g_ctx[o.device];
    std::lock_guard<std::mutex> lk(c.mu);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || o.device >= ndev) return BZ_ERR_DEVICE;
    HIP_OK(hipSetDevice(o.device));
    hipStream_t s = (hipStream_t)o.hip_stream;  // NULL: the null stream
    NoAllocDev &na = g_na[o.device];
    if (!na.ready) {
        st = noalloc_setup(o.device, na, s);
        if (st != BZ_OK) return st;
    }
    PlainGuard guard(&c);
    if (c.ready && c.have_last && c.last_stream != s) HIP_OK(hipStreamWaitEvent(s, c.done_ev, 0));

    const int flags = (o.check == BZ_CHECK_ROUND ? FLAG_ROUND : 0) | (o.no_termination ? FLAG_NO_TERM : 0) |
                      (o.identity_skip ? FLAG_SKIP : 0);
    const u64 max_cw = o.max_codewords ? o.max_codewords : DEFAULT_LIMIT;
    const int WF = (n + 31) / 32;
    int W = o.identity_skip ? (n - k + 31) / 32 : WF;
    if (W < 1) W = 1;
    const int grid = enum_grid(p, false, false, W, na.cu, o.blocks_per_cu ? o.blocks_per_cu : 64);
    if (grid < 1) return BZ_ERR_DEVICE;
    const u64 timeout = na.ticks_per_s * (u64)(o.wait_timeout_s > 0 ? o.wait_timeout_s : 120);
    NoAllocScratch *ws = na.ws;
    RunArgs a;
    a.n = n;
    a.k = k;
    a.flags = flags;
    a.U0 = n - k + 1;
    a.max_codewords = max_cw;
    a.grid = (uint32_t)grid;
    a.sweep_ops = plain_sweep_ops(p);
    a.timeout_ticks = timeout;
    a.rounds = nullptr;  // counted by the decomposition
    if (++na.epoch == 0) na.epoch = 1;
    a.spec = o.no_ahead ? nullptr : &ws->spec;
    a.epoch = na.epoch;
    a.pad = 0;
    HIP_OK(p == 3 ? launch_decompose<3>(WF, G, &ws->cs, ws->rows, a, s)
                  : launch_decompose<7>(WF, G, &ws->cs, ws->rows, a, s));
    EnumArgs ea;
    ea.k = k;
    ea.n = n;
    ea.flags = flags;
    ea.lookahead = LOOKAHEAD;
    ea.timeout_ticks = timeout;
    ea.res_out = nullptr;
    ea.flag_out = nullptr;
    ea.epoch = 0;
    ea.pair_stride = 0;
    HIP_OK(p == 3 ? launch_enum<3>(false, W, grid, &ws->cs, ws->rows, nullptr, ws->binom, nullptr, ea, s)
                  : launch_enum<7>(false, W, grid, &ws->cs, ws->rows, nullptr, ws->binom, nullptr, ea, s));
    CodeResult r;
    HIP_OK(hipMemcpyAsync(&r, &ws->cs.res, sizeof r, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return finish(p, n, k, flags, max_cw, r, out, plain_sweep_ops(p));
}

// =====================================================================
// Serving: continuous batching over a yielding persistent launch
// =====================================================================
//
// Requests queue on the host.  Each round the host admits queued requests
// into free slots (memory: one CodeState, packed rows and a generator per
// slot), decomposes the new slots, orders every active slot (arrival order, or
// shortest predicted work first with the work-predictor network) and launches
// the persistent enumeration over them.  Codes that end raise a flag in mapped
// host memory, so their results are collected while the launch runs.  When new
// requests wait, the host raises the yield flag: workgroups finish the part
// they hold and exit, every code keeping its progress in its claim word, and
// the next round continues all of them together with the new ones.  All data
// that a launch reads was written before it started (kernel boundaries), and
// during a launch only atomics cross workgroups.

struct bz_server {
    int dev = 0;
    DevCtx *c = nullptr;
    hipStream_t run = nullptr;  // the launches
    hipEvent_t round_done = nullptr;
    bz_server_options o{};
    int slots = 0, grid = 0, decomp_grid = 0, flags = 0;
    u64 max_cw = 0, timeout = 0, rows_per_slot = 0, g_per_slot = 0, pairs_per_slot = 0;
    // device
    CodeState *cs = nullptr;
    u64 *claims = nullptr;  // one claim word per slot, contiguous
    BatchCode *codes = nullptr;
    u32 *rows = nullptr;
    uint4 *pairs = nullptr;  // pair tables, pairs_per_slot 16-byte units per slot
    uint8_t *g = nullptr;
    BatchState *bs = nullptr;
    int32_t *order_d = nullptr, *new_d = nullptr;
    float *feat_d = nullptr, *pred_d = nullptr, *mlp_d = nullptr;
    // pinned host
    BatchCode *codes_h = nullptr;
    uint8_t *g_h = nullptr;
    uint32_t *yield_h = nullptr, *done_h = nullptr;  // mapped host memory
    uint32_t *yield_dev = nullptr, *done_dev = nullptr;  // the same, as device addresses
    CodeResult *res_h = nullptr;    // mapped: a code's result block, written before its done flag
    CodeResult *res_dev = nullptr;
    int32_t *order_h = nullptr, *new_h = nullptr;
    float *pred_h = nullptr, *qfeat_h = nullptr;
    // bookkeeping
    struct Req {
        int p, n, k;
        u64 tag;
        std::vector<uint8_t> G;
        float qpred = 0;         // predicted log10 work before the decomposition
        bool has_qpred = false;
    };
    std::deque<Req> queue;
    struct Slot {
        int state = 0;  // 0 free, 1 active
        int p = 0, n = 0, k = 0;
        u64 tag = 0;
        float prio = 0;       // predicted log10 work after the decomposition
        u64 seq = 0;
    };
    std::vector<Slot> slot;
    u64 seq = 0;
    u64 rounds = 0, yields = 0;
    bool running = false;
    int wmax = 2;
    std::mutex mu;
};

namespace {

void servers_hold(DevCtx &c) {
    // under srv_mu for the whole wait: no server starts a round (or is freed)
    // meanwhile; a round yields at the end of the part each workgroup holds
    std::lock_guard<std::mutex> lk(c.srv_mu);
    c.plain_active.store(1);
    for (bz_server *s : c.servers) {
        __atomic_store_n(s->yield_h, 1u, __ATOMIC_RELEASE);
        (void)hipEventSynchronize(s->round_done);  // complete at once if no round was launched
    }
}

void servers_release(DevCtx &c) {
    std::lock_guard<std::mutex> lk(c.srv_mu);
    c.plain_active.store(0);
}

void server_free(bz_server *s) {
    // teardown: errors are not actionable here
    if (s->run) (void)hipStreamSynchronize(s->run);
    for (void *p : {(void *)s->cs, (void *)s->claims, (void *)s->codes, (void *)s->rows, (void *)s->pairs,
                    (void *)s->g, (void *)s->bs, (void *)s->order_d, (void *)s->new_d, (void *)s->feat_d,
                    (void *)s->pred_d, (void *)s->mlp_d})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)s->codes_h, (void *)s->g_h, (void *)s->yield_h, (void *)s->done_h, (void *)s->res_h,
                    (void *)s->order_h, (void *)s->new_h, (void *)s->pred_h, (void *)s->qfeat_h})
        if (p) (void)hipHostFree(p);
    if (s->round_done) (void)hipEventDestroy(s->round_done);
    if (s->run) (void)hipStreamDestroy(s->run);
    delete s;
}

// Harvest codes that ended and rebuild their traces.  The kernel that ended a
// code wrote its result block to mapped host memory before raising its done
// flag, so nothing is copied here: a copy would need a free compute unit, and
// a running round holds all of them.
int server_harvest(bz_server *s, int max_out, uint64_t *tags, bz_result *results, int32_t *statuses, int *n_out) {
    std::vector<int> done;
    for (int i = 0; i < s->slots && (int)done.size() < max_out - *n_out; i++)
        if (s->slot[(size_t)i].state == 1 && __atomic_load_n(&s->done_h[i], __ATOMIC_ACQUIRE) != 0) done.push_back(i);
    if (done.empty()) return BZ_OK;
    for (int i : done) {
        bz_server::Slot &sl = s->slot[(size_t)i];
        const int k = *n_out;
        tags[k] = sl.tag;
        statuses[k] = finish(sl.p, sl.n, sl.k, s->flags, s->max_cw, s->res_h[i], &results[k],
                             s->codes_h[i].sweep_ops);
        (*n_out)++;
        sl.state = 0;
        __atomic_store_n(&s->done_h[i], 0u, __ATOMIC_RELEASE);
    }
    return BZ_OK;
}

template <int WMAX>
hipError_t server_launch(bz_server *s, int nactive) {
    CodeState *css = s->cs;
    u64 *clm = s->claims;
    const BatchCode *cds = s->codes;
    int nc = nactive;
    const u32 *rows = s->rows;
    const uint4 *prs = s->pairs;
    const u64 *bin = s->c->binom;
    BatchState *bs = s->bs;
    u64 to = s->timeout;
    const int32_t *order = s->order_d;
    const uint32_t *yield = s->yield_dev;
    uint32_t *done = s->done_dev;
    CodeResult *resm = s->res_dev;
    void *args[] = {&css, &clm, &cds, &nc, &rows, &prs, &bin, &bs, &to, &order, &yield, &done, &resm};
    return hipLaunchKernel((const void *)enum_batch_kernel<WMAX>, dim3(s->grid), dim3(256), args, 0, s->run);
}

// Predicted policy: the network's work estimate for the queued requests that
// have none yet (inputs p, n, k; the rank deficit of the last information
// set is only known after the decomposition and is taken as 0), then the
// queue in ascending estimate (ties in arrival order).
int server_queue_predictions(bz_server *s) {
    std::vector<size_t> need;
    for (size_t i = 0; i < s->queue.size(); i++)
        if (!s->queue[i].has_qpred) need.push_back(i);
    for (size_t lo = 0; lo < need.size(); lo += (size_t)s->slots) {
        const int nq = (int)std::min(need.size() - lo, (size_t)s->slots);
        for (int j = 0; j < nq; j++) {
            const bz_server::Req &r = s->queue[need[lo + (size_t)j]];
            mlp_features(r.p, r.n, r.k, 0, s->qfeat_h + 4 * j);
        }
        HIP_OK(hipMemcpyAsync(s->feat_d, s->qfeat_h, sizeof(float) * 4 * (size_t)nq, hipMemcpyHostToDevice, s->run));
        mlp_forward_kernel<<<(nq + 255) / 256, 256, 0, s->run>>>(s->mlp_d, s->feat_d, nq, s->pred_d, nullptr);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(s->pred_h, s->pred_d, sizeof(float) * (size_t)nq, hipMemcpyDeviceToHost, s->run));
        HIP_OK(hipStreamSynchronize(s->run));
        for (int j = 0; j < nq; j++) {
            bz_server::Req &r = s->queue[need[lo + (size_t)j]];
            r.qpred = s->pred_h[j];
            r.has_qpred = true;
        }
    }
    if (!need.empty())
        std::stable_sort(s->queue.begin(), s->queue.end(),
                         [](const bz_server::Req &a, const bz_server::Req &b) { return a.qpred < b.qpred; });
    return BZ_OK;
}

// Admit queued requests into free slots (and, with a budget, while their
// predicted work fits it), decompose them, order the active slots and start
// the next round.
int server_round(bz_server *s) {
    std::vector<int> fresh;
    const bool predicted = s->o.policy == BZ_SERVE_PREDICTED;
    if (predicted && !s->queue.empty()) {
        // an order is only needed when the queue does not fit the free slots or
        // a work budget applies (otherwise every queued request is admitted)
        int free_slots = 0;
        for (const auto &sl : s->slot) free_slots += sl.state == 0;
        if (s->o.admit_budget > 0 || (int)s->queue.size() > free_slots) {
            const int st = server_queue_predictions(s);
            if (st != BZ_OK) return st;
        }
    }
    double admitted_work = 0.0;
    for (int i = 0; i < s->slots && !s->queue.empty(); i++) {
        bz_server::Slot &sl = s->slot[(size_t)i];
        if (sl.state != 0) continue;
        if (predicted && s->o.admit_budget > 0) {
            const double w = std::pow(10.0, (double)s->queue.front().qpred);
            if (!fresh.empty() && admitted_work + w > s->o.admit_budget) break;
            admitted_work += w;
        }
        bz_server::Req r = std::move(s->queue.front());
        s->queue.pop_front();
        sl.state = 1;
        sl.p = r.p;
        sl.n = r.n;
        sl.k = r.k;
        sl.tag = r.tag;
        sl.seq = s->seq++;
        std::memcpy(s->g_h + (size_t)i * s->g_per_slot, r.G.data(), r.G.size());
        BatchCode &b = s->codes_h[i];
        b.g_offset = (u64)i * s->g_per_slot;
        b.row_offset = (u64)i * s->rows_per_slot;
        b.max_codewords = s->max_cw;
        b.p = r.p;
        b.n = r.n;
        b.k = r.k;
        b.flags = s->flags;
        b.U0 = r.n - r.k + 1;
        b.WF = (r.n + 31) / 32;
        b.W = s->o.identity_skip ? (r.n - r.k + 31) / 32 : b.WF;
        if (b.W < 1) b.W = 1;
        b.sweep_ops = DEFAULT_SWEEP_OPS;
        b.pair_stride = (uint32_t)pair_table_units(r.p, r.k, b.W);
        b.pair_offset = (u64)i * s->pairs_per_slot;
        s->new_h[fresh.size()] = i;
        fresh.push_back(i);
    }
    if (!fresh.empty()) {
        const int nf = (int)fresh.size();
        for (int i : fresh)
            HIP_OK(hipMemcpyAsync(s->g + (size_t)i * s->g_per_slot, s->g_h + (size_t)i * s->g_per_slot,
                                  (size_t)s->codes_h[i].n * s->codes_h[i].k, hipMemcpyHostToDevice, s->run));
        HIP_OK(hipMemcpyAsync(s->codes, s->codes_h, sizeof(BatchCode) * (size_t)s->slots, hipMemcpyHostToDevice,
                              s->run));
        HIP_OK(hipMemcpyAsync(s->new_d, s->new_h, sizeof(int32_t) * (size_t)nf, hipMemcpyHostToDevice, s->run));
        decompose_batch_kernel<<<nf, 64, 0, s->run>>>(s->g, s->codes, s->cs, s->claims, s->rows, s->pairs,
                                                      (uint32_t)s->decomp_grid, s->bs, s->new_d, s->done_dev,
                                                      s->res_dev);
        HIP_OK(hipGetLastError());
        if (s->o.policy == BZ_SERVE_PREDICTED) {
            features_kernel<<<(nf + 63) / 64, 64, 0, s->run>>>(s->cs, s->new_d, nf, s->feat_d);
            mlp_forward_kernel<<<(nf + 255) / 256, 256, 0, s->run>>>(s->mlp_d, s->feat_d, nf, s->pred_d, nullptr);
            HIP_OK(hipGetLastError());
            HIP_OK(hipMemcpyAsync(s->pred_h, s->pred_d, sizeof(float) * (size_t)nf, hipMemcpyDeviceToHost, s->run));
            HIP_OK(hipStreamSynchronize(s->run));
            for (int j = 0; j < nf; j++) s->slot[(size_t)fresh[(size_t)j]].prio = s->pred_h[j];
        }
    }
    // active slots in priority order; the predictor only orders work
    std::vector<int> act;
    int wmax = 1;
    for (int i = 0; i < s->slots; i++)
        if (s->slot[(size_t)i].state == 1) {
            act.push_back(i);
            if (s->codes_h[i].W > wmax) wmax = s->codes_h[i].W;
        }
    if (act.empty()) return BZ_OK;
    if (s->o.policy == BZ_SERVE_PREDICTED)
        std::stable_sort(act.begin(), act.end(), [&](int a, int b) {
            return s->slot[(size_t)a].prio < s->slot[(size_t)b].prio;
        });
    else
        std::stable_sort(act.begin(), act.end(),
                         [&](int a, int b) { return s->slot[(size_t)a].seq < s->slot[(size_t)b].seq; });
    for (size_t j = 0; j < act.size(); j++) s->order_h[j] = act[j];
    // a plain call on the device holds it: the round starts at a later poll
    std::lock_guard<std::mutex> lk(s->c->srv_mu);
    if (s->c->plain_active.load()) return BZ_OK;
    HIP_OK(hipMemcpyAsync(s->order_d, s->order_h, sizeof(int32_t) * act.size(), hipMemcpyHostToDevice, s->run));
    __atomic_store_n(s->yield_h, 0u, __ATOMIC_RELEASE);
    HIP_OK(wmax <= 2 && s->wmax <= 2 ? server_launch<2>(s, (int)act.size()) : server_launch<4>(s, (int)act.size()));
    HIP_OK(hipEventRecord(s->round_done, s->run));
    s->running = true;
    s->rounds++;
    return BZ_OK;
}

}  // namespace

extern "C" {

void bz_default_server_options(bz_server_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->slots = 1024;
    o->check = BZ_CHECK_STAGE;
    o->identity_skip = 1;
}

int bz_server_start(const bz_server_options *opt, bz_server **out) {
    if (!out) return BZ_ERR_ARG;
    *out = nullptr;
    bz_server_options o;
    if (opt) o = *opt;
    else bz_default_server_options(&o);
    if (o.slots == 0) o.slots = 1024;
    if (o.slots < 1 || o.slots > BZ_MAX_BATCH || (o.policy != BZ_SERVE_FIFO && o.policy != BZ_SERVE_PREDICTED))
        return BZ_ERR_ARG;
    if (o.policy == BZ_SERVE_PREDICTED && !o.mlp_params) return BZ_ERR_ARG;
    if (o.check != BZ_CHECK_STAGE && o.check != BZ_CHECK_ROUND) return BZ_ERR_ARG;
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 64 || o.max_n < 0 || o.max_n > BZ_MAX_N || o.cooperative)
        return BZ_ERR_ARG;
    if (!(o.admit_budget >= 0.0)) return BZ_ERR_ARG;
    DevCtx *c = nullptr;
    int st = get_ctx(o.device, &c);
    if (st != BZ_OK) return st;
    HIP_OK(hipSetDevice(o.device));
    bz_server *s = new bz_server();
    s->dev = o.device;
    s->c = c;
    s->o = o;
    s->slots = o.slots;
    s->flags = (o.check == BZ_CHECK_ROUND ? FLAG_ROUND : 0) | (o.identity_skip ? FLAG_SKIP : 0);
    s->max_cw = o.max_codewords ? o.max_codewords : DEFAULT_LIMIT;
    s->timeout = c->ticks_per_s * (u64)(o.wait_timeout_s > 0 ? o.wait_timeout_s : 120);
    const int max_n = o.max_n ? o.max_n : BZ_MAX_N;
    s->wmax = (max_n + 31) / 32 <= 2 ? 2 : 4;
    s->rows_per_slot = batch_row_words(max_n, 1);
    s->pairs_per_slot = max_pair_units(max_n, o.identity_skip ? 1 : 0, false);
    s->g_per_slot = (u64)(((max_n * BZ_MAX_K) + 255) / 256 * 256);
    s->grid = batch_grid(s->wmax, c->cu, o.blocks_per_cu ? o.blocks_per_cu : 64);  // default: as many as fit
    s->decomp_grid = s->grid * 8;  // smaller parts: a yield waits for at most one short part
    s->slot.resize((size_t)s->slots);
    const size_t ns = (size_t)s->slots;
    bool ok = s->grid > 0 && hipStreamCreateWithFlags(&s->run, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&s->round_done, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(&s->cs, sizeof(CodeState) * ns) == hipSuccess &&
              hipMalloc(&s->claims, sizeof(u64) * ns) == hipSuccess &&
              hipMalloc(&s->codes, sizeof(BatchCode) * ns) == hipSuccess &&
              hipMalloc(&s->rows, sizeof(u32) * s->rows_per_slot * ns) == hipSuccess &&
              hipMalloc(&s->pairs, sizeof(uint4) * (s->pairs_per_slot * ns + PAIR_PAD_UNITS)) == hipSuccess &&
              hipMalloc(&s->g, s->g_per_slot * ns) == hipSuccess && hipMalloc(&s->bs, sizeof(BatchState)) == hipSuccess &&
              hipMalloc(&s->order_d, sizeof(int32_t) * ns) == hipSuccess &&
              hipMalloc(&s->new_d, sizeof(int32_t) * ns) == hipSuccess &&
              hipMalloc(&s->feat_d, sizeof(float) * 4 * ns) == hipSuccess &&
              hipMalloc(&s->pred_d, sizeof(float) * ns) == hipSuccess &&
              hipMalloc(&s->mlp_d, sizeof(float) * MLP_NPARAM) == hipSuccess &&
              hipHostMalloc(&s->codes_h, sizeof(BatchCode) * ns, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&s->g_h, s->g_per_slot * ns, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&s->yield_h, sizeof(uint32_t), hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
              hipHostMalloc(&s->done_h, sizeof(uint32_t) * ns, hipHostMallocMapped | hipHostMallocCoherent) ==
                  hipSuccess &&
              hipHostMalloc(&s->res_h, sizeof(CodeResult) * ns, hipHostMallocMapped | hipHostMallocCoherent) ==
                  hipSuccess &&
              hipHostMalloc(&s->order_h, sizeof(int32_t) * ns, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&s->new_h, sizeof(int32_t) * ns, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&s->pred_h, sizeof(float) * ns, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&s->qfeat_h, sizeof(float) * 4 * ns, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        server_free(s);
        return BZ_ERR_NOMEM;
    }
    if (hipHostGetDevicePointer((void **)&s->yield_dev, s->yield_h, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&s->done_dev, s->done_h, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&s->res_dev, s->res_h, 0) != hipSuccess) {
        server_free(s);
        return BZ_ERR_DEVICE;
    }
    *s->yield_h = 0;
    std::memset(s->done_h, 0, sizeof(uint32_t) * ns);
    zero_batch_state<<<1, 1, 0, s->run>>>(s->bs);
    if (o.mlp_params &&
        hipMemcpyAsync(s->mlp_d, o.mlp_params, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, s->run) != hipSuccess) {
        server_free(s);
        return BZ_ERR_DEVICE;
    }
    if (hipStreamSynchronize(s->run) != hipSuccess) {
        server_free(s);
        return BZ_ERR_DEVICE;
    }
    {
        std::lock_guard<std::mutex> lk(c->srv_mu);
        c->servers.push_back(s);
    }
    *out = s;
    return BZ_OK;
}

int bz_server_submit(bz_server *s, int p, int n, int k, const uint8_t *G, uint64_t tag) {
    if (!s) return BZ_ERR_ARG;
    const int st = check_args(p, n, k, G, G);
    if (st != BZ_OK) return st;
    const int max_n = s->o.max_n ? s->o.max_n : BZ_MAX_N;
    if (n > max_n) return BZ_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    bz_server::Req r;
    r.p = p;
    r.n = n;
    r.k = k;
    r.tag = tag;
    r.G.assign(G, G + (size_t)n * k);
    s->queue.push_back(std::move(r));
    return BZ_OK;
}

int bz_server_poll(bz_server *s, int max_out, uint64_t *tags, bz_result *results, int32_t *statuses, int *n_out,
                   int *in_flight) {
    if (!s || max_out < 0 || !n_out || (max_out > 0 && (!tags || !results || !statuses))) return BZ_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    HIP_OK(hipSetDevice(s->dev));
    *n_out = 0;
    int st = server_harvest(s, max_out, tags, results, statuses, n_out);
    if (st != BZ_OK) return st;
    if (s->running) {
        const hipError_t q = hipEventQuery(s->round_done);
        if (q == hipSuccess) {
            s->running = false;
        } else if (q != hipErrorNotReady) {
            return BZ_ERR_DEVICE;
        } else if (!s->queue.empty()) {
            bool free_slot = false;
            for (const auto &sl : s->slot) free_slot |= sl.state == 0;
            // new work is waiting and fits: let the round end at the next part boundary
            if (free_slot && __atomic_exchange_n(s->yield_h, 1u, __ATOMIC_ACQ_REL) == 0u) s->yields++;
        }
    }
    if (!s->running) {
        BatchState bsh;
        HIP_OK(hipMemcpy(&bsh, s->bs, sizeof bsh, hipMemcpyDeviceToHost));
        if (bsh.status != BZ_OK) return BZ_ERR_DEVICE;
        st = server_harvest(s, max_out, tags, results, statuses, n_out);
        if (st != BZ_OK) return st;
        st = server_round(s);
        if (st != BZ_OK) return st;
    }
    if (in_flight) {
        int act = 0;
        for (const auto &sl : s->slot) act += sl.state;
        *in_flight = act + (int)s->queue.size();
    }
    return BZ_OK;
}

int bz_server_stats(bz_server *s, uint64_t *rounds, uint64_t *yields) {
    if (!s) return BZ_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (rounds) *rounds = s->rounds;
    if (yields) *yields = s->yields;
    return BZ_OK;
}

int bz_server_stop(bz_server *s) {
    if (!s) return BZ_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->yield_h) __atomic_store_n(s->yield_h, 1u, __ATOMIC_RELEASE);
    }
    {
        std::lock_guard<std::mutex> lk(s->c->srv_mu);
        auto &v = s->c->servers;
        v.erase(std::remove(v.begin(), v.end(), s), v.end());
    }
    (void)hipSetDevice(s->dev);
    server_free(s);
    return BZ_OK;
}

int bz_release(int device) {
    if (device < 0 || device >= MAX_DEV) return BZ_ERR_ARG;
    std::lock_guard<std::mutex> li(g_init_mu);
    DevCtx &c = g_ctx[device];
    std::lock_guard<std::mutex> lk(c.mu);
    {
        std::lock_guard<std::mutex> ls(c.srv_mu);
        if (!c.servers.empty()) return BZ_ERR_ARG;
    }
    if (!c.ready) return BZ_OK;
    int cur = 0;
    const bool had = hipGetDevice(&cur) == hipSuccess;
    HIP_OK(hipSetDevice(device));
    release_ctx(c);
    if (had) (void)hipSetDevice(cur);
    return BZ_OK;
}

}  // extern "C"
