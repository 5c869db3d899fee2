// Host side of the C ABI declared in include/hubga.h: argument validation,
// workspace carve-up, stream-ordered kernel pipelines, state I/O.
#include "../../include/hubga.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"

using namespace hubga;

namespace {

thread_local std::string g_init_error;

constexpr uint32_t kStateMagic = 0x31414748u;   // "HGA1"
constexpr int kProfilePairs = 8192;

struct Layout {
    size_t total = 0;
    size_t take(size_t bytes)
    {
        size_t off = total;
        total += (bytes + 255) & ~(size_t)255;
        return off;
    }
};

bool is_valid_combo(int prec, int kern)
{
    return (prec == GA_PREC_FP64 && kern == GA_KERN_PLAIN) ||
           (prec == GA_PREC_FP32 && (kern == GA_KERN_PLAIN || kern == GA_KERN_BATCHED)) ||
           ((prec == GA_PREC_SPLIT_BF16 || prec == GA_PREC_SPLIT3_BF16) && kern == GA_KERN_BATCHED);
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

std::string check_params(const ga_params *q)
{
    if (!q) return "params is NULL";
    if (q->n < 1 || q->n > kMaxN) return "n must be in [1, " + std::to_string(kMaxN) + "]";
    if (q->p < 1 || q->p > q->n || q->p > kMaxP) return "p must be in [1, min(n, " + std::to_string(kMaxP) + ")]";
    if (!finite_nonneg(q->chi) || !finite_nonneg(q->alpha) || !finite_nonneg(q->delta))
        return "chi, alpha and delta must be finite and >= 0";
    if (!std::isfinite(q->scale) || !(q->scale > 0.0)) return "scale must be finite and > 0";
    if (q->island_size < 2 || q->island_size % 2 || q->island_size > kMaxIsland)
        return "island_size must be even and in [2, " + std::to_string(kMaxIsland) + "]";
    if (q->population < q->island_size || q->population % q->island_size || q->population > 65536)
        return "population must be a multiple of island_size and <= 65536";
    if (q->n1 < 1) return "n1 must be >= 1";
    if (q->elitist != 0 && q->elitist != 1) return "elitist must be 0 or 1";
    if (q->c_symmetric != 0 && q->c_symmetric != 1) return "c_symmetric must be 0 or 1";
    if (q->multihop != 0 && q->multihop != 1) return "multihop must be 0 or 1";
    if (!is_valid_combo(q->precision, q->kernel))
        return "precision/kernel must be FP64+PLAIN, FP32+PLAIN, FP32+BATCHED, SPLIT_BF16+BATCHED or "
               "SPLIT3_BF16+BATCHED";
    return "";
}

Dims make_dims(const ga_params *q, ga_dtype cdt, ga_dtype wdt)
{
    Dims d{};
    d.n = q->n;
    d.p = q->p;
    d.S = q->population;
    d.m = q->island_size;
    d.R = d.S / d.m;
    d.n_pad = ((d.n + kPad - 1) / kPad) * kPad;
    d.n_mtiles = d.n_pad / kMfmaMinRows;
    d.mfma_cfg = 0;
    // up to 512 candidates per generation get the column-parallel exact
    // re-evaluation; any further ones the one-workgroup path
    d.tot = std::min(d.S, 512);
    d.n1 = q->n1;
    d.elitist = q->elitist;
    d.prec = q->precision;
    d.kern = q->kernel;
    d.c_f32 = cdt == GA_DT_F32;
    d.sym = q->c_symmetric;
    d.multihop = q->multihop;
    d.w_f32 = wdt == GA_DT_F32;
    d.chi = q->chi;
    d.alpha = q->alpha;
    d.delta = q->delta;
    d.scale = q->scale;
    d.seed = q->seed;
    return d;
}

// Offsets of every device buffer; the same walk sizes and carves.
struct Carve {
    size_t C, Ct, Ct32, W, W32, Ctr, Whi, Wlo, Wmd, O, D, dsum, hubs, kidx, cost, parts, eps, cmax, Ch32, partial, anc, anc_cost,
        anc_parts, best, best_cost, gen, stats, cand, cand_cnt, cand_cost, cand_parts, kidx_one, scratch, tbuf, slot_r, slot_c, slot_s, slot_done, handled, choice, total_slots, extra_r, extra_c, nextra, sync,
        enum_state, enum_best, binom;
    size_t total;
};

Carve carve(const Dims &d, int c_symmetric)
{
    Layout L;
    Carve c{};
    const size_t n2 = (size_t)d.n * d.n, np2 = (size_t)d.n_pad * d.n_pad;
    const size_t cs = d.c_f32 ? 4 : 8, ws = d.w_f32 ? 4 : 8;
    const bool split = split_mode(d.prec);
    // C, its transpose and the FP32 copy carry one row more: the FP32 copy's
    // extra row is +inf, the allocation scan's padding hub.
    c.C = L.take((n2 + d.n) * cs);
    c.Ct = c_symmetric ? c.C : L.take((n2 + d.n) * cs);
    c.Ct32 = d.c_f32 ? c.Ct : L.take((n2 + d.n) * 4);
    c.W = L.take(n2 * ws);
    c.W32 = (d.prec == kFP32 && !d.w_f32) ? L.take(n2 * 4) : (size_t)-1;
    c.Ctr = d.multihop ? L.take(n2 * 8) : (size_t)-1;
    // one pair of split buffers, in the layout the current tile configuration reads
    c.Whi = split ? L.take(np2 * 2) : (size_t)-1;
    c.Wlo = split ? L.take(np2 * 2) : (size_t)-1;
    c.Wmd = d.prec == kSplit3BF16 ? L.take(np2 * 2) : (size_t)-1;
    c.O = L.take((size_t)d.n * 8);
    c.D = L.take((size_t)d.n * 8);
    c.dsum = L.take((size_t)d.n * 8);
    c.hubs = L.take((size_t)d.S * d.p * 4);
    c.kidx = L.take((size_t)d.S * d.n_pad * 2);
    c.cost = L.take((size_t)d.S * 8);
    c.parts = L.take((size_t)d.S * 24);
    c.eps = L.take((size_t)d.S * 8);
    c.cmax = L.take((size_t)d.S * 4);
    const bool vec = d.prec == kFP32 && d.kern == GA_KERN_BATCHED;
    c.Ch32 = split || vec ? L.take((size_t)d.S * d.p * d.p * 4) : (size_t)-1;
    c.partial = split ? L.take((size_t)d.n_mtiles * d.S * d.p * 8) : vec ? L.take(vec_partial_bytes(d)) : (size_t)-1;
    c.anc = L.take((size_t)d.R * d.p * 4);
    c.anc_cost = L.take((size_t)d.R * 8);
    c.anc_parts = L.take((size_t)d.R * 24);
    c.best = L.take((size_t)d.p * 4);
    c.best_cost = L.take(32);
    c.gen = L.take(8);
    c.stats = L.take(32);
    c.cand = L.take((size_t)d.S * 4);
    c.cand_cnt = L.take((size_t)d.R * 4);
    c.cand_cost = L.take((size_t)d.S * 8);
    c.cand_parts = L.take((size_t)d.S * 24);
    c.kidx_one = L.take((size_t)d.n_pad * 2);
    c.scratch = L.take((size_t)d.n);
    c.tbuf = L.take((size_t)(d.prec == kFP64 ? 1 : d.tot) * d.n * 8);   // FP64: the column sums of P0
    c.slot_r = L.take((size_t)d.tot * 4);
    c.slot_c = L.take((size_t)d.tot * 4);
    c.slot_s = L.take((size_t)d.tot * 4);
    c.slot_done = L.take((size_t)d.tot * 4);
    c.handled = L.take((size_t)d.R * 4);
    c.choice = L.take((size_t)d.R * 4);
    c.total_slots = L.take(4);
    c.extra_r = L.take((size_t)d.S * 4);
    c.extra_c = L.take((size_t)d.S * 4);
    c.nextra = L.take(4);
    c.sync = L.take(8);
    c.enum_state = L.take(sizeof(EnumState));
    c.enum_best = L.take((size_t)d.p * 4);
    c.binom = L.take((size_t)(d.n + 1) * (d.p + 1) * 8);
    c.total = L.total;
    return c;
}

template <typename T>
T *at(void *base, size_t off)
{
    return off == (size_t)-1 ? nullptr : (T *)((char *)base + off);
}

}  // namespace

struct ga_ctx {
    ga_params prm{};
    Dims d{};
    DevPtrs P{};
    hipStream_t st = nullptr;
    void *ws = nullptr;
    bool own_ws = false;
    bool poisoned = false;
    std::string err;
    // kernel timing
    bool prof_on = false;
    std::vector<hipEvent_t> ev;
    int ev_used = 0;
    // one captured generation, replayed by ga_step (needs a non-null stream)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_failed = false;
    int static_dev = -1;   // >= 0: created by ga_init_static on this device (static storage)
    // exhaustive search: the binomial table is copied to the device on first use
    bool binom_ready = false;
    uint64_t nsets = 0;    // C(n, p), saturated at 2^63
    int wlayout = -1;      // WLayout held in the split buffers (-1: none yet)
};

// ------------------------------------------------- allocation-free init --
// ga_init_static's workspace: one array per device, resident from module load
// until the process ends.  Host code never passes `scratch` itself to a
// kernel or copy (in host code the name is a stand-in, not a device address):
// it takes the address hipGetSymbolAddress returns for the current device.
namespace {
constexpr size_t kStaticWorkspaceBytes = (size_t)32 << 20;
constexpr int kMaxStaticDevices = 64;
}  // namespace
__device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {
struct StaticSlot {
    void *ptr = nullptr;   // scratch on this device
    bool resolved = false;
    bool busy = false;     // a live context holds the array
    alignas(ga_ctx) unsigned char ctx_mem[sizeof(ga_ctx)];
};
StaticSlot g_static[kMaxStaticDevices];
std::mutex g_static_mu;
}  // namespace

struct ga_batch {
    hipStream_t st = nullptr;
    int cfg = 7;
    std::vector<ga_ctx *> ctxs;
    std::vector<ga_ctx *> grouped;   // stepped by the grouped launches
    std::vector<ga_ctx *> solo;      // stepped by their own generation on side streams
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;      // [0] fork, [1 + k] join of side stream k
    // grouped contexts: matrix-core job table, then the TickJob table.  The
    // device table is rewritten in stream order; its host staging is a ring of
    // pinned buffers, so a recomposition waits only for a copy kStageRing
    // recompositions old.
    // The device table: the composition header (GroupHdr), the matrix-core
    // job table and the TickJob table at fixed offsets sized for kMaxPoolJobs
    // contexts, so a captured generation's pointers stay valid for every
    // composition.
    static constexpr int kStageRing = 8;
    static constexpr size_t kHdrBytes = 256;
    void *d_tab = nullptr;
    void *h_tab[kStageRing] = {};
    hipEvent_t tab_copied[kStageRing] = {};
    int stage = 0;
    size_t tab_cap = 0, tick_off = 0;
    int njobs = 0, total_tiles = 0, min_p = 0, sel_threads = 64;
    int round_robin = 0;   // some context is folded: tiles go round robin over the XCDs
    int blocks[kTickPhases] = {};
    size_t lds_recheck = 0, lds_recheck_wide = 0;
    // One grouped generation captured as a graph, its grids sized to a
    // capacity; every composition that fits replays it (the kernels read the
    // composition from the header), a larger one is captured anew.
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_failed = false;
    int cap_blocks[kTickPhases] = {};
    int cap_grid = 0, cap_kins = 0, cap_sel = 0;
    size_t cap_lds = 0, cap_lds_wide = 0;
};

namespace {

ga_status fail(ga_ctx *ctx, ga_status s, const std::string &msg)
{
    if (ctx) {
        ctx->err = msg;
        if (s == GA_ERR_DEVICE) ctx->poisoned = true;
    } else {
        g_init_error = msg;
    }
    return s;
}

#define HIPCHK(expr)                                                                                      \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return fail(ctx, GA_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CTXCHK(ctx)                                                     \
    do {                                                                \
        if (!(ctx)) return GA_ERR_INVALID;                              \
        if ((ctx)->poisoned) return GA_ERR_STATE;                       \
    } while (0)

// Two events around the dominant evaluation kernel when profiling is on.
void prof_events(ga_ctx *ctx, hipEvent_t *a, hipEvent_t *b)
{
    *a = *b = nullptr;
    if (!ctx->prof_on || ctx->ev_used + 2 > (int)ctx->ev.size()) return;
    *a = ctx->ev[ctx->ev_used];
    *b = ctx->ev[ctx->ev_used + 1];
    ctx->ev_used += 2;
}

// The split buffers into the layout tile configuration cfg reads (split
// mode), enqueued on the context's stream when it differs from the layout
// they hold.  Never called during graph capture.
ga_status ensure_w_layout(ga_ctx *ctx, int cfg)
{
    if (!split_mode(ctx->d.prec)) return GA_OK;
    const int want = mfma_w_layout(ctx->d, cfg);
    if (want == ctx->wlayout) return GA_OK;
    HIPCHK(launch_w_layout(ctx->P, ctx->d, want, ctx->st));
    ctx->wlayout = want;
    return GA_OK;
}

// Evaluate `count` sorted hub sets at `hubs` (device) into P.cost / P.parts /
// P.eps, hub positions into `kidx`, on stream s; with ops.anc set, the
// allocation kernel first builds the sets (the generation's operators).
ga_status run_eval(ga_ctx *ctx, const int32_t *hubs, int count, uint16_t *kidx, hipStream_t s,
                   const AllocOps &ops = AllocOps{})
{
    const Dims &d = ctx->d;
    const DevPtrs &P = ctx->P;
    hipEvent_t a, b;
    prof_events(ctx, &a, &b);
    if (d.prec == kFP64) {
        HIPCHK(launch_alloc(P, d, hubs, count, kidx, 0, 0, s, ops));
        if (a) HIPCHK(hipEventRecord(a, s));
        HIPCHK(launch_eval_exact(P, d, hubs, kidx, count, P.cost, P.parts, P.eps, s));
        if (b) HIPCHK(hipEventRecord(b, s));
    } else if (d.prec == kFP32 && d.kern == GA_KERN_BATCHED) {
        HIPCHK(launch_alloc(P, d, hubs, count, kidx, 1, 1, s, ops));
        HIPCHK(launch_eval_vec(P, d, kidx, count, s, a, b));
    } else if (d.prec == kFP32) {
        HIPCHK(launch_alloc(P, d, hubs, count, kidx, 1, 0, s, ops));
        if (a) HIPCHK(hipEventRecord(a, s));
        HIPCHK(launch_eval_fp32(P, d, hubs, kidx, count, s));
        if (b) HIPCHK(hipEventRecord(b, s));
    } else {
        HIPCHK(launch_alloc(P, d, hubs, count, kidx, 1, 1, s, ops));
        HIPCHK(launch_eval_split(P, d, kidx, count, s, a, b));
    }
    return GA_OK;
}

ga_status run_eval(ga_ctx *ctx, const int32_t *hubs, int count, uint16_t *kidx)
{
    return run_eval(ctx, hubs, count, kidx, ctx->st);
}

// One generation on stream s: operators (in the allocation kernel, one
// child per workgroup), evaluation, selection.
ga_status run_generation(ga_ctx *ctx, hipStream_t s)
{
    const Dims &d = ctx->d;
    const DevPtrs &P = ctx->P;
    AllocOps ops;
    ops.anc = P.anc;
    ops.children = P.hubs;
    ops.gen = P.gen;
    ops.seed = d.seed;
    ops.m = d.m;
    ops.slot_counters[0] = P.total;
    ops.slot_counters[1] = P.nextra;
    ga_status st = run_eval(ctx, P.hubs, d.S, P.kidx, s, ops);
    if (st != GA_OK) return st;
    HIPCHK(launch_select(P, d, d.prec == kFP64, s, 1));
    return GA_OK;
}

ga_status run_generation(ga_ctx *ctx) { return run_generation(ctx, ctx->st); }

void drop_graph(ga_ctx *ctx)
{
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->gexec = nullptr;
    ctx->graph = nullptr;
}

// Capture one generation on the context's stream; false if the stream cannot
// be captured (then generations are launched directly).
bool capture_generation(ga_ctx *ctx)
{
    if (!ctx->st || ctx->graph_failed) return false;
    if (hipStreamBeginCapture(ctx->st, hipStreamCaptureModeRelaxed) != hipSuccess) {
        ctx->graph_failed = true;
        return false;
    }
    ga_status gs = run_generation(ctx);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->st, &g);
    if (gs != GA_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        ctx->poisoned = false;   // a failed capture enqueued nothing
        ctx->graph_failed = true;
        (void)hipGetLastError();
        return false;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        ctx->graph_failed = true;
        (void)hipGetLastError();
        return false;
    }
    ctx->graph = g;
    ctx->gexec = x;
    return true;
}

template <typename T>
std::string check_matrix(const void *M, int n, bool split_limit)
{
    const T *x = (const T *)M;
    const size_t n2 = (size_t)n * n;
    for (size_t k = 0; k < n2; ++k) {
        double v = (double)x[k];
        if (!std::isfinite(v) || v < 0.0) return "entry " + std::to_string(k) + " is negative or not finite";
        if (split_limit && v > 3.38e38) return "entry " + std::to_string(k) + " exceeds the bf16 range";
    }
    return "";
}

template <typename T>
bool symmetric(const void *M, int n)
{
    const T *x = (const T *)M;
    constexpr int B = 64;   // blocks of B x B, so the transposed reads stay in cache
    for (int bi = 0; bi < n; bi += B)
        for (int bj = bi; bj < n; bj += B)
            for (int i = bi; i < std::min(n, bi + B); ++i)
                for (int j = std::max(bj, i + 1); j < std::min(n, bj + B); ++j)
                    if (x[(size_t)i * n + j] != x[(size_t)j * n + i]) return false;
    return true;
}

std::string sort_check_hubs(const int32_t *in, int p, int n, int32_t *out)
{
    std::memcpy(out, in, sizeof(int32_t) * p);
    std::sort(out, out + p);
    if (out[0] < 0 || out[p - 1] >= n) return "hub id out of range";
    for (int k = 1; k < p; ++k)
        if (out[k] == out[k - 1]) return "repeated hub id";
    return "";
}

}  // namespace

extern "C" {

void ga_params_default(ga_params *q, int32_t n, int32_t hubs)
{
    if (!q) return;
    std::memset(q, 0, sizeof(*q));
    q->n = n;
    q->p = hubs;
    q->chi = 3.0;
    q->alpha = 0.75;
    q->delta = 2.0;
    q->scale = 1.0;
    q->seed = 1;
    q->population = 64;
    q->island_size = 64;
    q->n1 = 10;
    q->elitist = 1;
    q->precision = GA_PREC_FP64;
    q->kernel = GA_KERN_PLAIN;
    q->c_symmetric = 0;
    q->multihop = 0;
}

size_t ga_workspace_bytes(const ga_params *q, ga_dtype cdt, ga_dtype wdt)
{
    if (!check_params(q).empty()) return 0;
    if ((cdt != GA_DT_F64 && cdt != GA_DT_F32) || (wdt != GA_DT_F64 && wdt != GA_DT_F32)) return 0;
    return carve(make_dims(q, cdt, wdt), q->c_symmetric).total;
}

// Frees what ga_init took (the workspace if the library allocated it) and the
// context itself; a context in static storage is destroyed in place, its
// device slot released only when release_slot is set.
static void release_ctx(ga_ctx *ctx, bool release_slot)
{
    if (ctx->own_ws) (void)hipFree(ctx->ws);
    const int sd = ctx->static_dev;
    if (sd < 0) {
        delete ctx;
        return;
    }
    ctx->~ga_ctx();
    if (release_slot) {
        std::lock_guard<std::mutex> g(g_static_mu);
        g_static[sd].busy = false;
    }
}

// ga_init and ga_init_static: static_dev >= 0 builds the context in that
// device's static storage on d_workspace (that device's static array).
static ga_status init_ctx(const ga_params *q, const void *C, ga_dtype cdt, const void *W, ga_dtype wdt,
                          void *d_workspace, size_t ws_bytes, void *hip_stream, ga_ctx **out, int static_dev)
{
    ga_ctx *ctx = nullptr;
    try {
        if (!out) return fail(nullptr, GA_ERR_INVALID, "out is NULL");
        *out = nullptr;
        std::string e = check_params(q);
        if (!e.empty()) return fail(nullptr, GA_ERR_INVALID, e);
        if ((cdt != GA_DT_F64 && cdt != GA_DT_F32) || (wdt != GA_DT_F64 && wdt != GA_DT_F32))
            return fail(nullptr, GA_ERR_INVALID, "unknown dtype");
        if (!C || !W) return fail(nullptr, GA_ERR_INVALID, "C and W must be host arrays");
        const bool split = q->precision == GA_PREC_SPLIT_BF16 || q->precision == GA_PREC_SPLIT3_BF16;
        e = cdt == GA_DT_F32 ? check_matrix<float>(C, q->n, false) : check_matrix<double>(C, q->n, false);
        if (!e.empty()) return fail(nullptr, GA_ERR_INVALID, "C: " + e);
        e = wdt == GA_DT_F32 ? check_matrix<float>(W, q->n, split) : check_matrix<double>(W, q->n, split);
        if (!e.empty()) return fail(nullptr, GA_ERR_INVALID, "W: " + e);
        if (q->c_symmetric && !(cdt == GA_DT_F32 ? symmetric<float>(C, q->n) : symmetric<double>(C, q->n)))
            return fail(nullptr, GA_ERR_INVALID, "c_symmetric is set but C is not symmetric");
        Dims d = make_dims(q, cdt, wdt);
        Carve c = carve(d, q->c_symmetric);
        {
            static std::once_flag once;
            static hipError_t prep_err = hipSuccess;
            std::call_once(once, [] {
                int dev = 0, max_lds = 65536, optin = 0;
                if (hipGetDevice(&dev) == hipSuccess) {
                    (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
                    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess &&
                        optin > max_lds)
                        max_lds = optin;
                }
                (void)hipGetLastError();
                prep_err = prepare_plain_kernels(max_lds);
                if (prep_err == hipSuccess) prep_err = prepare_recheck_kernels(max_lds);
                if (prep_err == hipSuccess) prep_err = prepare_enum_kernels(max_lds);
            });
            if (prep_err != hipSuccess)
                return fail(nullptr, GA_ERR_DEVICE, std::string("kernel attributes: ") + hipGetErrorString(prep_err));
        }
        if (make_dims(q, cdt, wdt).n > 0) {
            int dev = 0, max_lds = 65536, optin = 0;
            if (hipGetDevice(&dev) == hipSuccess) {
                (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
                if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess &&
                    optin > max_lds)
                    max_lds = optin;
            }
            (void)hipGetLastError();
            const size_t need = std::max(recheck_lds(d.n, d.p), recheck_wide_lds(d.n, d.p)) + 4096;   // + static LDS
            if (need > (size_t)max_lds)
                return fail(nullptr, GA_ERR_INVALID, "n too large for this device's LDS (exact kernels)");
        }
        if (d_workspace && ws_bytes < c.total)
            return fail(nullptr, GA_ERR_OOM,
                        "workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(c.total));
        if (((uintptr_t)d_workspace) % 256)
            return fail(nullptr, GA_ERR_INVALID, "workspace must be 256-byte aligned");
        ctx = static_dev >= 0 ? new (g_static[static_dev].ctx_mem) ga_ctx() : new (std::nothrow) ga_ctx();
        if (!ctx) return fail(nullptr, GA_ERR_OOM, "host allocation failed");
        ctx->static_dev = static_dev;
        ctx->prm = *q;
        ctx->d = d;
        ctx->st = (hipStream_t)hip_stream;
        if (d_workspace) {
            ctx->ws = d_workspace;
        } else {
            hipError_t he = hipMalloc(&ctx->ws, c.total);
            if (he != hipSuccess) {
                release_ctx(ctx, false);
                return fail(nullptr, GA_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(he));
            }
            ctx->own_ws = true;
        }
        void *b = ctx->ws;
        DevPtrs &P = ctx->P;
        P.C = at<void>(b, c.C);
        P.Ct = at<void>(b, c.Ct);
        P.Ct32 = at<float>(b, c.Ct32);
        P.W = at<void>(b, c.W);
        P.W32 = at<float>(b, c.W32);
        P.Ctr = at<double>(b, c.Ctr);
        P.Whi = at<uint16_t>(b, c.Whi);
        P.Wlo = at<uint16_t>(b, c.Wlo);
        P.Wmd = at<uint16_t>(b, c.Wmd);
        P.Whsw = P.Wfhsw = P.Whi;
        P.Wlsw = P.Wflsw = P.Wlo;
        P.O = at<double>(b, c.O);
        P.D = at<double>(b, c.D);
        P.dsum = at<double>(b, c.dsum);
        P.hubs = at<int32_t>(b, c.hubs);
        P.kidx = at<uint16_t>(b, c.kidx);
        P.cost = at<double>(b, c.cost);
        P.parts = at<double>(b, c.parts);
        P.eps = at<double>(b, c.eps);
        P.cmax = at<int32_t>(b, c.cmax);
        P.Ch32 = at<float>(b, c.Ch32);
        P.partial = at<double>(b, c.partial);
        P.anc = at<int32_t>(b, c.anc);
        P.anc_cost = at<double>(b, c.anc_cost);
        P.anc_parts = at<double>(b, c.anc_parts);
        P.best = at<int32_t>(b, c.best);
        P.best_cost = at<double>(b, c.best_cost);
        P.gen = at<int64_t>(b, c.gen);
        P.stats = at<int64_t>(b, c.stats);
        P.cand = at<int32_t>(b, c.cand);
        P.cand_cnt = at<int32_t>(b, c.cand_cnt);
        P.cand_cost = at<double>(b, c.cand_cost);
        P.cand_parts = at<double>(b, c.cand_parts);
        P.kidx_one = at<uint16_t>(b, c.kidx_one);
        P.scratch = at<uint8_t>(b, c.scratch);
        P.tbuf = at<double>(b, c.tbuf);
        P.slot_r = at<int32_t>(b, c.slot_r);
        P.slot_c = at<int32_t>(b, c.slot_c);
        P.slot_s = at<int32_t>(b, c.slot_s);
        P.slot_done = at<int32_t>(b, c.slot_done);
        P.handled = at<int32_t>(b, c.handled);
        P.choice = at<int32_t>(b, c.choice);
        P.total = at<int32_t>(b, c.total_slots);
        P.extra_r = at<int32_t>(b, c.extra_r);
        P.extra_c = at<int32_t>(b, c.extra_c);
        P.nextra = at<int32_t>(b, c.nextra);
        P.sync = at<int>(b, c.sync);
        P.enum_state = at<EnumState>(b, c.enum_state);
        P.enum_best = at<int32_t>(b, c.enum_best);
        P.binom = at<uint64_t>(b, c.binom);

        const size_t n2 = (size_t)d.n * d.n;
        auto dev_fail = [&](hipError_t he, const char *what) {
            std::string m = std::string(what) + ": " + hipGetErrorString(he);
            release_ctx(ctx, false);
            return fail(nullptr, GA_ERR_DEVICE, m);
        };
        hipError_t he;
        if ((he = hipMemcpyAsync(P.C, C, n2 * (d.c_f32 ? 4 : 8), hipMemcpyHostToDevice, ctx->st)) != hipSuccess)
            return dev_fail(he, "copy C");
        if ((he = hipMemcpyAsync(P.W, W, n2 * (d.w_f32 ? 4 : 8), hipMemcpyHostToDevice, ctx->st)) != hipSuccess)
            return dev_fail(he, "copy W");
        if ((he = launch_prep(P, d, ctx->st)) != hipSuccess) return dev_fail(he, "prep");
        if ((he = launch_shortest_paths(P, d, ctx->st)) != hipSuccess) return dev_fail(he, "shortest paths");
        if (split_mode(d.prec)) {
            if ((he = launch_w_layout(P, d, mfma_w_layout(d, d.mfma_cfg), ctx->st)) != hipSuccess)
                return dev_fail(he, "split of W");
            ctx->wlayout = mfma_w_layout(d, d.mfma_cfg);
        }
        // ancestor P0: middle nodes, nearest-hub allocation, exact cost (Sec. 4.1)
        if ((he = launch_middle_nodes(P, d, P.best, P.scratch, ctx->st)) != hipSuccess)
            return dev_fail(he, "middle nodes");
        if ((he = launch_alloc(P, d, P.best, 1, P.kidx_one, 0, 0, ctx->st)) != hipSuccess)
            return dev_fail(he, "alloc P0");
        if ((he = launch_p0_exact(P, d, ctx->st)) != hipSuccess) return dev_fail(he, "eval P0");
        if ((he = launch_init_state(P, d, ctx->st)) != hipSuccess) return dev_fail(he, "init state");
        if ((he = hipStreamSynchronize(ctx->st)) != hipSuccess) return dev_fail(he, "sync");
        *out = ctx;
        return GA_OK;
    } catch (...) {
        if (ctx) release_ctx(ctx, false);
        return fail(nullptr, GA_ERR_OOM, "exception in ga_init");
    }
}

ga_status ga_init(const ga_params *q, const void *C, ga_dtype cdt, const void *W, ga_dtype wdt, void *d_workspace,
                  size_t ws_bytes, void *hip_stream, ga_ctx **out)
{
    return init_ctx(q, C, cdt, W, wdt, d_workspace, ws_bytes, hip_stream, out, -1);
}

ga_status ga_init_static(const ga_params *q, const void *C, ga_dtype cdt, const void *W, ga_dtype wdt,
                         void *hip_stream, ga_ctx **out)
{
    if (!out) return fail(nullptr, GA_ERR_INVALID, "out is NULL");
    *out = nullptr;
    const std::string e = check_params(q);
    if (!e.empty()) return fail(nullptr, GA_ERR_INVALID, e);
    const size_t need = ga_workspace_bytes(q, cdt, wdt);
    if (need == 0) return fail(nullptr, GA_ERR_INVALID, "unknown dtype");
    if (need > kStaticWorkspaceBytes)
        return fail(nullptr, GA_ERR_INVALID,
                    "ga_init_static: the context needs " + std::to_string(need) + " workspace bytes, more than the " +
                        std::to_string(kStaticWorkspaceBytes) + " of the static workspace; use ga_init");
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return fail(nullptr, GA_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(he));
    if (dev < 0 || dev >= kMaxStaticDevices) return fail(nullptr, GA_ERR_INVALID, "ga_init_static: device id too large");
    StaticSlot &slot = g_static[dev];
    {
        std::lock_guard<std::mutex> g(g_static_mu);
        if (!slot.resolved) {   // once per device, with the device current
            void *ptr = nullptr;
            he = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (he != hipSuccess || !ptr)
                return fail(nullptr, GA_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                                        hipGetErrorString(he));
            slot.ptr = ptr;
            slot.resolved = true;
        }
        if (slot.busy)
            return fail(nullptr, GA_ERR_STATE,
                        "ga_init_static: a live context holds this device's static workspace; ga_free it first");
        slot.busy = true;
    }
    ga_status st = init_ctx(q, C, cdt, W, wdt, slot.ptr, kStaticWorkspaceBytes, hip_stream, out, dev);
    if (st != GA_OK) {
        std::lock_guard<std::mutex> g(g_static_mu);
        slot.busy = false;
    }
    return st;
}

ga_status ga_evaluate(ga_ctx *ctx, const int32_t *hubs, int32_t count, double *cost_out, double *parts_out,
                      int32_t *alloc_out, double *eps_out)
{
    CTXCHK(ctx);
    try {
        const Dims &d = ctx->d;
        if (!hubs || !cost_out || count < 0) return fail(ctx, GA_ERR_INVALID, "hubs and cost_out are required");
        std::vector<int32_t> sorted((size_t)count * d.p);
        for (int s = 0; s < count; ++s) {
            std::string e = sort_check_hubs(hubs + (size_t)s * d.p, d.p, d.n, &sorted[(size_t)s * d.p]);
            if (!e.empty()) return fail(ctx, GA_ERR_INVALID, "hub set " + std::to_string(s) + ": " + e);
        }
        ga_status ls = ensure_w_layout(ctx, d.mfma_cfg);
        if (ls != GA_OK) return ls;
        std::vector<double> c((size_t)d.S), pr((size_t)3 * d.S), ep((size_t)d.S);
        std::vector<uint16_t> kx;
        if (alloc_out) kx.resize((size_t)d.S * d.n_pad);
        for (int s0 = 0; s0 < count; s0 += d.S) {
            const int cnt = std::min(d.S, count - s0);
            HIPCHK(hipMemcpyAsync(ctx->P.hubs, &sorted[(size_t)s0 * d.p], sizeof(int32_t) * cnt * d.p,
                                  hipMemcpyHostToDevice, ctx->st));
            ga_status st = run_eval(ctx, ctx->P.hubs, cnt, ctx->P.kidx);
            if (st != GA_OK) return st;
            HIPCHK(hipMemcpyAsync(c.data(), ctx->P.cost, 8 * cnt, hipMemcpyDeviceToHost, ctx->st));
            HIPCHK(hipMemcpyAsync(pr.data(), ctx->P.parts, 24 * cnt, hipMemcpyDeviceToHost, ctx->st));
            HIPCHK(hipMemcpyAsync(ep.data(), ctx->P.eps, 8 * cnt, hipMemcpyDeviceToHost, ctx->st));
            if (alloc_out)
                HIPCHK(hipMemcpyAsync(kx.data(), ctx->P.kidx, 2 * (size_t)cnt * d.n_pad, hipMemcpyDeviceToHost,
                                      ctx->st));
            HIPCHK(hipStreamSynchronize(ctx->st));
            for (int s = 0; s < cnt; ++s) {
                cost_out[s0 + s] = c[s];
                if (parts_out)
                    for (int q = 0; q < 3; ++q) parts_out[3 * (size_t)(s0 + s) + q] = pr[3 * (size_t)s + q];
                if (eps_out) eps_out[s0 + s] = ep[s];
                if (alloc_out) {
                    const int32_t *h = &sorted[(size_t)(s0 + s) * d.p];
                    for (int i = 0; i < d.n; ++i)
                        alloc_out[(size_t)(s0 + s) * d.n + i] = h[kx[(size_t)s * d.n_pad + i]];
                }
            }
        }
        return GA_OK;
    } catch (...) {
        return fail(ctx, GA_ERR_OOM, "host allocation failed in ga_evaluate");
    }
}

ga_status ga_evaluate_dev(ga_ctx *ctx, const int32_t *d_hubs, int32_t count, uint16_t *d_kidx, double *d_cost)
{
    CTXCHK(ctx);
    const Dims &d = ctx->d;
    if (!d_hubs || !d_cost || count < 1 || count > d.S)
        return fail(ctx, GA_ERR_INVALID, "need 1 <= count <= population and device hubs/cost");
    ga_status s = ensure_w_layout(ctx, d.mfma_cfg);
    if (s != GA_OK) return s;
    HIPCHK(launch_copy_clamp(d_hubs, ctx->P.hubs, count * d.p, d.n, ctx->st));
    s = run_eval(ctx, ctx->P.hubs, count, ctx->P.kidx);
    if (s != GA_OK) return s;
    HIPCHK(hipMemcpyAsync(d_cost, ctx->P.cost, 8 * (size_t)count, hipMemcpyDeviceToDevice, ctx->st));
    if (d_kidx)
        HIPCHK(hipMemcpy2DAsync(d_kidx, 2 * (size_t)d.n, ctx->P.kidx, 2 * (size_t)d.n_pad, 2 * (size_t)d.n, count,
                                hipMemcpyDeviceToDevice, ctx->st));
    return GA_OK;
}

ga_status ga_enumerate(ga_ctx *ctx, int64_t first, int64_t count, int32_t *hubs_out, double *cost_out,
                       double *parts_out, int64_t *rank_out, double *costs_all, double *eps_all, int64_t *rechecks_out)
{
    CTXCHK(ctx);
    try {
        const Dims &d = ctx->d;
        const DevPtrs &P = ctx->P;
        constexpr uint64_t kSat = 1ull << 63;
        if (!ctx->binom_ready) {   // Pascal's triangle, saturating
            const int w = d.p + 1;
            std::vector<uint64_t> t((size_t)(d.n + 1) * w, 0);
            for (int m = 0; m <= d.n; ++m) {
                t[(size_t)m * w] = 1;
                for (int j = 1; j <= std::min(m, d.p); ++j) {
                    const uint64_t a = t[(size_t)(m - 1) * w + j - 1], b = t[(size_t)(m - 1) * w + j];
                    t[(size_t)m * w + j] = (a >= kSat || b >= kSat || a + b >= kSat) ? kSat : a + b;
                }
            }
            HIPCHK(hipMemcpyAsync(P.binom, t.data(), t.size() * 8, hipMemcpyHostToDevice, ctx->st));
            HIPCHK(hipStreamSynchronize(ctx->st));
            ctx->nsets = t[(size_t)d.n * w + d.p];
            ctx->binom_ready = true;
        }
        const uint64_t total = ctx->nsets;
        if (total >= (1ull << 62)) return fail(ctx, GA_ERR_INVALID, "C(n, p) is 2^62 or more: too many hub sets");
        if (first < 0 || (uint64_t)first >= total) return fail(ctx, GA_ERR_INVALID, "first must be in [0, C(n, p))");
        if (count < 0) count = (int64_t)(total - (uint64_t)first);
        if (count == 0 || (uint64_t)count > total - (uint64_t)first)
            return fail(ctx, GA_ERR_INVALID, "count must be in [1, C(n, p) - first], or -1");
        ga_status ls = ensure_w_layout(ctx, d.mfma_cfg);
        if (ls != GA_OK) return ls;
        HIPCHK(launch_enum_init(P, ctx->st));
        for (int64_t off = 0; off < count; off += d.S) {
            const int cnt = (int)std::min<int64_t>(d.S, count - off);
            HIPCHK(launch_enum_unrank(P, d, first + off, cnt, ctx->st));
            ga_status st = run_eval(ctx, P.hubs, cnt, P.kidx);
            if (st != GA_OK) return st;
            HIPCHK(launch_enum_select(P, d, first + off, cnt, ctx->st));
            if (costs_all)
                HIPCHK(hipMemcpyAsync(costs_all + off, P.cost, 8 * (size_t)cnt, hipMemcpyDeviceToHost, ctx->st));
            if (eps_all)
                HIPCHK(hipMemcpyAsync(eps_all + off, P.eps, 8 * (size_t)cnt, hipMemcpyDeviceToHost, ctx->st));
        }
        EnumState es;
        std::vector<int32_t> h(d.p);
        HIPCHK(hipMemcpyAsync(&es, P.enum_state, sizeof(es), hipMemcpyDeviceToHost, ctx->st));
        HIPCHK(hipMemcpyAsync(h.data(), P.enum_best, 4 * (size_t)d.p, hipMemcpyDeviceToHost, ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));
        if (hubs_out) std::memcpy(hubs_out, h.data(), 4 * (size_t)d.p);
        if (cost_out) *cost_out = es.best_cost;
        if (parts_out) std::memcpy(parts_out, es.best_parts, 24);
        if (rank_out) *rank_out = es.best_rank;
        if (rechecks_out) *rechecks_out = es.rechecks;
        return GA_OK;
    } catch (...) {
        return fail(ctx, GA_ERR_OOM, "host allocation failed in ga_enumerate");
    }
}

ga_status ga_step(ga_ctx *ctx, int32_t generations)
{
    CTXCHK(ctx);
    if (generations < 0) return fail(ctx, GA_ERR_INVALID, "generations must be >= 0");
    if (generations == 0) return GA_OK;
    ga_status ls = ensure_w_layout(ctx, ctx->d.mfma_cfg);
    if (ls != GA_OK) return ls;
    if (!ctx->prof_on && (ctx->gexec || capture_generation(ctx))) {
        for (int g = 0; g < generations; ++g) HIPCHK(hipGraphLaunch(ctx->gexec, ctx->st));
        return GA_OK;
    }
    for (int g = 0; g < generations; ++g) {
        ga_status s = run_generation(ctx);
        if (s != GA_OK) return s;
    }
    return GA_OK;
}

ga_status ga_best(ga_ctx *ctx, int32_t *hubs_out, int32_t *alloc_out, double *cost_out, double *parts_out,
                  int64_t *generation_out)
{
    CTXCHK(ctx);
    const Dims &d = ctx->d;
    std::vector<int32_t> h(d.p);
    double bc[4];
    int64_t g;
    std::vector<uint16_t> kx;
    if (alloc_out) {
        HIPCHK(launch_alloc(ctx->P, d, ctx->P.best, 1, ctx->P.kidx_one, 0, 0, ctx->st));
        kx.resize(d.n_pad);
        HIPCHK(hipMemcpyAsync(kx.data(), ctx->P.kidx_one, 2 * (size_t)d.n_pad, hipMemcpyDeviceToHost, ctx->st));
    }
    HIPCHK(hipMemcpyAsync(h.data(), ctx->P.best, 4 * (size_t)d.p, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipMemcpyAsync(bc, ctx->P.best_cost, 32, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipMemcpyAsync(&g, ctx->P.gen, 8, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    if (hubs_out) std::memcpy(hubs_out, h.data(), 4 * (size_t)d.p);
    if (cost_out) *cost_out = bc[0];
    if (parts_out) std::memcpy(parts_out, bc + 1, 24);
    if (generation_out) *generation_out = g;
    if (alloc_out)
        for (int i = 0; i < d.n; ++i) alloc_out[i] = h[kx[i]];
    return GA_OK;
}

ga_status ga_solve(ga_ctx *ctx, int32_t generations, int32_t *hubs_out, int32_t *alloc_out, double *cost_out)
{
    ga_status s = ga_step(ctx, generations);
    if (s != GA_OK) return s;
    return ga_best(ctx, hubs_out, alloc_out, cost_out, nullptr, nullptr);
}

ga_status ga_population(ga_ctx *ctx, int32_t *hubs_out, double *cost_out)
{
    CTXCHK(ctx);
    const Dims &d = ctx->d;
    if (hubs_out) HIPCHK(hipMemcpyAsync(hubs_out, ctx->P.hubs, 4 * (size_t)d.S * d.p, hipMemcpyDeviceToHost, ctx->st));
    if (cost_out) HIPCHK(hipMemcpyAsync(cost_out, ctx->P.cost, 8 * (size_t)d.S, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    return GA_OK;
}

ga_status ga_ancestors(ga_ctx *ctx, int32_t *hubs_out, double *cost_out)
{
    CTXCHK(ctx);
    const Dims &d = ctx->d;
    if (hubs_out) HIPCHK(hipMemcpyAsync(hubs_out, ctx->P.anc, 4 * (size_t)d.R * d.p, hipMemcpyDeviceToHost, ctx->st));
    if (cost_out) HIPCHK(hipMemcpyAsync(cost_out, ctx->P.anc_cost, 8 * (size_t)d.R, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    return GA_OK;
}

// State blob: header {magic, n, p, S, m, seed, g} then anc (R*p int32),
// anc_cost (R), anc_parts (3R), best (p int32), best_cost + parts (4).
ga_status ga_get_state(ga_ctx *ctx, void *buf, size_t *bytes)
{
    CTXCHK(ctx);
    if (!bytes) return fail(ctx, GA_ERR_INVALID, "bytes is NULL");
    const Dims &d = ctx->d;
    const size_t hdr = 64;
    const size_t need = hdr + 4 * (size_t)d.R * d.p + 8 * (size_t)d.R + 24 * (size_t)d.R + 4 * (size_t)d.p + 32;
    if (!buf) {
        *bytes = need;
        return GA_OK;
    }
    if (*bytes < need) return fail(ctx, GA_ERR_INVALID, "state buffer too small");
    char *o = (char *)buf;
    std::memset(o, 0, hdr);
    uint32_t hv[5] = {kStateMagic, (uint32_t)d.n, (uint32_t)d.p, (uint32_t)d.S, (uint32_t)d.m};
    std::memcpy(o, hv, sizeof(hv));
    std::memcpy(o + 24, &ctx->prm.seed, 8);
    char *q = o + hdr;
    HIPCHK(hipMemcpyAsync(o + 32, ctx->P.gen, 8, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipMemcpyAsync(q, ctx->P.anc, 4 * (size_t)d.R * d.p, hipMemcpyDeviceToHost, ctx->st));
    q += 4 * (size_t)d.R * d.p;
    HIPCHK(hipMemcpyAsync(q, ctx->P.anc_cost, 8 * (size_t)d.R, hipMemcpyDeviceToHost, ctx->st));
    q += 8 * (size_t)d.R;
    HIPCHK(hipMemcpyAsync(q, ctx->P.anc_parts, 24 * (size_t)d.R, hipMemcpyDeviceToHost, ctx->st));
    q += 24 * (size_t)d.R;
    HIPCHK(hipMemcpyAsync(q, ctx->P.best, 4 * (size_t)d.p, hipMemcpyDeviceToHost, ctx->st));
    q += 4 * (size_t)d.p;
    HIPCHK(hipMemcpyAsync(q, ctx->P.best_cost, 32, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    *bytes = need;
    return GA_OK;
}

ga_status ga_set_state(ga_ctx *ctx, const void *buf, size_t bytes)
{
    CTXCHK(ctx);
    const Dims &d = ctx->d;
    const size_t hdr = 64;
    const size_t need = hdr + 4 * (size_t)d.R * d.p + 8 * (size_t)d.R + 24 * (size_t)d.R + 4 * (size_t)d.p + 32;
    if (!buf || bytes != need) return fail(ctx, GA_ERR_STATE, "state blob has the wrong size");
    const char *o = (const char *)buf;
    uint32_t hv[5];
    uint64_t seed;
    std::memcpy(hv, o, sizeof(hv));
    std::memcpy(&seed, o + 24, 8);
    if (hv[0] != kStateMagic || hv[1] != (uint32_t)d.n || hv[2] != (uint32_t)d.p || hv[3] != (uint32_t)d.S ||
        hv[4] != (uint32_t)d.m || seed != ctx->prm.seed)
        return fail(ctx, GA_ERR_STATE, "state blob belongs to a different configuration");
    const char *q = o + hdr;
    HIPCHK(hipMemcpyAsync(ctx->P.gen, o + 32, 8, hipMemcpyHostToDevice, ctx->st));
    HIPCHK(hipMemcpyAsync(ctx->P.anc, q, 4 * (size_t)d.R * d.p, hipMemcpyHostToDevice, ctx->st));
    q += 4 * (size_t)d.R * d.p;
    HIPCHK(hipMemcpyAsync(ctx->P.anc_cost, q, 8 * (size_t)d.R, hipMemcpyHostToDevice, ctx->st));
    q += 8 * (size_t)d.R;
    HIPCHK(hipMemcpyAsync(ctx->P.anc_parts, q, 24 * (size_t)d.R, hipMemcpyHostToDevice, ctx->st));
    q += 24 * (size_t)d.R;
    HIPCHK(hipMemcpyAsync(ctx->P.best, q, 4 * (size_t)d.p, hipMemcpyHostToDevice, ctx->st));
    q += 4 * (size_t)d.p;
    HIPCHK(hipMemcpyAsync(ctx->P.best_cost, q, 32, hipMemcpyHostToDevice, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    return GA_OK;
}

ga_status ga_stats(ga_ctx *ctx, int64_t stats[4])
{
    CTXCHK(ctx);
    if (!stats) return fail(ctx, GA_ERR_INVALID, "stats is NULL");
    HIPCHK(hipMemcpyAsync(stats, ctx->P.stats, 32, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    return GA_OK;
}

ga_status ga_profile_enable(ga_ctx *ctx, int32_t enable)
{
    CTXCHK(ctx);
    if (enable) {
        HIPCHK(hipStreamSynchronize(ctx->st));
        if (ctx->ev.empty()) {
            ctx->ev.resize(kProfilePairs * 2);
            for (auto &e : ctx->ev) HIPCHK(hipEventCreate(&e));
        }
        ctx->ev_used = 0;
    }
    ctx->prof_on = enable != 0;
    return GA_OK;
}

ga_status ga_profile_read(ga_ctx *ctx, double *ms_total, int64_t *launches)
{
    CTXCHK(ctx);
    HIPCHK(hipStreamSynchronize(ctx->st));
    double tot = 0.0;
    for (int k = 0; k + 1 < ctx->ev_used; k += 2) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev[k], ctx->ev[k + 1]));
        tot += ms;
    }
    if (ms_total) *ms_total = tot;
    if (launches) *launches = ctx->ev_used / 2;
    return GA_OK;
}

ga_status ga_set_stream(ga_ctx *ctx, void *hip_stream)
{
    CTXCHK(ctx);
    hipStream_t ns = (hipStream_t)hip_stream;
    if (ns == ctx->st) return GA_OK;
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e1 = hipEventRecord(ev, ctx->st);
    hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(ns, ev, 0) : e1;
    (void)hipEventDestroy(ev);   // released once the recorded work completes
    HIPCHK(e2);
    ctx->st = ns;
    ctx->graph_failed = false;   // a capture refused on the old stream may succeed on this one
    return GA_OK;
}

int32_t ga_tile_config_count(void) { return mfma_num_configs(); }

ga_status ga_tile_config_info(int32_t cfg, int32_t *rows, int32_t *cols, int32_t *ktile)
{
    if (cfg < 0 || cfg >= mfma_num_configs()) return fail(nullptr, GA_ERR_INVALID, "no such tile configuration");
    if (rows) *rows = mfma_rows_per_tile(cfg);
    if (cols) *cols = mfma_cols_per_tile(cfg);
    if (ktile) *ktile = mfma_k_tile(cfg);
    return GA_OK;
}

ga_status ga_set_tile_config(ga_ctx *ctx, int32_t cfg)
{
    CTXCHK(ctx);
    if (cfg < 0 || cfg >= mfma_num_configs()) return fail(ctx, GA_ERR_INVALID, "no such tile configuration");
    if (ctx->d.prec == kSplit3BF16 && !mfma_split3_config(cfg))
        return fail(ctx, GA_ERR_INVALID, "the three-part split runs in tile configurations 0, 2, 3 and 5 only");
    if (ctx->d.mfma_cfg != cfg) drop_graph(ctx);
    ctx->d.mfma_cfg = cfg;
    return ensure_w_layout(ctx, cfg);
}

ga_status ga_evaluation_folded(ga_ctx *ctx, int32_t *folded)
{
    CTXCHK(ctx);
    if (!folded) return fail(ctx, GA_ERR_INVALID, "folded is NULL");
    *folded = ctx->d.prec == kSplitBF16 && mfma_folds(ctx->d, ctx->d.mfma_cfg);
    return GA_OK;
}

}  // extern "C"

// ------------------------------------------------------------- batches --

namespace {

// Offset of the TickJob table in a batch's device table, and its size.
size_t batch_tick_offset()
{
    return ga_batch::kHdrBytes + ((mfma_job_bytes() * kMaxPoolJobs + 255) & ~(size_t)255);
}
size_t batch_table_bytes() { return batch_tick_offset() + sizeof(TickJob) * kMaxPoolJobs; }

// One grouped generation: the six grouped launches with the given grids
// (workgroups per phase, matrix-core workgroups, hub-position transfers,
// selection block size, re-evaluation LDS); the kernels take the composition
// from the table's header.
hipError_t launch_grouped(const ga_batch *b, const int *grid, int mfma_grid, int kins, int sel_threads,
                          size_t lds_recheck, size_t lds_recheck_wide)
{
    const GroupHdr *hdr = (const GroupHdr *)b->d_tab;
    const void *mjobs = (const char *)b->d_tab + ga_batch::kHdrBytes;
    const TickJob *tjobs = (const TickJob *)((const char *)b->d_tab + batch_tick_offset());
    const int nj = b->njobs;
    hipError_t e;
    if ((e = launch_ga_ops_group(hdr, tjobs, nj, grid[kTickOps], b->st)) != hipSuccess) return e;
    if ((e = launch_alloc_group(hdr, tjobs, nj, grid[kTickAlloc], b->st)) != hipSuccess) return e;
    if ((e = launch_mfma_group(hdr, mjobs, mfma_grid, b->cfg, kins, b->st)) != hipSuccess) return e;
    if ((e = launch_finalize_group(hdr, tjobs, nj, grid[kTickFinal], b->st)) != hipSuccess) return e;
    if ((e = launch_select1_group(hdr, tjobs, nj, grid[kTickSel1], sel_threads, b->st)) != hipSuccess) return e;
    return launch_recheck_group(hdr, tjobs, nj, lds_recheck, lds_recheck_wide, b->st);
}

void drop_batch_graph(ga_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

int grid_cap(int need)   // a power of two, at least 8
{
    int c = 8;
    while (c < need) c *= 2;
    return c;
}

// Keep the captured grouped generation when the current composition fits
// its grids; otherwise capture one whose grids have room to grow.  A stream
// that cannot be captured leaves direct launches.
void capture_batch_generation(ga_batch *b)
{
    const int kins = mfma_group_kins(b->cfg, b->min_p);
    bool fits = b->gexec && kins <= b->cap_kins && b->sel_threads <= b->cap_sel && b->lds_recheck <= b->cap_lds &&
                b->lds_recheck_wide <= b->cap_lds_wide && b->total_tiles <= b->cap_grid;
    for (int q = 0; q < kTickPhases && fits; ++q) fits = b->blocks[q] <= b->cap_blocks[q];
    if (fits || b->graph_failed) return;
    drop_batch_graph(b);
    int caps[kTickPhases];
    for (int q = 0; q < kTickPhases; ++q) caps[q] = grid_cap(b->blocks[q]);
    const int cap_grid = grid_cap(b->total_tiles), cap_kins = std::max(kins, b->cap_kins);
    const int cap_sel = std::max(b->sel_threads, b->cap_sel);
    const size_t cap_lds = std::max(b->lds_recheck, b->cap_lds);
    const size_t cap_lds_wide = std::max(b->lds_recheck_wide, b->cap_lds_wide);
    if (hipStreamBeginCapture(b->st, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        b->graph_failed = true;
        return;
    }
    const hipError_t le = launch_grouped(b, caps, cap_grid, cap_kins, cap_sel, cap_lds, cap_lds_wide);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(b->st, &g);
    hipGraphExec_t x = nullptr;
    if (le != hipSuccess || ee != hipSuccess || !g || hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        b->graph_failed = true;
        return;
    }
    b->graph = g;
    b->gexec = x;
    memcpy(b->cap_blocks, caps, sizeof(caps));
    b->cap_grid = cap_grid;
    b->cap_kins = cap_kins;
    b->cap_sel = cap_sel;
    b->cap_lds = cap_lds;
    b->cap_lds_wide = cap_lds_wide;
}

}  // namespace

extern "C" {

ga_status ga_batch_create(void *hip_stream, int32_t tile_config, ga_batch **out)
{
    if (!out) return fail(nullptr, GA_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!hip_stream) return fail(nullptr, GA_ERR_INVALID, "a batch needs a non-null stream");
    if (tile_config < 0 || tile_config >= mfma_num_configs() || !mfma_pipelined(tile_config))
        return fail(nullptr, GA_ERR_INVALID, "the batch tile configuration must be a pipelined one");
    ga_batch *b = new (std::nothrow) ga_batch();
    if (!b) return fail(nullptr, GA_ERR_OOM, "host allocation failed");
    b->st = (hipStream_t)hip_stream;
    b->cfg = tile_config;
    for (auto &ev : b->tab_copied)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ga_batch_free(b);
            return fail(nullptr, GA_ERR_DEVICE, "event");
        }
    // the device table and its pinned staging ring, at their full size
    b->tab_cap = batch_table_bytes();
    if (hipMalloc(&b->d_tab, b->tab_cap) != hipSuccess) {
        ga_batch_free(b);
        return fail(nullptr, GA_ERR_OOM, "job table");
    }
    for (auto &h : b->h_tab)
        if (hipHostMalloc(&h, b->tab_cap, 0) != hipSuccess) {
            ga_batch_free(b);
            return fail(nullptr, GA_ERR_OOM, "job table staging");
        }
    *out = b;
    return GA_OK;
}

ga_status ga_batch_set(ga_batch *b, ga_ctx *const *ctxs, int32_t count)
{
    if (!b || (count > 0 && !ctxs) || count < 0) return GA_ERR_INVALID;
    for (int i = 0; i < count; ++i) {
        if (!ctxs[i]) return fail(nullptr, GA_ERR_INVALID, "NULL context in batch");
        if (ctxs[i]->poisoned) return GA_ERR_STATE;
        if (ctxs[i]->st != b->st) return fail(nullptr, GA_ERR_INVALID, "batch contexts must use the batch's stream");
        for (int k = 0; k < i; ++k)
            if (ctxs[k] == ctxs[i]) return fail(nullptr, GA_ERR_INVALID, "context listed twice");
    }
    hipError_t e;
    // split-bf16 contexts whose hub count the tile configuration takes are
    // grouped; the others step alone (their own generation graph) beside them
    std::vector<ga_ctx *> grouped, solo;
    for (int i = 0; i < count; ++i) {
        ga_ctx *c = ctxs[i];
        if (c->d.prec == kSplitBF16 && mfma_groupable(c->d, b->cfg) && (int)grouped.size() < kMaxPoolJobs)
            grouped.push_back(c);
        else
            solo.push_back(c);
    }
    for (ga_ctx *c : grouped)
        if (ensure_w_layout(c, b->cfg) != GA_OK) return fail(nullptr, GA_ERR_DEVICE, "split of W: " + c->err);
    for (ga_ctx *c : solo) {
        if (ensure_w_layout(c, c->d.mfma_cfg) != GA_OK) return fail(nullptr, GA_ERR_DEVICE, "split of W: " + c->err);
        if (!c->gexec && !c->prof_on) (void)capture_generation(c);
    }
    const int njobs = (int)grouped.size();
    std::vector<const DevPtrs *> P;
    std::vector<const Dims *> D;
    std::vector<TickJob> tj(njobs);
    int min_p = 1 << 30, sel_threads = 64, round_robin = 0;
    int blocks[kTickPhases] = {};
    size_t lds_recheck = 0, lds_recheck_wide = 0;
    for (int j = 0; j < njobs; ++j) {
        const ga_ctx *c = grouped[j];
        const Dims &d = c->d;
        P.push_back(&c->P);
        D.push_back(&c->d);
        min_p = std::min(min_p, d.p);
        round_robin |= (int)mfma_folds(d, b->cfg);
        sel_threads = std::max(sel_threads, select_threads(d.m));
        lds_recheck = std::max(lds_recheck, recheck_lds(d.n, d.p));
        lds_recheck_wide = std::max(lds_recheck_wide, recheck_wide_lds(d.n, d.p));
        TickJob &J = tj[j];
        memset(&J, 0, sizeof(J));
        J.P = c->P;
        J.d = d;
        J.n_mt = mfma_partial_tiles(d, b->cfg);
        J.blocks[kTickOps] = ga_ops_blocks(d);
        J.blocks[kTickAlloc] = alloc_blocks(d.S);   // a multiple of 8: every context starts on XCD 0
        J.blocks[kTickFinal] = finalize_blocks(d.S);
        J.blocks[kTickSel1] = d.R;   // the re-evaluation draws from one pool of all contexts' items
        for (int q = 0; q < kTickPhases; ++q) {
            J.start[q] = blocks[q];
            blocks[q] += J.blocks[q];
        }
    }
    if (njobs && std::max(lds_recheck, lds_recheck_wide) > recheck_group_lds_cap())
        return fail(nullptr, GA_ERR_INVALID, "batch: re-evaluation LDS exceeds the device limit");
    // tables (header, matrix-core jobs, TickJobs), copied in stream order
    // after earlier generations, into the fixed layout
    const size_t tick_off = batch_tick_offset();
    if (njobs) {
        const int k = b->stage;
        b->stage = (k + 1) % ga_batch::kStageRing;
        if ((e = hipEventSynchronize(b->tab_copied[k])) != hipSuccess)   // this staging buffer's last copy
            return fail(nullptr, GA_ERR_DEVICE, hipGetErrorString(e));
        b->total_tiles = mfma_fill_jobs(P.data(), D.data(), njobs, b->cfg, (char *)b->h_tab[k] + ga_batch::kHdrBytes);
        memcpy((char *)b->h_tab[k] + tick_off, tj.data(), sizeof(TickJob) * njobs);
        GroupHdr hdr{};
        hdr.njobs = njobs;
        hdr.total_tiles = b->total_tiles;
        hdr.round_robin = round_robin;
        memcpy(hdr.blocks, blocks, sizeof(blocks));
        memcpy(b->h_tab[k], &hdr, sizeof(hdr));
        const size_t head = ga_batch::kHdrBytes + mfma_job_bytes() * njobs;
        if ((e = hipMemcpyAsync(b->d_tab, b->h_tab[k], head, hipMemcpyHostToDevice, b->st)) != hipSuccess ||
            (e = hipMemcpyAsync((char *)b->d_tab + tick_off, (char *)b->h_tab[k] + tick_off,
                                sizeof(TickJob) * njobs, hipMemcpyHostToDevice, b->st)) != hipSuccess)
            return fail(nullptr, GA_ERR_DEVICE, hipGetErrorString(e));
        if ((e = hipEventRecord(b->tab_copied[k], b->st)) != hipSuccess)
            return fail(nullptr, GA_ERR_DEVICE, hipGetErrorString(e));
    } else {
        b->total_tiles = 0;
    }
    b->tick_off = tick_off;
    b->njobs = njobs;
    b->min_p = min_p;
    b->round_robin = round_robin;
    b->sel_threads = sel_threads;
    b->lds_recheck = lds_recheck;
    b->lds_recheck_wide = lds_recheck_wide;
    memcpy(b->blocks, blocks, sizeof(blocks));
    // side streams (default priority) for the contexts stepped alone
    const int nside = std::min((int)solo.size(), 16);
    while ((int)b->side.size() < nside) {
        hipStream_t s2;
        if ((e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking)) != hipSuccess)
            return fail(nullptr, GA_ERR_DEVICE, hipGetErrorString(e));
        b->side.push_back(s2);
    }
    while ((int)b->ev.size() < 1 + 16) {
        hipEvent_t ev;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
            return fail(nullptr, GA_ERR_DEVICE, hipGetErrorString(e));
        b->ev.push_back(ev);
    }
    b->ctxs.assign(ctxs, ctxs + count);
    b->grouped = grouped;
    b->solo = solo;
    return GA_OK;
}

ga_status ga_batch_step(ga_batch *b, int32_t generations)
{
    if (!b || generations < 0) return GA_ERR_INVALID;
    if (b->ctxs.empty() || generations == 0) return GA_OK;
    const int nsolo = (int)b->solo.size();
    const int nside = std::min(nsolo, (int)b->side.size());
    auto dev_fail = [&](hipError_t e, const char *what) {
        for (auto *c : b->ctxs) c->poisoned = true;
        return fail(nullptr, GA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    const int nj = b->njobs;
    hipError_t e;
    // a member evaluated on its own since (another tile configuration) gets
    // the batch's layout of the W split back first
    for (ga_ctx *c : b->grouped)
        if (ensure_w_layout(c, b->cfg) != GA_OK) return dev_fail(hipErrorUnknown, "split of W");
    for (ga_ctx *c : b->solo)
        if (ensure_w_layout(c, c->d.mfma_cfg) != GA_OK) return dev_fail(hipErrorUnknown, "split of W");
    if (nj) capture_batch_generation(b);   // a no-op while the composition fits the captured graph
    for (int g = 0; g < generations; ++g) {
        if (nsolo) {   // fork: every alone-stepped context starts after the previous generation
            if ((e = hipEventRecord(b->ev[0], b->st)) != hipSuccess) return dev_fail(e, "fork");
            for (int k = 0; k < nside; ++k)
                if ((e = hipStreamWaitEvent(b->side[k], b->ev[0], 0)) != hipSuccess) return dev_fail(e, "fork wait");
            for (int i = 0; i < nsolo; ++i) {
                ga_ctx *c = b->solo[i];
                hipStream_t s2 = b->side[i % nside];
                if (c->gexec) {
                    if ((e = hipGraphLaunch(c->gexec, s2)) != hipSuccess) return dev_fail(e, "generation graph");
                } else if (run_generation(c, s2) != GA_OK) {
                    return dev_fail(hipErrorUnknown, "generation");
                }
            }
        }
        if (nj) {
            if (b->gexec)
                e = hipGraphLaunch(b->gexec, b->st);
            else
                e = launch_grouped(b, b->blocks, ((b->total_tiles + 7) / 8) * 8,
                                   mfma_group_kins(b->cfg, b->min_p), b->sel_threads, b->lds_recheck,
                                   b->lds_recheck_wide);
            if (e != hipSuccess) return dev_fail(e, "grouped generation");
        }
        if (nsolo)   // join
            for (int k = 0; k < nside; ++k) {
                if ((e = hipEventRecord(b->ev[1 + k], b->side[k])) != hipSuccess) return dev_fail(e, "join");
                if ((e = hipStreamWaitEvent(b->st, b->ev[1 + k], 0)) != hipSuccess) return dev_fail(e, "join wait");
            }
    }
    return GA_OK;
}

void ga_batch_free(ga_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->st);
    for (auto s2 : b->side) (void)hipStreamSynchronize(s2);
    for (auto s2 : b->side) (void)hipStreamDestroy(s2);
    for (auto ev : b->ev) (void)hipEventDestroy(ev);
    for (auto ev : b->tab_copied)
        if (ev) (void)hipEventDestroy(ev);
    drop_batch_graph(b);
    if (b->d_tab) (void)hipFree(b->d_tab);
    for (auto h : b->h_tab)
        if (h) (void)hipHostFree(h);
    delete b;
}

const char *ga_status_str(ga_status s)
{
    switch (s) {
    case GA_OK: return "GA_OK";
    case GA_ERR_INVALID: return "GA_ERR_INVALID";
    case GA_ERR_OOM: return "GA_ERR_OOM";
    case GA_ERR_DEVICE: return "GA_ERR_DEVICE";
    case GA_ERR_STATE: return "GA_ERR_STATE";
    }
    return "GA_UNKNOWN";
}

const char *ga_last_error(const ga_ctx *ctx) { return ctx ? ctx->err.c_str() : g_init_error.c_str(); }

void ga_free(ga_ctx *ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->st);
    drop_graph(ctx);
    for (auto &e : ctx->ev) (void)hipEventDestroy(e);
    release_ctx(ctx, true);
}

}  // extern "C"
