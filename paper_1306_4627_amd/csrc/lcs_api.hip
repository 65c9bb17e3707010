// lcs_api.hip -- C ABI of the LCS library (see include/lcs.h): contexts,
// validation, symbol remap tables, device memory, launch sequences, HIP
// graphs and result copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <utility>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "api_internal.hpp"
#include "kernels.hpp"
#include "lcs.h"
#include "plan.hpp"

using namespace lcs;

#define LCS_VERSION_STRING "lcs-mi355x 0.1 (gfx950)"

// Shape of a batch as the autotuner's cache sees it: flags, alphabet size,
// and base-2 logarithms of the pair count, the longest X and Y, and (in
// quarters) the total cell count.
struct TuneKey {
    uint32_t flags, sigma, lcount, lm, ln, lcells4;
    bool operator<(const TuneKey &o) const {
        return std::tie(flags, sigma, lcount, lm, ln, lcells4) <
               std::tie(o.flags, o.sigma, o.lcount, o.lm, o.ln, o.lcells4);
    }
};

struct lcs_ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    size_t budget = 0;
    size_t in_use = 0;
    int num_cus = 0;
    int clock_khz = 0;      // peak shader clock the device reports
    std::string arch;
    std::map<TuneKey, std::pair<lcs_tuning, float>> tune_cache;   // autotuner results
    std::map<std::tuple<const void *, int, size_t>, int> occupancy;   // kernel, block, LDS -> groups per CU
    std::mutex mu;   // guards in_use, tune_cache and occupancy (a request server uses them from its thread)
};

namespace {

struct ClassDev {
    int wpl = 1;
    uint32_t nitems = 0, ntb = 0;
    uint32_t *it_T = nullptr;
    int32_t *it_prev = nullptr;
    uint8_t *it_feeds = nullptr;
    uint32_t *it_depth = nullptr;
    uint64_t *it_ck = nullptr, *it_cb = nullptr, *it_xf = nullptr;
    int32_t *ln_pair = nullptr;
    uint32_t *ln_word0 = nullptr, *ln_skew = nullptr;
    uint64_t *ln_ys = nullptr;
    uint32_t *tb_pair = nullptr, *tb_item = nullptr, *tb_lane0 = nullptr;
    uint32_t *tb_band0 = nullptr, *tb_strip0 = nullptr;
    uint32_t *sp_t = nullptr, *sp_s = nullptr, *fx_t = nullptr, *fx_s = nullptr, *sl_t = nullptr;
    uint32_t nsp = 0, nfx = 0, nsl = 0, strip_bands = 1;
    uint32_t *cross = nullptr, *strip_res = nullptr;
    uint64_t *ckpt = nullptr;
    uint32_t *cbits = nullptr;
    uint64_t *xfer = nullptr;
    uint64_t *xsum = nullptr;          // threshold pass: running sums handed up chains
    uint64_t *trace = nullptr;         // schedule records of the fill items (LCS_FILL_TRACE)
    uint32_t *plain_ctr = nullptr;     // plain mode: kQueues queue counters per pair
    uint32_t *q_fill = nullptr, *q_spec = nullptr, *q_fix = nullptr, *q_seal = nullptr;
    // the pass's fill launch: per-SIMD rank counters and band counters of
    // its first-item bands (zeroed with the queue counters), band size and
    // count (0 = no bands)
    uint32_t *simd_rank = nullptr, *band_next = nullptr;
    uint32_t fill_band_size = 0, fill_nbands = 0;
    uint32_t fill_grid = 1, sp_grid = 1, fx_grid = 1, sl_grid = 1;
    int fill_waves = 4;                // waves per fill work-group
    int nb = 1;                        // traceback tiles per band recomputed together
    int nbands = 1;                    // traceback bands recomputed together
    int seal_nb = 1, seal_nbands = 1;  // the same for the seal pass (one-wave groups)
    int tb_waves = 4;                  // waves per work-group of the speculative and fix-up passes
    uint32_t prio_half = 1;            // half the longest fill item's steps (wave priorities)
    // plain mode: one launch per pair and pass
    std::vector<uint32_t> pl_pair;     // pair of each launch
    std::vector<uint32_t> pl_begin, pl_end, pl_tb;  // item range, index in tb list
    std::vector<uint32_t> pl_sp, pl_nsp, pl_fx, pl_nfx, pl_sl;  // ticket ranges (pl_sl: -1 = none)
    // traceback rounds: per item the history offsets in the round buffer,
    // per round its items and tickets (device), the ranges (host), four
    // queue counters per round (refill, speculative, fix-up, seal) and grids
    uint32_t n_rounds = 0;
    uint64_t *it_rb = nullptr, *it_rcb = nullptr;
    uint32_t *rd_items = nullptr;
    uint32_t *rd_sp_t = nullptr, *rd_sp_s = nullptr, *rd_fx_t = nullptr, *rd_fx_s = nullptr;
    uint32_t *rd_sl_t = nullptr, *rd_sl_top = nullptr, *rd_sl_lo = nullptr;
    uint32_t *q_round = nullptr;
    std::vector<uint32_t> rd_item_off, rd_sp_off, rd_fx_off, rd_sl_off;
    std::vector<uint32_t> rd_fill_grid, rd_sp_grid, rd_fx_grid, rd_sl_grid;
};

// queue counters per class (and per pair in plain mode): fill, speculative,
// fix-up and seal passes
constexpr int kQueues = 4;

// Automatic middle-column split: pairs of at least this many symbols on
// both sides.
constexpr uint64_t kSplitMinSide = 4096;

// Bump allocator over one device allocation.
struct Carver {
    char *base = nullptr;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
};

}  // namespace

struct lcs_batch {
    lcs_ctx *ctx = nullptr;
    lcs::BatchHooks hooks;         // stream and memory of server-owned batches
    bool ext_mem = false;          // device memory came from hooks.alloc
    uint32_t flags = 0;
    int sigma = 0;
    int ckpt = 0;
    bool plain = false;
    uint32_t spin_limit = 1u << 26;
    Plan plan;
    uint64_t npairs = 0;
    std::vector<uint64_t> m, n;
    std::vector<uint64_t> out_off_host;   // worst-case slot of each pair
    uint64_t out_bytes = 0;
    void *dev = nullptr;
    size_t dev_bytes = 0;
    size_t upload_bytes = 0;       // host-written prefix of the allocation
    size_t readback_bytes = 0;     // lengths, error word and strings, from out_len
    uint8_t *lut = nullptr, *xbytes = nullptr, *xcodes = nullptr, *ybytes = nullptr;
    uint64_t xarena = 0, yarena = 0;
    uint64_t *pair_xoff = nullptr, *pair_yoff = nullptr, *pair_out = nullptr, *out_len = nullptr;
    uint64_t *pair_diag = nullptr, *diag = nullptr;   // diag lives in zero64
    uint64_t diag_words = 0;
    // emit items: (pair, first bitmap word) per 64 bitmap words, pair order
    std::vector<uint32_t> em_pair_host, em_w0_host, em_first_host;
    uint32_t *em_pair = nullptr, *em_w0 = nullptr;
    std::vector<uint64_t> diag_off_host;
    uint32_t *pair_m = nullptr, *pair_n = nullptr;
    SegInfo *seg = nullptr;        // Y-stream regions
    uint32_t *blk_seg = nullptr;   // region of each 64-element block of the Y stream
    uint16_t *ystream = nullptr;
    uint8_t *out = nullptr;
    uint32_t *zero = nullptr;
    uint64_t nzero = 0;
    uint64_t *zero64 = nullptr;
    uint64_t nzero64 = 0;
    uint32_t *error = nullptr;
    uint64_t *clk = nullptr;       // clock counters of the last fill launch
    uint64_t *junk = nullptr;      // fill: target of reads and stores a chunk does not need
    // pairs split at the middle column (lengths only): the plan holds two
    // halves per split pair, pairs npairs.. of the device pair tables; the
    // reversed X codes of the second halves follow the X-code arena, 64
    // bytes past its end; each half's last column goes to vcols
    uint64_t nvirt = 0;
    uint64_t xrev = 0;
    std::vector<HalfInfo> halves_host;
    HalfInfo *halves = nullptr;
    uint64_t *pair_vbase = nullptr;
    uint64_t *vcols = nullptr;
    uint64_t vwords = 0;
    uint32_t v_pair0 = 0;
    std::vector<uint64_t> vbase_host;
    // threshold pass: per-pair target length (host copy and device) and
    // answer word (0 open, 1 reaches the target, 2 cannot; read back with the
    // lengths)
    uint32_t *thr_t = nullptr, *thr_dec = nullptr;
    std::vector<uint32_t> thr_host;
    bool thr_set = false;
    std::vector<ClassDev> cls;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool ran = false;
    bool timed_fill = false;     // the last pass recorded the fill events
    bool no_events = false;      // created without HIP events (allocation-free entry point)
    bool rounds = false;         // traceback in rounds (history of a set of items at a time)
    uint64_t *round_buf = nullptr;
    uint64_t history_bytes = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------

static thread_local char g_last_error[256] = "";

static void note_error(const char *what, hipError_t e) {
    std::snprintf(g_last_error, sizeof g_last_error, "%s: %s (%d)", what, hipGetErrorString(e),
                  (int)e);
}

static int fill_mode(uint32_t flags) {
    return (flags & LCS_WANT_TRACEBACK) ? kFillTraceback
                                        : (flags & LCS_THRESHOLD) ? kFillThreshold : kFillLength;
}

static lcs_status dev_err(hipError_t e) {
    return e == hipSuccess ? LCS_OK : (e == hipErrorOutOfMemory ? LCS_ERR_NOMEM : LCS_ERR_DEVICE);
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) {                        \
            note_error(#expr, e_);                     \
            return dev_err(e_);                        \
        }                                              \
    } while (0)

// --------------------------------------------------------------------------
// fixed device scratch of the allocation-free entry point
// --------------------------------------------------------------------------

// Every device this library runs on holds one copy of this array from the
// moment the library's code object is loaded until the process ends.  In
// host code its name only stands in for the symbol: the device address of a
// device's copy comes from hipGetSymbolAddress with that device current
// (lcs_create does this once per device) and is the only handle host code
// passes on.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
struct ScratchSlot {
    std::mutex use;            // held for the whole of one call on the device
    bool resolved = false;
    void *ptr = nullptr;       // this device's copy of `scratch`
    hipError_t err = hipSuccess;
};
static ScratchSlot g_scratch[kMaxDevices];
static std::mutex g_scratch_init;

// Resolve the device address of `scratch` on `device` (which must be
// current), once per device.
static void resolve_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_init);
    ScratchSlot &sl = g_scratch[device];
    if (sl.resolved) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    sl.err = e;
    sl.ptr = e == hipSuccess ? ptr : nullptr;
    sl.resolved = true;
}

// Build the byte -> code table: codes 0..size-1 in the order the alphabet
// lists its symbols; valid[b] says whether byte b belongs to the alphabet.
static lcs_status make_lut(const lcs_alphabet *a, uint8_t lut[256], bool valid[256], int *sigma) {
    if (!a || a->size < 1 || a->size > 256) return LCS_ERR_ARG;
    std::memset(lut, 0, 256);
    for (int k = 0; k < 256; ++k) valid[k] = false;
    if (!a->symbols) {
        if (a->size != 256) return LCS_ERR_ARG;
        for (int k = 0; k < 256; ++k) { lut[k] = (uint8_t)k; valid[k] = true; }
    } else {
        for (int k = 0; k < a->size; ++k) {
            uint8_t s = a->symbols[k];
            if (valid[s]) return LCS_ERR_ARG;   // repeated symbol
            valid[s] = true;
            lut[s] = (uint8_t)k;
        }
    }
    *sigma = a->size;
    return LCS_OK;
}

static bool all_in(const uint8_t *s, uint64_t len, const bool valid[256]) {
    // branch-free over blocks of 4 KiB, one test per block
    for (uint64_t k = 0; k < len;) {
        const uint64_t e = std::min<uint64_t>(len, k + 4096);
        unsigned ok = 1;
        for (; k < e; ++k) ok &= (unsigned)valid[s[k]];
        if (!ok) return false;
    }
    return true;
}

// Host threads for work over `bytes` of input: one per 4 MiB, at most 16.
static int host_threads(uint64_t bytes) {
    const uint64_t hc = std::max(1u, std::thread::hardware_concurrency());
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(std::min<uint64_t>(bytes >> 22, hc), 16));
}

// fn(t) for t in [0, T): the calling thread takes t = 0, T - 1 more threads
// the rest (the calling thread runs the tasks of any thread that cannot be
// started).
template <class F>
static void run_threads(int T, F fn) {
    std::vector<std::thread> th;
    int t = 1;
    try {
        for (; t < T; ++t) th.emplace_back(fn, t);
    } catch (...) {
        for (; t < T; ++t) fn(t);
    }
    fn(0);
    for (std::thread &x : th) x.join();
}

// Pair ranges of T tasks with about the same bytes of X and Y each.
static std::vector<uint64_t> pair_ranges(const lcs_pair *pairs, uint64_t count, int T) {
    uint64_t total = 0;
    for (uint64_t k = 0; k < count; ++k) total += pairs[k].m + pairs[k].n;
    std::vector<uint64_t> lo((size_t)T + 1, count);
    lo[0] = 0;
    uint64_t acc = 0;
    int t = 1;
    for (uint64_t k = 0; k < count && t < T; ++k) {
        acc += pairs[k].m + pairs[k].n;
        while (t < T && acc * (uint64_t)T >= total * (uint64_t)t) lo[(size_t)t++] = k + 1;
    }
    return lo;
}

static lcs_status check_pairs(const lcs_pair *pairs, uint64_t count) {
    if (count && !pairs) return LCS_ERR_ARG;
    for (uint64_t k = 0; k < count; ++k) {
        const lcs_pair &p = pairs[k];
        if ((p.m && !p.x) || (p.n && !p.y)) return LCS_ERR_ARG;
        if (p.m > LCS_MAX_LEN || p.n > LCS_MAX_LEN) return LCS_ERR_TOO_LONG;
    }
    return LCS_OK;
}

static lcs_status check_tuning(const lcs_tuning *t) {
    if (!t) return LCS_OK;
    if (t->words_per_lane != 0 && t->words_per_lane != 1 && t->words_per_lane != 2 &&
        t->words_per_lane != 4 && t->words_per_lane != 8)
        return LCS_ERR_ARG;
    if (t->ckpt_interval != 0 && t->ckpt_interval != 64 && t->ckpt_interval != 128 &&
        t->ckpt_interval != 256)
        return LCS_ERR_ARG;
    if (t->persistent_waves < 0 || t->plain < 0 || t->plain > 1) return LCS_ERR_ARG;
    if (t->link_items < 0 || t->tb_round_kib < 0) return LCS_ERR_ARG;
    if (t->halves < 0 || t->halves > 2) return LCS_ERR_ARG;
    if (t->strip_rows < 0 || t->tb_tiles < 0 || t->tb_tiles > 8 || t->tb_bands < 0 ||
        t->tb_bands > 16 || t->tb_tiles * t->tb_bands > 64)
        return LCS_ERR_ARG;
    return LCS_OK;
}

static void fill_plan_config(PlanConfig &cfg, int sigma, uint32_t flags, const lcs_tuning *t) {
    cfg.wpl = t ? t->words_per_lane : 0;
    cfg.traceback = (flags & LCS_WANT_TRACEBACK) != 0;
    cfg.ckpt = (t && t->ckpt_interval) ? t->ckpt_interval : 64;
    cfg.sigma = sigma;
    cfg.plain = t && t->plain;
    cfg.strip_rows = (t && t->strip_rows) ? t->strip_rows : 4096;
    cfg.round_bytes = (cfg.traceback && t && t->tb_round_kib > 0) ? (uint64_t)t->tb_round_kib * 1024 : 0;
    // Linked runs of chains: by default up to 64 items for the traceback
    // fill, whose longer steps the 6-8% fewer lane-steps pay for (4096-pair
    // related batch: fill 5.96 -> 5.39 ms), and none for the lengths-only and
    // threshold fills, where the longer waits inside a run cancel the gain or
    // more (threshold at 90%: 5.25 -> 5.51 ms); traceback rounds refill whole
    // items and need unlinked chains.
    cfg.link_items = (t && t->link_items) ? t->link_items
                                          : (cfg.traceback && !cfg.plain && !cfg.round_bytes) ? 64 : 1;
}

static void stats_from_plan(const Plan &p, uint64_t npairs, lcs_batch_stats *out) {
    std::memset(out, 0, sizeof *out);
    out->pairs = npairs;
    out->cells = p.cells;
    out->groups = p.items;
    out->lanes = p.lanes;
    out->lane_steps = p.lane_steps;
    int w = 0;
    for (const ClassPlan &c : p.classes) w = std::max(w, c.wpl);
    out->words_per_lane = w;
    out->ckpt_interval = p.cfg.traceback ? p.cfg.ckpt : 0;
    out->classes = (int32_t)p.classes.size();
    out->flags = p.cfg.traceback ? (int32_t)LCS_WANT_TRACEBACK : 0;
    uint64_t rw = 0, full = 0;
    for (const ClassPlan &c : p.classes) {
        out->tb_rounds = std::max<int32_t>(out->tb_rounds, (int32_t)c.n_rounds);
        rw = std::max(rw, c.round_words);
        full += (c.ck_words + 1) * 8 + (c.cb_words + 1) * 4;
    }
    if (p.cfg.traceback) out->history_bytes = p.cfg.round_bytes ? (rw + 1) * 8 : full;
}

// Planner messages to status codes.
static lcs_status plan_status(const std::string &why) {
    if (why.find("longer") != std::string::npos || why.find("too long") != std::string::npos ||
        why.find("too many") != std::string::npos)
        return LCS_ERR_TOO_LONG;
    if (why.find("round capacity") != std::string::npos) return LCS_ERR_NOMEM;
    return LCS_ERR_UNSUPPORTED;
}

// --------------------------------------------------------------------------
// status, version
// --------------------------------------------------------------------------

extern "C" const char *lcs_status_str(int s) {
    switch (s) {
        case LCS_PENDING: return "pending (queued or running)";
        case LCS_OK: return "ok";
        case LCS_ERR_ARG: return "invalid argument";
        case LCS_ERR_SYMBOL: return "symbol not in alphabet";
        case LCS_ERR_NOMEM: return "out of memory (device budget or host)";
        case LCS_ERR_DEVICE: return "device error (no gfx950 device or HIP failure)";
        case LCS_ERR_BUFFER: return "output buffer too small";
        case LCS_ERR_TOO_LONG: return "sequence too long";
        case LCS_ERR_UNSUPPORTED: return "unsupported tuning or alphabet";
        default: return "unknown status";
    }
}

extern "C" const char *lcs_version(void) { return LCS_VERSION_STRING; }

extern "C" const char *lcs_last_error(void) { return g_last_error; }

// --------------------------------------------------------------------------
// context
// --------------------------------------------------------------------------

extern "C" lcs_status lcs_create(lcs_ctx **out, int device, size_t mem_budget_bytes) {
    if (!out) return LCS_ERR_ARG;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) {
        note_error("hipGetDeviceCount", e);
        return LCS_ERR_DEVICE;
    }
    if (device < 0 || device >= count) {
        std::snprintf(g_last_error, sizeof g_last_error, "device %d out of range (%d visible)",
                      device, count);
        return LCS_ERR_DEVICE;
    }
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        std::snprintf(g_last_error, sizeof g_last_error, "device %d is %s, not gfx950", device,
                      prop.gcnArchName);
        return LCS_ERR_DEVICE;
    }
    HIP_TRY(hipSetDevice(device));
    resolve_scratch(device);
    std::unique_ptr<lcs_ctx> c(new (std::nothrow) lcs_ctx());
    if (!c) return LCS_ERR_NOMEM;
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->clock_khz = prop.clockRate;
    c->arch = prop.gcnArchName;
    HIP_TRY(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
    c->stream = c->own_stream;
    size_t fr = 0, tot = 0;
    e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) {
        note_error("hipMemGetInfo", e);
        (void)hipStreamDestroy(c->own_stream);
        return LCS_ERR_DEVICE;
    }
    c->budget = mem_budget_bytes ? mem_budget_bytes : (size_t)(fr * 0.9);
    *out = c.release();
    return LCS_OK;
}

extern "C" void lcs_destroy(lcs_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->own_stream) {
        (void)hipStreamSynchronize(ctx->own_stream);
        (void)hipStreamDestroy(ctx->own_stream);
    }
    delete ctx;
}

extern "C" lcs_status lcs_device_info(lcs_ctx *ctx, int32_t *compute_units, int32_t *peak_clock_khz) {
    if (!ctx) return LCS_ERR_ARG;
    if (compute_units) *compute_units = ctx->num_cus;
    if (peak_clock_khz) *peak_clock_khz = ctx->clock_khz;
    return LCS_OK;
}

extern "C" lcs_status lcs_set_stream(lcs_ctx *ctx, void *hip_stream) {
    if (!ctx) return LCS_ERR_ARG;
    ctx->stream = hip_stream ? (hipStream_t)hip_stream : ctx->own_stream;
    return LCS_OK;
}

extern "C" lcs_status lcs_synchronize(lcs_ctx *ctx) {
    if (!ctx) return LCS_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCS_ERR_DEVICE;
    return dev_err(hipStreamSynchronize(ctx->stream));
}

// --------------------------------------------------------------------------
// batches
// --------------------------------------------------------------------------

static void free_batch(lcs_batch *b) {
    if (!b) return;
    if (b->ctx) (void)hipSetDevice(b->ctx->device);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipEvent_t &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->dev) {
        if (b->ext_mem) {
            b->hooks.release(b->hooks.user, b->dev);
        } else {
            (void)hipFree(b->dev);
            if (b->ctx) {
                std::lock_guard<std::mutex> lk(b->ctx->mu);
                b->ctx->in_use -= b->dev_bytes;
            }
        }
    }
    delete b;
}

// Lay out (or, with base == nullptr, just size) the device memory of a batch.
static size_t carve(lcs_batch *b, char *base) {
    Carver cv;
    cv.base = base;
    const Plan &p = b->plan;
    const uint64_t np = b->npairs;
    // ---- written from the host (one upload of [0, upload_bytes)) ----
    b->lut = cv.take<uint8_t>(256);
    b->xbytes = cv.take<uint8_t>(b->xarena + 64);
    b->ybytes = cv.take<uint8_t>(b->yarena + 64);
    const uint64_t npp = np + b->nvirt;   // pairs of the plan: the halves of split pairs too
    b->pair_xoff = cv.take<uint64_t>(npp + 1);
    b->pair_yoff = cv.take<uint64_t>(npp + 1);
    b->pair_out = cv.take<uint64_t>(np + 1);
    b->pair_diag = cv.take<uint64_t>(np + 1);
    b->em_pair = cv.take<uint32_t>(b->em_pair_host.size() + 1);
    b->em_w0 = cv.take<uint32_t>(b->em_w0_host.size() + 1);
    b->pair_m = cv.take<uint32_t>(npp + 1);
    b->pair_n = cv.take<uint32_t>(npp + 1);
    b->halves = cv.take<HalfInfo>(b->halves_host.size() + 1);
    b->pair_vbase = cv.take<uint64_t>(b->nvirt + 1);
    const bool thr = (b->flags & LCS_THRESHOLD) != 0;
    b->thr_t = thr ? cv.take<uint32_t>(np + 1) : nullptr;
    const size_t ns = p.segs.size();
    b->seg = cv.take<SegInfo>(ns + 1);
    b->blk_seg = cv.take<uint32_t>(p.ys_elems / 64 + 1);
    b->cls.resize(p.classes.size());
    for (size_t ci = 0; ci < p.classes.size(); ++ci) {
        const ClassPlan &C = p.classes[ci];
        ClassDev &D = b->cls[ci];
        D.wpl = C.wpl;
        D.nitems = (uint32_t)C.it_T.size();
        D.ntb = (uint32_t)C.tb_pair.size();
        D.it_T = cv.take<uint32_t>(D.nitems);
        D.it_prev = cv.take<int32_t>(D.nitems);
        D.it_feeds = cv.take<uint8_t>(D.nitems);
        D.it_depth = cv.take<uint32_t>(D.nitems);
        D.it_ck = cv.take<uint64_t>(D.nitems);
        D.it_cb = cv.take<uint64_t>(D.nitems);
        D.it_xf = cv.take<uint64_t>(D.nitems);
        D.ln_pair = cv.take<int32_t>(C.ln_pair.size());
        D.ln_word0 = cv.take<uint32_t>(C.ln_pair.size());
        D.ln_skew = cv.take<uint32_t>(C.ln_pair.size());
        D.ln_ys = cv.take<uint64_t>(C.ln_pair.size());
        D.tb_pair = cv.take<uint32_t>(D.ntb + 1);
        D.tb_item = cv.take<uint32_t>(D.ntb + 1);
        D.tb_lane0 = cv.take<uint32_t>(D.ntb + 1);
        D.tb_band0 = cv.take<uint32_t>(C.tb_band0.size() + 1);
        D.tb_strip0 = cv.take<uint32_t>(C.tb_strip0.size() + 1);
        D.nsp = (uint32_t)C.sp_t.size();
        D.nfx = (uint32_t)C.fx_t.size();
        D.nsl = (uint32_t)C.sl_t.size();
        D.strip_bands = C.strip_bands;
        D.sp_t = cv.take<uint32_t>(D.nsp + 1);
        D.sp_s = cv.take<uint32_t>(D.nsp + 1);
        D.fx_t = cv.take<uint32_t>(D.nfx + 1);
        D.fx_s = cv.take<uint32_t>(D.nfx + 1);
        D.sl_t = cv.take<uint32_t>(D.nsl + 1);
        D.n_rounds = C.n_rounds;
        if (C.n_rounds) {
            D.it_rb = cv.take<uint64_t>(D.nitems);
            D.it_rcb = cv.take<uint64_t>(D.nitems);
            D.rd_items = cv.take<uint32_t>(C.rd_items.size() + 1);
            D.rd_sp_t = cv.take<uint32_t>(C.rd_sp_t.size() + 1);
            D.rd_sp_s = cv.take<uint32_t>(C.rd_sp_s.size() + 1);
            D.rd_fx_t = cv.take<uint32_t>(C.rd_fx_t.size() + 1);
            D.rd_fx_s = cv.take<uint32_t>(C.rd_fx_s.size() + 1);
            D.rd_sl_t = cv.take<uint32_t>(C.rd_sl_t.size() + 1);
            D.rd_sl_top = cv.take<uint32_t>(C.rd_sl_top.size() + 1);
            D.rd_sl_lo = cv.take<uint32_t>(C.rd_sl_lo.size() + 1);
        }
    }
    cv.off = (cv.off + 255) & ~(size_t)255;
    b->upload_bytes = cv.off;
    // ---- read back after a pass (one copy of [out_len, end of out)) ----
    b->out_len = cv.take<uint64_t>(np + 1);
    b->thr_dec = thr ? cv.take<uint32_t>(np + 1) : nullptr;
    // zeroed before every pass, 32-bit: error word, then per class the fill
    // and traceback queue counters and (plain mode) kQueues counters per pair
    uint64_t nz = 1;
    for (size_t ci = 0; ci < p.classes.size(); ++ci) {
        const ClassPlan &C = p.classes[ci];
        nz += kQueues;
        if (b->plain) nz += kQueues * C.tb_pair.size();
        else nz += kSimdKeys + kMaxBands;
        nz += kQueues * C.n_rounds;
    }
    b->zero = cv.take<uint32_t>(nz);
    b->nzero = nz;
    b->error = b->zero;
    b->out = cv.take<uint8_t>(b->out_bytes + 64);
    b->readback_bytes = (size_t)((char *)(b->out + b->out_bytes) - (char *)b->out_len);
    // ---- device only ----
    b->clk = cv.take<uint64_t>(4);
    b->junk = cv.take<uint64_t>(kJunkWords);
    b->xcodes = cv.take<uint8_t>(b->xarena + 64 + b->xrev + 64);
    b->ystream = cv.take<uint16_t>(p.ys_elems + 64);
    b->vcols = cv.take<uint64_t>(b->vwords + 1);
    // zeroed before every pass, 64-bit: traceback bitmaps, then the carry
    // hand-over words of every class
    uint64_t nz64 = (b->flags & LCS_WANT_TRACEBACK) ? b->diag_words : 0;
    const bool traced = (b->flags & LCS_FILL_TRACE) != 0;
    for (const ClassPlan &C : p.classes)
        nz64 += C.xf_words + (thr ? C.xf_words / 2 : 0) + (traced ? C.it_T.size() * kTraceWords : 0);
    b->zero64 = cv.take<uint64_t>(nz64 + 1);
    b->nzero64 = nz64;
    b->diag = b->zero64;
    uint64_t z64 = (b->flags & LCS_WANT_TRACEBACK) ? b->diag_words : 0;
    uint64_t zc = 1;
    // traceback history: every item's at once, or one round buffer shared by
    // the rounds of every class (they run one after another)
    b->history_bytes = 0;
    b->round_buf = nullptr;
    if (b->rounds) {
        uint64_t rw = 0;
        for (const ClassPlan &C : p.classes) rw = std::max(rw, C.round_words);
        b->round_buf = cv.take<uint64_t>(rw + 1);
        b->history_bytes = (rw + 1) * 8;
    }
    for (size_t ci = 0; ci < p.classes.size(); ++ci) {
        const ClassPlan &C = p.classes[ci];
        ClassDev &D = b->cls[ci];
        D.cross = cv.take<uint32_t>(C.n_bands + 1);
        D.strip_res = cv.take<uint32_t>(2 * C.n_strips + 2);
        if (b->rounds) {
            D.ckpt = b->round_buf;
            D.cbits = (uint32_t *)b->round_buf;
        } else {
            D.ckpt = cv.take<uint64_t>(C.ck_words + 1);
            D.cbits = cv.take<uint32_t>(C.cb_words + 1);
            if (b->flags & LCS_WANT_TRACEBACK) b->history_bytes += (C.ck_words + 1) * 8 + (C.cb_words + 1) * 4;
        }
        D.xfer = b->zero64 ? b->zero64 + z64 : nullptr;
        z64 += C.xf_words;
        if (thr) {
            D.xsum = b->zero64 ? b->zero64 + z64 : nullptr;
            z64 += C.xf_words / 2;
        }
        if (traced) {
            D.trace = b->zero64 ? b->zero64 + z64 : nullptr;
            z64 += C.it_T.size() * kTraceWords;
        }
        D.q_fill = b->zero ? b->zero + zc : nullptr;
        D.q_spec = b->zero ? b->zero + zc + 1 : nullptr;
        D.q_fix = b->zero ? b->zero + zc + 2 : nullptr;
        D.q_seal = b->zero ? b->zero + zc + 3 : nullptr;
        zc += kQueues;
        D.plain_ctr = b->zero ? b->zero + zc : nullptr;
        if (b->plain) {
            zc += kQueues * D.ntb;
        } else {
            D.simd_rank = b->zero ? b->zero + zc : nullptr;
            D.band_next = b->zero ? b->zero + zc + kSimdKeys : nullptr;
            zc += kSimdKeys + kMaxBands;
        }
        D.q_round = b->zero ? b->zero + zc : nullptr;
        zc += kQueues * C.n_rounds;
    }
    return cv.off + 256;
}

// Persistent grid: as many work-groups as can be resident, capped by work.
static uint32_t resident_grid(lcs_ctx *ctx, const void *fn, size_t lds, uint64_t work_groups,
                              int cap, int block = kFillBlock) {
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->occupancy.find(std::make_tuple(fn, block, lds));
        if (it != ctx->occupancy.end()) per_cu = it->second;
    }
    if (per_cu == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->occupancy[std::make_tuple(fn, block, lds)] = per_cu;
    }
    uint64_t g = (uint64_t)per_cu * (uint64_t)ctx->num_cus;
    if (cap > 0) g = std::min<uint64_t>(g, (uint64_t)cap);
    g = std::min<uint64_t>(g, std::max<uint64_t>(work_groups, 1));
    return (uint32_t)std::max<uint64_t>(g, 1);
}

static lcs_status build_batch(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                              const lcs_alphabet *alphabet, uint32_t flags,
                              const lcs_tuning *tuning, lcs_batch **out,
                              const BatchHooks *hooks = nullptr, bool no_events = false) {
    if (!ctx || !out) return LCS_ERR_ARG;
    if (flags & ~(uint32_t)(LCS_WANT_TRACEBACK | LCS_USE_GRAPH | LCS_THRESHOLD | LCS_FILL_TRACE))
        return LCS_ERR_ARG;
    if ((flags & LCS_THRESHOLD) && (flags & LCS_WANT_TRACEBACK)) return LCS_ERR_ARG;
    lcs_status st = check_pairs(pairs, count);
    if (st) return st;
    st = check_tuning(tuning);
    if (st) return st;
    uint8_t lut[256];
    bool valid[256];
    int sigma = 0;
    st = make_lut(alphabet, lut, valid, &sigma);
    if (st) return st;
    {
        // every byte against the alphabet, before anything is allocated
        uint64_t in_bytes = 0;
        for (uint64_t k = 0; k < count; ++k) in_bytes += pairs[k].m + pairs[k].n;
        const int T = host_threads(in_bytes);
        const std::vector<uint64_t> rg = pair_ranges(pairs, count, T);
        std::vector<uint8_t> bad((size_t)T, 0);
        run_threads(T, [&](int t) {
            for (uint64_t k = rg[(size_t)t]; k < rg[(size_t)t + 1]; ++k)
                if (!all_in(pairs[k].x, pairs[k].m, valid) || !all_in(pairs[k].y, pairs[k].n, valid)) {
                    bad[(size_t)t] = 1;
                    return;
                }
        });
        for (uint8_t v : bad)
            if (v) return LCS_ERR_SYMBOL;
    }
    std::unique_ptr<lcs_batch> b(new (std::nothrow) lcs_batch());
    if (!b) return LCS_ERR_NOMEM;
    b->ctx = ctx;
    b->flags = flags;
    b->sigma = sigma;
    b->plain = tuning && tuning->plain;
    b->npairs = count;
    std::vector<PairShape> shapes(count);
    b->m.resize(count);
    b->n.resize(count);
    b->out_off_host.resize(count + 1);
    uint64_t xa = 0, ya = 0, oo = 0;
    std::vector<uint64_t> xoff(count + 1), yoff(count + 1);
    for (uint64_t k = 0; k < count; ++k) {
        shapes[k].m = b->m[k] = pairs[k].m;
        shapes[k].n = b->n[k] = pairs[k].n;
        xoff[k] = xa;
        yoff[k] = ya;
        xa += (pairs[k].m + 63) / 64 * 64;   // padded: the fill reads whole dwords
        ya += pairs[k].n;
        b->out_off_host[k] = oo;
        oo += std::min(pairs[k].m, pairs[k].n);
    }
    b->out_off_host[count] = oo;
    b->diag_off_host.assign(count + 1, 0);
    if (flags & LCS_WANT_TRACEBACK) {
        uint64_t dw = 0;
        for (uint64_t k = 0; k < count; ++k) {
            b->diag_off_host[k] = dw;
            dw += (pairs[k].m + 63) / 64;
        }
        b->diag_words = dw;
        b->em_first_host.assign(count + 1, 0);
        for (uint64_t k = 0; k < count; ++k) {
            b->em_first_host[k] = (uint32_t)b->em_pair_host.size();
            const uint64_t W = (pairs[k].m + 63) / 64;
            for (uint64_t w0 = 0; w0 < W; w0 += 64) {
                b->em_pair_host.push_back((uint32_t)k);
                b->em_w0_host.push_back((uint32_t)w0);
            }
        }
        b->em_first_host[count] = (uint32_t)b->em_pair_host.size();
    }
    b->xarena = xa;
    b->yarena = ya;
    b->out_bytes = (flags & LCS_WANT_TRACEBACK) ? oo : 0;
    PlanConfig cfg;
    fill_plan_config(cfg, sigma, flags, tuning);
    cfg.cus = ctx->num_cus;
    if (max_wpl(sigma) == 0) return LCS_ERR_UNSUPPORTED;
    if (cfg.wpl && !wpl_fits(sigma, cfg.wpl)) return LCS_ERR_UNSUPPORTED;
    // Middle-column split (lengths only): pair k becomes two halves, pairs
    // count + 2s (X against Y[0, h)) and count + 2s + 1 (X reversed against
    // Y[h, n) reversed), h = n / 2; pair k itself is planned empty and its
    // length written by the combine.
    std::vector<uint32_t> hm(count + 1, 0), hn(count + 1, 0);
    for (uint64_t k = 0; k < count; ++k) {
        hm[k] = (uint32_t)pairs[k].m;
        hn[k] = (uint32_t)pairs[k].n;
    }
    {
        std::vector<uint64_t> split;
        const int hv = tuning ? tuning->halves : 0;
        if (!(flags & (LCS_WANT_TRACEBACK | LCS_THRESHOLD)) && !b->plain && hv != 1) {
            if (hv == 2) {
                for (uint64_t k = 0; k < count; ++k)
                    if (pairs[k].m >= 1 && pairs[k].n >= 2) split.push_back(k);
            } else {
                uint64_t lanes = 0;   // at one word per lane, split pairs counted twice
                for (uint64_t k = 0; k < count; ++k) {
                    const bool c = pairs[k].m >= kSplitMinSide && pairs[k].n >= kSplitMinSide;
                    lanes += (c ? 2 : 1) * ((pairs[k].m + 63) / 64);
                    if (c) split.push_back(k);
                }
                if (lanes * 4 > (uint64_t)ctx->num_cus * 16 * 64) split.clear();
            }
        }
        b->nvirt = 2 * split.size();
        xoff.resize(count + b->nvirt + 1, 0);
        yoff.resize(count + b->nvirt + 1, 0);
        hm.resize(count + b->nvirt + 1, 0);
        hn.resize(count + b->nvirt + 1, 0);
        uint64_t roff = xa + 64, vw = 0;
        std::vector<uint64_t> vbase;
        for (size_t si = 0; si < split.size(); ++si) {
            const uint64_t k = split[si], m = pairs[k].m, n = pairs[k].n, h = n / 2;
            const uint64_t f = count + 2 * si, r = f + 1, W = (m + 63) / 64;
            shapes[k].m = 0;
            shapes.push_back(PairShape{m, h});
            shapes.push_back(PairShape{m, n - h});
            xoff[f] = xoff[k];
            xoff[r] = roff;
            yoff[f] = yoff[k];
            yoff[r] = yoff[k] + h;
            hm[f] = hm[r] = (uint32_t)m;
            hn[f] = (uint32_t)h;
            hn[r] = (uint32_t)(n - h);
            HalfInfo hi{};
            hi.xsrc = xoff[k];
            hi.xdst = roff;
            hi.vf = vw;
            hi.vb = vw + W;
            hi.pair = (uint32_t)k;
            hi.m = (uint32_t)m;
            b->halves_host.push_back(hi);
            vbase.push_back(vw);
            vbase.push_back(vw + W);
            vw += 2 * W;
            roff += (m + 63) / 64 * 64;
        }
        b->xrev = roff - (xa + 64);
        b->vwords = vw;
        b->v_pair0 = (uint32_t)count;
        b->vbase_host = std::move(vbase);
    }
    std::string why = build_plan(shapes, cfg, b->plan);
    if (!why.empty()) return plan_status(why);
    b->ckpt = cfg.ckpt;
    b->rounds = cfg.round_bytes != 0;
    size_t need = carve(b.get(), nullptr);
    // A traceback whose full history does not fit the memory this batch may
    // take runs in rounds, the round buffer sized to what the other buffers
    // leave (shrunk until the whole batch fits, or NOMEM below).
    if ((flags & LCS_WANT_TRACEBACK) && !b->plain && !b->rounds) {
        size_t avail = 0;
        if (hooks && hooks->alloc) {
            avail = hooks->avail;
        } else {
            std::lock_guard<std::mutex> lk(ctx->mu);
            avail = ctx->budget > ctx->in_use ? ctx->budget - ctx->in_use : 0;
        }
        if (avail && need > avail && need - b->history_bytes < avail) {
            size_t rb = avail - (need - b->history_bytes);
            for (int tries = 0; tries < 6 && rb >= 4096; ++tries) {
                PlanConfig c2 = cfg;
                c2.round_bytes = rb & ~(size_t)4095;
                c2.link_items = 1;
                Plan p2;
                if (!build_plan(shapes, c2, p2).empty()) break;   // an item larger than the rounds
                b->plan = std::move(p2);
                b->rounds = true;
                cfg = c2;
                need = carve(b.get(), nullptr);
                if (need <= avail) break;
                rb -= std::min(rb, need - avail + 4096);
            }
        }
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return LCS_ERR_DEVICE;
    void *mem = nullptr;
    if (hooks && hooks->alloc) {
        b->hooks = *hooks;
        mem = hooks->alloc(hooks->user, need);
        if (!mem) return LCS_ERR_NOMEM;
        b->ext_mem = true;
    } else {
        if (hooks) b->hooks.stream = hooks->stream;
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->in_use + need > ctx->budget) return LCS_ERR_NOMEM;
        hipError_t e = hipMalloc(&mem, need);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? LCS_ERR_NOMEM : LCS_ERR_DEVICE;
        ctx->in_use += need;
    }
    b->dev = mem;
    b->dev_bytes = need;
    carve(b.get(), (char *)mem);
    lcs_batch *bp = b.release();

    // ---- host staging of everything the device needs ----
    auto fail = [&](lcs_status s) {
        free_batch(bp);
        return s;
    };
    // the host image of [0, upload_bytes): every host-written region at its
    // device offset, sent with one copy
    // (X and Y are copied by host threads; every other byte of the image is
    // zeroed once, and each pair's X padding with its copy)
    char *const dev0 = (char *)bp->dev;
    const size_t img_bytes = bp->upload_bytes;
    std::unique_ptr<uint8_t[]> image_buf(new (std::nothrow) uint8_t[img_bytes ? img_bytes : 1]);
    if (!image_buf) return fail(LCS_ERR_NOMEM);
    uint8_t *const img = image_buf.get();
    {
        const size_t xo = (size_t)((char *)bp->xbytes - dev0), yo = (size_t)((char *)bp->ybytes - dev0);
        if (!(xo + xa <= yo && yo + ya <= img_bytes)) return fail(LCS_ERR_DEVICE);
        std::memset(img, 0, xo);
        std::memset(img + xo + xa, 0, yo - (xo + xa));
        std::memset(img + yo + ya, 0, img_bytes - (yo + ya));
        const int T = host_threads(xa + ya);
        const std::vector<uint64_t> rg = pair_ranges(pairs, count, T);
        run_threads(T, [&](int t) {
            for (uint64_t k = rg[(size_t)t]; k < rg[(size_t)t + 1]; ++k) {
                const uint64_t m = pairs[k].m, pad = (m + 63) / 64 * 64;
                if (m) std::memcpy(img + xo + xoff[k], pairs[k].x, m);
                if (pad > m) std::memset(img + xo + xoff[k] + m, 0, pad - m);
                if (pairs[k].n) std::memcpy(img + yo + yoff[k], pairs[k].y, pairs[k].n);
            }
        });
    }
    const Plan &p = bp->plan;
    const size_t ns = p.segs.size();
    std::vector<SegInfo> seginfo(ns + 1);
    for (size_t s = 0; s < ns; ++s) {
        const Segment &sg = p.segs[s];
        if (sg.len > 0xffffffffull) return fail(LCS_ERR_TOO_LONG);
        SegInfo &si = seginfo[s];
        si.begin = sg.begin;
        si.len = (uint32_t)sg.len;
        si.pre = sg.pre;
        si.shift = sg.shift;
        si.n = 0;
        si.yoff = 0;
        if (sg.pair != kNoPair) {
            si.n = hn[sg.pair];
            si.yoff = yoff[sg.pair];
            if (sg.pair >= count && ((sg.pair - count) & 1)) si.shift |= kSegReversed;
        }
    }
    hipStream_t st0 = bp->hooks.stream ? bp->hooks.stream : ctx->own_stream;
    auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        const size_t off = (size_t)((char *)dst - dev0);
        if (off + bytes > img_bytes) return hipErrorInvalidValue;
        std::memcpy(img + off, src, bytes);
        return hipSuccess;
    };
#define UP(dst, src, bytes)                          \
    do {                                             \
        hipError_t e_ = up((dst), (src), (bytes));   \
        if (e_ != hipSuccess) return fail(dev_err(e_)); \
    } while (0)
    UP(bp->lut, lut, 256);
    UP(bp->pair_xoff, xoff.data(), (count + bp->nvirt) * 8);
    UP(bp->pair_yoff, yoff.data(), (count + bp->nvirt) * 8);
    UP(bp->pair_out, bp->out_off_host.data(), count * 8);
    UP(bp->pair_diag, bp->diag_off_host.data(), count * 8);
    UP(bp->em_pair, bp->em_pair_host.data(), bp->em_pair_host.size() * 4);
    UP(bp->em_w0, bp->em_w0_host.data(), bp->em_w0_host.size() * 4);
    UP(bp->pair_m, hm.data(), (count + bp->nvirt) * 4);
    UP(bp->pair_n, hn.data(), (count + bp->nvirt) * 4);
    UP(bp->halves, bp->halves_host.data(), bp->halves_host.size() * sizeof(HalfInfo));
    UP(bp->pair_vbase, bp->vbase_host.data(), bp->vbase_host.size() * 8);
    UP(bp->seg, seginfo.data(), ns * sizeof(SegInfo));
    {
        // regions are whole 64-element blocks, back to back
        std::vector<uint32_t> bs(p.ys_elems / 64, 0);
        for (size_t k = 0; k < ns; ++k) {
            const uint64_t b0 = p.segs[k].begin / 64, nb = (p.segs[k].len + 63) / 64;
            for (uint64_t q = b0; q < b0 + nb && q < bs.size(); ++q) bs[q] = (uint32_t)k;
        }
        UP(bp->blk_seg, bs.data(), bs.size() * 4);
    }
    for (size_t ci = 0; ci < p.classes.size(); ++ci) {
        const ClassPlan &C = p.classes[ci];
        ClassDev &D = bp->cls[ci];
        UP(D.it_T, C.it_T.data(), C.it_T.size() * 4);
        UP(D.it_prev, C.it_prev.data(), C.it_prev.size() * 4);
        UP(D.it_feeds, C.it_feeds.data(), C.it_feeds.size());
        UP(D.it_depth, C.it_depth.data(), C.it_depth.size() * 4);
        UP(D.it_ck, C.it_ck.data(), C.it_ck.size() * 8);
        UP(D.it_cb, C.it_cb.data(), C.it_cb.size() * 8);
        UP(D.it_xf, C.it_xf.data(), C.it_xf.size() * 8);
        UP(D.ln_pair, C.ln_pair.data(), C.ln_pair.size() * 4);
        UP(D.ln_word0, C.ln_word0.data(), C.ln_word0.size() * 4);
        UP(D.ln_skew, C.ln_skew.data(), C.ln_skew.size() * 4);
        UP(D.ln_ys, C.ln_ys.data(), C.ln_ys.size() * 8);
        UP(D.tb_pair, C.tb_pair.data(), C.tb_pair.size() * 4);
        UP(D.tb_item, C.tb_item.data(), C.tb_item.size() * 4);
        UP(D.tb_lane0, C.tb_lane0.data(), C.tb_lane0.size() * 4);
        UP(D.tb_band0, C.tb_band0.data(), C.tb_band0.size() * 4);
        UP(D.tb_strip0, C.tb_strip0.data(), C.tb_strip0.size() * 4);
        UP(D.sp_t, C.sp_t.data(), C.sp_t.size() * 4);
        UP(D.sp_s, C.sp_s.data(), C.sp_s.size() * 4);
        UP(D.fx_t, C.fx_t.data(), C.fx_t.size() * 4);
        UP(D.fx_s, C.fx_s.data(), C.fx_s.size() * 4);
        UP(D.sl_t, C.sl_t.data(), C.sl_t.size() * 4);
        if (C.n_rounds) {
            UP(D.it_rb, C.it_rb.data(), C.it_rb.size() * 8);
            UP(D.it_rcb, C.it_rcb.data(), C.it_rcb.size() * 8);
            UP(D.rd_items, C.rd_items.data(), C.rd_items.size() * 4);
            UP(D.rd_sp_t, C.rd_sp_t.data(), C.rd_sp_t.size() * 4);
            UP(D.rd_sp_s, C.rd_sp_s.data(), C.rd_sp_s.size() * 4);
            UP(D.rd_fx_t, C.rd_fx_t.data(), C.rd_fx_t.size() * 4);
            UP(D.rd_fx_s, C.rd_fx_s.data(), C.rd_fx_s.size() * 4);
            UP(D.rd_sl_t, C.rd_sl_t.data(), C.rd_sl_t.size() * 4);
            UP(D.rd_sl_top, C.rd_sl_top.data(), C.rd_sl_top.size() * 4);
            UP(D.rd_sl_lo, C.rd_sl_lo.data(), C.rd_sl_lo.size() * 4);
            D.rd_item_off = C.rd_item_off;
            D.rd_sp_off = C.rd_sp_off;
            D.rd_fx_off = C.rd_fx_off;
            D.rd_sl_off = C.rd_sl_off;
        }
        const int cap = tuning ? tuning->persistent_waves : 0;
        {
            const int fw = fill_block(C.wpl, sigma) / 64;   // waves per fill work-group
            D.fill_waves = fw;
            // with traceback rounds the pass's fill stores no history
            const int mode = bp->rounds ? (int)kFillLength : fill_mode(flags);
            D.fill_grid = resident_grid(ctx, fill_symbol(C.wpl, mode, raw_stream(sigma, C.wpl), sigma),
                                        fill_lds_bytes(C.wpl, sigma, mode), (D.nitems + fw - 1) / fw,
                                        cap > 0 ? (cap + fw - 1) / fw : 0, 64 * fw);
            // first-item bands: one band per wave every SIMD holds (four
            // SIMDs per CU), each as many places as there are SIMDs
            {
                const uint64_t simds = (uint64_t)ctx->num_cus * 4;
                uint64_t nbd = simds ? (uint64_t)D.fill_grid * (uint64_t)fw / simds : 0;
                nbd = std::min<uint64_t>(nbd, kMaxBands);
                if (simds) nbd = std::min<uint64_t>(nbd, D.nitems / simds);
                D.fill_nbands = bp->plain ? 0 : (uint32_t)nbd;
                D.fill_band_size = D.fill_nbands ? (uint32_t)simds : 0;
            }
            const void *tfn = fill_symbol(C.wpl, kFillTraceback, raw_stream(sigma, C.wpl), sigma);
            const size_t tlds = fill_lds_bytes(C.wpl, sigma, kFillTraceback);
            for (uint32_t r = 0; r < C.n_rounds; ++r) {
                const uint32_t ni = C.rd_item_off[r + 1] - C.rd_item_off[r];
                D.rd_fill_grid.push_back(resident_grid(ctx, tfn, tlds, (ni + fw - 1) / fw,
                                                       cap > 0 ? (cap + fw - 1) / fw : 0, 64 * fw));
            }
        }
        // the fill's wave priorities are set by the steps an item has left,
        // at fractions of the longest item
        {
            uint32_t mt = 0;
            for (uint32_t T : C.it_T) mt = std::max(mt, T);
            D.prio_half = std::max<uint32_t>(mt / 2, 1);
        }
        // traceback recompute rounds: by default tiles spanning about 256
        // columns per band and as many bands (up to four) as fit about 10 KiB
        // of LDS per wave (more LDS per wave costs more in resident waves than
        // it saves in rounds)
        {
            const size_t slot = tb_lds_bytes(C.wpl, sigma, cfg.ckpt, 1, 1) / (kTbBlock / 64);
            const int span = std::max(1, 256 / cfg.ckpt);
            const int room = std::max(1, (int)((10 * 1024) / slot));
            D.nb = (tuning && tuning->tb_tiles) ? tuning->tb_tiles : std::min(span, room);
            const int fit = (int)((10 * 1024) / (slot * D.nb));
            D.nbands = (tuning && tuning->tb_bands) ? tuning->tb_bands : std::max(1, std::min(4, fit));
            if (D.nb * D.nbands > 64 ||
                tb_lds_bytes(C.wpl, sigma, cfg.ckpt, D.nb, D.nbands) > 160 * 1024)
                return fail(LCS_ERR_ARG);
        }
        // The seal pass walks each pair's strips one after another, one wave
        // per pair: with so few waves LDS costs no residency, so its rounds
        // recompute up to 64 tiles (one per lane) over up to 16 bands, in
        // work-groups of one wave -- one batch of global reads per 16 bands
        // instead of per two.
        {
            D.seal_nb = D.nb;
            int bands = std::max(D.nbands, std::min(16, 64 / D.nb));
            while (bands > D.nbands && tb_lds_bytes(C.wpl, sigma, cfg.ckpt, D.nb, bands, 1) > 160 * 1024)
                --bands;
            D.seal_nbands = bands;
        }
        // With at most one strip per compute unit the speculative and fix-up
        // walks are as lone as the seal's, and take its work-groups of one
        // wave and its larger rounds (the 4096 x 4096 pair's pass: 0.57 ->
        // 0.53 ms)
        if (!bp->plain && !bp->rounds && !(tuning && (tuning->tb_tiles || tuning->tb_bands)) &&
            D.nsp <= (uint32_t)ctx->num_cus)
            D.tb_waves = 1;
        {
            const void *sym = tb_symbol(C.wpl, cfg.ckpt);
            const size_t lds = tb_lds_bytes(C.wpl, sigma, cfg.ckpt, D.nb, D.nbands);
            const size_t slds = tb_lds_bytes(C.wpl, sigma, cfg.ckpt, D.seal_nb, D.seal_nbands, 1);
            if (D.tb_waves == 1) {
                D.sp_grid = resident_grid(ctx, sym, slds, D.nsp, cap, 64);
                D.fx_grid = resident_grid(ctx, sym, slds, D.nfx, cap, 64);
            } else {
                D.sp_grid = resident_grid(ctx, sym, lds, (D.nsp + 3) / 4, cap > 0 ? (cap + 3) / 4 : 0);
                D.fx_grid = resident_grid(ctx, sym, lds, (D.nfx + 3) / 4, cap > 0 ? (cap + 3) / 4 : 0);
            }
            D.sl_grid = resident_grid(ctx, sym, slds, D.nsl, cap, 64);
            for (uint32_t r = 0; r < C.n_rounds; ++r) {
                const uint32_t nsp = C.rd_sp_off[r + 1] - C.rd_sp_off[r];
                const uint32_t nfx = C.rd_fx_off[r + 1] - C.rd_fx_off[r];
                const uint32_t nsl = C.rd_sl_off[r + 1] - C.rd_sl_off[r];
                D.rd_sp_grid.push_back(resident_grid(ctx, sym, lds, (nsp + 3) / 4, cap > 0 ? (cap + 3) / 4 : 0));
                D.rd_fx_grid.push_back(resident_grid(ctx, sym, lds, (nfx + 3) / 4, cap > 0 ? (cap + 3) / 4 : 0));
                D.rd_sl_grid.push_back(resident_grid(ctx, sym, slds, nsl, cap, 64));
            }
        }
        if (bp->plain) {
            // one launch per pair: items of a pair are consecutive, and so
            // are the tickets of one traceback entry in each pass
            std::vector<uint32_t> sp_first(D.ntb + 1, D.nsp), fx_first(D.ntb + 1, D.nfx),
                sl_of(D.ntb, 0xffffffffu);
            for (uint32_t k = D.nsp; k-- > 0;) sp_first[C.sp_t[k]] = k;
            for (uint32_t k = D.nfx; k-- > 0;) fx_first[C.fx_t[k]] = k;
            for (uint32_t k = 0; k < D.nsl; ++k) sl_of[C.sl_t[k]] = k;
            for (uint32_t t = 0; t < D.ntb; ++t) {
                const uint32_t pr = C.tb_pair[t];
                uint32_t first = C.tb_item[t], last = first;
                while (last + 1 < D.nitems && C.it_prev[last + 1] == (int32_t)last) ++last;
                D.pl_pair.push_back(pr);
                D.pl_begin.push_back(first);
                D.pl_end.push_back(last + 1);
                D.pl_tb.push_back(t);
                uint32_t nsp = 0, nfx = 0;
                for (uint32_t k = sp_first[t]; k < D.nsp && C.sp_t[k] == t; ++k) ++nsp;
                for (uint32_t k = fx_first[t]; k < D.nfx && C.fx_t[k] == t; ++k) ++nfx;
                D.pl_sp.push_back(sp_first[t]);
                D.pl_nsp.push_back(nsp);
                D.pl_fx.push_back(fx_first[t]);
                D.pl_nfx.push_back(nfx);
                D.pl_sl.push_back(sl_of[t]);
            }
        }
    }
#undef UP
    if (bp->upload_bytes &&
        hipMemcpyAsync(bp->dev, img, bp->upload_bytes, hipMemcpyHostToDevice, st0) != hipSuccess)
        return fail(LCS_ERR_DEVICE);
    if (hipStreamSynchronize(st0) != hipSuccess) return fail(LCS_ERR_DEVICE);
    bp->no_events = no_events;
    if (!no_events)
        for (hipEvent_t &ev : bp->ev)
            if (hipEventCreate(&ev) != hipSuccess) return fail(LCS_ERR_DEVICE);
    *out = bp;
    return LCS_OK;
}

extern "C" lcs_status lcs_batch_create(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                                       const lcs_alphabet *alphabet, uint32_t flags,
                                       const lcs_tuning *tuning, lcs_batch **out) {
    return build_batch(ctx, pairs, count, alphabet, flags, tuning, out);
}

// Enqueue the whole pass.  ev (optional) receives: before prep, before
// fill, after fill, after traceback.
static lcs_status enqueue(lcs_batch *b, hipStream_t s, bool events) {
    const Plan &p = b->plan;
    PrepArgs pa{};
    pa.lut = b->lut;
    pa.xbytes = b->xbytes;
    pa.xcodes = b->xcodes;
    pa.xarena = b->xarena;
    pa.ybytes = b->ybytes;
    pa.seg = b->seg;
    pa.nseg = (uint32_t)p.segs.size();
    pa.blk_seg = b->blk_seg;
    pa.nblk = p.ys_elems / 64;
    pa.ystream = b->ystream;
    pa.sentinel = (uint32_t)b->sigma;
    pa.out_len = b->out_len;
    pa.npairs = (uint32_t)b->npairs;
    pa.zero_words = b->zero;
    pa.nzero = b->nzero;
    pa.zero64 = b->zero64;
    pa.nzero64 = b->nzero64;
    if (b->flags & LCS_THRESHOLD) {
        pa.pair_m = b->pair_m;
        pa.pair_n = b->pair_n;
        pa.thr_t = b->thr_t;
        pa.thr_dec = b->thr_dec;
    }
    pa.halves = b->halves;
    pa.nhalves = (uint32_t)b->halves_host.size();
    if (events) HIP_TRY(hipEventRecord(b->ev[0], s));
    HIP_TRY(launch_prep(pa, b->xarena + 64, s));
    if (events) HIP_TRY(hipEventRecord(b->ev[1], s));
    const bool tb = (b->flags & LCS_WANT_TRACEBACK) != 0;
    const int mode = fill_mode(b->flags);
    auto fill_args = [&](size_t ci) {
        const ClassDev &D = b->cls[ci];
        FillArgs fa{};
        fa.xcodes = b->xcodes;
        fa.pair_xoff = b->pair_xoff;
        fa.pair_m = b->pair_m;
        fa.ystream = b->ystream;
        fa.it_T = D.it_T;
        fa.it_prev = D.it_prev;
        fa.it_feeds = D.it_feeds;
        fa.it_depth = D.it_depth;
        fa.it_ck = D.it_ck;
        fa.it_cb = D.it_cb;
        fa.it_xf = D.it_xf;
        fa.ln_pair = D.ln_pair;
        fa.ln_word0 = D.ln_word0;
        fa.ln_skew = D.ln_skew;
        fa.ln_ys = D.ln_ys;
        fa.out_len = b->out_len;
        if (!b->halves_host.empty()) {
            fa.out_v = b->vcols;
            fa.pair_vbase = b->pair_vbase;
            fa.v_pair0 = b->v_pair0;
        }
        fa.ckpt = D.ckpt;
        fa.cbits = D.cbits;
        fa.xfer = D.xfer;
        fa.queue = D.q_fill;
        fa.simd_rank = D.simd_rank;
        fa.band_next = D.band_next;
        fa.band_size = D.fill_band_size;
        fa.nbands = D.fill_nbands;
        fa.error = b->error;
        fa.junk = b->junk;
        fa.item_begin = 0;
        fa.item_end = D.nitems;
        fa.prio_half = D.prio_half;
        fa.spin_limit = b->spin_limit;
        fa.sigma = b->sigma;
        fa.ckpt_every = b->ckpt;
        fa.clk = b->clk;
        fa.trace = D.trace;
        if (mode == kFillThreshold) {
            fa.pair_n = b->pair_n;
            fa.thr_t = b->thr_t;
            fa.thr_dec = b->thr_dec;
            fa.xsum = D.xsum;
        }
        return fa;
    };
    auto tb_args = [&](size_t ci, int32_t mode) {
        const ClassDev &D = b->cls[ci];
        TbArgs ta{};
        ta.xcodes = b->xcodes;
        ta.pair_xoff = b->pair_xoff;
        ta.pair_m = b->pair_m;
        ta.pair_n = b->pair_n;
        ta.pair_diag = b->pair_diag;
        ta.diag = b->diag;
        ta.ystream = b->ystream;
        ta.it_T = D.it_T;
        ta.it_ck = D.it_ck;
        ta.it_cb = D.it_cb;
        ta.ln_skew = D.ln_skew;
        ta.ln_ys = D.ln_ys;
        ta.ckpt = D.ckpt;
        ta.cbits = D.cbits;
        ta.tb_pair = D.tb_pair;
        ta.tb_item = D.tb_item;
        ta.tb_lane0 = D.tb_lane0;
        ta.tb_band0 = D.tb_band0;
        ta.tb_strip0 = D.tb_strip0;
        ta.cross = D.cross;
        ta.strip_res = D.strip_res;
        ta.strip_bands = D.strip_bands;
        ta.sigma = b->sigma;
        ta.ckpt_every = b->ckpt;
        ta.nb = D.nb;
        ta.nbands = D.nbands;
        ta.ysh = raw_stream(b->sigma, D.wpl) ? 0 : 9 + __builtin_ctz((unsigned)D.wpl);
        ta.mode = mode;
        if (mode != kTbSeal && D.tb_waves == 1) {
            ta.nb = D.seal_nb;
            ta.nbands = D.seal_nbands;
        }
        if (mode == kTbSpec) {
            ta.tk_t = D.sp_t;
            ta.tk_s = D.sp_s;
            ta.nticket = D.nsp;
            ta.queue = D.q_spec;
        } else if (mode == kTbFix) {
            ta.tk_t = D.fx_t;
            ta.tk_s = D.fx_s;
            ta.nticket = D.nfx;
            ta.queue = D.q_fix;
        } else {
            ta.nb = D.seal_nb;
            ta.nbands = D.seal_nbands;
            ta.tk_t = D.sl_t;
            ta.tk_s = nullptr;     // every seal runs from the pair's top strip down
            ta.tk_lo = nullptr;
            ta.nticket = D.nsl;
            ta.queue = D.q_seal;
        }
        return ta;
    };
    EmitArgs ea{};
    ea.xbytes = b->xbytes;
    ea.pair_xoff = b->pair_xoff;
    ea.pair_m = b->pair_m;
    ea.pair_n = b->pair_n;
    ea.pair_diag = b->pair_diag;
    ea.diag = b->diag;
    ea.pair_out = b->pair_out;
    ea.out_len = b->out_len;
    ea.out = b->out;
    ea.em_pair = b->em_pair;
    ea.em_w0 = b->em_w0;
    ea.nitems = (uint32_t)b->em_pair_host.size();
    ea.error = b->error;
    if (!b->plain) {
        // with traceback rounds the pass's fill computes lengths and the
        // carry words handed between items only
        const int fwd_mode = b->rounds ? (int)kFillLength : mode;
        for (size_t ci = 0; ci < b->cls.size(); ++ci) {
            const ClassDev &D = b->cls[ci];
            if (!D.nitems) continue;
            HIP_TRY(launch_fill(D.wpl, fwd_mode, fill_args(ci), D.fill_grid, s));
        }
        if (events) HIP_TRY(hipEventRecord(b->ev[2], s));
        if (!b->halves_host.empty()) {
            HalvesArgs ha{};
            ha.halves = b->halves;
            ha.nhalves = (uint32_t)b->halves_host.size();
            ha.v = b->vcols;
            ha.out_len = b->out_len;
            HIP_TRY(launch_halves(ha, s));
        }
        if (tb) {
            for (size_t ci = 0; ci < b->cls.size(); ++ci) {
                const ClassDev &D = b->cls[ci];
                if (!D.ntb) continue;
                if (!D.n_rounds) {
                    HIP_TRY(launch_tb(D.wpl, tb_args(ci, kTbSpec), D.sp_grid, D.tb_waves, s));
                    if (D.nfx) HIP_TRY(launch_tb(D.wpl, tb_args(ci, kTbFix), D.fx_grid, D.tb_waves, s));
                    if (D.nsl) HIP_TRY(launch_tb(D.wpl, tb_args(ci, kTbSeal), D.sl_grid, 1, s));
                    continue;
                }
                // rounds: refill the round's items with their history in the
                // round buffer (their carry-in words from the items below are
                // already stored by the pass's fill), then walk the strips
                // they hold, from where the earlier rounds left the path
                for (uint32_t r = 0; r < D.n_rounds; ++r) {
                    uint32_t *q = D.q_round + (size_t)kQueues * r;
                    FillArgs fa = fill_args(ci);
                    fa.item_list = D.rd_items;
                    fa.item_begin = D.rd_item_off[r];
                    fa.item_end = D.rd_item_off[r + 1];
                    fa.it_ck = D.it_rb;
                    fa.it_cb = D.it_rcb;
                    fa.out_len = nullptr;
                    fa.queue = q;
                    fa.band_size = 0;
                    fa.nbands = 0;
                    fa.clk = nullptr;
                    fa.trace = nullptr;
                    HIP_TRY(launch_fill(D.wpl, kFillTraceback, fa, D.rd_fill_grid[r], s));
                    TbArgs ta = tb_args(ci, kTbSpec);
                    ta.it_ck = D.it_rb;
                    ta.it_cb = D.it_rcb;
                    ta.tk_t = D.rd_sp_t + D.rd_sp_off[r];
                    ta.tk_s = D.rd_sp_s + D.rd_sp_off[r];
                    ta.nticket = D.rd_sp_off[r + 1] - D.rd_sp_off[r];
                    ta.queue = q + 1;
                    if (ta.nticket) HIP_TRY(launch_tb(D.wpl, ta, D.rd_sp_grid[r], 4, s));
                    ta.mode = kTbFix;
                    ta.tk_t = D.rd_fx_t + D.rd_fx_off[r];
                    ta.tk_s = D.rd_fx_s + D.rd_fx_off[r];
                    ta.nticket = D.rd_fx_off[r + 1] - D.rd_fx_off[r];
                    ta.queue = q + 2;
                    if (ta.nticket) HIP_TRY(launch_tb(D.wpl, ta, D.rd_fx_grid[r], 4, s));
                    ta.mode = kTbSeal;
                    ta.tk_t = D.rd_sl_t + D.rd_sl_off[r];
                    ta.tk_s = D.rd_sl_top + D.rd_sl_off[r];
                    ta.tk_lo = D.rd_sl_lo + D.rd_sl_off[r];
                    ta.nticket = D.rd_sl_off[r + 1] - D.rd_sl_off[r];
                    ta.queue = q + 3;
                    ta.nb = D.seal_nb;
                    ta.nbands = D.seal_nbands;
                    if (ta.nticket) HIP_TRY(launch_tb(D.wpl, ta, D.rd_sl_grid[r], 1, s));
                }
            }
            HIP_TRY(launch_emit(ea, s));
        }
    } else {
        // plain per-pair: every pair gets its own fill launch (and its own
        // traceback launch), in order
        for (size_t ci = 0; ci < b->cls.size(); ++ci) {
            const ClassDev &D = b->cls[ci];
            uint32_t *ctr = D.plain_ctr;
            for (size_t k = 0; k < D.pl_pair.size(); ++k) {
                FillArgs fa = fill_args(ci);
                fa.item_begin = D.pl_begin[k];
                fa.item_end = D.pl_end[k];
                fa.queue = ctr + kQueues * k;
                fa.band_size = 0;
                fa.nbands = 0;
                uint32_t g = (fa.item_end - fa.item_begin + D.fill_waves - 1) / D.fill_waves;
                HIP_TRY(launch_fill(D.wpl, mode, fa, g, s));
                if (tb) {
                    TbArgs ta = tb_args(ci, kTbSpec);
                    ta.tk_t += D.pl_sp[k];
                    ta.tk_s += D.pl_sp[k];
                    ta.nticket = D.pl_nsp[k];
                    ta.queue = ctr + kQueues * k + 1;
                    HIP_TRY(launch_tb(D.wpl, ta, (ta.nticket + 3) / 4, 4, s));
                    if (D.pl_nfx[k]) {
                        ta = tb_args(ci, kTbFix);
                        ta.tk_t += D.pl_fx[k];
                        ta.tk_s += D.pl_fx[k];
                        ta.nticket = D.pl_nfx[k];
                        ta.queue = ctr + kQueues * k + 2;
                        HIP_TRY(launch_tb(D.wpl, ta, (ta.nticket + 3) / 4, 4, s));
                    }
                    if (D.pl_sl[k] != 0xffffffffu) {
                        ta = tb_args(ci, kTbSeal);
                        ta.tk_t += D.pl_sl[k];
                        ta.nticket = 1;
                        ta.queue = ctr + kQueues * k + 3;
                        HIP_TRY(launch_tb(D.wpl, ta, 1, 1, s));
                    }
                    const uint32_t pr = D.pl_pair[k];
                    EmitArgs e1 = ea;
                    e1.em_pair += b->em_first_host[pr];
                    e1.em_w0 += b->em_first_host[pr];
                    e1.nitems = b->em_first_host[pr + 1] - b->em_first_host[pr];
                    HIP_TRY(launch_emit(e1, s));
                }
            }
        }
        if (events) HIP_TRY(hipEventRecord(b->ev[2], s));
    }
    if (events) HIP_TRY(hipEventRecord(b->ev[3], s));
    return LCS_OK;
}

// Launch one pass.  Graph batches capture the sequence once (with the HIP
// event records as graph nodes, so per-pass timings stay readable) and replay
// it; the others enqueue the kernels directly.
static lcs_status launch_pass(lcs_batch *b, bool eager) {
    lcs_ctx *ctx = b->ctx;
    if ((b->flags & LCS_THRESHOLD) && !b->thr_set) return LCS_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCS_ERR_DEVICE;
    hipStream_t s = b->hooks.stream ? b->hooks.stream : ctx->stream;
    if ((b->flags & LCS_USE_GRAPH) && !b->plain && !eager) {
        if (!b->gexec) {
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            lcs_status st = enqueue(b, s, false);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(s, &g);
            if (st != LCS_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            HIP_TRY(e);
            b->graph = g;
            HIP_TRY(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
        }
        HIP_TRY(hipEventRecord(b->ev[0], s));
        HIP_TRY(hipGraphLaunch(b->gexec, s));
        HIP_TRY(hipEventRecord(b->ev[3], s));
        b->timed_fill = false;
    } else {
        lcs_status st = enqueue(b, s, !b->no_events);
        if (st) return st;
        b->timed_fill = !b->no_events;
    }
    b->ran = true;
    return LCS_OK;
}

extern "C" lcs_status lcs_batch_run(lcs_batch *b) {
    if (!b) return LCS_ERR_ARG;
    return launch_pass(b, false);
}

static lcs_status finish(lcs_batch *b) {
    if (!b->ran) return LCS_ERR_ARG;
    lcs_ctx *ctx = b->ctx;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCS_ERR_DEVICE;
    HIP_TRY(hipStreamSynchronize(b->hooks.stream ? b->hooks.stream : ctx->stream));
    uint32_t err = 0;
    HIP_TRY(hipMemcpy(&err, b->error, 4, hipMemcpyDeviceToHost));
    if (err) {
        std::snprintf(g_last_error, sizeof g_last_error, "kernel error flag %u (%s)", err,
                      (err & 1u) ? "a carry hand-over wait ran out of polls"
                                 : "a traceback disagrees with its length");
        return LCS_ERR_DEVICE;
    }
    return LCS_OK;
}

// Wait for the last pass and copy its results to the host in one piece:
// the lengths and the error word, and with `strings` also the LCS bytes (the
// three regions are adjacent on the device).  LCS_ERR_DEVICE if a kernel set
// the error word.
// Byte vector whose growth leaves the new bytes uninitialized: a read-back
// image is overwritten by the copy at once.
template <class T>
struct NoInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <class U>
    NoInitAlloc(const NoInitAlloc<U> &) {}
    template <class U>
    void construct(U *p) noexcept {
        ::new ((void *)p) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
using HostBytes = std::vector<uint8_t, NoInitAlloc<uint8_t>>;

static lcs_status readback(lcs_batch *b, bool strings, HostBytes &host) {
    if (!b->ran) return LCS_ERR_ARG;
    lcs_ctx *ctx = b->ctx;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCS_ERR_DEVICE;
    HIP_TRY(hipStreamSynchronize(b->hooks.stream ? b->hooks.stream : ctx->stream));
    const size_t err_off = (size_t)((char *)b->error - (char *)b->out_len);
    const size_t bytes = strings ? std::max(b->readback_bytes, err_off + 4) : err_off + 4;
    host.resize(bytes);
    HIP_TRY(hipMemcpy(host.data(), b->out_len, bytes, hipMemcpyDeviceToHost));
    uint32_t err = 0;
    std::memcpy(&err, host.data() + err_off, 4);
    if (err) {
        std::snprintf(g_last_error, sizeof g_last_error, "kernel error flag %u (%s)", err,
                      (err & 1u) ? "a carry hand-over wait ran out of polls"
                                 : "a traceback disagrees with its length");
        return LCS_ERR_DEVICE;
    }
    return LCS_OK;
}

// Threshold pass: answers and lengths from a read-back image (a pair
// answered before its last column has no length).
static lcs_status threshold_results(const lcs_batch *b, const HostBytes &host,
                                    uint8_t *out_pass, uint64_t *out_len) {
    const uint64_t *L = (const uint64_t *)host.data();
    const uint32_t *dec = (const uint32_t *)(host.data() + ((char *)b->thr_dec - (char *)b->out_len));
    for (uint64_t k = 0; k < b->npairs; ++k) {
        uint64_t len = LCS_LENGTH_UNKNOWN;
        uint8_t pass = 0;
        if (dec[k] == 1u || dec[k] == 2u) {
            pass = dec[k] == 1u;
        } else if (dec[k] == 0u) {
            if (L[k] > std::min(b->m[k], b->n[k])) return LCS_ERR_DEVICE;
            len = L[k];
            pass = L[k] >= b->thr_host[k];
        } else {
            return LCS_ERR_DEVICE;
        }
        if (out_pass) out_pass[k] = pass;
        if (out_len) out_len[k] = len;
    }
    return LCS_OK;
}

extern "C" lcs_status lcs_batch_lengths(lcs_batch *b, uint64_t *out_lens) {
    if (!b || (b->npairs && !out_lens)) return LCS_ERR_ARG;
    HostBytes host;
    lcs_status st = readback(b, false, host);
    if (st) return st;
    if (b->flags & LCS_THRESHOLD) return threshold_results(b, host, nullptr, out_lens);
    if (b->npairs) std::memcpy(out_lens, host.data(), b->npairs * 8);
    return LCS_OK;
}

// Least L in [0, m] whose similarity (100 * L) / m reaches pct (which is at
// most 100, and (100 * m) / m is exactly 100); the similarity is
// non-decreasing in L, so a binary search finds it.
static uint32_t target_length(uint64_t m, double pct) {
    if (m == 0) return 0;
    auto sim = [&](uint64_t L) { return (100.0 * (double)L) / (double)m; };
    if (sim(0) >= pct) return 0;
    uint64_t lo = 0, hi = m;   // sim(lo) < pct <= sim(hi)
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (sim(mid) >= pct) hi = mid;
        else lo = mid;
    }
    return (uint32_t)hi;
}

extern "C" lcs_status lcs_batch_set_threshold(lcs_batch *b, double min_percent) {
    if (!b || !(b->flags & LCS_THRESHOLD)) return LCS_ERR_ARG;
    if (!(min_percent >= 0.0 && min_percent <= 100.0)) return LCS_ERR_ARG;
    lcs_ctx *ctx = b->ctx;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCS_ERR_DEVICE;
    hipStream_t s = b->hooks.stream ? b->hooks.stream : ctx->stream;
    // earlier passes may still read the old targets
    HIP_TRY(hipStreamSynchronize(s));
    b->thr_host.assign(b->npairs + 1, 0);
    for (uint64_t k = 0; k < b->npairs; ++k) b->thr_host[k] = target_length(b->m[k], min_percent);
    if (b->npairs) {
        HIP_TRY(hipMemcpyAsync(b->thr_t, b->thr_host.data(), b->npairs * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    b->thr_set = true;
    return LCS_OK;
}

extern "C" lcs_status lcs_batch_decisions(lcs_batch *b, uint8_t *out_pass, uint64_t *out_len) {
    if (!b || !(b->flags & LCS_THRESHOLD)) return LCS_ERR_ARG;
    if (b->npairs && !out_pass) return LCS_ERR_ARG;
    HostBytes host;
    lcs_status st = readback(b, false, host);
    if (st) return st;
    return threshold_results(b, host, out_pass, out_len);
}

extern "C" lcs_status lcs_batch_tracebacks(lcs_batch *b, uint8_t *out_arena, uint64_t arena_cap,
                                           uint64_t *out_offsets, uint64_t *out_lens) {
    if (!b) return LCS_ERR_ARG;
    if (!(b->flags & LCS_WANT_TRACEBACK)) return LCS_ERR_ARG;
    if (b->npairs && (!out_offsets || !out_lens)) return LCS_ERR_ARG;
    if (arena_cap < b->out_off_host[b->npairs]) return LCS_ERR_BUFFER;
    if (b->out_off_host[b->npairs] && !out_arena) return LCS_ERR_ARG;
    HostBytes host;
    lcs_status st = readback(b, true, host);
    if (st) return st;
    const uint64_t *L = (const uint64_t *)host.data();
    const uint8_t *raw = host.data() + ((char *)b->out - (char *)b->out_len);
    uint64_t o = 0;
    for (uint64_t k = 0; k < b->npairs; ++k) {
        if (L[k] > std::min(b->m[k], b->n[k])) return LCS_ERR_DEVICE;
        out_offsets[k] = o;
        out_lens[k] = L[k];
        o += L[k];
    }
    // the strings into the caller's arena, pairs split over host threads
    const int T = host_threads(o);
    const uint64_t np = b->npairs;
    run_threads(T, [&](int t) {
        const uint64_t k0 = np * (uint64_t)t / (uint64_t)T, k1 = np * (uint64_t)(t + 1) / (uint64_t)T;
        for (uint64_t k = k0; k < k1; ++k)
            if (L[k]) std::memcpy(out_arena + out_offsets[k], raw + b->out_off_host[k], L[k]);
    });
    return LCS_OK;
}

extern "C" lcs_status lcs_batch_info(const lcs_batch *b, lcs_batch_stats *out) {
    if (!b || !out) return LCS_ERR_ARG;
    stats_from_plan(b->plan, b->npairs, out);
    out->split_pairs = (int32_t)b->halves_host.size();
    out->device_bytes = b->dev_bytes;
    out->history_bytes = b->history_bytes;
    out->flags = (int32_t)b->flags;
    return LCS_OK;
}

extern "C" lcs_status lcs_batch_time(lcs_batch *b, int eager, float *total_ms, float *fill_ms) {
    if (!b) return LCS_ERR_ARG;
    lcs_status st = launch_pass(b, eager != 0);
    if (st) return st;
    st = finish(b);
    if (st) return st;
    float t = 0.f;
    if (total_ms) {
        HIP_TRY(hipEventElapsedTime(&t, b->ev[0], b->ev[3]));
        *total_ms = t;
    }
    if (fill_ms) {
        if (b->timed_fill) {
            HIP_TRY(hipEventElapsedTime(&t, b->ev[1], b->ev[2]));
            *fill_ms = t;
        } else {
            *fill_ms = -1.f;
        }
    }
    return LCS_OK;
}

extern "C" lcs_status lcs_batch_clock(lcs_batch *b, double *mhz) {
    if (!b || !mhz || !b->ran) return LCS_ERR_ARG;
    lcs_ctx *ctx = b->ctx;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCS_ERR_DEVICE;
    HIP_TRY(hipStreamSynchronize(b->hooks.stream ? b->hooks.stream : ctx->stream));
    uint64_t c[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(c, b->clk, sizeof c, hipMemcpyDeviceToHost));
    if (c[3] <= c[1] || c[2] <= c[0]) return LCS_ERR_DEVICE;
    // shader cycles per tick of the 100 MHz counter
    *mhz = 100.0 * (double)(c[2] - c[0]) / (double)(c[3] - c[1]);
    return LCS_OK;
}

extern "C" lcs_status lcs_batch_fill_trace(lcs_batch *b, lcs_fill_item *out, uint64_t cap,
                                           uint64_t *count) {
    if (!b || !count || !(b->flags & LCS_FILL_TRACE)) return LCS_ERR_ARG;
    uint64_t total = 0;
    for (const ClassDev &D : b->cls) total += D.nitems;
    *count = total;
    if (!out) return LCS_OK;
    if (cap < total || !b->ran) return LCS_ERR_ARG;
    lcs_ctx *ctx = b->ctx;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCS_ERR_DEVICE;
    HIP_TRY(hipStreamSynchronize(b->hooks.stream ? b->hooks.stream : ctx->stream));
    std::vector<uint64_t> raw(total * kTraceWords + 1);
    uint64_t at = 0;
    for (const ClassDev &D : b->cls) {
        if (D.nitems)
            HIP_TRY(hipMemcpy(raw.data() + at * kTraceWords, D.trace,
                              (size_t)D.nitems * kTraceWords * sizeof(uint64_t), hipMemcpyDeviceToHost));
        at += D.nitems;
    }
    // times relative to the earliest item taken, 100 MHz counter ticks to ns
    uint64_t t0 = UINT64_MAX;
    for (uint64_t k = 0; k < total; ++k)
        if (raw[k * kTraceWords + 2]) t0 = std::min(t0, raw[k * kTraceWords]);
    const auto ns = [&](uint64_t t) { return t >= t0 ? (t - t0) * 10 : 0; };
    at = 0;
    for (size_t ci = 0; ci < b->cls.size(); ++ci) {
        const ClassPlan &C = b->plan.classes[ci];
        for (uint64_t i = 0; i < b->cls[ci].nitems; ++i) {
            const uint64_t *r = raw.data() + (at + i) * kTraceWords;
            lcs_fill_item &o = out[at + i];
            o.ran = r[2] != 0;
            o.start_ns = o.ran ? ns(r[0]) : 0;
            o.first_step_ns = o.ran ? ns(r[1]) : 0;
            o.end_ns = o.ran ? ns(r[2]) : 0;
            o.wait_ns = r[3] * 10;
            o.steps = C.it_T[i];
            o.feeder = C.it_prev[i] >= 0 ? (int32_t)(at + (uint64_t)C.it_prev[i]) : -1;
            o.feeds = C.it_feeds[i] != 0;
            o.hw_id = (uint32_t)(r[4] >> 32);
            o.xcc_id = (uint32_t)r[4];
        }
        at += b->cls[ci].nitems;
    }
    return LCS_OK;
}

extern "C" void lcs_batch_destroy(lcs_batch *b) { free_batch(b); }

// --------------------------------------------------------------------------
// one-call entry points
// --------------------------------------------------------------------------

static const lcs_tuning kSinglePair = {1, 0, 0, 0};   // most lanes per pair

extern "C" lcs_status lcs_length(lcs_ctx *ctx, const uint8_t *x, uint64_t m, const uint8_t *y,
                                 uint64_t n, const lcs_alphabet *alphabet, uint64_t *out_len) {
    if (!ctx || !out_len) return LCS_ERR_ARG;
    lcs_pair p = {x, m, y, n};
    lcs_tuning t = kSinglePair;
    lcs_batch *b = nullptr;
    lcs_status st = build_batch(ctx, &p, 1, alphabet, 0, &t, &b);
    if (st) return st;
    st = lcs_batch_run(b);
    uint64_t L = 0;
    if (!st) st = lcs_batch_lengths(b, &L);
    free_batch(b);
    if (!st) *out_len = L;
    return st;
}

extern "C" lcs_status lcs_traceback(lcs_ctx *ctx, const uint8_t *x, uint64_t m, const uint8_t *y,
                                    uint64_t n, const lcs_alphabet *alphabet, uint8_t *out,
                                    uint64_t out_cap, uint64_t *out_len) {
    if (!ctx || !out_len) return LCS_ERR_ARG;
    if (out_cap < std::min(m, n)) return LCS_ERR_BUFFER;
    if (std::min(m, n) && !out) return LCS_ERR_ARG;
    lcs_pair p = {x, m, y, n};
    lcs_tuning t = kSinglePair;
    lcs_batch *b = nullptr;
    lcs_status st = build_batch(ctx, &p, 1, alphabet, LCS_WANT_TRACEBACK, &t, &b);
    if (st) return st;
    st = lcs_batch_run(b);
    uint64_t off = 0, L = 0;
    if (!st) st = lcs_batch_tracebacks(b, out, out_cap, &off, &L);
    free_batch(b);
    if (!st) *out_len = L;
    return st;
}

extern "C" lcs_status lcs_length_batch(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                                       const lcs_alphabet *alphabet, uint64_t *out_lens) {
    if (!ctx || (count && !out_lens)) return LCS_ERR_ARG;
    lcs_batch *b = nullptr;
    lcs_status st = build_batch(ctx, pairs, count, alphabet, 0, nullptr, &b);
    if (st) return st;
    st = lcs_batch_run(b);
    if (!st) st = lcs_batch_lengths(b, out_lens);
    free_batch(b);
    return st;
}

extern "C" lcs_status lcs_similarity_batch(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                                           const lcs_alphabet *alphabet, double *out_percent) {
    if (!ctx || (count && !out_percent)) return LCS_ERR_ARG;
    std::vector<uint64_t> L(count + 1, 0);
    lcs_status st = lcs_length_batch(ctx, pairs, count, alphabet, L.data());
    if (st) return st;
    for (uint64_t k = 0; k < count; ++k)
        out_percent[k] = pairs[k].m ? (100.0 * (double)L[k]) / (double)pairs[k].m : 100.0;
    return LCS_OK;
}

extern "C" lcs_status lcs_threshold_batch(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                                          const lcs_alphabet *alphabet, double min_percent,
                                          uint8_t *out_pass, uint64_t *out_len) {
    if (!ctx || (count && !out_pass)) return LCS_ERR_ARG;
    if (!(min_percent >= 0.0 && min_percent <= 100.0)) return LCS_ERR_ARG;
    lcs_batch *b = nullptr;
    lcs_status st = build_batch(ctx, pairs, count, alphabet, LCS_THRESHOLD, nullptr, &b);
    if (st) return st;
    st = lcs_batch_set_threshold(b, min_percent);
    if (!st) st = lcs_batch_run(b);
    if (!st) st = lcs_batch_decisions(b, out_pass, out_len);
    free_batch(b);
    return st;
}

extern "C" lcs_status lcs_traceback_batch(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                                          const lcs_alphabet *alphabet, uint8_t *out_arena,
                                          uint64_t arena_cap, uint64_t *out_offsets,
                                          uint64_t *out_lens) {
    if (!ctx || (count && (!out_offsets || !out_lens))) return LCS_ERR_ARG;
    lcs_status st = check_pairs(pairs, count);
    if (st) return st;
    uint64_t worst = 0;
    for (uint64_t k = 0; k < count; ++k) worst += std::min(pairs[k].m, pairs[k].n);
    if (arena_cap < worst) return LCS_ERR_BUFFER;
    if (worst && !out_arena) return LCS_ERR_ARG;
    lcs_batch *b = nullptr;
    st = build_batch(ctx, pairs, count, alphabet, LCS_WANT_TRACEBACK, nullptr, &b);
    if (st) return st;
    st = lcs_batch_run(b);
    if (!st) st = lcs_batch_tracebacks(b, out_arena, arena_cap, out_offsets, out_lens);
    free_batch(b);
    return st;
}

// --------------------------------------------------------------------------
// allocation-free entry point
// --------------------------------------------------------------------------

namespace {
struct ScratchUse {
    void *ptr;
    size_t cap;
};
void *scratch_alloc(void *user, size_t bytes) {
    ScratchUse *u = (ScratchUse *)user;
    if (bytes > u->cap) {
        std::snprintf(g_last_error, sizeof g_last_error,
                      "batch needs %zu bytes of device scratch; the fixed scratch holds %zu", bytes,
                      u->cap);
        return nullptr;
    }
    return u->ptr;
}
void scratch_release(void *, void *) {}
}  // namespace

extern "C" lcs_status lcs_traceback_batch_noalloc(lcs_ctx *ctx, const lcs_pair *pairs,
                                                  uint64_t count, const lcs_alphabet *alphabet,
                                                  uint8_t *out_arena, uint64_t arena_cap,
                                                  uint64_t *out_offsets, uint64_t *out_lens) {
    if (!ctx || (count && (!out_offsets || !out_lens))) return LCS_ERR_ARG;
    lcs_status st = check_pairs(pairs, count);
    if (st) return st;
    uint64_t worst = 0;
    for (uint64_t k = 0; k < count; ++k) worst += std::min(pairs[k].m, pairs[k].n);
    if (arena_cap < worst) return LCS_ERR_BUFFER;
    if (worst && !out_arena) return LCS_ERR_ARG;
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return LCS_ERR_DEVICE;
    ScratchSlot &sl = g_scratch[ctx->device];
    if (!sl.resolved || !sl.ptr) {
        if (sl.resolved) note_error("hipGetSymbolAddress(scratch)", sl.err);
        else std::snprintf(g_last_error, sizeof g_last_error, "device scratch not resolved");
        return LCS_ERR_DEVICE;
    }
    // one call at a time per device: the scratch keeps the last call's
    // contents, and every pass clears what must start at zero itself
    std::lock_guard<std::mutex> lk(sl.use);
    ScratchUse use{sl.ptr, kNoAllocScratchBytes};
    BatchHooks hooks;
    hooks.stream = ctx->stream;
    hooks.alloc = scratch_alloc;
    hooks.release = scratch_release;
    hooks.user = &use;
    // a batch whose full traceback history would not fit the array runs in
    // rounds sized to what its other buffers leave
    hooks.avail = kNoAllocScratchBytes;
    lcs_batch *b = nullptr;
    st = build_batch(ctx, pairs, count, alphabet, LCS_WANT_TRACEBACK, nullptr, &b, &hooks, true);
    if (st) return st;
    st = launch_pass(b, true);
    if (!st) st = lcs_batch_tracebacks(b, out_arena, arena_cap, out_offsets, out_lens);
    // nothing of this call may still run on the scratch once the next call
    // can take it
    if (hipStreamSynchronize(ctx->stream) != hipSuccess && !st) st = LCS_ERR_DEVICE;
    free_batch(b);
    return st;
}

extern "C" uint64_t lcs_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

// --------------------------------------------------------------------------
// host-only planning checks
// --------------------------------------------------------------------------

// --------------------------------------------------------------------------
// library-internal batch interface (request server)
// --------------------------------------------------------------------------

namespace lcs {

lcs_status batch_create(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                        const lcs_alphabet *alphabet, uint32_t flags, const lcs_tuning *tuning,
                        const BatchHooks *hooks, lcs_batch **out) {
    return build_batch(ctx, pairs, count, alphabet, flags, tuning, out, hooks);
}

lcs_status alphabet_check(const lcs_alphabet *a, const uint8_t *x, uint64_t m, const uint8_t *y,
                          uint64_t n, int *sigma) {
    uint8_t lut[256];
    bool valid[256];
    const lcs_status st = make_lut(a, lut, valid, sigma);
    if (st) return st;
    if ((m && !x) || (n && !y)) return LCS_ERR_ARG;
    if (m > LCS_MAX_LEN || n > LCS_MAX_LEN) return LCS_ERR_TOO_LONG;
    if (!all_in(x, m, valid) || !all_in(y, n, valid)) return LCS_ERR_SYMBOL;
    return LCS_OK;
}

int ctx_device(lcs_ctx *ctx) { return ctx->device; }

lcs_status ctx_reserve(lcs_ctx *ctx, size_t *bytes, void **mem) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    const size_t left = ctx->budget > ctx->in_use ? ctx->budget - ctx->in_use : 0;
    size_t want = *bytes ? *bytes : left / 2;
    want = (want + 255) & ~(size_t)255;
    if (want == 0 || want > left) return LCS_ERR_NOMEM;
    if (hipSetDevice(ctx->device) != hipSuccess) return LCS_ERR_DEVICE;
    const hipError_t e = hipMalloc(mem, want);
    if (e != hipSuccess) {
        note_error("hipMalloc", e);
        return dev_err(e);
    }
    ctx->in_use += want;
    *bytes = want;
    return LCS_OK;
}

void ctx_unreserve(lcs_ctx *ctx, void *mem, size_t bytes) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    (void)hipFree(mem);
    ctx->in_use -= bytes;
}

lcs_status batch_launch(lcs_batch *b) {
    if (!b) return LCS_ERR_ARG;
    return launch_pass(b, true);
}

int batch_query(lcs_batch *b) {
    if (!b || !b->ran) return LCS_ERR_ARG;
    const hipError_t e = hipEventQuery(b->ev[3]);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    note_error("hipEventQuery", e);
    return dev_err(e);
}

lcs_status batch_results(lcs_batch *b, std::vector<uint64_t> &lens,
                         std::vector<std::vector<uint8_t>> *strings) {
    lens.assign(b->npairs, 0);
    if (!(b->flags & LCS_WANT_TRACEBACK) || !strings) return lcs_batch_lengths(b, lens.data());
    const uint64_t cap = b->out_off_host[b->npairs];
    std::vector<uint8_t> arena(cap + 1);
    std::vector<uint64_t> offs(b->npairs);
    lcs_status st = lcs_batch_tracebacks(b, arena.data(), cap, offs.data(), lens.data());
    if (st) return st;
    strings->assign(b->npairs, {});
    for (uint64_t k = 0; k < b->npairs; ++k)
        (*strings)[k].assign(arena.data() + offs[k], arena.data() + offs[k] + lens[k]);
    return LCS_OK;
}

}  // namespace lcs

// --------------------------------------------------------------------------
// autotuner
// --------------------------------------------------------------------------

static uint32_t ilog2_u64(uint64_t v) { return v ? 63u - (uint32_t)__builtin_clzll(v) : 0u; }

// The shape a tuning is cached under: what the batch computes (graph replay
// and schedule records do not change the best tuning, so a batch tuned for
// graph replay also serves the request server's eager batches), the
// alphabet, and log2 buckets of the pair count, the longest X and Y and the
// cells.
static TuneKey tune_key(const lcs_pair *pairs, uint64_t count, int sigma, uint32_t flags) {
    flags &= (uint32_t)(LCS_WANT_TRACEBACK | LCS_THRESHOLD);
    uint64_t mm = 0, mn = 0;
    double cells = 0;
    for (uint64_t k = 0; k < count; ++k) {
        mm = std::max<uint64_t>(mm, pairs[k].m);
        mn = std::max<uint64_t>(mn, pairs[k].n);
        cells += (double)pairs[k].m * (double)pairs[k].n;
    }
    return TuneKey{flags, (uint32_t)sigma, ilog2_u64(count), ilog2_u64(mm), ilog2_u64(mn),
                   cells >= 1 ? (uint32_t)(4.0 * std::log2(cells)) : 0u};
}

namespace lcs {
bool tuning_cached(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count, int sigma, uint32_t flags,
                   lcs_tuning *out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto hit = ctx->tune_cache.find(tune_key(pairs, count, sigma, flags));
    if (hit == ctx->tune_cache.end()) return false;
    *out = hit->second.first;
    return true;
}
}  // namespace lcs

extern "C" lcs_status lcs_autotune(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                                   const lcs_alphabet *alphabet, uint32_t flags,
                                   lcs_tuning *best, float *best_ms) {
    if (!ctx || !best) return LCS_ERR_ARG;
    if (flags & ~(uint32_t)(LCS_WANT_TRACEBACK | LCS_USE_GRAPH)) return LCS_ERR_ARG;
    lcs_status st = check_pairs(pairs, count);
    if (st) return st;
    uint8_t lut[256];
    bool valid[256];
    int sigma = 0;
    st = make_lut(alphabet, lut, valid, &sigma);
    if (st) return st;
    if (max_wpl(sigma) == 0) return LCS_ERR_UNSUPPORTED;
    const TuneKey key = tune_key(pairs, count, sigma, flags);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto hit = ctx->tune_cache.find(key);
        if (hit != ctx->tune_cache.end()) {
            *best = hit->second.first;
            if (best_ms) *best_ms = hit->second.second;
            return LCS_OK;
        }
    }
    // one candidate: plan, one untimed pass, then the best of two timed passes
    auto measure = [&](const lcs_tuning &t, float *ms) -> lcs_status {
        lcs_batch *b = nullptr;
        lcs_status s2 = build_batch(ctx, pairs, count, alphabet, flags, &t, &b);
        if (s2) return s2;
        float tot = 0.f, f = 0.f, bestt = 1e30f;
        s2 = lcs_batch_time(b, 0, &tot, &f);
        for (int r = 0; r < 2 && !s2; ++r) {
            s2 = lcs_batch_time(b, 0, &tot, &f);
            bestt = std::min(bestt, tot);
        }
        free_batch(b);
        if (!s2) *ms = bestt;
        return s2;
    };
    lcs_tuning cur{};
    float cur_ms = 1e30f;
    bool any = false;
    auto consider = [&](const lcs_tuning &t) -> lcs_status {
        float ms = 0.f;
        lcs_status s2 = measure(t, &ms);
        if (s2 == LCS_ERR_NOMEM || s2 == LCS_ERR_TOO_LONG || s2 == LCS_ERR_UNSUPPORTED) return LCS_OK;
        if (s2) return s2;
        if (!any || ms < cur_ms) {
            cur = t;
            cur_ms = ms;
            any = true;
        }
        return LCS_OK;
    };
    // words per lane first, then (with tracebacks) the checkpoint interval
    // and the tiles per recompute round
    for (int w : {1, 2, 4, 8}) {
        if (!wpl_fits(sigma, w)) continue;
        lcs_tuning t{};
        t.words_per_lane = w;
        st = consider(t);
        if (st) return st;
    }
    if (!any) return LCS_ERR_NOMEM;
    if (flags & LCS_WANT_TRACEBACK) {
        const lcs_tuning base = cur;
        for (int k : {64, 128}) {
            lcs_tuning t = base;
            t.ckpt_interval = k;
            st = consider(t);
            if (st) return st;
        }
        const lcs_tuning base2 = cur;
        const int K = base2.ckpt_interval ? base2.ckpt_interval : 64;
        const int span = std::max(1, 256 / K);
        for (int nb : {span - 1, span + 1}) {
            if (nb < 1 || nb > 8) continue;
            lcs_tuning t = base2;
            t.tb_tiles = nb;
            t.tb_bands = 2;
            st = consider(t);
            if (st) return st;
        }
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->tune_cache[key] = {cur, cur_ms};
    }
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return LCS_OK;
}

static lcs_status plan_only(const uint64_t *m, const uint64_t *n, uint64_t count,
                            uint16_t alphabet_size, uint32_t flags, const lcs_tuning *tuning,
                            std::vector<PairShape> &shapes, Plan &plan) {
    if (count && (!m || !n)) return LCS_ERR_ARG;
    if (alphabet_size < 1 || alphabet_size > 256) return LCS_ERR_ARG;
    if (flags & ~(uint32_t)(LCS_WANT_TRACEBACK | LCS_USE_GRAPH | LCS_THRESHOLD | LCS_FILL_TRACE))
        return LCS_ERR_ARG;
    if ((flags & LCS_THRESHOLD) && (flags & LCS_WANT_TRACEBACK)) return LCS_ERR_ARG;
    lcs_status st = check_tuning(tuning);
    if (st) return st;
    if (max_wpl(alphabet_size) == 0) return LCS_ERR_UNSUPPORTED;
    if (tuning && tuning->words_per_lane && !wpl_fits(alphabet_size, tuning->words_per_lane))
        return LCS_ERR_UNSUPPORTED;
    shapes.resize(count);
    for (uint64_t k = 0; k < count; ++k) {
        if (m[k] > LCS_MAX_LEN || n[k] > LCS_MAX_LEN) return LCS_ERR_TOO_LONG;
        shapes[k].m = m[k];
        shapes[k].n = n[k];
    }
    PlanConfig cfg;
    fill_plan_config(cfg, alphabet_size, flags, tuning);
    std::string why = build_plan(shapes, cfg, plan);
    if (!why.empty()) return plan_status(why);
    return LCS_OK;
}

extern "C" lcs_status lcs_plan_describe(const uint64_t *m, const uint64_t *n, uint64_t count,
                                        uint16_t alphabet_size, uint32_t flags,
                                        const lcs_tuning *tuning, lcs_batch_stats *out) {
    if (!out) return LCS_ERR_ARG;
    std::vector<PairShape> shapes;
    Plan plan;
    lcs_status st = plan_only(m, n, count, alphabet_size, flags, tuning, shapes, plan);
    if (st) return st;
    stats_from_plan(plan, count, out);
    return LCS_OK;
}

extern "C" lcs_status lcs_plan_selfcheck(const uint64_t *m, const uint64_t *n, uint64_t count,
                                         uint16_t alphabet_size, uint32_t flags,
                                         const lcs_tuning *tuning) {
    std::vector<PairShape> shapes;
    Plan plan;
    lcs_status st = plan_only(m, n, count, alphabet_size, flags, tuning, shapes, plan);
    if (st) return st;
    std::string why = check_plan(shapes, plan);
    if (!why.empty()) {
        std::fprintf(stderr, "lcs_plan_selfcheck: %s\n", why.c_str());
        return LCS_ERR_ARG;
    }
    return LCS_OK;
}
