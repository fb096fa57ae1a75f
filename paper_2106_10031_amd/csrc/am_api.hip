// am_api.hip -- host side of the C ABI declared in include/am.h.
//
// Owns the device copy of the network, the seed buffers and the marching
// state, and drives the step loop of parallel marching (Algorithm 1 with all
// active cells solved at once): chain -> clip -> insert -> commit -> resolve
// per batch of active cells, one small device-to-host read of the counters
// per step to learn the next active range.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/am.h"
#include "am_internal.h"

namespace am {
void launch_clip(const DevNet &, const uint64_t *, const int *, const uint64_t *, const int *, long long, long long,
                 const int *, const unsigned long long *, long long, const double *, const ClipOut &,
                 const Candidates &, unsigned long long, Counters *, const PropArgs &, hipStream_t);
void launch_clip_f32(const DevNet &, const uint64_t *, const int *, const uint64_t *, const int *, long long,
                     long long, long long, const float *, const ClipOut &, const Candidates &, unsigned long long,
                     Counters *, double, double, double, int *, unsigned long long *, const PropArgs &, hipStream_t);
void launch_calib_split(const DevNet &, const uint64_t *, const int *, long long, const double *, const float *,
                        const int *, const int *, const double *, const long long *, unsigned long long *,
                        hipStream_t);
void launch_prop_score(const PropNet &, const float *, long long, float *, hipStream_t);
hipError_t persist_setup(const DevNet &, size_t, int *, size_t *, int *);
void launch_persist(const DevNet &, int, size_t, uint64_t *, int *, int *, uint64_t *, int *, double *, int, long long,
                    const ClipOut &, Counters *, const InlineInsert &, hipStream_t);
long long prop_param_count();
int prop_grad_blocks();
void launch_prop_grad(const float *, const unsigned char *, long long, const float *, float *, float *, double *,
                      hipStream_t);
void launch_prop_adam(float *, const float *, float *, float *, int, float, hipStream_t);
void launch_chain_bf16(const DevNet &, const uint64_t *, const int *, long long, long long, float *, hipStream_t);
void launch_chain(const DevNet &, const uint64_t *, const int *, long long, long long, const int *,
                  const unsigned long long *, double *, int, hipStream_t);
void launch_fused(const DevNet &, const uint64_t *, const int *, const int *, const uint64_t *, const int *, long long,
                  long long, long long, const ClipOut &, const Candidates &, unsigned long long, Counters *,
                  hipStream_t);
size_t fused_lds_bytes(const DevNet &);
hipError_t prepare_fused(size_t);
size_t fused_static_lds_bytes();
size_t chain_res_lds_bytes(const DevNet &);
hipError_t prepare_chain_res(size_t);
int prepare_chain_lb(const DevNet &, size_t);
void launch_rows_unpad(const DevNet &, long long, const void *, bool, double *, hipStream_t);
void launch_insert(const DevNet &, const Candidates &, const CellArrays &, unsigned long long *, unsigned long long,
                   Counters *, unsigned long long, long long, hipStream_t);
void launch_commit(const DevNet &, const Candidates &, uint64_t *, int *, int *, uint64_t *, int *, unsigned *, int *,
                   const uint64_t *, const int *, const int *, unsigned long long *, Counters *, unsigned long long,
                   unsigned long long, long long, hipStream_t);
hipError_t sort_tmp_bytes(long long, size_t *);
void launch_step_begin(Counters *, long long, long long, hipStream_t);
void launch_chain_dev(const DevNet &, const uint64_t *, const int *, Counters *, long long, double *, int,
                      hipStream_t);
void launch_clip_dev(const DevNet &, const uint64_t *, const int *, const uint64_t *, const int *, Counters *,
                     long long, long long, const double *, const ClipOut &, const Candidates &, unsigned long long,
                     const PropArgs &, hipStream_t);
void launch_split_step_dev(const DevNet &, const uint64_t *, const int *, const int *, const uint64_t *, const int *,
                           Counters *, long long, long long, double *, const ClipOut &, const Candidates &,
                           unsigned long long, double, double, double, int *, int, const PropArgs &, hipStream_t);
hipError_t launch_sort_cells(const unsigned *, long long, long long, unsigned *, int *, int *, void *, size_t,
                             hipStream_t);
void launch_resolve(const Candidates &, int *, const long long *, Counters *, unsigned long long, long long, hipStream_t,
                    long long = 0, long long = 0);
void launch_codes(const DevNet &, const double *, const int *, long long, uint64_t *, int *, double *, hipStream_t);
void launch_seed_rays(const DevNet &, const double *, const double *, const int *, long long, double, int, uint64_t *, int *,
                      int *, int *, hipStream_t);
void launch_seed_st(const DevNet &, const double *, const int *, long long, int, uint64_t *, int *, int *, int *,
                    int *, double *, hipStream_t);
size_t seed_st_lds_bytes(const DevNet &);
void launch_seed_cands(const DevNet &, const uint64_t *, const int *, const int *, const int *, long long,
                       const Candidates &, Counters *, unsigned long long, hipStream_t);
hipError_t scan_tmp_bytes(long long, size_t *);
hipError_t launch_fetch(const DevNet &, long long, const int *, const int *, const double *, const int *,
                        const uint64_t *, const int *, const int *, const long long *, int *, int *, long long *,
                        long long *, void *, size_t, long long, long long *, int *, double *, long long *,
                        uint64_t *, int *, int *, hipStream_t);
hipError_t weld_tmp_bytes(long long, size_t *);
hipError_t sorted_fetch_tmp_bytes(long long, size_t *);
size_t qecd_scratch_bytes(long long, long long);
hipError_t run_qecd(const double *, long long, const long long *, long long, const unsigned char *, long long, int,
                    void *, double *, long long *, long long *, long long *, int *, long long *, hipStream_t);
hipError_t launch_fetch_sorted(const DevNet &, long long, const int *, const int *, const double *, const int *,
                               const uint64_t *, const int *, const int *, const long long *, int *, int *, long long *,
                               long long *, void *, size_t, long long, int *, int *, int *, int *, uint64_t *,
                               uint64_t *, long long *, long long *, void *, size_t, long long *, int *, double *,
                               long long *, uint64_t *, int *, int *, hipStream_t);
hipError_t launch_weld(long long, long long, const long long *, const int *, const long long *, const int *,
                       const double *, int, long long, long long *, int *, int *, void *, size_t,
                       unsigned long long *, long long *, double *, hipStream_t);
void launch_triangles(long long, long long, const long long *, const long long *, long long *, long long,
                      hipStream_t);
}  // namespace am

using namespace am;

// ---- scratch of am_faces_noalloc: the FP64 chain rows of one batch of cells.
// One copy per GPU, part of the loaded code object (it lives until the process
// ends).  Host code must not use the array's name as a device address: each
// device's address comes from hipGetSymbolAddress, taken once per device when
// a context is created on it, and only that pointer is passed to kernels.
static constexpr size_t kNoAllocScratchBytes = 32ull << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on `device` (the current device); looked up once.
hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_scratch_ptr[device] = (double *)ptr;
    return hipSuccess;
}

double *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}
}  // namespace

struct am_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    am_allocator alloc{};        // all zero: hipMalloc / hipFree

    // network
    bool loaded = false;
    DevNet dn{};
    double *d_weights = nullptr;
    double *d_wfrag = nullptr;
    float *d_wfrag32 = nullptr;   // the fragments as FP32 when every weight is an FP32 number
    double *d_wcol = nullptr;
    uint16_t *d_wfrag16 = nullptr;
    int *d_fb_list = nullptr;                 // cells the split-BF16 pass hands to FP64
    unsigned long long *d_fb_count = nullptr;
    size_t lds_limit = 0;       // dynamic LDS a workgroup may use
    bool fused_ok = false;      // the fused kernel's rows fit in LDS
    bool prefer_fused = false;  // kernel_path 0 choice (the split path measured faster at width 90)
    double *d_bias = nullptr;
    uint64_t *d_zobrist = nullptr;

    // seeds
    uint64_t *d_seed_codes = nullptr;
    int *d_seed_am = nullptr;
    int *d_seed_status = nullptr;
    int *d_seed_shape = nullptr;
    long long n_seeds = 0;
    long long seed_cap = 0;
    bool seeds_have_status = false;

    // marching state
    long long cap_cells = 0;
    uint64_t *d_codes = nullptr;
    int *d_am = nullptr;
    int *d_shape = nullptr;
    uint64_t *d_hash = nullptr;
    int *d_hints = nullptr;     // [cap][3] lines to clip first (entry edge and its neighbours)
    unsigned *d_cell_key = nullptr;   // [cap] Morton key of each cell's entry edge midpoint
    unsigned *d_key_sorted = nullptr; // [chunk] scratch of the step sort
    int *d_order = nullptr;           // [chunk] a step's cells in key order
    int *d_ids = nullptr;             // [chunk] scratch of the step sort
    char *d_sort_tmp = nullptr;
    size_t sort_tmp = 0;
    int *d_fm = nullptr;
    int *d_fids = nullptr;         // [slot_cap] face corners: edge ids
    double *d_fverts = nullptr;    // [slot_cap][3] vertices
    int *d_fnbr = nullptr;         // [slot_cap] neighbour cells
    long long *d_foff = nullptr;   // [cap] first slot of each cell's face
    unsigned long long slot_cap = 0;
    int *d_fflags = nullptr;
    unsigned long long hcap = 0;
    unsigned long long *d_slots = nullptr;
    unsigned long long cand_cap = 0;
    Candidates cand{};
    long long chunk_cells = 0;
    double *d_rows = nullptr;
    size_t rows_bytes = 0;
    // persistent march: ready flags per cell, the epoch of the current march,
    // and one rows buffer per resident workgroup
    unsigned *d_ready = nullptr;
    long long ready_cap = 0;
    unsigned epoch = 0;
    double *d_prows = nullptr;
    size_t prows_bytes = 0;
    int persist_blocks = 0;      // 0: not set up for the loaded net
    int persist_variant = 0;     // chain of the persistent tile (0 dense, 1/2 ping-pong FP64/FP32 fragments)
    size_t persist_lds = 0;
    Counters *d_ctr = nullptr;
    Counters *h_ctr = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evk[4] = {nullptr, nullptr, nullptr, nullptr};   // per-step kernel timing
    std::vector<hipEvent_t> evs;   // device-driven steps launched directly: 4 per step of a batch

    // fetch scratch
    int *d_has = nullptr;
    int *d_fidx = nullptr;
    long long *d_mcount = nullptr;
    long long *d_voff = nullptr;
    char *d_scan = nullptr;
    size_t scan_bytes = 0;
    long long scan_n = 0;

    // graph of device-driven steps (opts.graph_steps), rebuilt when its key changes
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<long long> graph_key;

    // chain tile: column groups per workgroup by launch size (< 2^11, < 2^13,
    // < 2^15, larger), set by am_tune_chain or am_set_chain_groups
    int chain_g[4] = {1, 1, 1, 1};

    // learned form: scorer weights (FP16 matrices, FP32 vectors), counters,
    // collection buffers (caller-owned) and training scratch
    bool prop_loaded = false;
    long long prop_version = 0;
    PropArgs prop{};
    char *d_prop_w = nullptr;
    unsigned long long *d_prop_stats = nullptr;
    unsigned long long *d_prop_nsamp = nullptr;
    float *d_prop_scratch = nullptr;
    double *d_prop_loss = nullptr;
    double *h_prop_loss = nullptr;

    // weld scratch: union-find parents, root flags, vertex ids, scan space
    long long *d_weld_parent = nullptr;
    int *d_weld_root = nullptr;
    int *d_weld_vid = nullptr;
    char *d_weld_tmp = nullptr;
    size_t weld_tmp = 0;
    long long weld_n = 0;
    unsigned long long *d_weld_unpaired = nullptr;

    // canonical-order fetch scratch (per face)
    long long sf_cap = 0;
    int *d_sf_cell = nullptr, *d_sf_pa = nullptr, *d_sf_pb = nullptr, *d_sf_rank = nullptr;
    uint64_t *d_sf_ka = nullptr, *d_sf_kb = nullptr;
    long long *d_sf_mc = nullptr, *d_sf_vo = nullptr;
    char *d_sf_tmp = nullptr;
    size_t sf_tmp = 0;

    // staging of an AM_HOST fetch (grown when a call needs more)
    char *d_hstage = nullptr;
    size_t hstage_bytes = 0;

    // asynchronous march: the worker thread, its result
    std::thread worker;
    std::atomic<bool> busy{false};
    am_status async_status = AM_OK;
    am_march_stats async_stats{};

    // split-BF16 certificate of the loaded net, measured on a march's first
    // cells (calibrate_split): relative row error per unit of vertex
    // sensitivity, sign-test margin, vertices measured
    bool calib_ok = false;
    double calib_eps = 0.0, calib_margin = 0.0;
    long long calib_vertices = 0;
    unsigned long long *d_calib = nullptr;

    // simplification scratch (grown when a call needs more)
    char *d_qecd = nullptr;
    size_t qecd_bytes = 0;

    // last result
    bool have_result = false;
    long long res_cells = 0, res_faces = 0, res_fverts = 0;
};

namespace {

constexpr long long kChainBucket[3] = {1LL << 11, 1LL << 13, 1LL << 15};
constexpr int kChainVariants = 8;

int chain_groups(const am_ctx *ctx, long long n, int forced) {
    if (forced > 0) return forced;
    int b = 0;
    while (b < 3 && n >= kChainBucket[b]) ++b;
    return ctx->chain_g[b];
}

am_status fail(am_ctx *c, am_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ctx, AM_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

// Device memory of the context: the caller's allocator when one was given to
// am_create, else hipMalloc / hipFree.
template <class T>
void dfree(am_ctx *c, T *&p) {
    if (p) {
        if (c->alloc.release) c->alloc.release(c->alloc.user, (void *)p, c->device, (void *)c->stream);
        else (void)hipFree((void *)p);
    }
    p = nullptr;
}

template <class T>
am_status dalloc(am_ctx *ctx, T *&p, size_t count) {
    dfree(ctx, p);
    if (count == 0) count = 1;
    const size_t bytes = sizeof(T) * count;
    if (ctx->alloc.alloc) {
        p = (T *)ctx->alloc.alloc(ctx->alloc.user, bytes, ctx->device, (void *)ctx->stream);
        if (!p) return fail(ctx, AM_E_OOM, "the caller's allocator returned no memory for %zu bytes", bytes);
        return AM_OK;
    }
    hipError_t e = hipMalloc((void **)&p, bytes);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, AM_E_OOM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    return AM_OK;
}

#define TRY(expr)                    \
    do {                             \
        am_status s_ = (expr);       \
        if (s_ != AM_OK) return s_;  \
    } while (0)

// BF16 bits of a float, rounded to nearest even.
uint16_t bf16_bits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

double bf16_value(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// The captured steps hold device addresses and a copy of the net by value:
// every buffer or net change must drop them before anything is freed.
void drop_graph(am_ctx *c) {
    if (c->graph_exec) {
        if (c->cap_stream) (void)hipStreamSynchronize(c->cap_stream);
        (void)hipGraphExecDestroy(c->graph_exec);
    }
    c->graph_exec = nullptr;
    c->graph_key.clear();
}

void free_march(am_ctx *c) {
    drop_graph(c);
    dfree(c, c->d_ready);
    c->ready_cap = 0;
    dfree(c, c->d_prows);
    c->prows_bytes = 0;
    dfree(c, c->d_codes);
    dfree(c, c->d_am);
    dfree(c, c->d_shape);
    dfree(c, c->d_hash);
    dfree(c, c->d_hints);
    dfree(c, c->d_fm);
    dfree(c, c->d_fids);
    dfree(c, c->d_fverts);
    dfree(c, c->d_fnbr);
    dfree(c, c->d_foff);
    dfree(c, c->d_fflags);
    dfree(c, c->d_slots);
    dfree(c, c->cand.parent);
    dfree(c, c->cand.slot);
    dfree(c, c->cand.unit);
    dfree(c, c->cand.hash);
    dfree(c, c->cand.kind);
    dfree(c, c->cand.ref);
    dfree(c, c->cand.cell);
    dfree(c, c->cand.hint_prev);
    dfree(c, c->cand.hint_next);
    dfree(c, c->cand.key);
    dfree(c, c->d_cell_key);
    dfree(c, c->d_key_sorted);
    dfree(c, c->d_order);
    dfree(c, c->d_ids);
    dfree(c, c->d_sort_tmp);
    dfree(c, c->d_rows);
    dfree(c, c->d_fb_list);
    dfree(c, c->d_fb_count);
    dfree(c, c->d_has);
    dfree(c, c->d_fidx);
    dfree(c, c->d_mcount);
    dfree(c, c->d_voff);
    dfree(c, c->d_scan);
    c->cap_cells = 0;
    c->hcap = 0;
    c->cand_cap = 0;
    c->rows_bytes = 0;
    c->scan_n = 0;
    c->have_result = false;
}

void free_net(am_ctx *c) {
    drop_graph(c);
    dfree(c, c->d_weights);
    dfree(c, c->d_wfrag);
    dfree(c, c->d_wfrag32);
    dfree(c, c->d_wcol);
    dfree(c, c->d_wfrag16);
    dfree(c, c->d_bias);
    dfree(c, c->d_zobrist);
    dfree(c, c->d_seed_codes);
    dfree(c, c->d_seed_am);
    dfree(c, c->d_seed_status);
    dfree(c, c->d_seed_shape);
    c->n_seeds = c->seed_cap = 0;
    c->loaded = false;
}

am_status set_device(am_ctx *ctx) {
    HIPCHK(hipSetDevice(ctx->device));
    return AM_OK;
}

// Sizes every marching buffer for `cells` cells.
am_status ensure_march(am_ctx *ctx, long long cells) {
    if (cells <= ctx->cap_cells && ctx->d_codes) return AM_OK;
    free_march(ctx);
    const DevNet &n = ctx->dn;
    TRY(dalloc(ctx, ctx->d_codes, (size_t)cells * n.W));
    TRY(dalloc(ctx, ctx->d_am, cells));
    TRY(dalloc(ctx, ctx->d_shape, cells));
    TRY(dalloc(ctx, ctx->d_hash, cells));
    TRY(dalloc(ctx, ctx->d_hints, (size_t)cells * 3));
    TRY(dalloc(ctx, ctx->d_fm, cells));
    // face corners: kSlotsPerCell per cell of the capacity on average
    // (faces average about four corners), taken in order as faces are made
    ctx->slot_cap = (unsigned long long)cells * kSlotsPerCell + kMaxPoly;
    TRY(dalloc(ctx, ctx->d_fids, (size_t)ctx->slot_cap));
    TRY(dalloc(ctx, ctx->d_fverts, (size_t)ctx->slot_cap * 3));
    TRY(dalloc(ctx, ctx->d_fnbr, (size_t)ctx->slot_cap));
    TRY(dalloc(ctx, ctx->d_foff, (size_t)cells));
    TRY(dalloc(ctx, ctx->d_fflags, cells));
    unsigned long long h = 1;
    while (h < 2ull * (unsigned long long)cells) h <<= 1;
    ctx->hcap = h;
    TRY(dalloc(ctx, ctx->d_slots, h));
    // rows for one batch of active cells: at most ~1 GiB, at least 4096 cells
    const size_t per_cell = sizeof(double) * 4 * (size_t)n.R;
    long long chunk = (long long)((1ull << 30) / per_cell);
    chunk = std::max<long long>(4096, std::min<long long>(chunk, 1 << 18));
    chunk = (chunk + 3) & ~3LL;
    ctx->chunk_cells = chunk;
    TRY(dalloc(ctx, ctx->d_rows, (size_t)chunk * 4 * n.R));
    TRY(dalloc(ctx, ctx->d_fb_list, chunk));
    TRY(dalloc(ctx, ctx->d_fb_count, 1));
    ctx->rows_bytes = per_cell * chunk;
    // candidates: the seeds, or up to 16 edges per active cell on average
    ctx->cand_cap = (unsigned long long)std::max<long long>(16 * chunk, ctx->seed_cap + 64);
    TRY(dalloc(ctx, ctx->cand.parent, ctx->cand_cap));
    TRY(dalloc(ctx, ctx->cand.slot, ctx->cand_cap));
    TRY(dalloc(ctx, ctx->cand.unit, ctx->cand_cap));
    TRY(dalloc(ctx, ctx->cand.hash, ctx->cand_cap));
    TRY(dalloc(ctx, ctx->cand.kind, ctx->cand_cap));
    TRY(dalloc(ctx, ctx->cand.ref, ctx->cand_cap));
    TRY(dalloc(ctx, ctx->cand.cell, ctx->cand_cap));
    TRY(dalloc(ctx, ctx->cand.hint_prev, ctx->cand_cap));
    TRY(dalloc(ctx, ctx->cand.hint_next, ctx->cand_cap));
    TRY(dalloc(ctx, ctx->cand.key, ctx->cand_cap));
    TRY(dalloc(ctx, ctx->d_cell_key, (size_t)cells));
    TRY(dalloc(ctx, ctx->d_key_sorted, (size_t)chunk));
    TRY(dalloc(ctx, ctx->d_order, (size_t)chunk));
    TRY(dalloc(ctx, ctx->d_ids, (size_t)chunk));
    {
        size_t b = 0;
        HIPCHK(sort_tmp_bytes(chunk, &b));
        TRY(dalloc(ctx, ctx->d_sort_tmp, b));
        ctx->sort_tmp = b;
    }
    ctx->cap_cells = cells;
    return AM_OK;
}

am_status ensure_scan(am_ctx *ctx, long long n) {
    if (n <= ctx->scan_n && ctx->d_scan) return AM_OK;
    TRY(dalloc(ctx, ctx->d_has, n));
    TRY(dalloc(ctx, ctx->d_fidx, n));
    TRY(dalloc(ctx, ctx->d_mcount, n));
    TRY(dalloc(ctx, ctx->d_voff, n));
    size_t b = 0;
    HIPCHK(scan_tmp_bytes(n, &b));
    TRY(dalloc(ctx, ctx->d_scan, b));
    ctx->scan_bytes = b;
    ctx->scan_n = n;
    return AM_OK;
}

}  // namespace

extern "C" {

am_status am_create(am_ctx **out, int device, void *hip_stream, const am_allocator *alloc) {
    if (!out) return AM_E_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return AM_E_HIP;
    if (device < 0 || device >= count) return AM_E_INVALID;
    if (alloc && (!alloc->alloc) != (!alloc->release)) return AM_E_INVALID;   // both or neither
    am_ctx *ctx = new am_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (alloc) ctx->alloc = *alloc;
    if (hipSetDevice(device) != hipSuccess || hipHostMalloc((void **)&ctx->h_ctr, sizeof(Counters)) != hipSuccess ||
        dalloc(ctx, ctx->d_ctr, 1) != AM_OK ||
        hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
        hipEventCreate(&ctx->evk[0]) != hipSuccess || hipEventCreate(&ctx->evk[1]) != hipSuccess ||
        hipEventCreate(&ctx->evk[2]) != hipSuccess || hipEventCreate(&ctx->evk[3]) != hipSuccess) {
        am_destroy(ctx);
        return AM_E_HIP;
    }
    if (noalloc_scratch_init(device) != hipSuccess) {
        am_destroy(ctx);
        return AM_E_HIP;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 65536;
    ctx->lds_limit = (size_t)lds;
    ctx->prop.k = kPropK;
    ctx->prop.rho = 6.f;
    *out = ctx;
    return AM_OK;
}

void am_destroy(am_ctx *ctx) {
    if (!ctx) return;
    if (ctx->worker.joinable()) ctx->worker.join();
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    drop_graph(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    ctx->cap_stream = nullptr;
    free_march(ctx);
    free_net(ctx);
    dfree(ctx, ctx->d_prop_w);
    dfree(ctx, ctx->d_prop_stats);
    dfree(ctx, ctx->d_prop_nsamp);
    dfree(ctx, ctx->d_prop_scratch);
    dfree(ctx, ctx->d_prop_loss);
    dfree(ctx, ctx->d_weld_parent);
    dfree(ctx, ctx->d_weld_root);
    dfree(ctx, ctx->d_weld_vid);
    dfree(ctx, ctx->d_weld_tmp);
    dfree(ctx, ctx->d_weld_unpaired);
    dfree(ctx, ctx->d_sf_cell);
    dfree(ctx, ctx->d_sf_pa);
    dfree(ctx, ctx->d_sf_pb);
    dfree(ctx, ctx->d_sf_rank);
    dfree(ctx, ctx->d_sf_ka);
    dfree(ctx, ctx->d_sf_kb);
    dfree(ctx, ctx->d_sf_mc);
    dfree(ctx, ctx->d_sf_vo);
    dfree(ctx, ctx->d_sf_tmp);
    dfree(ctx, ctx->d_qecd);
    dfree(ctx, ctx->d_hstage);
    dfree(ctx, ctx->d_calib);
    if (ctx->h_prop_loss) (void)hipHostFree(ctx->h_prop_loss);
    dfree(ctx, ctx->d_ctr);
    if (ctx->h_ctr) (void)hipHostFree(ctx->h_ctr);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    for (auto &e : ctx->evk)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : ctx->evs)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

const char *am_last_error(const am_ctx *ctx) {
    if (!ctx) return "null context";
    if (ctx->busy) return "an asynchronous march is running on this context (am_wait)";
    return ctx->err.c_str();
}

static am_status load_impl(am_ctx *ctx, const am_net_desc *nd, int n_shapes, const double *shape_bias);

am_status am_load_net(am_ctx *ctx, const am_net_desc *nd) { return load_impl(ctx, nd, 1, nullptr); }

am_status am_load_batch(am_ctx *ctx, const am_net_desc *nd, int32_t n_shapes, const double *shape_bias) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (n_shapes < 1 || !shape_bias) return fail(ctx, AM_E_INVALID, "need n_shapes >= 1 and a bias table");
    return load_impl(ctx, nd, n_shapes, shape_bias);
}

static am_status load_impl(am_ctx *ctx, const am_net_desc *nd, int n_shapes, const double *shape_bias) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!nd || !nd->width || nd->n_layers < 2 || nd->n_layers > kMaxLayers || nd->n_blocks < 1 ||
        nd->n_blocks > kMaxBlocks || !nd->blk_dst || !nd->blk_src || !nd->blk_w || !nd->bias)
        return fail(ctx, AM_E_INVALID, "bad network descriptor (layers 2..%d, blocks 1..%d)", kMaxLayers,
                    kMaxBlocks);
    TRY(set_device(ctx));
    const int L2 = nd->n_layers;
    if (nd->width[0] != 3) return fail(ctx, AM_E_INVALID, "width[0] must be 3");
    if (nd->dtype != AM_F64 && nd->dtype != AM_F32) return fail(ctx, AM_E_INVALID, "dtype must be AM_F64 or AM_F32");
    if (nd->n_heads != 0 && nd->n_heads != nd->width[L2 - 1])
        return fail(ctx, AM_E_INVALID, "n_heads %d differs from the head layer's width %d", nd->n_heads,
                    nd->width[L2 - 1]);
    const bool f32src = nd->dtype == AM_F32;
    // element i of a source array, widened exactly to FP64
    auto src_at = [f32src](const void *a, size_t i) {
        return f32src ? (double)((const float *)a)[i] : ((const double *)a)[i];
    };
    for (int l = 1; l < L2; ++l)
        if (nd->width[l] < 1) return fail(ctx, AM_E_INVALID, "width[%d] < 1", l);
    long long N = 0;
    for (int l = 1; l < L2 - 1; ++l) N += nd->width[l];
    const int M = nd->width[L2 - 1];
    if (N > kMaxHidden) return fail(ctx, AM_E_INVALID, "N = %lld hidden units exceeds %d", N, kMaxHidden);
    if (M > kMaxHeads) return fail(ctx, AM_E_INVALID, "M = %d heads exceeds %d", M, kMaxHeads);
    std::vector<int> has_input(L2, 0);
    for (int b = 0; b < nd->n_blocks; ++b) {
        const int d = nd->blk_dst[b], s = nd->blk_src[b];
        if (!(0 <= s && s < d && d < L2)) return fail(ctx, AM_E_INVALID, "block %d: %d <- %d not feed-forward", b, d, s);
        if (!nd->blk_w[b]) return fail(ctx, AM_E_INVALID, "block %d has no weights", b);
        for (int b2 = 0; b2 < b; ++b2)
            if (nd->blk_dst[b2] == d && nd->blk_src[b2] == s)
                return fail(ctx, AM_E_INVALID, "duplicate block %d <- %d", d, s);
        has_input[d] = 1;
    }
    for (int l = 1; l < L2; ++l) {
        if (!has_input[l]) return fail(ctx, AM_E_INVALID, "layer %d has no input block", l);
        if (!shape_bias && !nd->bias[l]) return fail(ctx, AM_E_INVALID, "layer %d has no bias", l);
    }

    free_march(ctx);
    free_net(ctx);
    DevNet dn{};
    dn.n_layers = L2;
    dn.N = (int)N;
    dn.M = M;
    dn.W = std::max(1, (int)((N + 63) / 64));
    int row = 0, unit = 0, boff = 0;
    for (int l = 0; l < L2; ++l) {
        dn.width[l] = nd->width[l];
        if (l == 0) continue;
        dn.row_off[l] = row;
        dn.unit_off[l] = unit;
        dn.bias_off[l] = boff;
        row += nd->width[l];   // rows are indexed by unit
        unit += nd->width[l];
        boff += nd->width[l];
    }
    dn.R = row;
    // weights: each block padded to 16-row multiples and ld = 4-column multiples
    std::vector<double> hw;
    dn.n_blocks = nd->n_blocks;
    for (int b = 0; b < nd->n_blocks; ++b) {
        const int d = nd->blk_dst[b], s = nd->blk_src[b];
        const int nd_ = nd->width[d], ns = nd->width[s];
        const int ld = (ns + 3) & ~3, rows = (nd_ + 15) & ~15;
        dn.blk_dst[b] = d;
        dn.blk_src[b] = s;
        dn.blk_ld[b] = ld;
        dn.blk_off[b] = (long long)hw.size();
        hw.resize(hw.size() + (size_t)rows * ld, 0.0);
        double *dst = hw.data() + dn.blk_off[b];
        const void *src = nd->blk_w[b];
        for (int i = 0; i < nd_; ++i)
            for (int k = 0; k < ns; ++k) {
                const double w = src_at(src, (size_t)i * ns + k);
                if (!std::isfinite(w)) return fail(ctx, AM_E_INVALID, "block %d has a non-finite weight", b);
                dst[(size_t)i * ld + k] = w;
            }
    }
    // MFMA A fragments: per block, per 16-row tile, per K-step, 64 doubles in lane order
    std::vector<double> hf;
    for (int b = 0; b < nd->n_blocks; ++b) {
        const int ld = dn.blk_ld[b], rows = (nd->width[dn.blk_dst[b]] + 15) & ~15;
        const double *Wp = hw.data() + dn.blk_off[b];
        dn.blk_frag_off[b] = (long long)hf.size();
        for (int mt = 0; mt < rows / 16; ++mt)
            for (int ks = 0; ks < ld / 4; ++ks)
                for (int l = 0; l < 64; ++l) hf.push_back(Wp[(size_t)(mt * 16 + l % 16) * ld + ks * 4 + l / 16]);
    }
    // column-major copy of every block (rows padded to 16) for the gathered chain
    std::vector<double> hc;
    for (int b = 0; b < nd->n_blocks; ++b) {
        const int ld = dn.blk_ld[b], rows = (nd->width[dn.blk_dst[b]] + 15) & ~15, ns = nd->width[dn.blk_src[b]];
        const double *Wp = hw.data() + dn.blk_off[b];
        dn.blk_col_off[b] = (long long)hc.size();
        for (int k = 0; k < ns; ++k)
            for (int i = 0; i < rows; ++i) hc.push_back(Wp[(size_t)i * ld + k]);
    }
    // bias table [S][boff]: the net's own biases, or one row per shape
    // split-BF16 fragments (blocks from the input are copies and get none)
    std::vector<uint16_t> h16;
    for (int b = 0; b < nd->n_blocks; ++b) {
        const int d = dn.blk_dst[b], sr = dn.blk_src[b];
        const int nd_ = nd->width[d], ns = nd->width[sr];
        const int ld32 = (ns + 31) & ~31, rows16 = (nd_ + 15) & ~15;
        dn.blk_ld32[b] = ld32;
        dn.blk_frag16_off[b] = (long long)(h16.size() / 8);
        if (sr == 0) continue;
        const void *src = nd->blk_w[b];
        for (int mt = 0; mt < rows16 / 16; ++mt)
            for (int ks = 0; ks < ld32 / 32; ++ks)
                for (int t = 0; t < 3; ++t)
                    for (int l = 0; l < 64; ++l)
                        for (int u = 0; u < 8; ++u) {
                            const int i = mt * 16 + l % 16, k = ks * 32 + 8 * (l / 16) + u;
                            double w = (i < nd_ && k < ns) ? src_at(src, (size_t)i * ns + k) : 0.0;
                            uint16_t term = 0;
                            for (int tt = 0; tt <= t; ++tt) {   // w = h + m + l, each the rounded remainder
                                term = bf16_bits((float)w);
                                w -= bf16_value(term);
                            }
                            h16.push_back(term);
                        }
    }
    std::vector<double> hb((size_t)n_shapes * boff);
    for (int sh = 0; sh < n_shapes; ++sh)
        for (int l = 1; l < L2; ++l)
            for (int k = 0; k < nd->width[l]; ++k) {
                const double v = shape_bias ? shape_bias[(size_t)sh * boff + dn.bias_off[l] + k] : src_at(nd->bias[l], k);
                if (!std::isfinite(v)) return fail(ctx, AM_E_INVALID, "bias of shape %d layer %d is not finite", sh, l);
                hb[(size_t)sh * boff + dn.bias_off[l] + k] = v;
            }
    dn.S = n_shapes;
    dn.bias_stride = boff;
    std::vector<uint64_t> zob(N + M + n_shapes);
    uint64_t sm = 0x5eed0fa11c0de5ull;
    for (auto &z : zob) z = splitmix64(sm);

    // FP32 copy of the fragments when it is exact (fitted nets are stored in FP32)
    bool all_f32 = true;
    for (double w : hf)
        if ((double)(float)w != w) {
            all_f32 = false;
            break;
        }
    if (all_f32) {
        std::vector<float> hf32(hf.begin(), hf.end());
        TRY(dalloc(ctx, ctx->d_wfrag32, hf32.size()));
        HIPCHK(hipMemcpy(ctx->d_wfrag32, hf32.data(), sizeof(float) * hf32.size(), hipMemcpyHostToDevice));
    }
    {
        int wmax = 0;
        for (int l = 1; l < L2 - 1; ++l) wmax = std::max(wmax, nd->width[l]);
        dn.lb_kpad = (wmax + 31) & ~31;
    }
    TRY(dalloc(ctx, ctx->d_weights, hw.size()));
    TRY(dalloc(ctx, ctx->d_wfrag, hf.size()));
    TRY(dalloc(ctx, ctx->d_wcol, hc.size()));
    HIPCHK(hipMemcpy(ctx->d_wcol, hc.data(), sizeof(double) * hc.size(), hipMemcpyHostToDevice));
    TRY(dalloc(ctx, ctx->d_wfrag16, h16.size()));
    HIPCHK(hipMemcpy(ctx->d_wfrag16, h16.data(), sizeof(uint16_t) * h16.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_wfrag, hf.data(), sizeof(double) * hf.size(), hipMemcpyHostToDevice));
    TRY(dalloc(ctx, ctx->d_bias, hb.size()));
    TRY(dalloc(ctx, ctx->d_zobrist, zob.size()));
    HIPCHK(hipMemcpy(ctx->d_weights, hw.data(), sizeof(double) * hw.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_bias, hb.data(), sizeof(double) * hb.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_zobrist, zob.data(), sizeof(uint64_t) * zob.size(), hipMemcpyHostToDevice));
    dn.weights = ctx->d_weights;
    dn.wfrag = ctx->d_wfrag;
    dn.wfrag32 = ctx->d_wfrag32;
    dn.wcol = ctx->d_wcol;
    dn.wfrag16 = ctx->d_wfrag16;
    dn.bias = ctx->d_bias;
    dn.zobrist = ctx->d_zobrist;
    ctx->calib_ok = false;   // the split-BF16 certificate is measured per net
    ctx->persist_blocks = 0;  // the persistent tile is chosen per net
    dn.lb_ok = prepare_chain_lb(dn, ctx->lds_limit);
    (void)hipGetLastError();
    ctx->dn = dn;
    // the fused kernel keeps the rows of four cells in LDS next to 4 x 1.75 KiB of clip scratch
    const size_t fb = fused_lds_bytes(dn);
    ctx->fused_ok = fb + fused_static_lds_bytes() <= ctx->lds_limit && prepare_fused(fb) == hipSuccess;
    {
        const size_t rb = chain_res_lds_bytes(ctx->dn);
        if (rb > 0 && prepare_chain_res(rb) != hipSuccess) return fail(ctx, AM_E_HIP, "chain LDS attribute failed");
    }
    (void)hipGetLastError();
    ctx->loaded = true;
    return AM_OK;
}

am_status am_net_dims(const am_ctx *ctx, int32_t *n_hidden, int32_t *n_heads, int32_t *code_words,
                      int32_t *n_shapes) {
    if (!ctx || !ctx->loaded) return AM_E_STATE;
    if (n_shapes) *n_shapes = ctx->dn.S;
    if (n_hidden) *n_hidden = ctx->dn.N;
    if (n_heads) *n_heads = ctx->dn.M;
    if (code_words) *code_words = ctx->dn.W;
    return AM_OK;
}

am_status am_codes(am_ctx *ctx, const double *pts, const int32_t *shape_id, int64_t n, uint64_t *codes,
                   int32_t *argmax, double *F) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->loaded) return fail(ctx, AM_E_STATE, "no network loaded");
    if (n < 0 || (n > 0 && !pts)) return fail(ctx, AM_E_INVALID, "bad points");
    TRY(set_device(ctx));
    launch_codes(ctx->dn, pts, shape_id, n, codes, argmax, F, ctx->stream);
    HIPCHK(hipGetLastError());
    return AM_OK;
}

am_status am_chain(am_ctx *ctx, const uint64_t *codes, const int32_t *shape_id, int64_t n, int32_t precision,
                   double *rows) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->loaded) return fail(ctx, AM_E_STATE, "no network loaded");
    if (n < 0 || (n > 0 && (!codes || !rows)) || precision < 0 || precision > 1)
        return fail(ctx, AM_E_INVALID, "bad arguments");
    TRY(set_device(ctx));
    TRY(ensure_march(ctx, std::max<long long>(ctx->cap_cells, 1024)));
    for (long long lo = 0; lo < n; lo += ctx->chunk_cells) {
        const long long hi = std::min<long long>(n, lo + ctx->chunk_cells);
        if (precision == 1) {
            launch_chain_bf16(ctx->dn, codes, shape_id, lo, hi, (float *)ctx->d_rows, ctx->stream);
            launch_rows_unpad(ctx->dn, hi - lo, ctx->d_rows, true, rows + lo * 4 * (ctx->dn.N + ctx->dn.M),
                              ctx->stream);
        } else {
            launch_chain(ctx->dn, codes, shape_id, lo, hi, nullptr, nullptr, ctx->d_rows,
                     chain_groups(ctx, hi - lo, 0), ctx->stream);
            launch_rows_unpad(ctx->dn, hi - lo, ctx->d_rows, false, rows + lo * 4 * (ctx->dn.N + ctx->dn.M),
                              ctx->stream);
        }
    }
    HIPCHK(hipGetLastError());
    return AM_OK;
}

am_status am_faces(am_ctx *ctx, const uint64_t *codes, const int32_t *argmax, const int32_t *shape_id, int64_t n,
                   int32_t max_m, int32_t *m, int32_t *ids, double *verts, int32_t *flags) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->loaded) return fail(ctx, AM_E_STATE, "no network loaded");
    if (n < 0 || max_m < 3 || max_m > kMaxPoly || (n > 0 && (!codes || !m || !ids || !verts)))
        return fail(ctx, AM_E_INVALID, "bad arguments (max_m must be 3..%d)", kMaxPoly);
    TRY(set_device(ctx));
    TRY(ensure_march(ctx, std::max<long long>(ctx->cap_cells, 1024)));
    for (long long lo = 0; lo < n; lo += ctx->chunk_cells) {
        const long long hi = std::min<long long>(n, lo + ctx->chunk_cells);
        launch_chain(ctx->dn, codes, shape_id, lo, hi, nullptr, nullptr, ctx->d_rows,
                     chain_groups(ctx, hi - lo, 0), ctx->stream);
        ClipOut out{};
        out.m = m;
        out.ids = ids;
        out.verts = verts;
        out.nbr = nullptr;
        out.flags = flags;
        out.stride = max_m;
        out.out_base = 0;
        Candidates none{};
        launch_clip(ctx->dn, codes, argmax, nullptr, nullptr, lo, hi, nullptr, nullptr, 0, ctx->d_rows, out, none, 0,
                    nullptr, PropArgs{}, ctx->stream);
    }
    HIPCHK(hipGetLastError());
    return AM_OK;
}

am_status am_faces_noalloc(am_ctx *ctx, const uint64_t *codes, const int32_t *argmax, const int32_t *shape_id,
                           int64_t n, int32_t max_m, int32_t *m, int32_t *ids, double *verts, int32_t *flags) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->loaded) return fail(ctx, AM_E_STATE, "no network loaded");
    if (n < 0 || max_m < 3 || max_m > kMaxPoly || (n > 0 && (!codes || !m || !ids || !verts)))
        return fail(ctx, AM_E_INVALID, "bad arguments (max_m must be 3..%d)", kMaxPoly);
    const size_t per_cell = sizeof(double) * 4 * (size_t)ctx->dn.R;
    const long long batch = (long long)(kNoAllocScratchBytes / per_cell);
    if (batch < 1)
        return fail(ctx, AM_E_INVALID,
                    "am_faces_noalloc: the rows of one cell need %zu bytes, more than its %zu-byte scratch",
                    per_cell, kNoAllocScratchBytes);
    TRY(set_device(ctx));
    double *rows = noalloc_scratch(ctx->device);
    if (!rows) return fail(ctx, AM_E_STATE, "am_faces_noalloc: no scratch address for device %d", ctx->device);
    for (long long lo = 0; lo < n; lo += batch) {
        const long long hi = std::min<long long>(n, lo + batch);
        launch_chain(ctx->dn, codes, shape_id, lo, hi, nullptr, nullptr, rows, chain_groups(ctx, hi - lo, 0),
                     ctx->stream);
        ClipOut out{};
        out.m = m;
        out.ids = ids;
        out.verts = verts;
        out.nbr = nullptr;
        out.flags = flags;
        out.stride = max_m;
        out.out_base = 0;
        Candidates none{};
        launch_clip(ctx->dn, codes, argmax, nullptr, nullptr, lo, hi, nullptr, nullptr, 0, rows, out, none, 0,
                    nullptr, PropArgs{}, ctx->stream);
    }
    HIPCHK(hipGetLastError());
    return AM_OK;
}

static am_status ensure_seed_cap(am_ctx *ctx, long long n) {
    if (n <= ctx->seed_cap && ctx->d_seed_codes) return AM_OK;
    TRY(dalloc(ctx, ctx->d_seed_codes, (size_t)n * ctx->dn.W));
    TRY(dalloc(ctx, ctx->d_seed_am, n));
    TRY(dalloc(ctx, ctx->d_seed_status, n));
    TRY(dalloc(ctx, ctx->d_seed_shape, n));
    ctx->seed_cap = n;
    return AM_OK;
}

am_status am_seed_rays(am_ctx *ctx, const double *orig, const double *dir, const int32_t *shape_id, int64_t n_rays,
                       double t_max, int32_t max_iter, int32_t *status_out) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->loaded) return fail(ctx, AM_E_STATE, "no network loaded");
    if (n_rays <= 0 || !orig || !dir) return fail(ctx, AM_E_INVALID, "need at least one ray");
    TRY(set_device(ctx));
    TRY(ensure_seed_cap(ctx, n_rays));
    if (!std::isfinite(t_max)) return fail(ctx, AM_E_INVALID, "t_max must be finite");
    launch_seed_rays(ctx->dn, orig, dir, shape_id, n_rays, t_max > 0.0 ? t_max : 1.0, max_iter > 0 ? max_iter : 200,
                     ctx->d_seed_codes,
                     ctx->d_seed_am, ctx->d_seed_shape, ctx->d_seed_status, ctx->stream);
    if (status_out)
        HIPCHK(hipMemcpyAsync(status_out, ctx->d_seed_status, sizeof(int) * n_rays, hipMemcpyDeviceToDevice,
                              ctx->stream));
    HIPCHK(hipGetLastError());
    ctx->n_seeds = n_rays;
    ctx->seeds_have_status = true;
    ctx->have_result = false;
    return AM_OK;
}

am_status am_seed_points_st(am_ctx *ctx, const double *pts, const int32_t *shape_id, int64_t n, int32_t max_iter,
                            int32_t *status_out, int32_t *iters_out, double *x_out) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->loaded) return fail(ctx, AM_E_STATE, "no network loaded");
    if (n <= 0 || !pts) return fail(ctx, AM_E_INVALID, "need at least one start point");
    if (max_iter < 0 || max_iter > 100000) return fail(ctx, AM_E_INVALID, "max_iter must be 0..100000");
    if (seed_st_lds_bytes(ctx->dn) > ctx->lds_limit)
        return fail(ctx, AM_E_INVALID, "sphere tracing needs %zu bytes of LDS (limit %zu)",
                    seed_st_lds_bytes(ctx->dn), ctx->lds_limit);
    TRY(set_device(ctx));
    TRY(ensure_seed_cap(ctx, n));
    launch_seed_st(ctx->dn, pts, shape_id, n, max_iter > 0 ? max_iter : 64, ctx->d_seed_codes, ctx->d_seed_am,
                   ctx->d_seed_shape, ctx->d_seed_status, iters_out, x_out, ctx->stream);
    if (status_out)
        HIPCHK(hipMemcpyAsync(status_out, ctx->d_seed_status, sizeof(int) * n, hipMemcpyDeviceToDevice,
                              ctx->stream));
    HIPCHK(hipGetLastError());
    ctx->n_seeds = n;
    ctx->seeds_have_status = true;
    ctx->have_result = false;
    return AM_OK;
}

am_status am_seed_cells(am_ctx *ctx, const uint64_t *codes, const int32_t *argmax, const int32_t *shape_id,
                        int64_t n) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->loaded) return fail(ctx, AM_E_STATE, "no network loaded");
    if (n <= 0 || !codes) return fail(ctx, AM_E_INVALID, "need at least one seed cell");
    TRY(set_device(ctx));
    TRY(ensure_seed_cap(ctx, n));
    HIPCHK(hipMemcpyAsync(ctx->d_seed_codes, codes, sizeof(uint64_t) * n * ctx->dn.W, hipMemcpyDeviceToDevice,
                          ctx->stream));
    if (argmax)
        HIPCHK(hipMemcpyAsync(ctx->d_seed_am, argmax, sizeof(int) * n, hipMemcpyDeviceToDevice, ctx->stream));
    else
        HIPCHK(hipMemsetAsync(ctx->d_seed_am, 0, sizeof(int) * n, ctx->stream));
    if (shape_id)
        HIPCHK(hipMemcpyAsync(ctx->d_seed_shape, shape_id, sizeof(int) * n, hipMemcpyDeviceToDevice, ctx->stream));
    else
        HIPCHK(hipMemsetAsync(ctx->d_seed_shape, 0, sizeof(int) * n, ctx->stream));
    ctx->n_seeds = n;
    ctx->seeds_have_status = false;
    ctx->have_result = false;
    return AM_OK;
}

am_status am_seed_points(am_ctx *ctx, const double *pts, const int32_t *shape_id, int64_t n) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->loaded) return fail(ctx, AM_E_STATE, "no network loaded");
    if (n <= 0 || !pts) return fail(ctx, AM_E_INVALID, "need at least one seed point");
    TRY(set_device(ctx));
    TRY(ensure_seed_cap(ctx, n));
    launch_codes(ctx->dn, pts, shape_id, n, ctx->d_seed_codes, ctx->d_seed_am, nullptr, ctx->stream);
    HIPCHK(hipGetLastError());
    if (shape_id)
        HIPCHK(hipMemcpyAsync(ctx->d_seed_shape, shape_id, sizeof(int) * n, hipMemcpyDeviceToDevice, ctx->stream));
    else
        HIPCHK(hipMemsetAsync(ctx->d_seed_shape, 0, sizeof(int) * n, ctx->stream));
    ctx->n_seeds = n;
    ctx->seeds_have_status = false;
    ctx->have_result = false;
    return AM_OK;
}

static am_status march_impl(am_ctx *ctx, const am_march_opts *opts, am_march_stats *stats);

am_status am_march(am_ctx *ctx, const am_march_opts *opts, am_march_stats *stats) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (ctx->worker.joinable()) ctx->worker.join();   // an asynchronous march nobody waited for
    if (opts && opts->async) {
        const am_march_opts o = *opts;
        ctx->busy = true;
        ctx->worker = std::thread([ctx, o]() {
            am_march_stats st{};
            const am_status r = march_impl(ctx, &o, &st);
            ctx->async_stats = st;
            ctx->async_status = r;
            ctx->busy = false;
        });
        return AM_OK;
    }
    return march_impl(ctx, opts, stats);
}

am_status am_wait(am_ctx *ctx, am_march_stats *stats) {
    if (!ctx) return AM_E_INVALID;
    if (!ctx->worker.joinable()) {
        if (stats) *stats = am_march_stats{};
        return fail(ctx, AM_E_STATE, "no asynchronous march to wait for");
    }
    ctx->worker.join();
    if (stats) *stats = ctx->async_stats;
    return ctx->async_status;
}

am_status am_busy(const am_ctx *ctx, int32_t *busy) {
    if (!ctx || !busy) return AM_E_INVALID;
    *busy = ctx->busy ? 1 : 0;
    return AM_OK;
}

// Measures the split-BF16 certificate's constants for the loaded net on the
// first n (<= chunk / 2) cells of the march: their FP64 rows and faces (at the
// start of the rows and face buffers, which the march overwrites) against
// their FP32 rows (k_calib_split).  row_eps = 8 x the largest ratio of vertex
// error to first-order sensitivity, margin = 8 x the largest sign-test error
// of a row at a vertex relative to |c|_1 (1 + |v|_inf); with fewer than 512
// vertices measured, at least 5e-6 and 1.6e-5.
static am_status calibrate_split(am_ctx *ctx, long long n) {
    const DevNet &net = ctx->dn;
    hipStream_t s = ctx->stream;
    if (!ctx->d_calib) TRY(dalloc(ctx, ctx->d_calib, 4));
    double *r64 = ctx->d_rows;
    float *r32 = (float *)(ctx->d_rows + (size_t)n * net.R * 4);
    HIPCHK(hipMemsetAsync(ctx->d_calib, 0, 4 * sizeof(unsigned long long), s));
    launch_chain(net, ctx->d_codes, ctx->d_shape, 0, n, nullptr, nullptr, r64, 1, s);
    ClipOut out{};
    out.m = ctx->d_fm;
    out.ids = ctx->d_fids;
    out.verts = ctx->d_fverts;
    out.nbr = nullptr;
    out.flags = ctx->d_fflags;
    out.stride = kMaxPoly;
    out.out_base = 0;
    out.off = ctx->d_foff;
    out.slot_n = ctx->d_calib + 3;   // its own slot counter: the march's starts at 0
    out.slot_cap = ctx->slot_cap;
    const Candidates none{};
    launch_clip(net, ctx->d_codes, ctx->d_am, nullptr, nullptr, 0, n, nullptr, nullptr, 0, r64, out, none, 0, nullptr,
                PropArgs{}, s);
    launch_chain_bf16(net, ctx->d_codes, ctx->d_shape, 0, n, r32, s);
    launch_calib_split(net, ctx->d_codes, ctx->d_am, n, r64, r32, ctx->d_fm, ctx->d_fids, ctx->d_fverts, ctx->d_foff,
                       ctx->d_calib, s);
    unsigned long long h[3] = {0, 0, 0};
    HIPCHK(hipMemcpyAsync(h, ctx->d_calib, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    double ratio = 0.0, marg = 0.0;
    memcpy(&ratio, &h[0], sizeof ratio);
    memcpy(&marg, &h[1], sizeof marg);
    ctx->calib_vertices = (long long)h[2];
    ctx->calib_eps = std::max(1e-7, 8.0 * ratio);
    ctx->calib_margin = std::max(1e-7, 8.0 * marg);
    if (ctx->calib_vertices < 512) {
        ctx->calib_eps = std::max(ctx->calib_eps, 5e-6);
        ctx->calib_margin = std::max(ctx->calib_margin, 1.6e-5);
    }
    ctx->calib_ok = true;
    return AM_OK;
}

static am_status march_impl(am_ctx *ctx, const am_march_opts *opts, am_march_stats *stats) {
    if (!ctx->loaded) return fail(ctx, AM_E_STATE, "no network loaded");
    if (ctx->n_seeds <= 0) return fail(ctx, AM_E_STATE, "no seeds");
    TRY(set_device(ctx));
    am_march_opts o{};
    if (opts) o = *opts;
    const long long cap = o.max_cells > 0 ? o.max_cells : (1LL << 20);
    if (cap >= (1LL << 31)) return fail(ctx, AM_E_INVALID, "max_cells must be < 2^31");
    if (cap < ctx->n_seeds) return fail(ctx, AM_E_INVALID, "max_cells smaller than the seed count");
    TRY(ensure_march(ctx, cap));
    if (ctx->cand_cap < (unsigned long long)ctx->n_seeds) {
        ctx->cap_cells = 0;   // force a re-size with room for the seeds
        TRY(ensure_march(ctx, cap));
    }
    if (o.kernel_path < 0 || o.kernel_path > 3) return fail(ctx, AM_E_INVALID, "kernel_path must be 0..3");
    if (o.wait_limit < 0) return fail(ctx, AM_E_INVALID, "wait_limit must be >= 0");
    const bool persistent = o.kernel_path == 3;
    if (persistent && (o.precision != 0 || o.propose != 0 || ctx->prop.samples || o.face_routine != 0 ||
                       o.graph_steps != 0 || o.max_steps != 0))
        return fail(ctx, AM_E_INVALID, "the persistent march runs the plain FP64 form (no precision, proposals, "
                                       "sample collection, pivoting, graph_steps or max_steps)");
    if (o.precision < 0 || o.precision > 1) return fail(ctx, AM_E_INVALID, "precision must be 0 or 1");
    if (o.precision == 1 && o.kernel_path == 2)
        return fail(ctx, AM_E_INVALID, "the split-BF16 form runs on the split path");
    if (o.kernel_path == 2 && !ctx->fused_ok)
        return fail(ctx, AM_E_INVALID, "the fused kernel needs %zu bytes of LDS (limit %zu)",
                    fused_lds_bytes(ctx->dn) + fused_static_lds_bytes(), ctx->lds_limit);
    if (o.propose < 0 || o.propose > 3) return fail(ctx, AM_E_INVALID, "propose must be 0..3");
    if (o.chain_groups < 0 || o.chain_groups > kChainVariants)
        return fail(ctx, AM_E_INVALID, "chain_groups must be 0..%d", kChainVariants);
    if (o.graph_steps < 0 || o.graph_steps > 64) return fail(ctx, AM_E_INVALID, "graph_steps must be 0..64");
    if (o.graph_steps > 0 && (ctx->prop.samples || o.kernel_path == 2))
        return fail(ctx, AM_E_INVALID, "device-driven steps run the split path without sample collection");
    if (o.face_routine < 0 || o.face_routine > 1) return fail(ctx, AM_E_INVALID, "face_routine must be 0 or 1");
    if (o.face_routine == 1 && (o.precision != 0 || o.propose != 0 || ctx->prop.samples || o.kernel_path == 2 ||
                                o.graph_steps > 0))
        return fail(ctx, AM_E_INVALID, "pivoting runs the plain FP64 split path with host-driven steps");
    if (o.propose == 1 && !ctx->prop_loaded) return fail(ctx, AM_E_STATE, "no proposal scorer loaded");
    const bool collecting = ctx->prop.samples != nullptr;
    if ((o.propose != 0 || collecting) && o.kernel_path == 2)
        return fail(ctx, AM_E_INVALID, "proposals and sample collection run on the split path");
    const bool fused = !persistent && o.precision == 0 && o.propose == 0 && !collecting &&
                       (o.kernel_path == 2 || (o.kernel_path == 0 && ctx->prefer_fused && ctx->fused_ok));
    PropArgs pa = ctx->prop;
    pa.mode = o.propose;
    pa.face_routine = o.face_routine;
    if (o.propose != 0) {
        if (!ctx->d_prop_stats) TRY(dalloc(ctx, ctx->d_prop_stats, (size_t)kPropStats * kPropSlots));
        pa.stats = ctx->d_prop_stats;
        HIPCHK(hipMemsetAsync(ctx->d_prop_stats, 0, sizeof(unsigned long long) * kPropStats * kPropSlots,
                              ctx->stream));
    } else {
        pa.stats = nullptr;
    }
    const double vtol = o.vertex_tol > 0.0 ? o.vertex_tol : 1e-5;
    am_march_stats st{};
    st.fused = fused ? 1 : 0;
    hipStream_t s = ctx->stream;
    const DevNet &net = ctx->dn;
    ctx->have_result = false;

    HIPCHK(hipEventRecord(ctx->ev0, s));
    HIPCHK(hipMemsetAsync(ctx->d_ctr, 0, sizeof(Counters), s));
    HIPCHK(hipMemsetAsync(ctx->d_slots, 0, sizeof(unsigned long long) * ctx->hcap, s));
    const unsigned long long hmask = ctx->hcap - 1;

    // seeds -> cells 0..S-1 (deduplicated)
    const CellArrays ca{ctx->d_codes, ctx->d_am, ctx->d_shape, ctx->d_seed_codes, ctx->d_seed_am, ctx->d_seed_shape};
    launch_seed_cands(net, ctx->d_seed_codes, ctx->d_seed_am, ctx->d_seed_shape,
                      ctx->seeds_have_status ? ctx->d_seed_status : nullptr, ctx->n_seeds, ctx->cand, ctx->d_ctr,
                      ctx->cand_cap, s);
    launch_insert(net, ctx->cand, ca, ctx->d_slots, hmask, ctx->d_ctr, ctx->cand_cap, ctx->n_seeds, s);
    launch_commit(net, ctx->cand, ctx->d_codes, ctx->d_am, ctx->d_shape, ctx->d_hash, ctx->d_hints,
                  ctx->d_cell_key, ctx->d_fm,
                  ctx->d_seed_codes, ctx->d_seed_am, ctx->d_seed_shape, ctx->d_slots, ctx->d_ctr, ctx->cand_cap,
                  (unsigned long long)cap, ctx->n_seeds, s);
    HIPCHK(hipMemcpyAsync(ctx->h_ctr, ctx->d_ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    st.seeds_in = (long long)ctx->h_ctr->n_cand;
    long long lo = 0, hi = (long long)ctx->h_ctr->n_cells;
    st.seed_cells = hi;
    if (ctx->h_ctr->overflowed()) {
        st.required_cells = hi;
        if (stats) *stats = st;
        return fail(ctx, AM_E_CAPACITY, "seed insertion overflowed the capacities");
    }
    if (hi == 0) {
        if (stats) *stats = st;
        return fail(ctx, AM_E_SEED, "no ray produced a seed");
    }

    // the split-BF16 certificate of this net: measured once, on up to 2048
    // seed cells, before their faces are computed for the march
    if (o.precision == 1 && !ctx->calib_ok) TRY(calibrate_split(ctx, std::min<long long>(hi, 2048)));
    // sign-test margin: the caller's, else the measured one; each vertex adds
    // its own error estimate to it
    const double margin = o.margin > 0.0 ? o.margin : ctx->calib_margin;
    if (o.precision == 1) {
        st.split_row_eps = ctx->calib_eps;
        st.split_margin = margin;
        st.calib_vertices = ctx->calib_vertices;
    }
    ClipOut out{};
    out.m = ctx->d_fm;
    out.ids = ctx->d_fids;
    out.verts = ctx->d_fverts;
    out.nbr = ctx->d_fnbr;
    out.flags = ctx->d_fflags;
    out.stride = kMaxPoly;
    out.out_base = 0;
    out.off = ctx->d_foff;
    out.slot_n = &ctx->d_ctr->slot_n;
    out.slot_cap = ctx->slot_cap;
    const long long seed_cells = hi;
    // one device-driven step (graph_steps > 0): chain and clip of the range the
    // counters hold (split-BF16 with its FP64 redo, or FP64), then the hash
    // kernels; resolve takes the next range.  Events e[0..3], when given, mark
    // the chain, clip and hash phases.
    const long long gchunk = std::min<long long>(ctx->chunk_cells, 1LL << 14);
    int variant = chain_groups(ctx, gchunk, o.chain_groups);
    if (variant == 5) variant = 1;   // the gathered tile needs a sorted step
    auto dev_step = [&](hipStream_t q, hipEvent_t *e) -> hipError_t {
        hipError_t r = hipSuccess;
        if (e) r = hipEventRecord(e[0], q);
        if (o.precision == 1) {
            launch_split_step_dev(net, ctx->d_codes, ctx->d_shape, ctx->d_am, ctx->d_hash, ctx->d_hints, ctx->d_ctr,
                                  gchunk, seed_cells, ctx->d_rows, out, ctx->cand, ctx->cand_cap, margin, vtol,
                                  ctx->calib_eps, ctx->d_fb_list, variant, pa, q);
            if (e && r == hipSuccess) r = hipEventRecord(e[1], q);   // the split step is timed as chain
        } else {
            launch_chain_dev(net, ctx->d_codes, ctx->d_shape, ctx->d_ctr, gchunk, ctx->d_rows, variant, q);
            if (e && r == hipSuccess) r = hipEventRecord(e[1], q);
            launch_clip_dev(net, ctx->d_codes, ctx->d_am, ctx->d_hash, ctx->d_hints, ctx->d_ctr, gchunk, seed_cells,
                            ctx->d_rows, out, ctx->cand, ctx->cand_cap, pa, q);
        }
        if (e && r == hipSuccess) r = hipEventRecord(e[2], q);
        const long long nh = gchunk * 6;
        launch_insert(net, ctx->cand, ca, ctx->d_slots, hmask, ctx->d_ctr, ctx->cand_cap, nh, q);
        launch_commit(net, ctx->cand, ctx->d_codes, ctx->d_am, ctx->d_shape, ctx->d_hash, ctx->d_hints,
                      ctx->d_cell_key, ctx->d_fm, ctx->d_seed_codes, ctx->d_seed_am, ctx->d_seed_shape, ctx->d_slots,
                      ctx->d_ctr, ctx->cand_cap, (unsigned long long)cap, nh, q);
        launch_resolve(ctx->cand, ctx->d_fnbr, ctx->d_foff, ctx->d_ctr, ctx->cand_cap, nh, q, gchunk, cap);
        if (e && r == hipSuccess) r = hipEventRecord(e[3], q);
        return r;
    };
    if (persistent) {
        // one launch: workgroups take cells from the device-side queue until
        // none is left or in flight (k_march_persist)
        if (ctx->persist_blocks <= 0)
            HIPCHK(persist_setup(net, ctx->lds_limit, &ctx->persist_variant, &ctx->persist_lds, &ctx->persist_blocks));
        const size_t pb = (size_t)ctx->persist_blocks * 4 * (size_t)net.R * 4 * sizeof(double);
        if (ctx->prows_bytes < pb) {
            dfree(ctx, ctx->d_prows);
            ctx->prows_bytes = 0;
            TRY(dalloc(ctx, ctx->d_prows, pb / sizeof(double)));
            ctx->prows_bytes = pb;
        }
        if (ctx->ready_cap < cap) {
            dfree(ctx, ctx->d_ready);
            ctx->ready_cap = 0;
            TRY(dalloc(ctx, ctx->d_ready, (size_t)cap));
            HIPCHK(hipMemsetAsync(ctx->d_ready, 0, sizeof(unsigned) * (size_t)cap, s));
            ctx->ready_cap = cap;
            ctx->epoch = 0;
        }
        if (++ctx->epoch == 0) {   // flags of 2^32 marches ago could match: clear them
            HIPCHK(hipMemsetAsync(ctx->d_ready, 0, sizeof(unsigned) * (size_t)ctx->ready_cap, s));
            ctx->epoch = 1;
        }
        InlineInsert ins{};
        ins.codes = ctx->d_codes;
        ins.argmax = ctx->d_am;
        ins.shape = ctx->d_shape;
        ins.cell_hash = ctx->d_hash;
        ins.hints = ctx->d_hints;
        ins.face_m = ctx->d_fm;
        ins.slots = ctx->d_slots;
        ins.hmask = hmask;
        ins.ready = ctx->d_ready;
        ins.epoch = ctx->epoch;
        ins.cap_cells = (unsigned long long)cap;
        ins.spin_limit = o.wait_limit > 0 ? (unsigned long long)o.wait_limit : 1ull << 23;
        if (o.time_kernels) HIPCHK(hipEventRecord(ctx->evk[0], s));
        launch_persist(net, ctx->persist_variant, ctx->persist_lds, ctx->d_codes, ctx->d_shape, ctx->d_am,
                       ctx->d_hash, ctx->d_hints, ctx->d_prows, ctx->persist_blocks, seed_cells, out, ctx->d_ctr, ins,
                       s);
        HIPCHK(hipGetLastError());
        if (o.time_kernels) HIPCHK(hipEventRecord(ctx->evk[1], s));
        HIPCHK(hipMemcpyAsync(ctx->h_ctr, ctx->d_ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipGetLastError());
        if (o.time_kernels) {
            float a = 0.f;
            HIPCHK(hipEventElapsedTime(&a, ctx->evk[0], ctx->evk[1]));
            st.chain_ms = a;
            st.chain_launches = 1;
        }
        const Counters &c = *ctx->h_ctr;
        st.steps = 1;
        if (c.overflowed()) {
            st.required_cells = (long long)c.n_cells;
            st.cells = std::min<long long>((long long)c.n_cells, cap);
            if (stats) *stats = st;
            return fail(ctx, AM_E_CAPACITY,
                        "capacity exceeded (cells %llu/%lld, hash overflow %llu, faces without room for their "
                        "corners %llu)",
                        c.n_cells, cap, c.overflow_hash, c.overflow_slots);
        }
        if (c.stalled || c.done_cells != c.n_cells)
            return fail(ctx, AM_E_STALL, "persistent march stopped: %llu bounded waits ran out, %llu of %llu cells done",
                        c.stalled, c.done_cells, c.n_cells);
        lo = hi = 0;
    } else if (o.graph_steps > 0 && o.time_kernels) {
        // device-driven steps launched one by one (no graph), graph_steps per
        // counter read, HIP events around each kernel class of every step
        const size_t nev = (size_t)o.graph_steps * 4;
        while (ctx->evs.size() < nev) {
            hipEvent_t e = nullptr;
            HIPCHK(hipEventCreate(&e));
            ctx->evs.push_back(e);
        }
        launch_step_begin(ctx->d_ctr, gchunk, cap, s);   // later ranges: resolve ends each step
        for (;;) {
            const long long run0 = (long long)ctx->h_ctr->steps_run;
            for (int k = 0; k < o.graph_steps; ++k) {
                hipEvent_t *e = ctx->evs.data() + 4 * k;
                HIPCHK(dev_step(s, e));
            }
            HIPCHK(hipMemcpyAsync(ctx->h_ctr, ctx->d_ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            HIPCHK(hipGetLastError());
            const Counters &c = *ctx->h_ctr;
            // steps after the frontier ran dry only launched empty grids: time the ones that ran
            const long long ran = std::min<long long>((long long)c.steps_run - run0, o.graph_steps);
            for (long long k = 0; k < ran; ++k) {
                hipEvent_t *e = ctx->evs.data() + 4 * k;
                float a = 0.f, b = 0.f, c3 = 0.f;
                HIPCHK(hipEventElapsedTime(&a, e[0], e[1]));
                HIPCHK(hipEventElapsedTime(&b, e[1], e[2]));
                HIPCHK(hipEventElapsedTime(&c3, e[2], e[3]));
                st.chain_ms += a;
                st.clip_ms += b;
                st.hash_ms += c3;
                st.chain_launches++;
                st.clip_launches++;
                st.hash_launches += 3;
            }
            if (c.overflowed()) {
                st.required_cells = (long long)c.n_cells;
                st.cells = std::min<long long>((long long)c.n_cells, cap);
                st.steps = (long long)c.steps_run;
                if (stats) *stats = st;
                return fail(ctx, AM_E_CAPACITY,
                            "capacity exceeded (cells %llu/%lld, candidate overflow %llu, hash overflow %llu, "
                            "faces without room for their corners %llu)",
                            c.n_cells, cap, c.overflow_cand, c.overflow_hash, c.overflow_slots);
            }
            if (c.step_lo >= c.n_cells) break;
            if (o.max_steps > 0 && (long long)c.steps_run >= o.max_steps) break;
        }
        st.steps = (long long)ctx->h_ctr->steps_run;
        st.max_frontier = (long long)ctx->h_ctr->max_frontier;
        st.graph_launches = 0;
        lo = hi = 0;
    } else if (o.graph_steps > 0) {
        // device-driven steps, graph_steps per graph launch, one counter read
        // per launch
        auto bits = [](double x) {
            long long b;
            memcpy(&b, &x, sizeof b);
            return b;
        };
        const std::vector<long long> key = {(long long)o.graph_steps, gchunk, variant, (long long)ctx->d_codes,
                                            (long long)ctx->d_rows, (long long)ctx->cand.parent,
                                            (long long)ctx->d_slots, (long long)hmask, (long long)ctx->d_fm,
                                            (long long)ctx->d_foff, (long long)ctx->slot_cap,
                                            (long long)net.wfrag, (long long)net.bias, cap, seed_cells,
                                            (long long)ctx->cand_cap, (long long)o.precision, (long long)o.propose,
                                            bits(margin), bits(vtol), bits(ctx->calib_eps),
                                            (long long)ctx->d_fb_list, (long long)pa.stats, ctx->prop_version};
        if (!ctx->graph_exec || ctx->graph_key != key) {
            if (ctx->graph_exec) {
                HIPCHK(hipGraphExecDestroy(ctx->graph_exec));
                ctx->graph_exec = nullptr;
            }
            if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
            hipStream_t cs = ctx->cap_stream;
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            for (int k = 0; k < o.graph_steps; ++k) (void)dev_step(cs, nullptr);
            const hipError_t ce = hipStreamEndCapture(cs, &g);
            if (ce != hipSuccess) return fail(ctx, AM_E_HIP, "graph capture failed: %s", hipGetErrorString(ce));
            const hipError_t ie = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                ctx->graph_exec = nullptr;
                return fail(ctx, AM_E_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
            }
            ctx->graph_key = key;
        }
        long long launches = 0;
        launch_step_begin(ctx->d_ctr, gchunk, cap, s);   // later ranges: resolve ends each step
        for (;;) {
            HIPCHK(hipGraphLaunch(ctx->graph_exec, s));
            HIPCHK(hipMemcpyAsync(ctx->h_ctr, ctx->d_ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            HIPCHK(hipGetLastError());
            ++launches;
            const Counters &c = *ctx->h_ctr;
            if (c.overflowed()) {
                st.required_cells = (long long)c.n_cells;
                st.cells = std::min<long long>((long long)c.n_cells, cap);
                st.steps = (long long)c.steps_run;
                if (stats) *stats = st;
                return fail(ctx, AM_E_CAPACITY,
                            "capacity exceeded (cells %llu/%lld, candidate overflow %llu, hash overflow %llu, "
                            "faces without room for their corners %llu)",
                            c.n_cells, cap, c.overflow_cand, c.overflow_hash, c.overflow_slots);
            }
            if (c.step_lo >= c.n_cells) break;
            if (o.max_steps > 0 && (long long)c.steps_run >= o.max_steps) break;
        }
        st.steps = (long long)ctx->h_ctr->steps_run;
        st.max_frontier = (long long)ctx->h_ctr->max_frontier;
        st.graph_launches = launches;
        lo = hi = 0;
    }
    while (lo < hi) {
        if (o.max_steps > 0 && st.steps >= o.max_steps) break;
        const long long n = std::min<long long>(hi - lo, ctx->chunk_cells);
        st.max_frontier = std::max<long long>(st.max_frontier, hi - lo);
        HIPCHK(hipMemsetAsync(&ctx->d_ctr->n_cand, 0, sizeof(unsigned long long), s));
        const bool tk = o.time_kernels != 0;
        if (tk) HIPCHK(hipEventRecord(ctx->evk[0], s));
        if (fused) {
            launch_fused(net, ctx->d_codes, ctx->d_shape, ctx->d_am, ctx->d_hash, ctx->d_hints, lo, lo + n, seed_cells,
                         out, ctx->cand, ctx->cand_cap, ctx->d_ctr, s);
            if (tk) HIPCHK(hipEventRecord(ctx->evk[1], s));
        } else if (o.precision == 1) {
            // split-BF16 chain; faces it cannot certify go to the FP64 chain and clip
            HIPCHK(hipMemsetAsync(ctx->d_fb_count, 0, sizeof(unsigned long long), s));
            launch_chain_bf16(net, ctx->d_codes, ctx->d_shape, lo, lo + n, (float *)ctx->d_rows, s);
            if (tk) HIPCHK(hipEventRecord(ctx->evk[1], s));
            launch_clip_f32(net, ctx->d_codes, ctx->d_am, ctx->d_hash, ctx->d_hints, lo, lo + n, seed_cells,
                            (const float *)ctx->d_rows, out, ctx->cand, ctx->cand_cap, ctx->d_ctr, margin, vtol,
                            ctx->calib_eps, ctx->d_fb_list, ctx->d_fb_count, pa, s);
            launch_chain(net, ctx->d_codes, ctx->d_shape, 0, n, ctx->d_fb_list, ctx->d_fb_count, ctx->d_rows,
                         chain_groups(ctx, n, o.chain_groups), s);
            launch_clip(net, ctx->d_codes, ctx->d_am, ctx->d_hash, ctx->d_hints, 0, n, ctx->d_fb_list,
                        ctx->d_fb_count, seed_cells, ctx->d_rows, out, ctx->cand, ctx->cand_cap, ctx->d_ctr, pa, s);
        } else {
            // the gathered chain skips units off in all four cells of a tile:
            // order the step's cells by position first, so that tiles are local
            const int variant = chain_groups(ctx, n, o.chain_groups);
            const int *order = nullptr;
            if (variant == 5) {
                HIPCHK(launch_sort_cells(ctx->d_cell_key, lo, n, ctx->d_key_sorted, ctx->d_ids, ctx->d_order,
                                         ctx->d_sort_tmp, ctx->sort_tmp, s));
                order = ctx->d_order;
            }
            launch_chain(net, ctx->d_codes, ctx->d_shape, lo, lo + n, order, nullptr, ctx->d_rows, variant, s);
            if (tk) HIPCHK(hipEventRecord(ctx->evk[1], s));
            launch_clip(net, ctx->d_codes, ctx->d_am, ctx->d_hash, ctx->d_hints, lo, lo + n, order, nullptr,
                        seed_cells, ctx->d_rows, out, ctx->cand, ctx->cand_cap, ctx->d_ctr, pa, s);
        }
        if (tk) HIPCHK(hipEventRecord(ctx->evk[2], s));
        const long long nh = n * 6;
        launch_insert(net, ctx->cand, ca, ctx->d_slots, hmask, ctx->d_ctr, ctx->cand_cap, nh, s);
        launch_commit(net, ctx->cand, ctx->d_codes, ctx->d_am, ctx->d_shape, ctx->d_hash, ctx->d_hints,
                  ctx->d_cell_key, ctx->d_fm,
                      ctx->d_seed_codes, ctx->d_seed_am, ctx->d_seed_shape, ctx->d_slots, ctx->d_ctr, ctx->cand_cap,
                      (unsigned long long)cap, nh, s);
        launch_resolve(ctx->cand, ctx->d_fnbr, ctx->d_foff, ctx->d_ctr, ctx->cand_cap, nh, s);
        if (tk) HIPCHK(hipEventRecord(ctx->evk[3], s));
        HIPCHK(hipMemcpyAsync(ctx->h_ctr, ctx->d_ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipGetLastError());
        if (tk) {
            float a = 0.f, b = 0.f, c3 = 0.f;
            HIPCHK(hipEventElapsedTime(&a, ctx->evk[0], ctx->evk[1]));
            HIPCHK(hipEventElapsedTime(&b, ctx->evk[1], ctx->evk[2]));
            HIPCHK(hipEventElapsedTime(&c3, ctx->evk[2], ctx->evk[3]));
            st.chain_ms += a;
            st.clip_ms += b;
            st.hash_ms += c3;
            st.chain_launches++;
            st.clip_launches += fused ? 0 : 1;
            st.hash_launches += 3;
        }
        st.steps++;
        const Counters &c = *ctx->h_ctr;
        if (c.overflowed()) {
            st.required_cells = (long long)c.n_cells;
            st.cells = std::min<long long>((long long)c.n_cells, cap);
            if (stats) *stats = st;
            return fail(ctx, AM_E_CAPACITY,
                        "capacity exceeded (cells %llu/%lld, candidate overflow %llu, hash overflow %llu, "
                        "faces without room for their corners %llu)",
                        c.n_cells, cap, c.overflow_cand, c.overflow_hash, c.overflow_slots);
        }
        lo += n;
        hi = (long long)c.n_cells;
    }
    HIPCHK(hipEventRecord(ctx->ev1, s));
    HIPCHK(hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    const Counters &c = *ctx->h_ctr;
    st.cells = (long long)c.n_cells;

    st.domain_edges = (long long)c.domain_edges;
    st.escalated = (long long)c.escalated;
    st.pivot_cells = (long long)c.pivot_cells;
    st.pivot_fallback = (long long)c.pivot_fallback;
    if (o.propose != 0) {
        unsigned long long ps[kPropStats * kPropSlots];
        HIPCHK(hipMemcpy(ps, ctx->d_prop_stats, sizeof ps, hipMemcpyDeviceToHost));
        long long sum[kPropStats] = {0, 0, 0};
        for (int i = 0; i < kPropStats; ++i)
            for (int j = 0; j < kPropSlots; ++j) sum[i] += (long long)ps[i * kPropSlots + j];
        st.prop_cells = sum[0];
        st.prop_accepted = sum[1];
        st.prop_cuts = sum[2];
    }
    st.degenerate = (long long)c.degenerate;
    st.march_ms = ms;

    // faces and empty seeds: count through the fetch scan
    TRY(ensure_scan(ctx, std::max<long long>(st.cells, 1)));
    HIPCHK(launch_fetch(net, st.cells, ctx->d_fm, ctx->d_fids, ctx->d_fverts, ctx->d_fnbr, ctx->d_codes,
                        ctx->d_am, ctx->d_shape, ctx->d_foff, ctx->d_has, ctx->d_fidx, ctx->d_mcount, ctx->d_voff,
                        ctx->d_scan, ctx->scan_bytes, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                        nullptr, s));
    int last_idx = 0, last_has = 0;
    HIPCHK(hipMemcpyAsync(&last_idx, ctx->d_fidx + st.cells - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&last_has, ctx->d_has + st.cells - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<int> seed_m(seed_cells);
    HIPCHK(hipMemcpyAsync(seed_m.data(), ctx->d_fm, sizeof(int) * seed_cells, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    long long tail[2] = {0, 0};   // exclusive scan of the vertex counts and the last count
    HIPCHK(hipMemcpy(&tail[0], ctx->d_voff + st.cells - 1, sizeof(long long), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&tail[1], ctx->d_mcount + st.cells - 1, sizeof(long long), hipMemcpyDeviceToHost));
    st.faces = (long long)last_idx + last_has;
    st.face_verts = tail[0] + tail[1];
    st.triangles = st.face_verts - 2 * st.faces;
    for (int v : seed_m) st.seed_empty += v == 0;
    ctx->res_cells = st.cells;
    ctx->res_faces = st.faces;
    ctx->res_fverts = st.face_verts;
    ctx->have_result = true;
    if (stats) *stats = st;
    if (st.seed_empty == seed_cells && st.faces == 0) return fail(ctx, AM_E_SEED, "every seed face is empty");
    if (o.strict && st.degenerate > 0) return fail(ctx, AM_E_DEGENERATE, "%lld degenerate faces", st.degenerate);
    return AM_OK;
}

am_status am_get_counts(const am_ctx *ctx, int64_t *faces, int64_t *face_verts, int64_t *tris, int64_t *cells) {
    if (!ctx || ctx->busy || !ctx->have_result) return AM_E_STATE;
    if (faces) *faces = ctx->res_faces;
    if (face_verts) *face_verts = ctx->res_fverts;
    if (tris) *tris = ctx->res_fverts - 2 * ctx->res_faces;
    if (cells) *cells = ctx->res_cells;
    return AM_OK;
}

// Output arrays of a fetch, in caller memory (host or device).
struct FetchOut {
    int64_t *offsets;
    int32_t *ids;
    double *verts;
    int64_t *nbr;
    uint64_t *codes;
    int32_t *argmax;
    int32_t *shape_id;
};

static am_status fetch_device(am_ctx *ctx, bool sorted, const FetchOut &o);

// AM_HOST: the device fetch into a staging buffer kept by the context, then
// one copy per requested array into the caller's host memory.
static am_status fetch_any(am_ctx *ctx, int32_t where, bool sorted, const FetchOut &o) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (ctx->busy) return AM_E_STATE;
    if (where != AM_DEVICE && where != AM_HOST) return fail(ctx, AM_E_INVALID, "where must be AM_DEVICE or AM_HOST");
    if (!ctx->have_result) return fail(ctx, AM_E_STATE, "no march result");
    if (where == AM_DEVICE) return fetch_device(ctx, sorted, o);
    TRY(set_device(ctx));
    const long long F = ctx->res_faces, V = ctx->res_fverts, Wd = ctx->dn.W;
    const size_t sz[7] = {sizeof(int64_t) * (size_t)(F + 1), sizeof(int32_t) * (size_t)V, sizeof(double) * 3 * (size_t)V,
                          sizeof(int64_t) * (size_t)V,     sizeof(uint64_t) * (size_t)(F * Wd),
                          sizeof(int32_t) * (size_t)F,     sizeof(int32_t) * (size_t)F};
    void *host[7] = {o.offsets, o.ids, o.verts, o.nbr, o.codes, o.argmax, o.shape_id};
    size_t off[7], total = 0;
    for (int k = 0; k < 7; ++k) {
        off[k] = total;
        if (host[k]) total += (sz[k] + 255) & ~(size_t)255;
    }
    if (total > ctx->hstage_bytes || !ctx->d_hstage) {
        TRY(dalloc(ctx, ctx->d_hstage, total));
        ctx->hstage_bytes = total;
    }
    char *b = ctx->d_hstage;
    const FetchOut d{o.offsets ? (int64_t *)(b + off[0]) : nullptr, o.ids ? (int32_t *)(b + off[1]) : nullptr,
                     o.verts ? (double *)(b + off[2]) : nullptr,   o.nbr ? (int64_t *)(b + off[3]) : nullptr,
                     o.codes ? (uint64_t *)(b + off[4]) : nullptr, o.argmax ? (int32_t *)(b + off[5]) : nullptr,
                     o.shape_id ? (int32_t *)(b + off[6]) : nullptr};
    TRY(fetch_device(ctx, sorted, d));
    for (int k = 0; k < 7; ++k)
        if (host[k] && sz[k] > 0) HIPCHK(hipMemcpyAsync(host[k], b + off[k], sz[k], hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return AM_OK;
}

am_status am_fetch(am_ctx *ctx, int32_t where, int64_t *offsets, int32_t *ids, double *verts, int64_t *nbr,
                   uint64_t *codes, int32_t *argmax, int32_t *shape_id) {
    return fetch_any(ctx, where, false, FetchOut{offsets, ids, verts, nbr, codes, argmax, shape_id});
}

am_status am_fetch_sorted(am_ctx *ctx, int32_t where, int64_t *offsets, int32_t *ids, double *verts, int64_t *nbr,
                          uint64_t *codes, int32_t *argmax, int32_t *shape_id) {
    return fetch_any(ctx, where, true, FetchOut{offsets, ids, verts, nbr, codes, argmax, shape_id});
}

static am_status fetch_device(am_ctx *ctx, bool sorted, const FetchOut &o) {
    int64_t *offsets = o.offsets;
    int32_t *ids = o.ids;
    double *verts = o.verts;
    int64_t *nbr = o.nbr;
    uint64_t *codes = o.codes;
    int32_t *argmax = o.argmax;
    int32_t *shape_id = o.shape_id;
    TRY(set_device(ctx));
    TRY(ensure_scan(ctx, std::max<long long>(ctx->res_cells, 1)));
    if (!sorted) {
        HIPCHK(launch_fetch(ctx->dn, ctx->res_cells, ctx->d_fm, ctx->d_fids, ctx->d_fverts, ctx->d_fnbr, ctx->d_codes,
                            ctx->d_am, ctx->d_shape, ctx->d_foff, ctx->d_has, ctx->d_fidx, ctx->d_mcount, ctx->d_voff,
                            ctx->d_scan, ctx->scan_bytes, ctx->res_faces, (long long *)offsets, ids, verts,
                            (long long *)nbr, codes, argmax, shape_id, ctx->stream));
        return AM_OK;
    }
    const long long F = ctx->res_faces;
    if (F >= (1LL << 31)) return fail(ctx, AM_E_INVALID, "too many faces to sort");
    if (F > ctx->sf_cap || !ctx->d_sf_cell) {
        const long long n = std::max<long long>(F, 1);
        TRY(dalloc(ctx, ctx->d_sf_cell, n));
        TRY(dalloc(ctx, ctx->d_sf_pa, n));
        TRY(dalloc(ctx, ctx->d_sf_pb, n));
        TRY(dalloc(ctx, ctx->d_sf_rank, n));
        TRY(dalloc(ctx, ctx->d_sf_ka, n));
        TRY(dalloc(ctx, ctx->d_sf_kb, n));
        TRY(dalloc(ctx, ctx->d_sf_mc, n));
        TRY(dalloc(ctx, ctx->d_sf_vo, n));
        size_t b = 0;
        HIPCHK(sorted_fetch_tmp_bytes(n, &b));
        TRY(dalloc(ctx, ctx->d_sf_tmp, b));
        ctx->sf_tmp = b;
        ctx->sf_cap = n;
    }
    HIPCHK(launch_fetch_sorted(ctx->dn, ctx->res_cells, ctx->d_fm, ctx->d_fids, ctx->d_fverts, ctx->d_fnbr,
                               ctx->d_codes, ctx->d_am, ctx->d_shape, ctx->d_foff, ctx->d_has, ctx->d_fidx,
                               ctx->d_mcount, ctx->d_voff, ctx->d_scan, ctx->scan_bytes, F, ctx->d_sf_cell,
                               ctx->d_sf_pa, ctx->d_sf_pb, ctx->d_sf_rank, ctx->d_sf_ka, ctx->d_sf_kb, ctx->d_sf_mc,
                               ctx->d_sf_vo, ctx->d_sf_tmp, ctx->sf_tmp, (long long *)offsets, ids, verts,
                               (long long *)nbr, codes, argmax, shape_id, ctx->stream));
    return AM_OK;
}

// ---- quadric edge-collapse simplification

am_status am_simplify(am_ctx *ctx, int64_t n_verts, const double *vxyz, int64_t n_tris, const int64_t *tri,
                      const uint8_t *boundary, int64_t target_tris, int32_t max_rounds, double *v_out,
                      int64_t *tri_out, int64_t *n_verts_out, int64_t *n_tris_out, int32_t *rounds_out,
                      int64_t *n_bad) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (n_verts <= 0 || n_tris <= 0 || !vxyz || !tri || !v_out || !tri_out)
        return fail(ctx, AM_E_INVALID, "need vertices, triangles and output buffers");
    if (3 * n_verts >= (1LL << 31) || 3 * n_tris >= (1LL << 31))   // 32-bit ids index 3-wide rows
        return fail(ctx, AM_E_INVALID, "at most (2^31 - 1) / 3 vertices and as many triangles");
    if (target_tris < 0) return fail(ctx, AM_E_INVALID, "negative target");
    if (max_rounds <= 0) max_rounds = 256;
    if (max_rounds > 4096) return fail(ctx, AM_E_INVALID, "max_rounds must be at most 4096");
    TRY(set_device(ctx));
    const size_t qb = qecd_scratch_bytes(n_verts, n_tris);
    if (qb > ctx->qecd_bytes || !ctx->d_qecd) {   // kept by the context, grown when needed
        TRY(dalloc(ctx, ctx->d_qecd, qb));
        ctx->qecd_bytes = qb;
    }
    char *scratch = ctx->d_qecd;
    long long Vo = 0, To = 0, bad = 0;
    int rounds = 0;
    const hipError_t e = run_qecd(vxyz, n_verts, (const long long *)tri, n_tris, boundary, target_tris, max_rounds,
                                  scratch, v_out, (long long *)tri_out, &Vo, &To, &rounds, &bad, ctx->stream);
    (void)hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, AM_E_HIP, "simplification failed: %s", hipGetErrorString(e));
    if (n_verts_out) *n_verts_out = Vo;
    if (n_tris_out) *n_tris_out = To;
    if (rounds_out) *rounds_out = rounds;
    if (n_bad) *n_bad = bad;
    return AM_OK;
}

// ---- welded mesh

am_status am_weld(am_ctx *ctx, int64_t faces, const int64_t *offsets, const int32_t *ids, const int64_t *nbr,
                  const int32_t *argmax, const double *verts, int64_t corners, int64_t *corner_vertex,
                  double *vxyz, int64_t vxyz_rows, int64_t *n_vertices, int64_t *n_unpaired) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->loaded) return fail(ctx, AM_E_STATE, "no network loaded");
    if (faces < 0 || corners < 0 || vxyz_rows < 0) return fail(ctx, AM_E_INVALID, "negative size");
    if (corners >= (1LL << 31)) return fail(ctx, AM_E_INVALID, "at most 2^31 - 1 corners");
    if (faces > 0 && (!offsets || !ids || !nbr)) return fail(ctx, AM_E_INVALID, "offsets, ids and nbr are required");
    if (vxyz && !verts && corners > 0) return fail(ctx, AM_E_INVALID, "vxyz needs verts");
    if (corners > 0 && faces == 0) return fail(ctx, AM_E_INVALID, "corners without faces");
    TRY(set_device(ctx));
    if (faces > 0) {
        long long last = 0;   // the CSR end must be the corner count
        HIPCHK(hipMemcpy(&last, offsets + faces, sizeof(long long), hipMemcpyDeviceToHost));
        if (last != corners) return fail(ctx, AM_E_INVALID, "offsets[faces] = %lld, corners = %lld", last, corners);
    }
    if (corners > ctx->weld_n || !ctx->d_weld_parent) {
        const long long n = std::max<long long>(corners, 1);
        TRY(dalloc(ctx, ctx->d_weld_parent, n));
        TRY(dalloc(ctx, ctx->d_weld_root, n));
        TRY(dalloc(ctx, ctx->d_weld_vid, n));
        size_t b = 0;
        HIPCHK(weld_tmp_bytes(n, &b));
        TRY(dalloc(ctx, ctx->d_weld_tmp, b));
        ctx->weld_tmp = b;
        ctx->weld_n = n;
    }
    if (!ctx->d_weld_unpaired) TRY(dalloc(ctx, ctx->d_weld_unpaired, 1));
    HIPCHK(hipMemsetAsync(ctx->d_weld_unpaired, 0, sizeof(unsigned long long), ctx->stream));
    HIPCHK(launch_weld(faces, corners, (const long long *)offsets, ids, (const long long *)nbr, argmax, verts,
                       ctx->dn.N, vxyz ? vxyz_rows : 0, (long long *)ctx->d_weld_parent, ctx->d_weld_root,
                       ctx->d_weld_vid, ctx->d_weld_tmp, ctx->weld_tmp, ctx->d_weld_unpaired,
                       (long long *)corner_vertex, vxyz, ctx->stream));
    HIPCHK(hipGetLastError());
    long long V = 0;
    unsigned long long unp = 0;
    if (corners > 0) {
        int tail[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(&tail[0], ctx->d_weld_vid + corners - 1, sizeof(int), hipMemcpyDeviceToHost,
                              ctx->stream));
        HIPCHK(hipMemcpyAsync(&tail[1], ctx->d_weld_root + corners - 1, sizeof(int), hipMemcpyDeviceToHost,
                              ctx->stream));
        HIPCHK(hipMemcpyAsync(&unp, ctx->d_weld_unpaired, sizeof(unp), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        V = (long long)tail[0] + tail[1];
    }
    if (n_vertices) *n_vertices = V;
    if (n_unpaired) *n_unpaired = (int64_t)unp;
    if (vxyz && V > vxyz_rows)
        return fail(ctx, AM_E_INVALID, "vxyz has %lld rows, the mesh has %lld vertices", (long long)vxyz_rows, V);
    return AM_OK;
}

am_status am_triangles(am_ctx *ctx, int64_t faces, const int64_t *offsets, const int64_t *corner_vertex,
                       int64_t *tri, int64_t tri_rows) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (faces < 0 || tri_rows < 0) return fail(ctx, AM_E_INVALID, "negative size");
    if (faces > 0 && (!offsets || !corner_vertex || !tri))
        return fail(ctx, AM_E_INVALID, "offsets, corner_vertex and tri are required");
    TRY(set_device(ctx));
    if (faces > 0) {
        long long ends[2] = {0, 0};
        HIPCHK(hipMemcpy(&ends[0], offsets, sizeof(long long), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(&ends[1], offsets + faces, sizeof(long long), hipMemcpyDeviceToHost));
        if (ends[0] != 0 || ends[1] < 0) return fail(ctx, AM_E_INVALID, "offsets must start at 0");
        launch_triangles(faces, ends[1], (const long long *)offsets, (const long long *)corner_vertex,
                         (long long *)tri, tri_rows, ctx->stream);
    }
    HIPCHK(hipGetLastError());
    return AM_OK;
}

// ---- chain tile autotuner

am_status am_set_chain_groups(am_ctx *ctx, const int32_t *groups) {
    if (!ctx || !groups) return AM_E_INVALID;
    for (int b = 0; b < 4; ++b)
        if (groups[b] < 1 || groups[b] > kChainVariants)
            return fail(ctx, AM_E_INVALID, "chain tile variants are 1..%d", kChainVariants);
    for (int b = 0; b < 4; ++b) ctx->chain_g[b] = groups[b];
    return AM_OK;
}

am_status am_get_chain_groups(const am_ctx *ctx, int32_t *groups) {
    if (!ctx || !groups) return AM_E_INVALID;
    for (int b = 0; b < 4; ++b) groups[b] = ctx->chain_g[b];
    return AM_OK;
}

am_status am_tune_chain(am_ctx *ctx, int32_t reps, float *ms_out) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->have_result || ctx->res_cells <= 0) return fail(ctx, AM_E_STATE, "tuning needs a finished march");
    if (reps < 1 || reps > 100) return fail(ctx, AM_E_INVALID, "reps must be 1..100");
    TRY(set_device(ctx));
    const int nv = kChainVariants;
    const long long sizes[4] = {1LL << 10, 1LL << 12, 1LL << 14, 1LL << 16};
    hipStream_t s = ctx->stream;
    for (int b = 0; b < 4; ++b) {
        const long long n = std::min<long long>({sizes[b], ctx->res_cells, ctx->chunk_cells});
        float best = 0.f;
        int best_g = 1;
        for (int gi = 0; gi < nv; ++gi) {
            const int g = gi + 1;
            if (g >= 6 && !((ctx->dn.lb_ok >> (g - 6)) & 1)) {   // cannot run on this net
                if (ms_out) ms_out[b * nv + gi] = -1.f;
                continue;
            }
            launch_chain(ctx->dn, ctx->d_codes, ctx->d_shape, 0, n, nullptr, nullptr, ctx->d_rows, g, s);
            HIPCHK(hipEventRecord(ctx->evk[0], s));
            for (int r = 0; r < reps; ++r)
                launch_chain(ctx->dn, ctx->d_codes, ctx->d_shape, 0, n, nullptr, nullptr, ctx->d_rows, g, s);
            HIPCHK(hipEventRecord(ctx->evk[1], s));
            HIPCHK(hipEventSynchronize(ctx->evk[1]));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ctx->evk[0], ctx->evk[1]));
            ms /= (float)reps;
            if (ms_out) ms_out[b * nv + gi] = ms;
            if (gi == 0 || ms < best) {
                best = ms;
                best_g = g;
            }
        }
        ctx->chain_g[b] = best_g;
    }
    HIPCHK(hipGetLastError());
    return AM_OK;
}

// ---- learned form

int64_t am_prop_param_count(void) { return prop_param_count(); }

am_status am_prop_set(am_ctx *ctx, const float *params, int64_t n_params, int32_t k, float rho) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!params || n_params != prop_param_count())
        return fail(ctx, AM_E_INVALID, "the scorer has %lld parameters", prop_param_count());
    if (k < 1 || k > kPropK) return fail(ctx, AM_E_INVALID, "k must be 1..%d", kPropK);
    if (!(rho > 0.f) || !(rho < 1e6f)) return fail(ctx, AM_E_INVALID, "rho must be positive and finite");
    for (int64_t i = 0; i < n_params; ++i)
        if (!std::isfinite(params[i])) return fail(ctx, AM_E_INVALID, "non-finite scorer parameter %lld", (long long)i);
    TRY(set_device(ctx));
    const int H = kPropH, D = kPropD;
    // device image: W1 (FP16), W2 (FP16), b1, b2, w3 (FP32)
    std::vector<_Float16> w1((size_t)H * D), w2((size_t)H * H);
    for (int i = 0; i < H * D; ++i) w1[i] = (_Float16)params[i];
    const float *b1 = params + H * D, *W2 = b1 + H, *b2 = W2 + H * H, *w3 = b2 + H;
    for (int i = 0; i < H * H; ++i) w2[i] = (_Float16)W2[i];
    const size_t o_w2 = w1.size() * 2, o_b1 = o_w2 + w2.size() * 2, o_b2 = o_b1 + H * 4, o_w3 = o_b2 + H * 4,
                 total = o_w3 + H * 4;
    if (!ctx->d_prop_w) TRY(dalloc(ctx, ctx->d_prop_w, total));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipMemcpy(ctx->d_prop_w, w1.data(), w1.size() * 2, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_prop_w + o_w2, w2.data(), w2.size() * 2, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_prop_w + o_b1, b1, H * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_prop_w + o_b2, b2, H * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_prop_w + o_w3, w3, H * 4, hipMemcpyHostToDevice));
    PropNet &P = ctx->prop.net;
    P.W1 = (const _Float16 *)ctx->d_prop_w;
    P.W2 = (const _Float16 *)(ctx->d_prop_w + o_w2);
    P.b1 = (const float *)(ctx->d_prop_w + o_b1);
    P.b2 = (const float *)(ctx->d_prop_w + o_b2);
    P.w3 = (const float *)(ctx->d_prop_w + o_w3);
    P.b3 = w3[H];
    ctx->prop.k = k;
    ctx->prop.rho = rho;
    ctx->prop_loaded = true;
    ++ctx->prop_version;   // captured steps hold the scorer by value
    return AM_OK;
}

am_status am_prop_collect(am_ctx *ctx, float *samples, uint8_t *labels, int64_t cap, float rho) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    TRY(set_device(ctx));
    if (!samples || !labels || cap <= 0) {
        ctx->prop.samples = nullptr;
        ctx->prop.labels = nullptr;
        ctx->prop.cap = 0;
        return AM_OK;
    }
    if (!(rho > 0.f) || !(rho < 1e6f)) return fail(ctx, AM_E_INVALID, "rho must be positive and finite");
    if (!ctx->d_prop_nsamp) TRY(dalloc(ctx, ctx->d_prop_nsamp, 1));
    HIPCHK(hipMemsetAsync(ctx->d_prop_nsamp, 0, sizeof(unsigned long long), ctx->stream));
    ctx->prop.samples = samples;
    ctx->prop.labels = labels;
    ctx->prop.cap = (unsigned long long)cap;
    ctx->prop.n_samples = ctx->d_prop_nsamp;
    if (!ctx->prop_loaded) ctx->prop.rho = rho;
    else if (rho != ctx->prop.rho) return fail(ctx, AM_E_INVALID, "rho differs from the loaded scorer's");
    return AM_OK;
}

am_status am_prop_collected(am_ctx *ctx, int64_t *n) {
    if (!ctx || !n) return AM_E_INVALID;
    *n = 0;
    if (!ctx->d_prop_nsamp) return AM_OK;
    TRY(set_device(ctx));
    unsigned long long v = 0;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipMemcpy(&v, ctx->d_prop_nsamp, sizeof v, hipMemcpyDeviceToHost));
    *n = (int64_t)v;
    return AM_OK;
}

am_status am_prop_grad(am_ctx *ctx, const float *X, const uint8_t *y, int64_t n, const float *params, float *grad,
                       double *loss) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (n <= 0 || !X || !y || !params || !grad) return fail(ctx, AM_E_INVALID, "bad arguments");
    TRY(set_device(ctx));
    const long long P = prop_param_count();
    if (!ctx->d_prop_scratch) TRY(dalloc(ctx, ctx->d_prop_scratch, (size_t)prop_grad_blocks() * P + kPropH * kPropH));
    if (!ctx->d_prop_loss) TRY(dalloc(ctx, ctx->d_prop_loss, (size_t)prop_grad_blocks()));
    if (!ctx->h_prop_loss) HIPCHK(hipHostMalloc((void **)&ctx->h_prop_loss, sizeof(double) * prop_grad_blocks()));
    launch_prop_grad(X, y, n, params, grad, ctx->d_prop_scratch, ctx->d_prop_loss, ctx->stream);
    HIPCHK(hipGetLastError());
    if (loss) {
        HIPCHK(hipMemcpyAsync(ctx->h_prop_loss, ctx->d_prop_loss, sizeof(double) * prop_grad_blocks(),
                              hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        double sum = 0.0;
        for (int b = 0; b < prop_grad_blocks(); ++b) sum += ctx->h_prop_loss[b];
        *loss = sum / (double)n;
    }
    return AM_OK;
}

am_status am_prop_adam(am_ctx *ctx, float *params, const float *grad, float *m, float *v, int32_t step, float lr) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0.f)) return fail(ctx, AM_E_INVALID, "bad arguments");
    TRY(set_device(ctx));
    launch_prop_adam(params, grad, m, v, step, lr, ctx->stream);
    HIPCHK(hipGetLastError());
    return AM_OK;
}

am_status am_prop_score(am_ctx *ctx, const float *X, int64_t n, float *z) {
    if (!ctx) return AM_E_INVALID;
    if (ctx->busy) return AM_E_STATE;
    if (!ctx->prop_loaded) return fail(ctx, AM_E_STATE, "no proposal scorer loaded");
    if (n < 0 || (n > 0 && (!X || !z))) return fail(ctx, AM_E_INVALID, "bad arguments");
    TRY(set_device(ctx));
    if (n > 0) launch_prop_score(ctx->prop.net, X, n, z, ctx->stream);
    HIPCHK(hipGetLastError());
    return AM_OK;
}

}  // extern "C"
