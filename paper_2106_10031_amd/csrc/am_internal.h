// am_internal.h -- device data layout and wave-level helpers shared by the
// analytic-marching kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace am {

constexpr int kMaxLayers = 40;
constexpr int kMaxBlocks = 64;
constexpr int kMaxHidden = 8192;
constexpr int kMaxHeads = 64;
constexpr int kWave = 64;
constexpr int kMaxPoly = 64;      // polygon vertices held by one wave (one per lane)
constexpr int kSlotsPerCell = 8;  // face corners a march reserves per cell of its capacity (mean; faces hold up to 64)

// On-line tolerance of the halfplane clip: 2^-40 relative (see am.h).
constexpr double kTau = 9.094947017729282379150390625e-13;
// Half-size of the starting square in the plane frame: the box section lies
// within distance sqrt(3) of the plane's foot point.
constexpr double kSquareHalf = 2.0;

// Network as laid out in device memory.  Rows of the affine chain are kept
// per cell indexed by unit: layer l (1..L+1) occupies rows
// row_off[l] .. row_off[l] + width[l] - 1 with row_off[l] = unit_off[l], so
// row g holds hidden unit g and row N + i head i (R = N + M rows per cell).
struct DevNet {
    int n_layers;              // L + 2
    int N, M, W;               // hidden units, heads, code words
    int S;                     // shapes sharing the weights (1 for a single net)
    int bias_stride;           // doubles per shape in `bias` (sum of widths of layers >= 1)
    int R;                     // rows per cell (N + M)
    int width[kMaxLayers];
    int row_off[kMaxLayers];   // row offset of layer l (= unit_off[l])
    int unit_off[kMaxLayers];  // global unit offset (layer l >= 1; heads at N)
    int bias_off[kMaxLayers];  // offset of layer l's bias in `bias`
    int n_blocks;
    int blk_dst[kMaxBlocks], blk_src[kMaxBlocks];
    int blk_ld[kMaxBlocks];    // leading dimension (= src width rounded up to 4)
    long long blk_off[kMaxBlocks];   // offset of the block in `weights` (rows padded to 16)
    long long blk_frag_off[kMaxBlocks];   // offset of the block in `wfrag`
    const double *weights;     // blocks, row-major, zero padded to (16*ceil(n_dst/16)) x ld
    // the same blocks as MFMA A fragments: for 16-row tile mt and K-step ks,
    // 64 doubles in lane order, lane l = W[16 mt + l % 16][4 ks + l / 16]
    const double *wfrag;
    // split-BF16 fragments for v_mfma_f32_16x16x32_bf16: per block, tile mt,
    // K-step ks (32 wide) and term t (h, m, l: W = h + m + l), 64 lanes x 8
    // BF16, lane l element u = term of W[16 mt + l % 16][32 ks + 8 (l / 16) + u]
    const void *wfrag16;
    long long blk_frag16_off[kMaxBlocks];   // in units of 8 BF16 (16 bytes)
    int blk_ld32[kMaxBlocks];               // src width rounded up to 32
    // the same blocks column-major, rows padded to 16: element (i, k) at
    // wcol[blk_col_off + k * 16 ceil(n_dst / 16) + i] (gathered chain)
    const double *wcol;
    long long blk_col_off[kMaxBlocks];
    // the FP64 fragments as FP32 values when every weight is exactly an FP32
    // number (nullptr otherwise): half the bytes to stream, widened exactly
    const float *wfrag32;
    int lb_kpad;               // rows of the staged-B chain's LDS buffer (widest hidden layer, to 32)
    int lb_ok;                 // bit v - 6 set: staged-B chain variant v (6, 7, 8) can run
    const double *bias;        // [S][bias_stride]: shape s, layer l at s * bias_stride + bias_off[l]
    const uint64_t *zobrist;   // [N + M + S] keys of the cell fingerprint (units, heads, shapes)
};

// ---- learned form: a scorer ranks the constraint lines near the edge a
// cell was entered by; the best ones are clipped first, then every line is
// checked (the plain clip), so the face never depends on the scorer.
constexpr int kPropD = 32;       // features per line, zero padded (one MFMA K-step)
constexpr int kPropF = 8;        // features in use
constexpr int kPropH = 128;      // hidden width of the scorer
constexpr int kPropK = 16;       // most proposals per cell
constexpr int kPropSlots = 32;   // counters spread over this many slots
constexpr int kPropStats = 3;    // cells proposed, cells accepted, cuts in the check pass

struct PropNet {
    const _Float16 *W1;          // [kPropH][kPropD]
    const float *b1;             // [kPropH]
    const _Float16 *W2;          // [kPropH][kPropH]
    const float *b2;             // [kPropH]
    const float *w3;             // [kPropH]
    float b3;
};

struct PropArgs {
    int mode;                    // 0 off, 1 scorer, 2 distance order, 3 off but count cuts
    int face_routine;            // 0 clipping, 1 pivoting walk from the entry edge (FP64 rows)
    int k;                       // proposals per cell (<= kPropK)
    float rho;                   // candidates: distance to the entry midpoint <= rho x entry length
    PropNet net;
    float *samples;              // collection (nullptr: off): [cap][kPropD] features
    unsigned char *labels;       // [cap] 1 if the line carries an edge of the face
    unsigned long long cap;
    unsigned long long *n_samples;
    unsigned long long *stats;   // [kPropStats][kPropSlots]
};

// Candidate neighbour cells produced by one marching step.
struct Candidates {
    int *parent;       // cell the candidate was found from; < 0: seed -(1+index)
    int *slot;         // edge index in the parent's face
    int *unit;         // constraint id crossed (hidden unit or N + head)
    uint64_t *hash;    // fingerprint of the candidate's cell
    int *kind;         // insert outcome
    long long *ref;    // slot position (owner), cell id (found) or candidate (dup)
    int *cell;         // resolved cell id
    int *hint_prev;    // the parent's edges next to the crossed one (clip-order hints)
    int *hint_next;
    unsigned *key;     // Morton key of the crossed edge's midpoint (step ordering)
};

enum : int { kOwner = 0, kFound = 1, kDup = 2, kLost = 3 };

// Per-cell and per-seed arrays the code of a candidate may come from.
struct CellArrays {
    const uint64_t *codes;
    const int *argmax;
    const int *shape;
    const uint64_t *seed_codes;
    const int *seed_am;
    const int *seed_shape;
};

// Where the clip kernel writes faces.  With off == NULL, face f (output
// index cell - out_base) has `stride` slots at f * stride; otherwise each face
// takes m consecutive slots from the shared counter *slot_n (at most slot_cap
// in all) and off[f] records the first.
struct ClipOut {
    int *m;               // [cells] vertex count, 0 = empty face
    int *ids;             // [slots]
    double *verts;        // [slots][3]
    int *nbr;             // [slots] neighbour cell (-1 box edge) or NULL
    int *flags;           // [cells] or NULL
    int stride;           // most vertices of a face (<= kMaxPoly); slots per face without off
    long long out_base;   // output index = cell - out_base
    long long *off;       // [cells] first slot of each face, or NULL
    unsigned long long *slot_n;   // slots taken so far (with off)
    unsigned long long slot_cap;  // slots available (with off)
};

// Device-side counters of a march (one struct in device memory).
// The counters that many workgroups update or poll while a march runs
// (n_cells, slot_n, next_cell, done_cells, stop) each sit on a 128-byte line
// of their own, so that traffic on one does not queue behind another's.
struct Counters {
    alignas(128) unsigned long long n_cells;
    unsigned long long n_cand;
    unsigned long long overflow_cells;
    unsigned long long overflow_cand;
    unsigned long long overflow_hash;
    unsigned long long degenerate;
    unsigned long long domain_edges;
    unsigned long long face_verts;
    unsigned long long too_big;
    unsigned long long escalated;   // cells the split-BF16 pass handed to FP64
    // device-driven steps (graph launch): first cell and cell count of the
    // current step (adjacent: read as a pair), steps run
    unsigned long long step_lo;
    unsigned long long step_n;
    unsigned long long steps_run;
    unsigned long long pivot_cells;      // pivoting form: faces traced by the walk
    unsigned long long pivot_fallback;   // ... and cells clipped instead
    unsigned long long max_frontier;     // device-driven steps: largest frontier seen
    unsigned long long n_cand_prev;      // the step's candidate count, copied by commit for resolve
    unsigned long long fb_n;             // device-driven split-BF16 steps: cells handed to FP64
    unsigned long long overflow_slots;   // faces that found no room for their corners
    unsigned long long stalled;          // persistent march: bounded waits that ran out (the march failed)
    alignas(128) unsigned long long slot_n;   // face slots (corners) taken
    // persistent march: next cell id to hand out, cells finished, stop request
    alignas(128) unsigned long long next_cell;
    alignas(128) unsigned long long done_cells;
    alignas(128) unsigned long long stop;

    __host__ __device__ bool overflowed() const {
        return overflow_cells || overflow_cand || overflow_hash || overflow_slots;
    }
};

// ---- device hash set of discovered cells (open addressing, 64-bit slots).
// A committed slot holds tag(h) << 32 | cell id.  A slot being filled holds
// kPending plus a reference to where the candidate's code comes from.
constexpr uint64_t kPending = 1ull << 63;

__device__ __forceinline__ uint32_t slot_tag(uint64_t h) {
    return (uint32_t)((h >> 32) & 0x7fffffffu) | 0x40000000u;   // never zero
}

// Cross-workgroup data of the persistent march (new cells' records, hash
// slots, ready flags, queue counters) is read and written only with
// device-scope relaxed atomics: each such access is coherent across the XCDs
// by itself (it is performed at the device's coherence point), so no
// acquire or release fence is needed, and none of the cache-wide invalidate
// or write-back operations those fences imply is issued.  Order between a
// record and the flag that publishes it comes from publish_wait: the
// writer's record stores have completed before its flag store is issued, and
// a reader issues its record loads only after its flag load has returned.
template <typename T>
__device__ __forceinline__ T ld_dev(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_dev(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void publish_wait() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);   // the compiler keeps the order
    __builtin_amdgcn_s_waitcnt(0);             // every earlier memory access has completed
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// A cell's record as the persistent march holds it (copied to LDS from the
// cell arrays with device-scope loads): the clip reads this instead of the
// arrays, which another workgroup wrote.
struct CellRec {
    const uint64_t *code;
    int am;
    int shape;
    int hint[3];
    uint64_t hash;
};

// What the persistent march needs to insert a face's neighbours into the
// hash set as soon as the face is known (no candidate buffer): the cell
// arrays it appends to, the set, the ready flags (ready[c] == epoch once cell
// c's code and hints are written) and the bound on waits.
struct InlineInsert {
    uint64_t *codes;
    int *argmax;
    int *shape;
    uint64_t *cell_hash;
    int *hints;
    int *face_m;
    unsigned long long *slots;
    unsigned long long hmask;
    unsigned *ready;
    unsigned epoch;
    unsigned long long cap_cells;
    unsigned long long spin_limit;   // bound of one wait: naps (~64 cycles) of a queue poll, 16x polls of a slot
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Broadcast a value from lane `src` (uniform) to the whole wave.
__device__ __forceinline__ double bcast(double x, int src) {
    const uint64_t u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, src);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
    return __longlong_as_double(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int bcast(int x, int src) { return __builtin_amdgcn_readlane(x, src); }

// Value of `x` in lane `src` (per-lane source).
__device__ __forceinline__ double shfl(double x, int src) { return __shfl(x, src, kWave); }
__device__ __forceinline__ int shfl(int x, int src) { return __shfl(x, src, kWave); }

__device__ __forceinline__ double wave_sum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

__device__ __forceinline__ int wave_min(int x) {
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, kWave));
    return x;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int code_bit(const uint64_t *code, int g) {
    return (int)((code[g >> 6] >> (g & 63)) & 1ull);
}

// Wave-aggregated atomic add: every active lane with `want` gets a slot.
__device__ __forceinline__ unsigned long long wave_reserve(unsigned long long *ctr, bool want,
                                                           unsigned long long *base_out) {
    const uint64_t m = ballot(want);
    unsigned long long base = 0;
    const int leader = m ? __builtin_ctzll(m) : 0;
    if (m && lane_id() == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(m));
    base = (unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)base, leader) |
           ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(base >> 32), leader)
            << 32);
    *base_out = base;
    return base + (unsigned long long)__popcll(m & lanemask_lt());
}

}  // namespace am
