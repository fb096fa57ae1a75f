/*
 * am.h -- C ABI of the analytic-marching library for AMD MI355X (gfx950).
 *
 * The library meshes the exact zero-level set of a ReLU network F (Sec. 2.2
 * of Lei, Jia, Ma: "Learning and Meshing from Deep Implicit Surface Networks
 * Using an Efficient Implementation of Analytic Marching") as a polygon mesh
 * Z = {V, {P}}: one convex polygon (the analytic face, Eqn (AnalyticFace)) per
 * analytic cell, each with its vertices (Eqn (VertexEquationSystem)) and the
 * face across each of its edges.  Cells are visited by analytic marching
 * (Algorithm 1, parallel marching of Sec. 4.2.2): all cells of the active set
 * are solved at once on the GPU and their neighbours, found by flipping one
 * unit's state (Sec. 3.1), are deduplicated in a device hash set.
 *
 * Network model (Sec. 2.2, Sec. 5.1 shortcuts, Sec. 5.2 max pooling): layer 0
 * is the input x in R^3, layers 1..L are ReLU layers, layer L+1 holds M >= 1
 * heads and F(x) = max_i head_i(x).  A block (dst, src, W) adds W act[src] to
 * the pre-activation of layer dst for any src < dst (identity or linear
 * shortcuts are ordinary blocks); act[0] = x, act[l] = relu(pre[l]).
 *
 * Conventions (fixed; the CPU reference follows the same ones):
 *   - activation code: N = n_1 + ... + n_L bits, layer-major; bit g lives in
 *     bit (g % 64) of 64-bit word g / 64; a unit is on iff its
 *     pre-activation is > 0 (Eqn (NeuronState)).  W = max(1, ceil(N/64))
 *     words per code.  The argmax head j (lowest index on ties) is part of
 *     the cell's identity (Eqn (StateFuntionalMaxPoolingOperation)).
 *   - domain: the box [-1,1]^3.  Edge (constraint) ids: 0..N-1 hidden units,
 *     N+i the max-pool comparison with head i, -1..-6 the box planes
 *     x<=1, x>=-1, y<=1, y>=-1, z<=1, z>=-1 (no neighbour).
 *   - polygons run counter-clockwise seen from +grad F and start at the
 *     edge with the smallest id; vertex i starts edge i.
 *   - a vertex lies ON a constraint line when |c.[v;1]| <= 2^-40 *
 *     (|c_uv| (1 + |v_uv|) + |c_w|) in the plane frame; only constraints
 *     carrying an edge of positive length spawn neighbours.
 *
 * Memory: every pointer argument is either a host pointer or a device pointer
 * as stated per call.  The context owns its device scratch (allocated on
 * am_load_net / am_march from the allocator given to am_create, and freed by
 * am_destroy) and enqueues all work on the HIP stream given to am_create.
 * No call throws or aborts across the ABI; failures return a status and
 * am_last_error() describes them.  A
 * context must not be used from two threads at once.
 */
#ifndef AM_H
#define AM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AM_OK = 0,
    AM_E_INVALID = 1,    /* bad argument, bad network, NaN/Inf weights */
    AM_E_OOM = 2,        /* device allocation failed */
    AM_E_CAPACITY = 3,   /* a capacity in am_march_opts was too small; see stats */
    AM_E_SEED = 4,       /* no seed produced a non-empty face */
    AM_E_DEGENERATE = 5, /* strict mode: a degenerate face was met */
    AM_E_HIP = 6,        /* a HIP runtime call failed */
    AM_E_STATE = 7,      /* call out of order (e.g. march before load) */
    AM_E_STALL = 8       /* persistent march: a bounded device-side wait ran out (a cell's
                            code never appeared, or no cell finished for about a second
                            while one was in flight); the result is incomplete */
} am_status;

typedef struct am_ctx am_ctx;

/* Element type of the weights and biases of an am_net_desc. */
enum { AM_F64 = 0, AM_F32 = 1 };

/* Where am_fetch writes: caller DEVICE buffers (enqueued) or HOST memory
 * (the call synchronises). */
enum { AM_DEVICE = 0, AM_HOST = 1 };

/* Network description.  All pointers are HOST pointers, borrowed for the
 * call only (the weights are copied to the device, widened exactly to FP64). */
typedef struct {
    int32_t n_layers;             /* L + 2 (input, hidden layers, head layer) */
    const int32_t *width;         /* [n_layers]; width[0] must be 3 */
    int32_t n_blocks;
    const int32_t *blk_dst;       /* [n_blocks], 1 <= dst < n_layers */
    const int32_t *blk_src;       /* [n_blocks], 0 <= src < dst */
    const void *const *blk_w;     /* [n_blocks] row-major width[dst] x width[src], of type dtype */
    const void *const *bias;      /* [n_layers]; bias[l] has width[l] entries of type dtype, bias[0] unused */
    int32_t n_heads;              /* M >= 1 heads joined by a max (Sec. 5.2); 0 = width[n_layers-1],
                                     else it must equal width[n_layers-1] */
    int32_t dtype;                /* AM_F64 (0) or AM_F32 (1): element type of blk_w and bias */
} am_net_desc;

typedef struct {
    int64_t max_cells;    /* capacity of discovered cells (0: 1<<20); faces share room for 8
                             corners per cell of this capacity (faces average about 4), and a
                             march that needs more returns AM_E_CAPACITY */
    int32_t max_steps;    /* bound on marching steps (0: unbounded) */
    int32_t strict;       /* 1: return AM_E_DEGENERATE on a degenerate face */
    int32_t time_kernels; /* 1: time each kernel class with HIP events on the stream */
    int32_t kernel_path;  /* 0: the library's choice; 1: split (chain rows through HBM, then
                             the clip); 2: fused chain+clip in LDS (AM_E_INVALID if too big);
                             3: persistent march, one launch for the whole march (the
                             parallel marching of Sec. 4.2.2 without steps): as many
                             workgroups as fit on the device take four discovered cells at a
                             time from a device-side queue, compute their chain, clip them
                             and insert their neighbours into the hash set at once, until no
                             cell is left or in flight.  Plain FP64 form only (AM_E_INVALID
                             with precision, propose, sample collection, pivoting,
                             graph_steps or max_steps).  The cells, faces and adjacency are
                             those of the stepped march; cell ids are assigned in the order
                             cells are found, so only canonical fetches (am_fetch_sorted)
                             are reproducible from run to run */
    int32_t precision;    /* 0: FP64 chain and clip.  1: split-BF16 chain on matrix cores
                             (each operand = three BF16 terms, six products, FP32
                             accumulation), clip and vertex solves in FP64 on the FP32 rows;
                             a face is kept only if every vertex's estimated relative error
                             is at most `vertex_tol` and no other constraint comes within
                             `margin` + that estimate of a vertex (and no edge is that
                             short), else its cell is redone by the FP64 chain and clip.
                             The estimate is the vertex's first-order sensitivity to its
                             rows times a row error measured for each loaded net on the
                             first march's seed cells (stats.split_row_eps).  This is an
                             empirical certificate, not a bound: cells, cycles and
                             adjacency equal the FP64 result unless an unmeasured error
                             exceeds 8x the largest measured one */
    int32_t propose;      /* learned form (not in the paper, which sorts planes by distance
                             in its pivoting routine, Sec. 4.2.1): before the every-line clip,
                             clip the best k hidden lines near the edge the cell was entered
                             by.  0: off; 1: ranked by the scorer of am_prop_set; 2: ranked
                             by distance to that edge's midpoint; 3: off, but count cuts.
                             The every-line pass decides the face, so results equal
                             propose 0.  Cells without an entry edge (seeds) are not
                             proposed for. */
    int32_t chain_groups; /* affine-chain tile: 0 = the context's table (am_tune_chain); 1, 2
                             or 4 column groups of 16 (4, 8 or 16 cells per workgroup; more
                             cells share each streamed weight fragment); 3 = four cells
                             reading the previous layer's rows from LDS as the B operand
                             (layers of at most 128 units stay there; for nets up to 512
                             units wide each layer is staged there, masked, from global
                             memory); 5 = four cells whose K loop runs
                             only over the source units active in any of them (sources of at
                             most 1024 units; rows then differ from the dense sum in the last
                             bits); 6, 7 = 4 or 8 cells whose previous layer is written,
                             masked, by the producing MFMA tiles into LDS as the next B
                             operand, with weight fragments streamed one batch of K-steps
                             ahead (as FP32 when every weight is an FP32 number), one 16-row
                             output tile per wave (two if the widest layer is over 256); 8 =
                             as 6 with two output tiles per wave.  6..8 need layers of at
                             most 512 units and their LDS (widest hidden layer x 16 x 4 or 8
                             cells doubles); otherwise they run as 1.  Variants 1..4 and 6..8
                             sum in the same order (equal rows) */
    int32_t graph_steps;  /* > 0 (<= 64): device-driven steps, this many captured in one HIP
                             graph (built once per context and shape of the march, then
                             replayed) and one counter read per replay instead of per step.
                             Each step takes up to 16384 cells from the device-side frontier.
                             With time_kernels the same steps are launched one by one on the
                             stream instead (no graph), still one counter read per
                             graph_steps steps, with HIP events around each kernel class.
                             Every form of the split path (FP64 or split-BF16 with its FP64
                             redo, with or without proposals, one shape or a batch);
                             AM_E_INVALID with sample collection, kernel_path 2 or pivoting.
                             The gathered chain tile (5) is replaced by 1 */
    int32_t face_routine; /* 0: halfplane clipping; 1: pivoting (Sec. 4.2.1): each face with
                             an entry edge from its parent is traced vertex by vertex from
                             that edge (a ratio test over every line per vertex); seeds,
                             cells whose entry edge ends on a box plane or is degenerate, and
                             walks that do not close are clipped.  The faces are the same.
                             Plain FP64 form on the split path only (AM_E_INVALID with
                             precision, propose, sample collection, kernel_path 2 or
                             graph_steps) */
    int32_t async;        /* 1: enqueue the march on a worker thread and return at once;
                             am_wait blocks until it ends and returns its status and stats.
                             Until then every other call on the context returns AM_E_STATE
                             (am_busy tells whether it still runs) */
    double margin;        /* relative sign-test margin of precision 1 (0: the measured one,
                             stats.split_margin) */
    double vertex_tol;    /* precision 1: a cell is also redone in FP64 when a vertex's
                             estimated relative error (stats.split_row_eps x its first-order
                             sensitivity to the rows) exceeds this (0: 1e-5) */
    int32_t wait_limit;   /* kernel_path 3: bound of each wait of the march, in naps of about
                             64 cycles that a workgroup polling the queue may sleep while no
                             cell finishes anywhere (a wait for another wave's claim gets a
                             sixteenth of it in polls); a wait that runs out stops the march
                             with AM_E_STALL and the context can march again.  0: 1 << 23
                             (about 0.2 s); a tiny value forces the stall (tests of that
                             path).  Negative: AM_E_INVALID; ignored by the other paths */
} am_march_opts;

typedef struct {
    int64_t faces;            /* cells with a non-empty face */
    int64_t face_verts;       /* sum of polygon sizes */
    int64_t triangles;        /* sum of (m - 2): fan triangulation count */
    int64_t cells;            /* distinct cells discovered (incl. empty) */
    int64_t steps;            /* marching steps (frontier generations) */
    int64_t max_frontier;     /* largest frontier (cells discovered, not yet processed) */
    int64_t seeds_in;         /* seed cells before deduplication */
    int64_t seed_cells;       /* distinct seed cells */
    int64_t seed_empty;       /* seed cells whose face is empty */
    int64_t degenerate;       /* non-seed cells with an empty or degenerate face */
    int64_t domain_edges;     /* edges on the box */
    int64_t required_cells;   /* on AM_E_CAPACITY: the cell capacity needed so far */
    double march_ms;          /* device time of the march (HIP events) */
    /* with opts.time_kernels: summed HIP-event durations and launch counts */
    double chain_ms;          /* affine chain (FP64 MFMA); fused path: chain + clip */
    double clip_ms;           /* halfplane clip + vertex solve + candidates (split path) */
    double hash_ms;           /* insert + commit + resolve */
    int64_t chain_launches;
    int64_t clip_launches;
    int64_t hash_launches;
    int32_t fused;            /* 1 if the fused chain+clip kernel ran */
    int32_t pad;
    int64_t escalated;        /* precision 1: cells redone in FP64 */
    /* propose != 0, over cells with an entry edge: */
    int64_t prop_cells;       /* such cells */
    int64_t prop_accepted;    /* ... whose every-line pass cut nothing (the proposals and
                                 entry lines already gave the face) */
    int64_t prop_cuts;        /* lines that cut in their every-line passes */
    int64_t graph_launches;   /* graph_steps > 0: graph replays */
    int64_t pivot_cells;      /* face_routine 1: faces traced by pivoting */
    int64_t pivot_fallback;   /* face_routine 1: cells clipped instead (seeds, no usable entry
                                 edge, or a walk that did not close) */
    /* precision 1: the certificate's constants for the loaded net, measured on
       the first march's seed cells (at most 2048) against the FP64 chain and clip */
    double split_row_eps;     /* relative row error per unit of vertex sensitivity (8 x measured) */
    double split_margin;      /* sign-test margin used (opts.margin, else 8 x the measured one) */
    int64_t calib_vertices;   /* vertices those were measured on */
} am_march_stats;

/* Device memory supplier.  alloc returns `bytes` of device memory on
 * `device` for work on `stream` (a hipStream_t), or NULL on failure (the call
 * that needed it then returns AM_E_OOM); release returns a block alloc gave.
 * A caching allocator (PyTorch's) may hand a released block to the next
 * alloc on the same stream at once: the library enqueues all its work on
 * that stream.  `user` is passed back unchanged. */
typedef struct {
    void *(*alloc)(void *user, size_t bytes, int device, void *stream);
    void (*release)(void *user, void *ptr, int device, void *stream);
    void *user;
} am_allocator;

/* Creates a context on `device` that enqueues its work on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  Every device buffer the
 * context owns comes from `alloc` (copied; NULL = hipMalloc / hipFree),
 * except pinned host memory for its counters and the fixed scratch of
 * am_faces_noalloc.  AM_E_INVALID if alloc gives only one of its two
 * functions. */
am_status am_create(am_ctx **out, int device, void *hip_stream, const am_allocator *alloc);

/* Frees the context and every device buffer it owns.  NULL is a no-op. */
void am_destroy(am_ctx *ctx);

/* Text of the last failure on this context (owned by ctx; valid until the
 * next call on it). */
const char *am_last_error(const am_ctx *ctx);

/* Loads a network (Sec. 2.2, 5.1, 5.2); see am_net_desc.  Rejects widths
 * < 1, width[0] != 3, non-feed-forward or duplicate blocks, layers with no
 * input block, N > 8192 and NaN/Inf parameters with AM_E_INVALID.  Resets
 * any seeds and results. */
am_status am_load_net(am_ctx *ctx, const am_net_desc *net);

/* Loads S shapes that share one network's weights and differ in their
 * biases: shape_bias is a HOST array [S][n_1 + ... + n_L + M] (layers in
 * order), row s replacing the biases of every layer for shape s; the
 * descriptor's own bias pointers are ignored.  This covers a decoder whose
 * latent code enters layers linearly (the latent term W_z z_s folds into the
 * bias of each layer it feeds), e.g. a latent re-injected at an inner layer as
 * a linear shortcut (Sec. 5.1).  Cells of different shapes are different
 * cells (the shape id is part of a cell's identity); one march covers all of
 * them (parallel marching, Sec. 4.2.2).  Same checks as am_load_net. */
am_status am_load_batch(am_ctx *ctx, const am_net_desc *net, int32_t n_shapes, const double *shape_bias);

/* Dimensions of the loaded network: N hidden units, M heads, W code words,
 * S shapes (1 after am_load_net).  Any pointer may be NULL. */
am_status am_net_dims(const am_ctx *ctx, int32_t *n_hidden, int32_t *n_heads, int32_t *code_words,
                      int32_t *n_shapes);

/* Forward pass: code and F at n points (Eqns (NeuronState)-(MLPState)).
 * DEVICE pointers: pts [n][3] f64 and shape_id [n] i32 (NULL = shape 0) in;
 * codes [n][W] u64, argmax [n] i32, F [n] f64 out (any output may be NULL;
 * a shape id out of range gives argmax -1 and F = NaN).  Enqueued; returns
 * before the results are ready (synchronise the stream). */
am_status am_codes(am_ctx *ctx, const double *pts, const int32_t *shape_id, int64_t n, uint64_t *codes,
                   int32_t *argmax, double *F);

/* Affine chain (Lemma 1, Corollary 1): for each of n cells given by its
 * code, the rows Z[g] = (a, b, c, d) with pre_g(x) = a x + b y + c z + d
 * inside the cell, g = 0..N-1 hidden units then N..N+M-1 heads.  DEVICE
 * pointers: codes [n][W] u64 and shape_id [n] (NULL = shape 0) in;
 * rows [n][N+M][4] f64 out.  precision 0 = FP64 matrix cores, 1 = the
 * split-BF16 chain of am_march_opts.precision (rows rounded to FP32).
 * Enqueued. */
am_status am_chain(am_ctx *ctx, const uint64_t *codes, const int32_t *shape_id, int64_t n, int32_t precision,
                   double *rows);

/* Analytic faces of n given cells (Eqn (AnalyticFace) clipped to the box,
 * vertices by Eqn (VertexEquationSystem)), without marching.  DEVICE
 * pointers: codes [n][W], argmax [n], shape_id [n] in (argmax and shape_id
 * may be NULL = 0); m [n] i32 (0 = empty face),
 * ids [n][max_m] i32, verts [n][max_m][3] f64, flags [n] i32 out.
 * max_m must be in 3..64.  Enqueued. */
am_status am_faces(am_ctx *ctx, const uint64_t *codes, const int32_t *argmax, const int32_t *shape_id,
                   int64_t n, int32_t max_m, int32_t *m, int32_t *ids, double *verts, int32_t *flags);

/* am_faces without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, layout and results as am_faces (bit for bit).
 * The chain rows go through a fixed 32 MiB device scratch array that the
 * library holds on every GPU it runs on until the process ends; its address is
 * looked up when a context is created on the device.  n cells are processed
 * in batches of floor(32 MiB / (32 R)) cells (R = padded rows per cell, about
 * N + M), one batch after another on the context's stream.  The call itself
 * allocates nothing; a network whose single cell needs more than 32 MiB of
 * rows is rejected with AM_E_INVALID.  Every context on one GPU shares that
 * GPU's scratch: calls on different streams that overlap in time race (their
 * results are then undefined); calls on one stream do not.  Enqueued. */
am_status am_faces_noalloc(am_ctx *ctx, const uint64_t *codes, const int32_t *argmax, const int32_t *shape_id,
                           int64_t n, int32_t max_m, int32_t *m, int32_t *ids, double *verts, int32_t *flags);

/* Seeds by dichotomy along rays o + t d, t in [0, t_max] (Sec. 4.3.2; t_max
 * <= 0 means 1): bisect
 * until both bracket ends share one code (at most max_iter halvings, <= 0
 * means 200), then take the linear root inside that cell; the seed cell is
 * the code and argmax at the root.  DEVICE pointers: orig [R][3], dir [R][3]
 * f64, shape_id [R] i32 (NULL = all shape 0).  Rays without a sign change are
 * skipped (counted in status_out, a DEVICE [R] i32 array that may be NULL:
 * 0 ok, 1 no sign change, 2 no convergence, 3 shape id out of range).
 * Replaces any previous seeds; the seed cells are kept in the context for
 * am_march.  Enqueued. */
am_status am_seed_rays(am_ctx *ctx, const double *orig, const double *dir, const int32_t *shape_id,
                       int64_t n_rays, double t_max, int32_t max_iter, int32_t *status_out);

/* Seeds given directly as cells.  DEVICE pointers: codes [n][W] u64,
 * argmax [n] i32 and shape_id [n] i32 (NULL = all 0).  Seeds with an argmax
 * or shape id out of range are dropped.  Replaces any previous seeds.
 * Enqueued. */
am_status am_seed_cells(am_ctx *ctx, const uint64_t *codes, const int32_t *argmax, const int32_t *shape_id,
                        int64_t n);

/* Seeds from points (the start of Algorithm 1 is a point on the surface):
 * the cell of each point pts[i] (DEVICE [n][3] f64; shape_id DEVICE [n] i32
 * or NULL) by a forward pass (Eqns (NeuronState)-(MLPState)) is a seed.  A
 * point off the surface gives a cell whose face may be empty; it then adds
 * nothing (am_march returns AM_E_SEED only if every seed face is empty).  A
 * shape id out of range drops the point.  Replaces any previous seeds.
 * Enqueued. */
am_status am_seed_points(am_ctx *ctx, const double *pts, const int32_t *shape_id, int64_t n);

/* Sphere-tracing seeds (Sec. 4.3.1, Eqn (SphereTracing)), for SDF networks:
 * from each start point pts[i] (DEVICE [n][3] f64; shape_id DEVICE [n] i32 or
 * NULL), repeats x <- x - F(x) g / |g|^2 with g the gradient of F in the cell
 * of x (the paper's update with step size 1 when |g| = 1) until a step lands
 * in the cell it started from; that point lies on the cell's zero plane and
 * its code is the seed.  max_iter steps at most (0: 64).  Optional DEVICE
 * outputs: status_out [n] i32 (0 settled, 1 not within max_iter, 2 zero
 * gradient, 3 settled outside [-1,1]^3, 4 shape id out of range), iters_out
 * [n] i32, x_out [n][3] f64 (the last iterate).  Seeds with status != 0 are
 * skipped by the march.  AM_E_INVALID if the network needs more LDS than a
 * workgroup has (2 (3 + N + M) doubles + 2 W words).  Enqueued. */
am_status am_seed_points_st(am_ctx *ctx, const double *pts, const int32_t *shape_id, int64_t n, int32_t max_iter,
                            int32_t *status_out, int32_t *iters_out, double *x_out);

/* Marches from the current seeds (Algorithm 1, all active cells at once)
 * until the active set is empty.  Blocks until done unless opts->async (then
 * use am_wait; stats is not written).  opts may be NULL.  Returns
 * AM_E_CAPACITY (stats->required_cells set) when max_cells is too small;
 * AM_E_SEED when every seed face is empty. */
am_status am_march(am_ctx *ctx, const am_march_opts *opts, am_march_stats *stats);

/* Waits for the asynchronous march started by am_march (opts->async = 1):
 * returns that march's status and fills stats (may be NULL).  AM_E_STATE if
 * none was started since the last wait. */
am_status am_wait(am_ctx *ctx, am_march_stats *stats);

/* *busy = 1 while an asynchronous march runs on the context, else 0. */
am_status am_busy(const am_ctx *ctx, int32_t *busy);

/* Sizes of the last march's result: faces, polygon corners, fan triangles
 * (corners - 2 faces), cells discovered.  Any pointer may be NULL. */
am_status am_get_counts(const am_ctx *ctx, int64_t *faces, int64_t *face_verts, int64_t *tris, int64_t *cells);

/* Copies the last march's mesh into caller-owned buffers, faces in discovery
 * order:  offsets [F+1] i64 (CSR into the per-edge arrays), ids [V] i32 edge
 * constraint ids, verts [V][3] f64 (vertex i starts edge i), nbr [V] i64 face
 * index across edge i (-1 box edge, -2 neighbour cell has no face), codes
 * [F][W] u64, argmax [F] i32, shape_id [F] i32; F, V from am_get_counts.
 * where = AM_DEVICE: DEVICE buffers, enqueued.  where = AM_HOST: HOST memory;
 * the arrays are staged in device memory the context keeps, copied, and the
 * call synchronises.  Any pointer may be NULL to skip that output. */
am_status am_fetch(am_ctx *ctx, int32_t where, int64_t *offsets, int32_t *ids, double *verts, int64_t *nbr,
                   uint64_t *codes, int32_t *argmax, int32_t *shape_id);

/* As am_fetch (same `where`, buffers and layout), with the faces in canonical order:
 * sorted by shape id, then by code words (unsigned, word 0 first), then by
 * argmax; nbr holds indices in that order.  Every face's cycle starts at its
 * smallest edge id either way, so the output is independent of discovery
 * order and equals the CPU reference's mesh array for array.  A stable radix
 * sort per key word; device scratch of about 48 bytes per face is kept by
 * the context.  Enqueued. */
am_status am_fetch_sorted(am_ctx *ctx, int32_t where, int64_t *offsets, int32_t *ids, double *verts, int64_t *nbr,
                          uint64_t *codes, int32_t *argmax, int32_t *shape_id);

/* ---- Welded mesh: the output Z = {V, {P}} of Sec. 3, a shared vertex
 * array plus polygons that index it.  A march emits each face with its own
 * copy of its vertices; across a shared edge (edge i of face f, edge j of
 * face g = nbr[i], on the same constraint, or for a max-pool comparison edge
 * the neighbour's row N + argmax[f], N = hidden units of the loaded net)
 * the start of edge i is the end of edge j and vice versa.  Welding puts
 * corners joined that way into one vertex, by connectivity alone, so a
 * vertex where many faces meet is still one vertex.  Vertex ids run in the
 * order of each vertex's smallest corner index.
 *
 * DEVICE in: the am_fetch layout for `faces` faces and `corners` corners
 * (offsets [faces+1] with offsets[faces] == corners, ids [corners],
 * nbr [corners], argmax [faces] or NULL when the net has no max-pool, verts
 * [corners][3], needed only for vxyz).  DEVICE out (NULL to skip):
 * corner_vertex [corners] i64 vertex id of each corner; vxyz [vxyz_rows][3]
 * f64 vertex positions, taken from each vertex's smallest corner.  HOST
 * out: n_vertices; n_unpaired = edges whose neighbour lists no matching
 * edge back, plus faces with malformed offsets (0 for a march's mesh).
 * At most 2^31 - 1 corners.  Synchronises.  AM_E_INVALID when
 * offsets[faces] != corners or vxyz_rows < n_vertices (corner_vertex and
 * n_vertices are still valid then; the first vxyz_rows rows are written). */
am_status am_weld(am_ctx *ctx, int64_t faces, const int64_t *offsets, const int32_t *ids,
                  const int64_t *nbr, const int32_t *argmax, const double *verts, int64_t corners,
                  int64_t *corner_vertex, double *vxyz, int64_t vxyz_rows, int64_t *n_vertices,
                  int64_t *n_unpaired);

/* Fan triangulation of the welded polygons: face f with corners c0..c(m-1)
 * gives triangles (c0, ck, ck+1), k = 1..m-2, in face order, as vertex ids
 * from corner_vertex.  DEVICE: offsets [faces+1] (offsets[0] == 0),
 * corner_vertex [offsets[faces]] i64, tri [tri_rows][3] i64 out; tri_rows =
 * corners - 2 faces holds them all (rows past tri_rows are not written).
 * The polygons are convex (Sec. 3), so the fan covers each exactly.
 * Enqueued after a synchronous read of the two offset ends. */
am_status am_triangles(am_ctx *ctx, int64_t faces, const int64_t *offsets,
                       const int64_t *corner_vertex, int64_t *tri, int64_t tri_rows);

/* ---- Quadric edge-collapse simplification of a welded triangle mesh (the
 * post-processing of Sec. 4.4, with Garland and Heckbert's quadric error
 * metric; it gives up the exactness of the march).  Each vertex carries the
 * area-weighted quadric of its triangles' planes; an edge collapses to the
 * point minimising the summed quadric (or the best of its ends and midpoint).
 * Rounds in parallel: every vertex keeps its cheapest edge, an edge cheapest
 * at both ends claims the vertices of all triangles around it, and an edge
 * holding all its claims collapses if its ends share exactly two neighbours
 * and no surviving triangle turns by more than about 78 degrees; claims
 * repeat three times a round among edges whose neighbourhoods no collapse
 * of that round has touched.  Rounds stop
 * at target_tris live triangles (the last round's collapses are rationed, so
 * the count ends at the target or one below it: a collapse removes two),
 * when nothing collapses, or after max_rounds (0: 256; at most 4096).
 * Errors: AM_E_INVALID for empty inputs, a NULL buffer, a negative target,
 * 3 * n_verts or 3 * n_tris at or above 2^31, or max_rounds above 4096.
 *
 * DEVICE in: vxyz [n_verts][3] f64, tri [n_tris][3] i64 (vertex ids; the
 * welded mesh and its fan triangles, consistently oriented), boundary
 * [n_verts] u8 or NULL (flagged vertices never move).  DEVICE out (capacity
 * n_verts and n_tris rows): v_out, tri_out, compacted, vertex ids into v_out.
 * HOST out: n_verts_out, n_tris_out, rounds_out, n_bad (input triangles with
 * an id out of range or a repeated vertex, dropped).  Allocates its scratch
 * (about 165 B per vertex and 52 B per triangle) for the call; synchronises. */
am_status am_simplify(am_ctx *ctx, int64_t n_verts, const double *vxyz, int64_t n_tris, const int64_t *tri,
                      const uint8_t *boundary, int64_t target_tris, int32_t max_rounds, double *v_out,
                      int64_t *tri_out, int64_t *n_verts_out, int64_t *n_tris_out, int32_t *rounds_out,
                      int64_t *n_bad);

/* ---- Affine-chain tile autotuner.  The chain kernel has eight tile
 * variants (opts.chain_groups): 4, 8 or 16 cells per workgroup (1, 2 or 4
 * column groups of the 16-column FP64 MFMA tile; more cells share each
 * streamed weight fragment, fewer fill the chip at small frontiers); 3: four
 * cells reading the previous layer from LDS; 5: four cells whose K loop
 * skips the units that are off in all of them; 6, 7, 8: the staged-B chain
 * (see am_march_opts.chain_groups).  The context keeps one variant per
 * launch-size bucket (fewer than 2^11 cells, 2^13, 2^15, more); all start
 * at 1. */

/* Times the chain kernel on the first 2^10, 2^12, 2^14 and 2^16 cells of the
 * last march (fewer if it has fewer) for each variant, `reps` launches each,
 * and keeps the fastest per bucket.  ms_out (HOST, may be NULL) receives the
 * 4 x 8 average launch times (bucket-major; variants 1..8; -1 for a variant
 * that cannot run on the loaded net).  AM_E_STATE without a finished march. */
am_status am_tune_chain(am_ctx *ctx, int32_t reps, float *ms_out);

/* Sets / reads the 4 per-bucket variants (each 1..8; HOST arrays). */
am_status am_set_chain_groups(am_ctx *ctx, const int32_t *groups);
am_status am_get_chain_groups(const am_ctx *ctx, int32_t *groups);

/* ---- Learned form: constraint-proposal scorer.
 *
 * The scorer is a ReLU MLP  x (32 features, 8 used) -> 128 -> 128 -> 1 that
 * gives each hidden line near a cell's entry edge a logit; the best k are
 * clipped first (opts.propose = 1).  Parameters are FP32, flat, in the order
 *   W1 [128][32], b1 [128], W2 [128][128], b2 [128], w3 [128], b3
 * (am_prop_param_count() of them).  The features of a line, in the plane
 * frame of the cell, relative to the entry edge (the crossed line's segment
 * between the parent's two neighbouring edges, length h): its signed distance
 * from the edge's midpoint and from both endpoints, in units of h (clamped to
 * +-16); the cosine and sine of its normal against the edge direction; its
 * layer / L; its unit's state bit; log2(h) / 16.  Candidates are the lines
 * whose midpoint distance is at most rho h. */

/* Number of scorer parameters. */
int64_t am_prop_param_count(void);

/* Loads the scorer used by propose = 1: params is a HOST array of
 * am_prop_param_count() FP32 values (copied; matrices stored as FP16 on the
 * device).  k (1..16) lines are proposed per cell among candidates within
 * rho (> 0) entry lengths.  AM_E_INVALID on a wrong count or a non-finite
 * value. */
am_status am_prop_set(am_ctx *ctx, const float *params, int64_t n_params, int32_t k, float rho);

/* Training samples: every later march of this context appends, for each cell
 * with an entry edge and a face, one row per candidate line (within rho entry
 * lengths): samples [cap][32] FP32 features, labels [cap] u8 (1 if the line
 * carries an edge of the face).  DEVICE buffers owned by the caller; rows
 * beyond cap are dropped (am_prop_collected reports the total wanted).
 * NULL buffers or cap <= 0 turn collection off.  Resets the count. */
am_status am_prop_collect(am_ctx *ctx, float *samples, uint8_t *labels, int64_t cap, float rho);

/* Rows wanted by the marches since am_prop_collect (may exceed cap). */
am_status am_prop_collected(am_ctx *ctx, int64_t *n);

/* Mean binary cross-entropy of the scorer's logits on n rows (X [n][32] FP32,
 * y [n] u8, DEVICE) and its gradient: params and grad are DEVICE arrays of
 * am_prop_param_count() FP32.  FP32 arithmetic, partial sums in FP64.  loss
 * (HOST, may be NULL) receives the mean loss; then the call synchronises. */
am_status am_prop_grad(am_ctx *ctx, const float *X, const uint8_t *y, int64_t n, const float *params,
                       float *grad, double *loss);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected, step >= 1) on
 * DEVICE arrays params, grad, m, v of am_prop_param_count() FP32.  Enqueued. */
am_status am_prop_adam(am_ctx *ctx, float *params, const float *grad, float *m, float *v, int32_t step, float lr);

/* Logits of n feature rows (X [n][32] FP32, DEVICE) by the loaded scorer as
 * the proposing clip computes them (FP16 operands on matrix cores, FP32
 * accumulation) into z [n] FP32 (DEVICE).  Enqueued. */
am_status am_prop_score(am_ctx *ctx, const float *X, int64_t n, float *z);

#ifdef __cplusplus
}
#endif

#endif /* AM_H */
