// am_frontier.hip -- seeding, the device hash set of discovered cells, and the
// result compaction (gfx950).
//
// Marching (Algorithm 1 of the paper, parallel form of Sec. 4.2.2) keeps an
// active set and checks every newly inferred state against the states seen so
// far.  Here the active set is a contiguous range of cell ids, and a
// lock-free open-addressing hash set over 64-bit slots deduplicates the
// neighbour candidates of a whole step at once:
//   insert : each candidate probes from its fingerprint; an empty slot is
//            claimed with CAS as PENDING|tag|candidate; a slot with the same
//            tag is compared on the full code (committed cell or pending
//            candidate) and, if equal, the candidate is a duplicate;
//   commit : every claiming candidate gets the next cell id, writes its code
//            and turns its slot into tag|cell;
//   resolve: every candidate writes the neighbour cell id into its parent's
//            face.
// Fingerprints are Zobrist hashes (XOR of one random key per set bit and one
// per argmax head), so a flip updates them in O(1).
#include <hipcub/hipcub.hpp>

#include "am_internal.h"

namespace am {

// Where the code of candidate t comes from: a parent cell with one flip, or
// a seed code.
struct CodeRef {
    const uint64_t *base;
    int flip;     // unit to flip, -1 = none
    int am;
    int shape;
};

__device__ __forceinline__ CodeRef cand_code(const DevNet &net, const Candidates &cand, long long t,
                                             const CellArrays &ca) {
    CodeRef r;
    const int p = cand.parent[t];
    const uint64_t *codes = ca.codes;
    const int *argmax = ca.argmax;
    if (p >= 0) {
        const int u = cand.unit[t];
        r.shape = ca.shape[p];
        r.base = codes + (long long)p * net.W;
        if (u < net.N) {
            r.flip = u;
            r.am = argmax[p];
        } else {
            r.flip = -1;
            r.am = u - net.N;
        }
    } else {
        const long long s = -1LL - p;
        r.base = ca.seed_codes + s * net.W;
        r.flip = -1;
        r.am = ca.seed_am[s];
        r.shape = ca.seed_shape ? ca.seed_shape[s] : 0;
    }
    return r;
}

__device__ __forceinline__ uint64_t code_word(const CodeRef &r, int w) {
    uint64_t x = r.base[w];
    if (r.flip >= 0 && (r.flip >> 6) == w) x ^= 1ull << (r.flip & 63);
    return x;
}

// Eight words of each code are loaded before any is compared (the loads of
// a batch overlap, and the argmax and shape compare with the first batch).
__device__ __forceinline__ bool code_eq(int W, const CodeRef &a, const CodeRef &b) {
    bool eq = a.am == b.am && a.shape == b.shape;
    for (int w0 = 0; w0 < W; w0 += 8) {
        uint64_t x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int w = min(w0 + u, W - 1);   // a repeated last word compares as it did
            x[u] = code_word(a, w);
            y[u] = code_word(b, w);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) eq = eq && x[u] == y[u];
        if (!eq) return false;
    }
    return true;
}

// ------------------------------------------------------------------ insert

__global__ __launch_bounds__(256) void k_insert(DevNet net, Candidates cand, CellArrays ca, unsigned long long *slots,
                                                unsigned long long hmask, Counters *ctr,
                                                unsigned long long cand_cap) {
    const unsigned long long n = min(ctr->n_cand, cand_cap);
    for (unsigned long long t = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; t < n;
         t += (unsigned long long)gridDim.x * blockDim.x) {
        const uint64_t h = cand.hash[t];
        const unsigned long long tag = slot_tag(h);
        const CodeRef me = cand_code(net, cand, (long long)t, ca);
        unsigned long long pos = h & hmask;
        int kind = kLost;
        long long ref = -1;
        for (unsigned long long probe = 0; probe <= hmask; ++probe) {
            unsigned long long s = __hip_atomic_load(&slots[pos], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (s == 0) {
                const unsigned long long mine = kPending | (tag << 32) | (unsigned long long)t;
                s = atomicCAS(&slots[pos], 0ull, mine);
                if (s == 0) {
                    kind = kOwner;
                    ref = (long long)pos;
                    break;
                }
            }
            if (((s >> 32) & 0x7fffffffull) == tag) {
                const long long other = (long long)(s & 0xffffffffull);
                CodeRef o;
                if (s & kPending) {
                    o = cand_code(net, cand, other, ca);
                } else {
                    o.base = ca.codes + other * net.W;
                    o.flip = -1;
                    o.am = ca.argmax[other];
                    o.shape = ca.shape[other];
                }
                if (code_eq(net.W, me, o)) {
                    kind = (s & kPending) ? kDup : kFound;
                    ref = other;
                    break;
                }
            }
            pos = (pos + 1) & hmask;
        }
        if (kind == kLost) atomicAdd(&ctr->overflow_hash, 1ull);
        cand.kind[t] = kind;
        cand.ref[t] = ref;
    }
}

// ------------------------------------------------------------------ commit

__global__ __launch_bounds__(256) void k_commit(DevNet net, Candidates cand, uint64_t *codes, int *argmax,
                                                int *shape, uint64_t *cell_hash, int *hints, unsigned *cell_key,
                                                int *face_m,
                                                const uint64_t *seed_codes, const int *seed_am,
                                                const int *seed_shape, unsigned long long *slots, Counters *ctr,
                                                unsigned long long cand_cap, unsigned long long cap_cells) {
    const unsigned long long n = min(ctr->n_cand, cand_cap);
    // resolve reads this copy, so that a device-driven step can clear n_cand
    // for the next step while resolve runs
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->n_cand_prev = ctr->n_cand;
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    // every lane of the wave runs the same number of iterations (wave_reserve)
    const unsigned long long n_round = (n + 63) & ~63ull;
    for (unsigned long long t = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; t < n_round;
         t += stride) {
        const bool own = t < n && cand.kind[t] == kOwner;
        unsigned long long base;
        const unsigned long long id = wave_reserve(&ctr->n_cells, own, &base);
        if (!own) continue;
        if (id >= cap_cells) {
            atomicAdd(&ctr->overflow_cells, 1ull);
            cand.cell[t] = -1;
            continue;
        }
        const CellArrays ca{codes, argmax, shape, seed_codes, seed_am, seed_shape};
        const CodeRef me = cand_code(net, cand, (long long)t, ca);
        uint64_t *dst = codes + (long long)id * net.W;
        for (int w = 0; w < net.W; ++w) dst[w] = code_word(me, w);
        argmax[id] = me.am;
        shape[id] = me.shape;
        const uint64_t h = cand.hash[t];
        cell_hash[id] = h;
        const int p = cand.parent[t];
        int entry = -1, hp = -1, hn = -1;
        if (p >= 0) {
            const int u = cand.unit[t];
            entry = u < net.N ? u : net.N + argmax[p];   // the crossed plane, in this cell's ids
            hp = cand.hint_prev[t];
            hn = cand.hint_next[t];
        }
        hints[id * 3 + 0] = entry;
        hints[id * 3 + 1] = hp;
        hints[id * 3 + 2] = hn;
        if (cell_key) cell_key[id] = (p >= 0 && cand.key) ? cand.key[t] : 0u;
        face_m[id] = 0;
        slots[cand.ref[t]] = ((unsigned long long)slot_tag(h) << 32) | id;
        cand.cell[t] = (int)id;
    }
}

// ----------------------------------------------------------------- resolve

// With advance set (device-driven steps), one thread also ends the step and
// takes the next step's range (up to chunk cells of the frontier, none after
// an overflow) and clears the candidate and fallback counts: nothing else in
// this kernel reads the step fields, n_cand or fb_n.
__device__ void next_step_range(Counters *c, unsigned long long chunk, unsigned long long cap_cells) {
    const unsigned long long cells = c->n_cells < cap_cells ? c->n_cells : cap_cells;
    const bool bad = c->overflowed();
    const unsigned long long lo = c->step_lo;
    unsigned long long n = (!bad && cells > lo) ? cells - lo : 0ull;
    if (n > c->max_frontier) c->max_frontier = n;
    if (n > chunk) n = chunk;
    c->step_n = n;
    c->n_cand = 0ull;
    c->fb_n = 0ull;
}

__global__ __launch_bounds__(256) void k_resolve(Candidates cand, int *face_nbr, const long long *face_off, Counters *ctr,
                                                 unsigned long long cand_cap, unsigned long long chunk,
                                                 unsigned long long cap_cells, int advance) {
    const unsigned long long n = min(ctr->n_cand_prev, cand_cap);
    if (advance && blockIdx.x == 0 && threadIdx.x == 0) {
        ctr->step_lo += ctr->step_n;
        if (ctr->step_n) ctr->steps_run += 1ull;
        next_step_range(ctr, chunk, cap_cells);
    }
    for (unsigned long long t = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; t < n;
         t += (unsigned long long)gridDim.x * blockDim.x) {
        const int p = cand.parent[t];
        if (p < 0) continue;
        const int kind = cand.kind[t];
        int c = -1;
        if (kind == kOwner) c = cand.cell[t];
        else if (kind == kFound) c = (int)cand.ref[t];
        else if (kind == kDup) c = cand.cell[cand.ref[t]];
        face_nbr[face_off[p] + cand.slot[t]] = c;
    }
}

// ------------------------------------------------------------------- seeds

// Forward pass of one point by a workgroup (Sec. 2.2).  act: LDS of
// 3 + N + M doubles; code: LDS of W words.  Returns F = max over heads and
// the argmax (lowest index on ties) to every thread.
__device__ double wg_forward(const DevNet &net, int shape, const double x[3], double *act, uint64_t *code,
                             int *am_out) {
    const double *bias = net.bias + (long long)shape * net.bias_stride;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid < 3) act[tid] = x[tid];
    for (int w = tid; w < net.W; w += nt) code[w] = 0;
    __syncthreads();
    const int L2 = net.n_layers;
    for (int l = 1; l < L2; ++l) {
        const int nl = net.width[l];
        const int aoff = 3 + net.unit_off[l];
        for (int k = tid; k < nl; k += nt) {
            double acc = bias[net.bias_off[l] + k];
            for (int b = 0; b < net.n_blocks; ++b) {
                if (net.blk_dst[b] != l) continue;
                const int j = net.blk_src[b];
                const double *Wr = net.weights + net.blk_off[b] + (long long)k * net.blk_ld[b];
                const double *aj = act + (j == 0 ? 0 : 3 + net.unit_off[j]);
                const int nj = net.width[j];
                // sixteen weights of the row (wide loads, then L1 hits) and
                // activations are loaded at once; the last, partial chunk
                // clamps its indices; the products are summed in order q = 0, 1, ...
                int q0 = 0;
                for (; q0 + 16 <= nj; q0 += 16) {
                    double wv[16], av[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        wv[u] = Wr[q0 + u];
                        av[u] = aj[q0 + u];
                    }
#pragma unroll
                    for (int u = 0; u < 16; ++u) acc += wv[u] * av[u];
                }
                if (q0 < nj) {
                    double wv[16], av[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int q = min(q0 + u, nj - 1);
                        wv[u] = Wr[q];
                        av[u] = aj[q];
                    }
#pragma unroll
                    for (int u = 0; u < 16; ++u)
                        if (q0 + u < nj) acc += wv[u] * av[u];
                }
            }
            if (l < L2 - 1) {
                act[aoff + k] = acc > 0.0 ? acc : 0.0;
                if (acc > 0.0) {
                    const int g = net.unit_off[l] + k;
                    atomicOr((unsigned long long *)&code[g >> 6], 1ull << (g & 63));
                }
            } else {
                act[aoff + k] = acc;
            }
        }
        __syncthreads();
    }
    const double *heads = act + 3 + net.N;
    int best = 0;
    for (int i = 1; i < net.M; ++i)
        if (heads[i] > heads[best]) best = i;
    const double F = heads[best];
    *am_out = best;
    __syncthreads();
    return F;
}

__global__ __launch_bounds__(256) void k_codes(DevNet net, const double *pts, const int *shape_id, long long n,
                                               uint64_t *codes, int *argmax, double *Fout) {
    extern __shared__ double lds[];
    double *act = lds;
    uint64_t *code = (uint64_t *)(lds + 3 + net.N + net.M);
    for (long long p = blockIdx.x; p < n; p += gridDim.x) {
        double x[3] = {pts[p * 3], pts[p * 3 + 1], pts[p * 3 + 2]};
        int am;
        const int sh_in = shape_id ? shape_id[p] : 0;
        const bool sh_ok = sh_in >= 0 && sh_in < net.S;   // a bad id reports argmax -1, F = NaN
        const double F = wg_forward(net, sh_ok ? sh_in : 0, x, act, code, &am);
        if (codes)
            for (int w = threadIdx.x; w < net.W; w += blockDim.x) codes[p * net.W + w] = code[w];
        if (threadIdx.x == 0) {
            if (argmax) argmax[p] = sh_ok ? am : -1;
            if (Fout) Fout[p] = sh_ok ? F : __builtin_nan("");
        }
        __syncthreads();
    }
}

// Dichotomy along o + t d, t in [0, t_max]: keep a bracket with a sign change,
// halve it until both ends share one code, then take the linear root.
__global__ __launch_bounds__(256) void k_seed_rays(DevNet net, const double *orig, const double *dir,
                                                   const int *shape_id, long long n_rays, double t_max, int max_iter,
                                                   uint64_t *seed_codes, int *seed_am, int *seed_shape,
                                                   int *status) {
    extern __shared__ double lds[];
    double *act = lds;
    uint64_t *c_lo = (uint64_t *)(lds + 3 + net.N + net.M);
    uint64_t *c_hi = c_lo + net.W;
    uint64_t *c_m = c_hi + net.W;
    __shared__ int s_eq;
    for (long long r = blockIdx.x; r < n_rays; r += gridDim.x) {
        const double o[3] = {orig[r * 3], orig[r * 3 + 1], orig[r * 3 + 2]};
        const double d[3] = {dir[r * 3], dir[r * 3 + 1], dir[r * 3 + 2]};
        int a_lo, a_hi, a_m;
        double x[3];
        const int sh_in = shape_id ? shape_id[r] : 0;
        const bool sh_ok = sh_in >= 0 && sh_in < net.S;
        const int sh = sh_ok ? sh_in : 0;
        if (threadIdx.x == 0) seed_shape[r] = sh;
        double f_lo = wg_forward(net, sh, o, act, c_m, &a_lo);
        for (int w = threadIdx.x; w < net.W; w += blockDim.x) c_lo[w] = c_m[w];
        for (int i = 0; i < 3; ++i) x[i] = o[i] + t_max * d[i];
        double f_hi = wg_forward(net, sh, x, act, c_m, &a_hi);
        for (int w = threadIdx.x; w < net.W; w += blockDim.x) c_hi[w] = c_m[w];
        __syncthreads();
        int st = 0;
        double t_lo = 0.0, t_hi = t_max;
        if (!sh_ok) {
            st = 3;   // shape id out of range
        } else if ((f_lo > 0.0) == (f_hi > 0.0)) {
            st = 1;
        } else {
            for (int it = 0;; ++it) {
                if (threadIdx.x == 0) s_eq = (a_lo == a_hi);
                __syncthreads();
                for (int w = threadIdx.x; w < net.W; w += blockDim.x)
                    if (c_lo[w] != c_hi[w]) s_eq = 0;
                __syncthreads();
                const int eq = s_eq;
                __syncthreads();
                if (eq) break;
                if (it >= max_iter) {
                    st = 2;
                    break;
                }
                const double tm = 0.5 * (t_lo + t_hi);
                for (int i = 0; i < 3; ++i) x[i] = o[i] + tm * d[i];
                const double fm = wg_forward(net, sh, x, act, c_m, &a_m);
                if ((fm > 0.0) == (f_lo > 0.0)) {
                    t_lo = tm;
                    f_lo = fm;
                    a_lo = a_m;
                    for (int w = threadIdx.x; w < net.W; w += blockDim.x) c_lo[w] = c_m[w];
                } else {
                    t_hi = tm;
                    f_hi = fm;
                    a_hi = a_m;
                    for (int w = threadIdx.x; w < net.W; w += blockDim.x) c_hi[w] = c_m[w];
                }
                __syncthreads();
            }
        }
        if (st == 0) {
            const double ts = t_lo - f_lo * (t_hi - t_lo) / (f_hi - f_lo);
            for (int i = 0; i < 3; ++i) x[i] = o[i] + ts * d[i];
            wg_forward(net, sh, x, act, c_m, &a_m);
            for (int w = threadIdx.x; w < net.W; w += blockDim.x) seed_codes[r * net.W + w] = c_m[w];
            if (threadIdx.x == 0) seed_am[r] = a_m;
        } else {
            for (int w = threadIdx.x; w < net.W; w += blockDim.x) seed_codes[r * net.W + w] = 0;
            if (threadIdx.x == 0) seed_am[r] = 0;
        }
        if (threadIdx.x == 0 && status) status[r] = st;
        __syncthreads();
    }
}

// Gradient of the selected head in the cell of `code` by a reverse pass:
// the head's adjoint goes down through every block (l <- j), masked by the
// ReLU states of layer l's units (hidden layers only).  adj: LDS of
// 3 + N + M doubles.  Returns the xyz gradient to every thread.
__device__ void wg_grad(const DevNet &net, const uint64_t *code, int am, double *adj, double g[3]) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int total = 3 + net.N + net.M;
    for (int i = tid; i < total; i += nt) adj[i] = 0.0;
    __syncthreads();
    if (tid == 0) adj[3 + net.N + am] = 1.0;
    __syncthreads();
    const int L2 = net.n_layers;
    for (int l = L2 - 1; l >= 1; --l) {
        const int nl = net.width[l];
        const double *al = adj + 3 + net.unit_off[l];
        const bool hidden = l < L2 - 1;
        for (int b = 0; b < net.n_blocks; ++b) {
            if (net.blk_dst[b] != l) continue;
            const int j = net.blk_src[b];
            const int nj = net.width[j];
            double *aj = adj + (j == 0 ? 0 : 3 + net.unit_off[j]);
            const double *Wb = net.weights + net.blk_off[b];
            const int ld = net.blk_ld[b];
            for (int q = tid; q < nj; q += nt) {
                double acc = 0.0;
#pragma unroll 8
                for (int k = 0; k < nl; ++k) {
                    const double a = al[k];
                    if (a == 0.0 || (hidden && !code_bit(code, net.unit_off[l] + k))) continue;
                    acc += Wb[(long long)k * ld + q] * a;
                }
                aj[q] += acc;
            }
        }
        __syncthreads();
    }
    g[0] = adj[0];
    g[1] = adj[1];
    g[2] = adj[2];
    __syncthreads();
}

// Sphere-tracing seeds (Sec. 4.3.1, Eqn (SphereTracing)): from each start
// point, x <- x - F g / |g|^2 with g the gradient of F in the current cell
// (the paper's step of size 1 when |g| = 1), until a step lands in the cell
// it started from.  Status 0 settled, 1 max_iter steps without settling,
// 2 zero gradient, 3 settled outside [-1, 1]^3, 4 shape id out of range.
__global__ __launch_bounds__(256) void k_seed_st(DevNet net, const double *pts, const int *shape_id, long long n,
                                                 int max_iter, uint64_t *seed_codes, int *seed_am,
                                                 int *seed_shape, int *status, int *iters, double *x_out) {
    extern __shared__ double lds[];
    double *act = lds;
    double *adj = lds + 3 + net.N + net.M;
    uint64_t *c_cur = (uint64_t *)(adj + 3 + net.N + net.M);
    uint64_t *c_new = c_cur + net.W;
    __shared__ int s_eq;
    for (long long r = blockIdx.x; r < n; r += gridDim.x) {
        double x[3] = {pts[r * 3], pts[r * 3 + 1], pts[r * 3 + 2]};
        const int sh_in = shape_id ? shape_id[r] : 0;
        const bool sh_ok = sh_in >= 0 && sh_in < net.S;
        const int sh = sh_ok ? sh_in : 0;
        int a_cur = 0, a_new = 0, st = 1, it = 0;
        double F = wg_forward(net, sh, x, act, c_cur, &a_cur);
        if (!sh_ok) {
            st = 4;
        } else if (F == 0.0) {
            st = 0;
        } else {
            for (it = 0; it < max_iter;) {
                double g[3];
                wg_grad(net, c_cur, a_cur, adj, g);
                const double gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
                if (!(gg > 0.0)) {
                    st = 2;
                    break;
                }
                for (int i = 0; i < 3; ++i) x[i] -= F * g[i] / gg;
                const double Fq = wg_forward(net, sh, x, act, c_new, &a_new);
                ++it;
                if (threadIdx.x == 0) s_eq = (a_new == a_cur);
                __syncthreads();
                for (int w = threadIdx.x; w < net.W; w += blockDim.x)
                    if (c_new[w] != c_cur[w]) s_eq = 0;
                __syncthreads();
                const int eq = s_eq;
                __syncthreads();
                if (eq) {
                    st = 0;
                    break;
                }
                for (int w = threadIdx.x; w < net.W; w += blockDim.x) c_cur[w] = c_new[w];
                a_cur = a_new;
                F = Fq;
                __syncthreads();
            }
        }
        if (st == 0 && (fabs(x[0]) > 1.0 || fabs(x[1]) > 1.0 || fabs(x[2]) > 1.0)) st = 3;
        for (int w = threadIdx.x; w < net.W; w += blockDim.x) seed_codes[r * net.W + w] = st == 0 ? c_cur[w] : 0ull;
        if (threadIdx.x == 0) {
            seed_am[r] = st == 0 ? a_cur : 0;
            seed_shape[r] = sh;
            if (status) status[r] = st;
            if (iters) iters[r] = it;
            if (x_out) {
                x_out[r * 3] = x[0];
                x_out[r * 3 + 1] = x[1];
                x_out[r * 3 + 2] = x[2];
            }
        }
        __syncthreads();
    }
}

// Seeds with status 0 become candidates (parent = -(1 + seed index)).
__global__ __launch_bounds__(256) void k_seed_cands(DevNet net, const uint64_t *seed_codes, const int *seed_am,
                                                    const int *seed_shape, const int *seed_ok, long long n,
                                                    Candidates cand,
                                                    Counters *ctr, unsigned long long cand_cap) {
    const long long n_round = (n + 63) & ~63LL;
    for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < n_round;
         s += (long long)gridDim.x * blockDim.x) {
        const bool ok = s < n && (!seed_ok || seed_ok[s] == 0) && seed_am[s] >= 0 && seed_am[s] < net.M &&
                        seed_shape[s] >= 0 && seed_shape[s] < net.S;
        unsigned long long base;
        const unsigned long long idx = wave_reserve(&ctr->n_cand, ok, &base);
        if (!ok) continue;
        if (idx >= cand_cap) {
            atomicAdd(&ctr->overflow_cand, 1ull);
            continue;
        }
        uint64_t h = net.zobrist[net.N + seed_am[s]] ^ net.zobrist[net.N + net.M + seed_shape[s]];
        for (int w = 0; w < net.W; ++w) {
            uint64_t x = seed_codes[s * net.W + w];
            while (x) {
                const int b = __builtin_ctzll(x);
                x &= x - 1;
                const int g = w * 64 + b;
                if (g < net.N) h ^= net.zobrist[g];
            }
        }
        cand.parent[idx] = (int)(-1 - s);
        cand.slot[idx] = -1;
        cand.unit[idx] = -1;
        cand.hash[idx] = h;
    }
}

// ------------------------------------------------------------------- fetch

__global__ void k_face_flags(const int *face_m, long long n, int *has, long long *mcount) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const int m = face_m[c];
        has[c] = m > 0 ? 1 : 0;
        mcount[c] = m;
    }
}

// The outputs never alias the march's arrays, and each face's corners are
// taken four at a time with every load of the four issued before any store,
// so a face costs a few dependent round trips (neighbour id, then its face
// index) instead of three per corner.
__global__ void k_fetch(const DevNet net, long long n, const int *__restrict__ face_m, const int *__restrict__ fidx,
                        const long long *__restrict__ voff, const int *__restrict__ ids,
                        const double *__restrict__ verts, const int *__restrict__ nbr,
                        const uint64_t *__restrict__ codes, const int *__restrict__ argmax,
                        const int *__restrict__ shape, const long long *__restrict__ foff,
                        long long *__restrict__ o_off, int *__restrict__ o_ids, double *__restrict__ o_verts,
                        long long *__restrict__ o_nbr, uint64_t *__restrict__ o_codes, int *__restrict__ o_am,
                        int *__restrict__ o_shape) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const int m = face_m[c];
        if (m <= 0) continue;
        const long long f = fidx[c];
        const long long o = voff[c];
        const long long s0 = foff[c];
        if (o_off) o_off[f] = o;
        if (o_codes)
            for (int w = 0; w < net.W; ++w) o_codes[f * net.W + w] = codes[c * net.W + w];
        if (o_am) o_am[f] = argmax[c];
        if (o_shape) o_shape[f] = shape[c];
        for (int i0 = 0; i0 < m; i0 += 4) {
            int id[4], g[4], gm[4], gf[4];
            double x[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long long s = s0 + min(i0 + u, m - 1);
                id[u] = ids[s];
                x[u][0] = verts[s * 3 + 0];
                x[u][1] = verts[s * 3 + 1];
                x[u][2] = verts[s * 3 + 2];
                g[u] = o_nbr ? nbr[s] : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                gm[u] = g[u] >= 0 ? face_m[g[u]] : 0;
                gf[u] = g[u] >= 0 ? fidx[g[u]] : 0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (i0 + u >= m) break;
                const long long t = o + i0 + u;
                if (o_ids) o_ids[t] = id[u];
                if (o_verts) {
                    o_verts[t * 3 + 0] = x[u][0];
                    o_verts[t * 3 + 1] = x[u][1];
                    o_verts[t * 3 + 2] = x[u][2];
                }
                if (o_nbr) o_nbr[t] = g[u] < 0 ? -1 : (gm[u] > 0 ? (long long)gf[u] : -2);
            }
        }
    }
}

__global__ void k_fetch_tail(long long *o_off, long long F, const long long *voff, const int *face_m,
                             long long n) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && o_off) o_off[F] = n > 0 ? voff[n - 1] + face_m[n - 1] : 0;
}

// ---- canonical face order: faces sorted by shape id, then code words
// (unsigned, word 0 first), then argmax; neighbour indices follow the order.
// Least-significant-key-first passes of a stable radix sort over a face
// permutation.

__global__ void k_face_cells(const int *face_m, const int *fidx, long long n, int *face_cell) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x)
        if (face_m[c] > 0) face_cell[fidx[c]] = (int)c;
}

__global__ void k_iota_int(int *v, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        v[i] = (int)i;
}

// which >= 0: code word `which`; -1: argmax; -2: shape id.
__global__ void k_sort_key(const int *perm, const int *face_cell, const uint64_t *codes, const int *argmax,
                           const int *shape, int W, int which, long long F, uint64_t *keys) {
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < F;
         p += (long long)gridDim.x * blockDim.x) {
        const long long c = face_cell[perm[p]];
        uint64_t k;
        if (which >= 0) k = codes[c * W + which];
        else if (which == -1) k = (uint64_t)(uint32_t)argmax[c];
        else k = (uint64_t)(uint32_t)(shape ? shape[c] : 0);
        keys[p] = k;
    }
}

__global__ void k_sorted_counts(const int *perm, const int *face_cell, const int *face_m, long long F, int *rank,
                                long long *mcount) {
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < F;
         p += (long long)gridDim.x * blockDim.x) {
        const int f = perm[p];
        rank[f] = (int)p;
        mcount[p] = face_m[face_cell[f]];
    }
}

__global__ void k_fetch_sorted(const DevNet net, long long F, const int *perm, const int *face_cell,
                               const int *rank, const long long *voff, const int *face_m, const int *fidx,
                               const int *ids, const double *verts, const int *nbr, const uint64_t *codes,
                               const int *argmax, const int *shape, const long long *foff, long long *o_off,
                               int *o_ids, double *o_verts, long long *o_nbr, uint64_t *o_codes, int *o_am,
                               int *o_shape) {
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < F;
         p += (long long)gridDim.x * blockDim.x) {
        const long long c = face_cell[perm[p]];
        const int m = face_m[c];
        const long long o = voff[p];
        if (o_off) o_off[p] = o;
        if (o_codes)
            for (int w = 0; w < net.W; ++w) o_codes[p * net.W + w] = codes[c * net.W + w];
        if (o_am) o_am[p] = argmax[c];
        if (o_shape) o_shape[p] = shape[c];
        for (int i = 0; i < m; ++i) {
            const long long s = foff[c] + i;
            if (o_ids) o_ids[o + i] = ids[s];
            if (o_verts) {
                o_verts[(o + i) * 3 + 0] = verts[s * 3 + 0];
                o_verts[(o + i) * 3 + 1] = verts[s * 3 + 1];
                o_verts[(o + i) * 3 + 2] = verts[s * 3 + 2];
            }
            if (o_nbr) {
                const int g = nbr[s];
                o_nbr[o + i] = g < 0 ? -1 : (face_m[g] > 0 ? (long long)rank[fidx[g]] : -2);
            }
        }
    }
}

__global__ void k_sorted_tail(long long *o_off, long long F, const long long *voff, const long long *mcount) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && o_off) o_off[F] = F > 0 ? voff[F - 1] + mcount[F - 1] : 0;
}

// ---------------------------------------------------------------- launchers

static unsigned grid_for(long long n, int block = 256, long long cap = 2048) {
    long long b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

void launch_insert(const DevNet &net, const Candidates &cand, const CellArrays &ca, unsigned long long *slots,
                   unsigned long long hmask, Counters *ctr, unsigned long long cand_cap, long long n_hint,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_insert, dim3(grid_for(n_hint)), dim3(256), 0, st, net, cand, ca, slots, hmask, ctr, cand_cap);
}

void launch_commit(const DevNet &net, const Candidates &cand, uint64_t *codes, int *argmax, int *shape,
                   uint64_t *cell_hash, int *hints, unsigned *cell_key, int *face_m, const uint64_t *seed_codes,
                   const int *seed_am, const int *seed_shape, unsigned long long *slots, Counters *ctr,
                   unsigned long long cand_cap, unsigned long long cap_cells, long long n_hint, hipStream_t st) {
    hipLaunchKernelGGL(k_commit, dim3(grid_for(n_hint)), dim3(256), 0, st, net, cand, codes, argmax, shape, cell_hash,
                       hints, cell_key, face_m, seed_codes, seed_am, seed_shape, slots, ctr, cand_cap, cap_cells);
}

// Orders cells lo..lo+n-1 by their Morton keys: order[p] = the p-th cell.
// tmp must hold sort_tmp_bytes(n); keys_out and ids are n words of scratch.
__global__ void k_iota(int *ids, long long lo, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ids[i] = (int)(lo + i);
}

hipError_t sort_tmp_bytes(long long n, size_t *bytes) {
    return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, (const unsigned *)nullptr, (unsigned *)nullptr,
                                              (const int *)nullptr, (int *)nullptr, (int)n, 0, 30);
}

hipError_t launch_sort_cells(const unsigned *cell_key, long long lo, long long n, unsigned *keys_out, int *ids,
                             int *order, void *tmp, size_t tmp_bytes, hipStream_t st) {
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ids, lo, n);
    size_t tb = tmp_bytes;
    return hipcub::DeviceRadixSort::SortPairs(tmp, tb, cell_key + lo, keys_out, ids, order, (int)n, 0, 30, st);
}

void launch_resolve(const Candidates &cand, int *face_nbr, const long long *face_off, Counters *ctr,
                    unsigned long long cand_cap,
                    long long n_hint, hipStream_t st, long long chunk, long long cap_cells) {
    hipLaunchKernelGGL(k_resolve, dim3(grid_for(n_hint)), dim3(256), 0, st, cand, face_nbr, face_off, ctr, cand_cap,
                       (unsigned long long)(chunk > 0 ? chunk : 0), (unsigned long long)(cap_cells > 0 ? cap_cells : 0),
                       chunk > 0 ? 1 : 0);
}

size_t forward_lds_bytes(const DevNet &net, int code_bufs) {
    return sizeof(double) * (3 + net.N + net.M) + sizeof(uint64_t) * net.W * code_bufs;
}

void launch_codes(const DevNet &net, const double *pts, const int *shape_id, long long n, uint64_t *codes,
                  int *argmax, double *F, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_codes, dim3(grid_for(n, 1, 8192)), dim3(256), forward_lds_bytes(net, 1), st, net, pts,
                       shape_id, n, codes, argmax, F);
}

void launch_seed_rays(const DevNet &net, const double *orig, const double *dir, const int *shape_id, long long n,
                      double t_max, int max_iter, uint64_t *seed_codes, int *seed_am, int *seed_shape, int *status,
                      hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_seed_rays, dim3(grid_for(n, 1, 8192)), dim3(256), forward_lds_bytes(net, 3), st, net,
                       orig, dir, shape_id, n, t_max, max_iter, seed_codes, seed_am, seed_shape, status);
}

void launch_seed_st(const DevNet &net, const double *pts, const int *shape_id, long long n, int max_iter,
                    uint64_t *seed_codes, int *seed_am, int *seed_shape, int *status, int *iters, double *x_out,
                    hipStream_t st) {
    if (n <= 0) return;
    const size_t lds = sizeof(double) * 2 * (3 + net.N + net.M) + sizeof(uint64_t) * 2 * net.W;
    hipLaunchKernelGGL(k_seed_st, dim3(grid_for(n, 1, 8192)), dim3(256), lds, st, net, pts, shape_id, n, max_iter,
                       seed_codes, seed_am, seed_shape, status, iters, x_out);
}

size_t seed_st_lds_bytes(const DevNet &net) {
    return sizeof(double) * 2 * (3 + net.N + net.M) + sizeof(uint64_t) * 2 * net.W;
}

void launch_seed_cands(const DevNet &net, const uint64_t *seed_codes, const int *seed_am, const int *seed_shape,
                       const int *seed_ok, long long n, const Candidates &cand, Counters *ctr,
                       unsigned long long cand_cap, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_seed_cands, dim3(grid_for(n)), dim3(256), 0, st, net, seed_codes, seed_am, seed_shape,
                       seed_ok, n, cand, ctr, cand_cap);
}

// Compacts faces of cells 0..n-1 into CSR form.  tmp must hold scan_tmp_bytes(n).
hipError_t scan_tmp_bytes(long long n, size_t *bytes) {
    size_t a = 0, b = 0;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, a, (int *)nullptr, (int *)nullptr, (int)n);
    if (e != hipSuccess) return e;
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, b, (long long *)nullptr, (long long *)nullptr, (int)n);
    *bytes = a > b ? a : b;
    return e;
}

hipError_t launch_fetch(const DevNet &net, long long n, const int *face_m, const int *ids, const double *verts,
                        const int *nbr, const uint64_t *codes, const int *argmax, const int *shape,
                        const long long *foff,
                        int *has, int *fidx, long long *mcount, long long *voff, void *tmp, size_t tmp_bytes,
                        long long F, long long *o_off, int *o_ids, double *o_verts, long long *o_nbr,
                        uint64_t *o_codes, int *o_am, int *o_shape, hipStream_t st) {
    if (n <= 0) {
        if (o_off) return hipMemsetAsync(o_off, 0, sizeof(long long), st);
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_face_flags, dim3(grid_for(n)), dim3(256), 0, st, face_m, n, has, mcount);
    size_t tb = tmp_bytes;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(tmp, tb, has, fidx, (int)n, st);
    if (e != hipSuccess) return e;
    tb = tmp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(tmp, tb, mcount, voff, (int)n, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fetch, dim3(grid_for(n)), dim3(256), 0, st, net, n, face_m, fidx, voff, ids, verts, nbr,
                       codes, argmax, shape, foff, o_off, o_ids, o_verts, o_nbr, o_codes, o_am, o_shape);
    hipLaunchKernelGGL(k_fetch_tail, dim3(1), dim3(64), 0, st, o_off, F, voff, face_m, n);
    return hipGetLastError();
}

// Scratch of the canonical fetch for F faces: sort temporary bytes (the scan
// temporary of launch_fetch is reused for the sorted counts).
hipError_t sorted_fetch_tmp_bytes(long long F, size_t *bytes) {
    size_t a = 0, b = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                                      (const int *)nullptr, (int *)nullptr, (int)F, 0, 64);
    if (e != hipSuccess) return e;
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, b, (long long *)nullptr, (long long *)nullptr, (int)F);
    *bytes = a > b ? a : b;
    return e;
}

// As launch_fetch, faces in canonical order.  face_cell, perm_a, perm_b, rank
// [F] ints, keys_a, keys_b [F] u64, mcs, voffs [F] i64 scratch; tmp holds
// sorted_fetch_tmp_bytes(F) (and scan_tmp_bytes(n) for the cell scan).
hipError_t launch_fetch_sorted(const DevNet &net, long long n, const int *face_m, const int *ids,
                               const double *verts, const int *nbr, const uint64_t *codes, const int *argmax,
                               const int *shape, const long long *foff, int *has, int *fidx, long long *mcount,
                               long long *voff, void *scan_tmp, size_t scan_bytes, long long F, int *face_cell,
                               int *perm_a, int *perm_b, int *rank, uint64_t *keys_a, uint64_t *keys_b,
                               long long *mcs, long long *voffs, void *tmp, size_t tmp_bytes, long long *o_off,
                               int *o_ids, double *o_verts, long long *o_nbr, uint64_t *o_codes, int *o_am,
                               int *o_shape, hipStream_t st) {
    if (n <= 0 || F <= 0) {
        if (o_off) return hipMemsetAsync(o_off, 0, sizeof(long long), st);
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_face_flags, dim3(grid_for(n)), dim3(256), 0, st, face_m, n, has, mcount);
    size_t tb = scan_bytes;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(scan_tmp, tb, has, fidx, (int)n, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_face_cells, dim3(grid_for(n)), dim3(256), 0, st, face_m, fidx, n, face_cell);
    hipLaunchKernelGGL(k_iota_int, dim3(grid_for(F)), dim3(256), 0, st, perm_a, F);
    // least significant key first: argmax, code words W-1 .. 0, shape
    for (int pass = 0; pass < net.W + 2; ++pass) {
        const int which = pass == 0 ? -1 : (pass <= net.W ? net.W - pass : -2);
        if (which == -2 && net.S <= 1) break;
        if (which == -1 && net.M <= 1) continue;
        hipLaunchKernelGGL(k_sort_key, dim3(grid_for(F)), dim3(256), 0, st, perm_a, face_cell, codes, argmax, shape,
                           net.W, which, F, keys_a);
        tb = tmp_bytes;
        e = hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys_a, keys_b, perm_a, perm_b, (int)F, 0,
                                               which >= 0 ? 64 : 32, st);
        if (e != hipSuccess) return e;
        int *t = perm_a;
        perm_a = perm_b;
        perm_b = t;
    }
    hipLaunchKernelGGL(k_sorted_counts, dim3(grid_for(F)), dim3(256), 0, st, perm_a, face_cell, face_m, F, rank, mcs);
    tb = tmp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(tmp, tb, mcs, voffs, (int)F, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fetch_sorted, dim3(grid_for(F)), dim3(256), 0, st, net, F, perm_a, face_cell, rank, voffs,
                       face_m, fidx, ids, verts, nbr, codes, argmax, shape, foff, o_off, o_ids, o_verts, o_nbr,
                       o_codes, o_am, o_shape);
    hipLaunchKernelGGL(k_sorted_tail, dim3(1), dim3(64), 0, st, o_off, F, voffs, mcs);
    return hipGetLastError();
}

}  // namespace am
