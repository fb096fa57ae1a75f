// am_kernels.hip -- per-cell work of analytic marching on gfx950: the affine
// chain on FP64 matrix cores and the analytic face by halfplane clipping.
//
// Affine chain.  For a cell with activation code s, Lemma 1 and Corollary 1 of
// the paper give every pre-activation as an affine function of x inside the
// cell.  With the bias carried by the homogeneous coordinate, the rows Z_l
// (n_l x 4) obey
//     Z_0 = [I_3 | 0],
//     Z_l = sum over blocks (l <- j) of W_{l<-j} diag(s_j) Z_j  +  b_l e_4^T,
// where diag(s_0) = I (the input is never rectified); the shortcut blocks of
// Sec. 5.1 and the max-pooled heads of Sec. 5.2 are ordinary blocks.  Batched
// over cells this is a dense GEMM per layer, W (n_l x n_j) times the stacked
// masked rows [diag(s^(c)) Z_j^(c)]_c (n_j x 4C); a workgroup of four waves
// owns four cells = 16 columns, the N size of v_mfma_f64_16x16x4f64.  The
// mask diag(s_j) is applied while loading the B operand.
//
// Analytic face.  The face of a cell (Eqn (AnalyticFace)) is the part of the
// zero plane a_F . [x;1] = 0 where every oriented constraint
// (1 - 2 s_k) a_k . [x;1] <= 0 holds (Eqn (AnalyticCellSystem)), plus the
// max-pool sub-cell rows (a_F(i) - a_F(j)) . [x;1] <= 0 of Eqn
// (AnalyticCellSystemMaxPooling), inside the domain box.  Instead of the
// paper's pair enumeration (Algorithm 1) or pivoting (Sec. 4.2.1), one wave
// clips a polygon in a 2-D frame of the plane:
//   * lane i holds vertex i (frame coordinates, id of the edge it starts);
//   * constraints are tested 64 at a time, one per lane, against every
//     vertex (broadcast with readlane); only the lines that cut are applied;
//   * a cut is one Sutherland-Hodgman pass: each lane emits 0-2 vertices,
//     positions come from two ballots and a popcount (wave compaction), the
//     new polygon goes through the wave's LDS scratch.
// Vertices are then recomputed in FP64 from their two edge ids and the plane
// (Eqn (VertexEquationSystem)), and each edge on a hidden unit or head
// comparison becomes a neighbour candidate (state flip, Sec. 3.1).
#include <type_traits>

#include "am_internal.h"

namespace am {

typedef double v4d __attribute__((ext_vector_type(4)));

#ifndef AM_KCHUNK
#define AM_KCHUNK 8
#endif
constexpr int kKChunk = AM_KCHUNK;     // K-steps whose operands are loaded before their MFMAs issue
constexpr int kMaxWords = kMaxHidden / 64;

// Cells of a tile: positions p0..p0+ncell-1 of the active range, i.e. cell
// p0 + c, or list[p0 + c] when a cell list is given.
__device__ __forceinline__ long long tile_cell(const int *list, long long p0, int c) {
    return list ? (long long)list[p0 + c] : p0 + c;
}

// Stages the codes and shape ids of a tile's ncell (<= nmax) cells in LDS
// (ends with a barrier).
__device__ void stage_tile(const DevNet &net, const uint64_t *codes, const int *cell_shape,
                           const int *list, long long p0, int ncell, uint64_t *code_lds, int *shape_lds,
                           int nmax = 4) {
    for (int t = threadIdx.x; t < nmax * net.W; t += blockDim.x) {
        const int c = t / net.W;
        code_lds[t] = c < ncell ? codes[tile_cell(list, p0, c) * net.W + (t - c * net.W)] : 0ull;
    }
    if (threadIdx.x < nmax) {
        const int c = threadIdx.x;
        const int sh = (cell_shape && c < ncell) ? cell_shape[tile_cell(list, p0, c)] : 0;
        shape_lds[c] = (sh >= 0 && sh < net.S) ? sh : 0;
    }
    __syncthreads();
}

// Affine chain of the 4 G cells c0..c0+ncell-1 of a tile: G groups of 16 MFMA
// columns (cell = 4 g + col / 4, homogeneous component q = col % 4).  Element
// (row, cell, q) of the rows is zb[row * rs + cell * cs + q].  Each wave takes
// two 16-row output tiles at a time (mt and mt + nwaves), so that every A
// fragment (weights) feeds 2 G MFMAs and every B value feeds two: a tile of
// 4 G cells streams each weight block from L2 once.  Operands of KC K-steps
// are loaded before their MFMAs issue.  Ends with a barrier.
// With zl (LDS, 2 x kLdsRows x 16 doubles, G = 1), the rows of each layer of
// at most kLdsRows units are also kept in LDS (ping-pong by layer parity) and
// the next layer reads its B operand there instead of from global memory.
constexpr int kLdsRows = 128;

template <int G, int KC>
__device__ void chain_tile(const DevNet &net, const uint64_t *codes,
                           const int *cell_shape, const int *list, long long c0, int ncell, double *zb,
                           long long rs, long long cs, uint64_t *code_lds, int *shape_lds, double *zl = nullptr,
                           bool staged = false) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int col = lane & 15;       // MFMA column (B, D) / row within the tile (A)
    const int kq = lane >> 4;        // k within the K-step of 4 (A, B) / row offset (D)
    const int q = col & 3;           // homogeneous component of this column
    const int cl = col >> 2;         // cell of this column within its group
    if (!staged) stage_tile(net, codes, cell_shape, list, c0, ncell, code_lds, shape_lds, 4 * G);
    long long bias_base[G];
    const uint64_t *code[G];
    double *zc[G];
    bool cell_ok[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int c = 4 * g + cl;
        cell_ok[g] = c < ncell;
        bias_base[g] = (long long)shape_lds[c] * net.bias_stride;
        code[g] = code_lds + c * net.W;
        zc[g] = zb + c * cs + q;
    }

    for (int l = 1; l < net.n_layers; ++l) {
        const int nl = net.width[l];
        const int mtiles = (nl + 15) >> 4;
        for (int mt0 = wave; mt0 < mtiles; mt0 += 2 * nwaves) {
            const int mt1 = mt0 + nwaves;
            const bool two = mt1 < mtiles;
            v4d acc0[G], acc1[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                acc0[g] = v4d{0.0, 0.0, 0.0, 0.0};
                acc1[g] = v4d{0.0, 0.0, 0.0, 0.0};
            }
            for (int b = 0; b < net.n_blocks; ++b) {
                if (net.blk_dst[b] != l) continue;
                const int j = net.blk_src[b];
                const int ks_n = net.blk_ld[b] >> 2;
                const int nj = net.width[j];
                // A fragments: 64 doubles per (tile, K-step), already in lane order
                const double *fr0 = net.wfrag + net.blk_frag_off[b] + (long long)mt0 * ks_n * 64 + lane;
                const double *fr1 = fr0 + (long long)(mt1 - mt0) * ks_n * 64;
                if (j == 0) {
                    // Z_0 = [I | 0]: one K-step; row k of B is e_k for k < 3
                    const double bv = (kq < 3 && kq == q) ? 1.0 : 0.0;
                    const double a0 = fr0[0], a1 = two ? fr1[0] : 0.0;
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        acc0[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv, acc0[g], 0, 0, 0);
                        if (two) acc1[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv, acc1[g], 0, 0, 0);
                    }
                    continue;
                }
                const int uoff = net.unit_off[j];
                const long long roff = (long long)net.row_off[j] * rs;
                // B from LDS: the previous layer, kept there when it fits
                const double *zin = (zl && j == l - 1 && nj <= kLdsRows) ? zl + (j & 1) * kLdsRows * 16 + col
                                                                         : nullptr;
                for (int ks0 = 0; ks0 < ks_n; ks0 += KC) {
                    double a0[KC], a1[KC], bv[G][KC];
#pragma unroll
                    for (int u = 0; u < KC; ++u) {
                        const int ks = ks0 + u;
                        const bool kv = ks < ks_n;
                        const int k = ks * 4 + kq;
                        a0[u] = kv ? fr0[ks * 64] : 0.0;
                        a1[u] = (kv && two) ? fr1[ks * 64] : 0.0;
#pragma unroll
                        for (int g = 0; g < G; ++g)
                            bv[g][u] = (kv && k < nj && cell_ok[g] && code_bit(code[g], uoff + k))
                                           ? (zin ? zin[k * 16] : zc[g][roff + k * rs]) : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < KC; ++u) {
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            acc0[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], bv[g][u], acc0[g], 0, 0, 0);
                            if (two) acc1[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], bv[g][u], acc1[g], 0, 0, 0);
                        }
                    }
                }
            }
            // v_mfma_f64_16x16x4f64 leaves D[kq + 4 r][col] in register r of
            // lane (kq * 16 + col)
            double *zout = (zl && nl <= kLdsRows) ? zl + (l & 1) * kLdsRows * 16 + col : nullptr;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (!cell_ok[g]) continue;
                const double *bias = net.bias + bias_base[g] + net.bias_off[l];
                double *z0 = zc[g] + (long long)net.row_off[l] * rs;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i0 = mt0 * 16 + kq + 4 * r;
                    if (i0 < nl) {
                        const double v = acc0[g][r] + (q == 3 ? bias[i0] : 0.0);
                        z0[i0 * rs] = v;
                        if (zout) zout[i0 * 16] = v;
                    }
                    const int i1 = mt1 * 16 + kq + 4 * r;
                    if (two && i1 < nl) {
                        const double v = acc1[g][r] + (q == 3 ? bias[i1] : 0.0);
                        z0[i1 * rs] = v;
                        if (zout) zout[i1 * 16] = v;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---- staged chain: four cells per workgroup; before each layer the rows of
// the previous hidden layer (written by the workgroup to global memory) are
// copied once, masked by the cells' codes and zero padded to the K-steps,
// into one LDS buffer (widest hidden layer x 16 doubles, at most kResMax
// units), so the four waves read their B operand there instead of each
// fetching it through L1.  Shortcut sources are read from global memory as
// in the dense tile.  Ends with a barrier.
constexpr int kResMax = 512;

template <int KC>
__device__ void chain_tile_res(const DevNet &net, const uint64_t *__restrict__ codes,
                               const int *__restrict__ cell_shape, const int *list, long long c0, int ncell,
                               double *zb, long long rs, long long cs, uint64_t *code_lds, int *shape_lds,
                               double *zr) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    constexpr int nwaves = 4;
    const int col = lane & 15;
    const int kq = lane >> 4;
    const int q = col & 3;
    const int cl = col >> 2;
    stage_tile(net, codes, cell_shape, list, c0, ncell, code_lds, shape_lds, 4);
    const bool cell_ok = cl < ncell;
    const long long bias_base = (long long)shape_lds[cl] * net.bias_stride;
    const uint64_t *code = code_lds + cl * net.W;
    double *zc = zb + cl * cs + q;

    for (int l = 1; l < net.n_layers; ++l) {
        const int nl = net.width[l];
        const int mtiles = (nl + 15) >> 4;
        const int jp = l - 1;
        const int njp = net.width[jp];
        const int ldp = (njp + 3) & ~3;
        if (jp >= 1) {
            // stage the previous layer: element (k, cell, q) at zr[k * 16 + 4 cell + q]
            const int uoff = net.unit_off[jp];
            const long long roff = (long long)net.row_off[jp] * rs;
            for (int t = threadIdx.x; t < 16 * ldp; t += blockDim.x) {
                const int c = t / (4 * ldp);
                const int r = t - c * 4 * ldp;
                const int k = r >> 2, qq = r & 3;
                double v = 0.0;
                if (c < ncell && k < njp && code_bit(code_lds + c * net.W, uoff + k))
                    v = zb[c * cs + roff + (long long)k * rs + qq];
                zr[k * 16 + 4 * c + qq] = v;
            }
            __syncthreads();
        }
        for (int mt0 = wave; mt0 < mtiles; mt0 += 2 * nwaves) {
            const int mt1 = mt0 + nwaves;
            const bool two = mt1 < mtiles;
            v4d acc0 = v4d{0.0, 0.0, 0.0, 0.0}, acc1 = v4d{0.0, 0.0, 0.0, 0.0};
            for (int b = 0; b < net.n_blocks; ++b) {
                if (net.blk_dst[b] != l) continue;
                const int j = net.blk_src[b];
                const int ks_n = net.blk_ld[b] >> 2;
                const int nj = net.width[j];
                const double *fr0 = net.wfrag + net.blk_frag_off[b] + (long long)mt0 * ks_n * 64 + lane;
                const double *fr1 = fr0 + (long long)(mt1 - mt0) * ks_n * 64;
                if (j == 0) {
                    const double bv = (kq < 3 && kq == q) ? 1.0 : 0.0;
                    const double a0 = fr0[0], a1 = two ? fr1[0] : 0.0;
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv, acc0, 0, 0, 0);
                    if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv, acc1, 0, 0, 0);
                    continue;
                }
                if (j == jp) {
                    // staged: masked and padded, no bounds or code tests
                    const double *zin = zr + kq * 16 + col;
                    for (int ks0 = 0; ks0 < ks_n; ks0 += KC) {
                        double a0[KC], a1[KC], bv[KC];
#pragma unroll
                        for (int u = 0; u < KC; ++u) {
                            const int ks = ks0 + u;
                            const bool kv = ks < ks_n;
                            a0[u] = kv ? fr0[ks * 64] : 0.0;
                            a1[u] = (kv && two) ? fr1[ks * 64] : 0.0;
                            bv[u] = kv ? zin[ks * 64] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < KC; ++u) {
                            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], bv[u], acc0, 0, 0, 0);
                            if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], bv[u], acc1, 0, 0, 0);
                        }
                    }
                    continue;
                }
                const int uoff = net.unit_off[j];
                const long long roff = (long long)net.row_off[j] * rs;
                for (int ks0 = 0; ks0 < ks_n; ks0 += KC) {
                    double a0[KC], a1[KC], bv[KC];
#pragma unroll
                    for (int u = 0; u < KC; ++u) {
                        const int ks = ks0 + u;
                        const bool kv = ks < ks_n;
                        const int k = ks * 4 + kq;
                        a0[u] = kv ? fr0[ks * 64] : 0.0;
                        a1[u] = (kv && two) ? fr1[ks * 64] : 0.0;
                        bv[u] = (kv && k < nj && cell_ok && code_bit(code, uoff + k)) ? zc[roff + k * rs] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < KC; ++u) {
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], bv[u], acc0, 0, 0, 0);
                        if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], bv[u], acc1, 0, 0, 0);
                    }
                }
            }
            if (cell_ok) {
                const double *bias = net.bias + bias_base + net.bias_off[l];
                double *z0 = zc + (long long)net.row_off[l] * rs;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // v_mfma_f64_16x16x4f64 leaves D[kq + 4 r][col] in register r
                    const int i0 = mt0 * 16 + kq + 4 * r;
                    if (i0 < nl) z0[i0 * rs] = acc0[r] + (q == 3 ? bias[i0] : 0.0);
                    const int i1 = mt1 * 16 + kq + 4 * r;
                    if (two && i1 < nl) z0[i1 * rs] = acc1[r] + (q == 3 ? bias[i1] : 0.0);
                }
            }
        }
        __syncthreads();
    }
}

// ---- gathered chain: a tile's four cells share the MFMA columns, so a unit
// that is off in all four contributes only zeros.  For source layers of at
// most kListMax units the tile first lists the units active in any of its
// cells (LDS, ascending, padded with -1 to a multiple of 4) and the K loop
// runs over that list, loading A from the column-major weights (four
// 128-byte columns per K-step).  Products are summed in list order, so rows
// may differ from the dense kernel's in the last bits.
constexpr int kListMax = 1024;
constexpr int kListBlocks = 2;

// Builds the union list of source layer j over the tile's ncell cells;
// returns its length.  All threads; ends with a barrier.
__device__ int union_list(const DevNet &net, int j, const uint64_t *code_lds, int ncell, short *list,
                          int *cnt_lds) {
    const int nj = net.width[j], uoff = net.unit_off[j];
    const int nchunks = (nj + 63) >> 6;
    const int t = threadIdx.x;
    uint64_t mask = 0;
    if (t < nchunks) {
        const int u0 = uoff + t * 64;
        const int w = u0 >> 6, sh = u0 & 63;
        for (int c = 0; c < ncell; ++c) {
            const uint64_t *code = code_lds + c * net.W;
            mask |= code[w] >> sh;
            if (sh && w + 1 < net.W) mask |= code[w + 1] << (64 - sh);
        }
        const int rem = nj - t * 64;
        if (rem < 64) mask &= (1ull << rem) - 1ull;
        cnt_lds[t] = __popcll(mask);
    }
    __syncthreads();
    int base = 0, total = 0;
    for (int c = 0; c < nchunks; ++c) {
        const int v = cnt_lds[c];
        if (c < t) base += v;
        total += v;
    }
    if (t < nchunks) {
        int at = base;
        while (mask) {
            const int bit = __builtin_ctzll(mask);
            mask &= mask - 1ull;
            list[at++] = (short)(t * 64 + bit);
        }
    }
    if (t < 4 && total + t < ((total + 3) & ~3)) list[total + t] = -1;
    __syncthreads();
    return total;
}

template <int KC>
__device__ void chain_tile_gather(const DevNet &net, const uint64_t *__restrict__ codes,
                                  const int *__restrict__ cell_shape, const int *list, long long c0, int ncell,
                                  double *zb, long long rs, long long cs, uint64_t *code_lds, int *shape_lds,
                                  short *lists, int *cnt_lds) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int col = lane & 15;
    const int kq = lane >> 4;
    const int q = col & 3;
    const int cl = col >> 2;
    const bool cell_ok = cl < ncell;
    stage_tile(net, codes, cell_shape, list, c0, ncell, code_lds, shape_lds);
    const long long bias_base = (long long)shape_lds[cl] * net.bias_stride;
    const uint64_t *code = code_lds + cl * net.W;
    double *zc = zb + cl * cs + q;

    for (int l = 1; l < net.n_layers; ++l) {
        const int nl = net.width[l];
        const int mtiles = (nl + 15) >> 4;
        const int rows16 = mtiles * 16;
        int lb[kListBlocks], lcount[kListBlocks], nlist = 0;
        for (int b = 0; b < net.n_blocks; ++b) {
            const int j = net.blk_src[b];
            if (net.blk_dst[b] != l || j == 0 || net.width[j] > kListMax || nlist == kListBlocks) continue;
            lcount[nlist] = union_list(net, j, code_lds, ncell, lists + nlist * (kListMax + 4), cnt_lds);
            lb[nlist++] = b;
        }
        for (int mt0 = wave; mt0 < mtiles; mt0 += 2 * nwaves) {
            const int mt1 = mt0 + nwaves;
            const bool two = mt1 < mtiles;
            v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
            for (int b = 0; b < net.n_blocks; ++b) {
                if (net.blk_dst[b] != l) continue;
                const int j = net.blk_src[b];
                const int ks_n = net.blk_ld[b] >> 2;
                const int nj = net.width[j];
                const double *fr0 = net.wfrag + net.blk_frag_off[b] + (long long)mt0 * ks_n * 64 + lane;
                const double *fr1 = fr0 + (long long)(mt1 - mt0) * ks_n * 64;
                if (j == 0) {
                    const double bv = (kq < 3 && kq == q) ? 1.0 : 0.0;
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(fr0[0], bv, acc0, 0, 0, 0);
                    if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(fr1[0], bv, acc1, 0, 0, 0);
                    continue;
                }
                const int uoff = net.unit_off[j];
                const double *zj = zc + (long long)net.row_off[j] * rs;
                int li = -1;
                for (int t = 0; t < nlist; ++t)
                    if (lb[t] == b) li = t;
                if (li >= 0) {
                    const short *kl = lists + li * (kListMax + 4);
                    const int ksn = (lcount[li] + 3) >> 2;
                    const double *wc = net.wcol + net.blk_col_off[b] + mt0 * 16 + col;
                    const long long d1 = (long long)(mt1 - mt0) * 16;
                    for (int ks0 = 0; ks0 < ksn; ks0 += KC) {
                        double a0[KC], a1[KC], bv[KC];
#pragma unroll
                        for (int u = 0; u < KC; ++u) {
                            const int ks = ks0 + u;
                            const int k = ks < ksn ? (int)kl[ks * 4 + kq] : -1;
                            const long long wo = (long long)k * rows16;
                            a0[u] = k >= 0 ? wc[wo] : 0.0;
                            a1[u] = (k >= 0 && two) ? wc[wo + d1] : 0.0;
                            bv[u] = (k >= 0 && cell_ok && code_bit(code, uoff + k)) ? zj[k * rs] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < KC; ++u) {
                            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], bv[u], acc0, 0, 0, 0);
                            if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], bv[u], acc1, 0, 0, 0);
                        }
                    }
                    continue;
                }
                for (int ks0 = 0; ks0 < ks_n; ks0 += KC) {
                    double a0[KC], a1[KC], bv[KC];
#pragma unroll
                    for (int u = 0; u < KC; ++u) {
                        const int ks = ks0 + u;
                        const bool kv = ks < ks_n;
                        const int k = ks * 4 + kq;
                        a0[u] = kv ? fr0[ks * 64] : 0.0;
                        a1[u] = (kv && two) ? fr1[ks * 64] : 0.0;
                        bv[u] = (kv && k < nj && cell_ok && code_bit(code, uoff + k)) ? zj[k * rs] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < KC; ++u) {
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], bv[u], acc0, 0, 0, 0);
                        if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], bv[u], acc1, 0, 0, 0);
                    }
                }
            }
            if (cell_ok) {
                const double *bias = net.bias + bias_base + net.bias_off[l];
                double *z0 = zc + (long long)net.row_off[l] * rs;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i0 = mt0 * 16 + kq + 4 * r;
                    if (i0 < nl) z0[i0 * rs] = acc0[r] + (q == 3 ? bias[i0] : 0.0);
                    const int i1 = mt1 * 16 + kq + 4 * r;
                    if (two && i1 < nl) z0[i1 * rs] = acc1[r] + (q == 3 ? bias[i1] : 0.0);
                }
            }
        }
        __syncthreads();
    }
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// x = h + m + l with h, m, l in BF16 (each the rounded remainder of the last):
// 24 significant bits, as many as FP32 holds.
__device__ __forceinline__ void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l) {
    h = (__bf16)x;
    const float r1 = x - (float)h;
    m = (__bf16)r1;
    l = (__bf16)(r1 - (float)m);
}

// Affine chain of four cells in split-BF16 on matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Each operand is split into
// three BF16 terms; the six products hh, hm, mh, mm, hl, lh are accumulated,
// which keeps about 24 bits (terms below 2^-24 relative are dropped).  Rows
// are FP32, element (row, cell, q) at zb[row * rs + cell * cs + q]; blocks
// from the input are exact copies of W's x, y, z columns and bypass the
// matrix cores.  Layout (16x16x32 BF16): A[i][k] in lane (i + 16 (k/8)),
// element k % 8; B[k][j] in lane (j + 16 (k/8)); D[4 (l/16) + r][l % 16] in
// register r of lane l.
__device__ void chain_tile_bf16(const DevNet &net, const uint64_t *__restrict__ codes,
                                const int *__restrict__ cell_shape, const int *list, long long c0, int ncell,
                                float *zb, long long rs, long long cs, uint64_t *code_lds, int *shape_lds) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int col = lane & 15;
    const int kq = lane >> 4;
    const int q = col & 3;
    const int cl = col >> 2;
    const bool cell_ok = cl < ncell;
    stage_tile(net, codes, cell_shape, list, c0, ncell, code_lds, shape_lds);
    const long long bias_base = (long long)shape_lds[cl] * net.bias_stride;
    const uint64_t *code = code_lds + cl * net.W;
    float *zc = zb + cl * cs + q;

    for (int l = 1; l < net.n_layers; ++l) {
        const int nl = net.width[l];
        const int mtiles = (nl + 15) >> 4;
        for (int mt0 = wave; mt0 < mtiles; mt0 += 2 * nwaves) {
            const int mt1 = mt0 + nwaves;
            const bool two = mt1 < mtiles;
            v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
            int b_in = -1;
            for (int b = 0; b < net.n_blocks; ++b) {
                if (net.blk_dst[b] != l) continue;
                const int j = net.blk_src[b];
                if (j == 0) {
                    b_in = b;
                    continue;
                }
                const int ks_n = net.blk_ld32[b] >> 5;
                const int nj = net.width[j];
                const v8bf *fr0 = reinterpret_cast<const v8bf *>(net.wfrag16) + net.blk_frag16_off[b] +
                                  (long long)mt0 * ks_n * 3 * 64 + lane;
                const v8bf *fr1 = fr0 + (long long)(mt1 - mt0) * ks_n * 3 * 64;
                const int uoff = net.unit_off[j];
                const float *zj = zc + (long long)net.row_off[j] * rs;
                for (int ks = 0; ks < ks_n; ++ks) {
                    const int kb = ks * 32 + 8 * kq;
                    v8bf bh, bm, bl;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int k = kb + u;
                        const float v = (k < nj && cell_ok && code_bit(code, uoff + k)) ? zj[k * rs] : 0.f;
                        __bf16 h, m, lo;
                        split3(v, h, m, lo);
                        bh[u] = h;
                        bm[u] = m;
                        bl[u] = lo;
                    }
                    const v8bf ah = fr0[(ks * 3 + 0) * 64], am = fr0[(ks * 3 + 1) * 64], al = fr0[(ks * 3 + 2) * 64];
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc0, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc0, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc0, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, acc0, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, acc0, 0, 0, 0);
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc0, 0, 0, 0);
                    if (two) {
                        const v8bf ch = fr1[(ks * 3 + 0) * 64], cm = fr1[(ks * 3 + 1) * 64],
                                   cl3 = fr1[(ks * 3 + 2) * 64];
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cl3, bh, acc1, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch, bl, acc1, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cm, bm, acc1, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cm, bh, acc1, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch, bm, acc1, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch, bh, acc1, 0, 0, 0);
                    }
                }
            }
            if (cell_ok) {
                const double *bias = net.bias + bias_base + net.bias_off[l];
                float *z0 = zc + (long long)net.row_off[l] * rs;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i0 = mt0 * 16 + 4 * kq + r;
                    const int i1 = mt1 * 16 + 4 * kq + r;
                    if (i0 < nl) {
                        double v = (double)acc0[r] + (q == 3 ? bias[i0] : 0.0);
                        if (b_in >= 0 && q < 3) v += net.weights[net.blk_off[b_in] + (long long)i0 * net.blk_ld[b_in] + q];
                        z0[i0 * rs] = (float)v;
                    }
                    if (two && i1 < nl) {
                        double v = (double)acc1[r] + (q == 3 ? bias[i1] : 0.0);
                        if (b_in >= 0 && q < 3) v += net.weights[net.blk_off[b_in] + (long long)i1 * net.blk_ld[b_in] + q];
                        z0[i1 * rs] = (float)v;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Hidden lines the precision check can list per cell (more: the cell is redone in FP64).
constexpr int kNearMax = 256;

struct PolyScratch {
    double a[kMaxPoly];
    double b[kMaxPoly];
    double r[kMaxPoly];
    int e[kMaxPoly];
    int near[kNearMax];   // hidden lines the precision check must revisit
};

struct Poly {
    double a, b;   // this lane's vertex in the plane frame
    double r;      // 1 + |(a, b)|, the vertex scale of the on-line tolerance
    int e;         // id of the edge starting at this vertex
    int m;         // vertex count (uniform)
};

enum : int { kFlagEmpty = 1, kFlagDegen = 2, kFlagSingular = 4, kFlagTooBig = 8 };

// One Sutherland-Hodgman pass with the halfplane cu a + cv b + cw <= 0 (id);
// nrm = |(cu, cv)| scales the on-line tolerance.
// Returns false when the polygon has no interior left.
__device__ bool sh_clip(Poly &P, double cu, double cv, double cw, double nrm, int id, PolyScratch &s,
                        int &flags) {
    const int lane = lane_id();
    const bool act = lane < P.m;
    const double d = cu * P.a + cv * P.b + cw;
    const double tol = kTau * (nrm * P.r + fabs(cw));
    const int cls = !act ? 0 : (d > tol ? 1 : (d < -tol ? -1 : 0));
    const uint64_t outm = ballot(act && cls == 1);
    if (!outm) return true;
    const uint64_t inm = ballot(act && cls == -1);
    if (!inm) {
        P.m = 0;
        return false;
    }
    const int j = (lane + 1 >= P.m) ? 0 : lane + 1;
    const double ja = shfl(P.a, j), jb = shfl(P.b, j), jd = shfl(d, j);
    const int jc = shfl(cls, j);
    const bool c1 = act && cls != 1;
    const bool c2 = act && ((cls == -1 && jc == 1) || (cls == 1 && jc == -1));
    const uint64_t b1 = ballot(c1), b2 = ballot(c2);
    const uint64_t lt = lanemask_lt();
    const int pos = __popcll(b1 & lt) + __popcll(b2 & lt);
    const int nm = __popcll(b1) + __popcll(b2);
    if (nm > kMaxPoly) {
        flags |= kFlagTooBig;
        P.m = 0;
        return false;
    }
    if (c1) {
        s.a[pos] = P.a;
        s.b[pos] = P.b;
        s.r[pos] = P.r;
        s.e[pos] = (cls == 0 && jc == 1) ? id : P.e;
    }
    if (c2) {
        const double t = d / (d - jd);
        const double xa = P.a + t * (ja - P.a);
        const double xb = P.b + t * (jb - P.b);
        const int p2 = pos + (c1 ? 1 : 0);
        s.a[p2] = xa;
        s.b[p2] = xb;
        s.r[p2] = 1.0 + sqrt(xa * xa + xb * xb);
        s.e[p2] = (cls == -1) ? id : P.e;
    }
    wave_lds_sync();
    P.m = nm;
    if (lane < nm) {
        P.a = s.a[lane];
        P.b = s.b[lane];
        P.r = s.r[lane];
        P.e = s.e[lane];
    }
    wave_lds_sync();
    return true;
}

// Oriented constraint row of id (feasible side <= 0), widened to FP64.
template <typename RowT>
__device__ __forceinline__ void constraint_row(const DevNet &net, int id, const uint64_t *code, int am,
                                               const RowT *rb, long long rs, double c[4]) {
    if (id < 0) {
        const int t = -id - 1;
        const int ax = t >> 1;
        c[0] = c[1] = c[2] = 0.0;
        c[ax] = (t & 1) ? -1.0 : 1.0;
        c[3] = -1.0;
    } else if (id < net.N) {
        const RowT *z = rb + (long long)(id) * rs;
        const double sg = code_bit(code, id) ? -1.0 : 1.0;
        c[0] = sg * z[0];
        c[1] = sg * z[1];
        c[2] = sg * z[2];
        c[3] = sg * z[3];
    } else {
        const RowT *zi = rb + (long long)(id) * rs;
        const RowT *zj = rb + (long long)(net.N + am) * rs;
        c[0] = zi[0] - zj[0];
        c[1] = zi[1] - zj[1];
        c[2] = zi[2] - zj[2];
        c[3] = zi[3] - zj[3];
    }
}

// Largest row sum of |A^-1| for a 3x3 matrix (adjugate / determinant).
__device__ double inv_norm3(const double A[3][3]) {
    const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    if (det == 0.0) return __builtin_inf();
    const double i00 = c00, i01 = A[0][2] * A[2][1] - A[0][1] * A[2][2], i02 = A[0][1] * A[1][2] - A[0][2] * A[1][1];
    const double i10 = c01, i11 = A[0][0] * A[2][2] - A[0][2] * A[2][0], i12 = A[0][2] * A[1][0] - A[0][0] * A[1][2];
    const double i20 = c02, i21 = A[0][1] * A[2][0] - A[0][0] * A[2][1], i22 = A[0][0] * A[1][1] - A[0][1] * A[1][0];
    const double r0 = fabs(i00) + fabs(i01) + fabs(i02);
    const double r1 = fabs(i10) + fabs(i11) + fabs(i12);
    const double r2 = fabs(i20) + fabs(i21) + fabs(i22);
    return fmax(r0, fmax(r1, r2)) / fabs(det);
}

// The split-BF16 certificate scales each vertex's first-order sensitivity to
// the rows, |A^-1|_inf max_k (|A_k|_1 |x|_inf + |r_k|) / max(1, |x|_inf), by a
// relative row error eps measured for the loaded net (k_calib_split, on the
// first cells of a march, against the FP64 chain and clip) and passed in
// Fallback::row_eps.

// Solves A x = r (3x3) by elimination with row pivoting; false if singular.
__device__ bool solve3(double A[3][3], double r[3], double x[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int i = c + 1; i < 3; ++i)
            if (fabs(A[i][c]) > fabs(A[p][c])) p = i;
        if (A[p][c] == 0.0) return false;
        if (p != c) {
            for (int k = 0; k < 3; ++k) {
                const double t = A[c][k];
                A[c][k] = A[p][k];
                A[p][k] = t;
            }
            const double t = r[c];
            r[c] = r[p];
            r[p] = t;
        }
        const double inv = 1.0 / A[c][c];
        for (int i = c + 1; i < 3; ++i) {
            const double f = A[i][c] * inv;
            for (int k = c; k < 3; ++k) A[i][k] -= f * A[c][k];
            r[i] -= f * r[c];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double s = r[i];
        for (int k = i + 1; k < 3; ++k) s -= A[i][k] * x[k];
        x[i] = s / A[i][i];
    }
    return true;
}

// Cells whose face the split-BF16 path cannot certify, for the FP64 path.
struct Fallback {
    int *list;
    unsigned long long *count;
    unsigned long long cap;
    double row_eps;    // relative error of the FP32 rows per unit of vertex sensitivity
};

// Precision check of a face computed from approximate rows: true when a
// constraint that is not an edge of the polygon comes within margin + est_i
// of vertex i (relative to |c|_1 (1 + |v|_inf); est_i is the vertex's own
// estimated relative error, held by lane i), or when an edge is that short;
// then the exact face may differ and the cell must be redone in FP64.  The
// hidden lines checked are the n_near ones the clip listed in `near`: every
// other hidden line stayed farther than that from an intermediate polygon,
// which contains the final one.  Max-pool and box lines are all checked.
template <typename RowT>
__device__ bool margin_ambiguous(const DevNet &net, const uint64_t *code, int am, const RowT *rb, long long rs,
                                 int m, int e, double vx, double vy, double vz, double est, double margin,
                                 const int *near, int n_near) {
    const int lane = lane_id();
    bool amb = false;
    const int jn = lane + 1 >= m ? 0 : lane + 1;
    const double wx = shfl(vx, jn), wy = shfl(vy, jn), wz = shfl(vz, jn);
    const double west = shfl(est, jn);
    if (lane < m) {
        const double sc = 1.0 + fmax(fabs(vx), fmax(fabs(vy), fabs(vz)));
        if (fmax(fabs(wx - vx), fmax(fabs(wy - vy), fabs(wz - vz))) <= (margin + est + west) * sc) amb = true;
    }
    const int total = n_near + net.M + 6;
    for (int base = 0; base < total; base += kWave) {
        const int t = base + lane;
        bool valid = t < total;
        int id;
        if (t < n_near) {
            id = near[t];
        } else if (t < n_near + net.M) {
            id = net.N + (t - n_near);
            if (t - n_near == am) valid = false;
        } else {
            id = -1 - (t - n_near - net.M);
        }
        bool isedge = false;
        for (int k = 0; k < m; ++k) isedge |= bcast(e, k) == id;
        double c[4] = {0.0, 0.0, 0.0, 0.0};
        const bool test = valid && !isedge;
        if (test) constraint_row(net, id, code, am, rb, rs, c);
        const double cn = fabs(c[0]) + fabs(c[1]) + fabs(c[2]) + fabs(c[3]);
        for (int i = 0; i < m; ++i) {
            const double xi = bcast(vx, i), yi = bcast(vy, i), zi = bcast(vz, i);
            const double ti = margin + bcast(est, i);
            const double d = c[0] * xi + c[1] * yi + c[2] * zi + c[3];
            const double sc = 1.0 + fmax(fabs(xi), fmax(fabs(yi), fabs(zi)));
            if (test && d > -ti * cn * sc) amb = true;
        }
    }
    return ballot(amb) != 0;
}

// 30-bit Morton key of a point of [-1, 1]^3 (10 bits per axis), used to order
// a step's cells so that the four cells of a chain tile lie close together.
__device__ __forceinline__ unsigned spread10(unsigned v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ __forceinline__ unsigned morton_key(double x, double y, double z) {
    auto q = [](double t) {
        const double u = fmin(1.0, fmax(0.0, 0.5 * (t + 1.0)));
        return (unsigned)fmin(1023.0, u * 1024.0);
    };
    return spread10(q(x)) | (spread10(q(y)) << 1) | (spread10(q(z)) << 2);
}

// ---------------------------------------------------------------- learned form

typedef _Float16 v8h __attribute__((ext_vector_type(8)));

// The edge a cell was entered by, in its plane frame: the crossed line and the
// parent's two edges beside it bound this face too, so their intersections are
// two vertices of it (generic position).  Uniform over the wave.
struct EntryEdge {
    double v1a, v1b, v2a, v2b;   // endpoints
    double qa, qb;               // midpoint
    double ta, tb;               // unit direction v1 -> v2
    double h;                    // length
    int id[3];                   // the three lines (entry, previous, next)
};

// Unit-normal 2-D line of constraint `id` in the frame: a x + b y + o <= 0 inside.
template <typename RowT>
__device__ bool frame_line(const DevNet &net, int id, const uint64_t *code, int am, const RowT *rb, long long rs,
                           const double u[3], const double v[3], const double p0[3], double &a, double &b,
                           double &o) {
    double c[4];
    constraint_row(net, id, code, am, rb, rs, c);
    const double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
    const double cv = c[0] * v[0] + c[1] * v[1] + c[2] * v[2];
    const double cw = c[0] * p0[0] + c[1] * p0[1] + c[2] * p0[2] + c[3];
    const double n = sqrt(cu * cu + cv * cv);
    if (!(n > 0.0)) return false;
    a = cu / n;
    b = cv / n;
    o = cw / n;
    return true;
}

template <typename RowT>
__device__ bool entry_edge(const DevNet &net, const int *hints, long long cell, const uint64_t *code, int am,
                           const RowT *rb, long long rs, const double u[3], const double v[3], const double p0[3],
                           EntryEdge &E) {
    if (!hints) return false;
    double a[3], b[3], o[3];
    for (int h = 0; h < 3; ++h) {
        const int id = hints[cell * 3 + h];
        if (id < 0 || id >= net.N + net.M || id == net.N + am) return false;
        E.id[h] = id;
        if (!frame_line(net, id, code, am, rb, rs, u, v, p0, a[h], b[h], o[h])) return false;
    }
    const double d1 = a[0] * b[1] - a[1] * b[0], d2 = a[0] * b[2] - a[2] * b[0];
    if (fabs(d1) < 1e-9 || fabs(d2) < 1e-9) return false;
    E.v1a = (b[0] * o[1] - b[1] * o[0]) / d1;
    E.v1b = (a[1] * o[0] - a[0] * o[1]) / d1;
    E.v2a = (b[0] * o[2] - b[2] * o[0]) / d2;
    E.v2b = (a[2] * o[0] - a[0] * o[2]) / d2;
    const double da = E.v2a - E.v1a, db = E.v2b - E.v1b;
    E.h = sqrt(da * da + db * db);
    if (!(E.h > 1e-12) || !(E.h < 8.0)) return false;
    E.ta = da / E.h;
    E.tb = db / E.h;
    E.qa = 0.5 * (E.v1a + E.v2a);
    E.qb = 0.5 * (E.v1b + E.v2b);
    return true;
}

__device__ __forceinline__ float clamp16(double x) { return (float)fmin(16.0, fmax(-16.0, x)); }

// Features of the unit-normal line (a, b, o) of hidden unit g, relative to the
// entry edge: signed distances of its midpoint and endpoints in entry lengths,
// the line's direction against the edge, the unit's depth and state, and the
// edge length.  Returns the midpoint distance in entry lengths.
__device__ double line_features(const DevNet &net, const EntryEdge &E, int g, int bit, double a, double b, double o,
                                float f[kPropF]) {
    const double ih = 1.0 / E.h;
    const double s = (a * E.qa + b * E.qb + o) * ih;
    int layer = 1;
    while (layer + 1 < net.n_layers - 1 && g >= net.unit_off[layer + 1]) ++layer;
    f[0] = clamp16(s);
    f[1] = clamp16((a * E.v1a + b * E.v1b + o) * ih);
    f[2] = clamp16((a * E.v2a + b * E.v2b + o) * ih);
    f[3] = (float)(a * E.ta + b * E.tb);
    f[4] = (float)(b * E.ta - a * E.tb);
    f[5] = (float)layer / (float)(net.n_layers - 2);
    f[6] = (float)bit;
    f[7] = (float)(log2(E.h) * (1.0 / 16.0));
    return s;
}

__device__ __forceinline__ float wave_max_f(float x) {
    for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, kWave));
    return x;
}

// Logits of the first `rows` rows of feats [64][kPropD] (FP16) by the scorer
// relu(W1 x + b1) -> relu(W2 . + b2) -> w3 . + b3, on v_mfma_f32_16x16x32_f16
// with FP32 accumulation; hs is [16][kPropH] FP16 LDS scratch.  Lane r gets
// row r's logit (rows >= `rows`: unspecified).
__device__ float prop_score(const PropNet &P, const _Float16 *feats, _Float16 *hs, int rows) {
    const int lane = lane_id();
    const int r16 = lane & 15, q = lane >> 4;
    float z = 0.f;
    for (int c = 0; c * 16 < rows; ++c) {
        const v8h bx = *(const v8h *)(feats + (16 * c + r16) * kPropD + 8 * q);
#pragma unroll
        for (int i = 0; i < kPropH / 16; ++i) {
            const v8h aw = *(const v8h *)(P.W1 + (16 * i + r16) * kPropD + 8 * q);
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(aw, bx, acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int h = 16 * i + 4 * q + r;   // D[4 q + r][r16] of tile i
                hs[r16 * kPropH + h] = (_Float16)fmaxf(acc[r] + P.b1[h], 0.f);
            }
        }
        wave_lds_sync();
        float part = 0.f;
#pragma unroll 2
        for (int i = 0; i < kPropH / 16; ++i) {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < kPropH / 32; ++ks) {
                const v8h aw = *(const v8h *)(P.W2 + (16 * i + r16) * kPropH + 32 * ks + 8 * q);
                const v8h bh = *(const v8h *)(hs + r16 * kPropH + 32 * ks + 8 * q);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(aw, bh, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int h = 16 * i + 4 * q + r;
                part += P.w3[h] * fmaxf(acc[r] + P.b2[h], 0.f);
            }
        }
        wave_lds_sync();
        part += __shfl_xor(part, 16, kWave);
        part += __shfl_xor(part, 32, kWave);
        if (q == c) z = part + P.b3;
    }
    return z;
}

// Per-wave LDS of the proposing clip.
struct alignas(16) PropScratch {
    _Float16 feats[kWave * kPropD];
    _Float16 hs[16 * kPropH];
    int ids[kWave];
};

// Merges this lane's candidate (s, id; s = -inf for none) into the running
// top-k list held by lanes 0..k-1 (tk_s, tk_id), best first.
__device__ void topk_merge(float s, int id, float &tk_s, int &tk_id, int k) {
    const int lane = lane_id();
    // the list changes only if a candidate beats the current k-th best
    const float kth = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, tk_s), k - 1));
    if (!ballot(s > kth)) return;
    float s2 = lane < k ? tk_s : -INFINITY;
    const int id2 = tk_id;
    float ns = -INFINITY;
    int nid = -1;
    for (int t = 0; t < k; ++t) {
        const float m = wave_max_f(fmaxf(s, s2));
        if (m == -INFINITY) break;
        const uint64_t w1 = ballot(s == m), w2 = ballot(s2 == m);
        int pick_id;
        if (w1) {
            const int src = __builtin_ctzll(w1);
            pick_id = __builtin_amdgcn_readlane(id, src);
            if (lane == src) s = -INFINITY;
        } else {
            const int src = __builtin_ctzll(w2);
            pick_id = __builtin_amdgcn_readlane(id2, src);
            if (lane == src) s2 = -INFINITY;
        }
        if (lane == t) {
            ns = m;
            nid = pick_id;
        }
    }
    tk_s = ns;
    tk_id = nid;
}

// Proposal pass: ranks the hidden lines near the entry edge (distance to its
// midpoint <= rho entry lengths, the entry lines themselves excluded) by the
// scorer (mode 1) or by that distance (mode 2, the order the paper's pivoting
// routine sorts planes in) and returns the best k ids in lanes 0..k-1
// (-1: none).
template <typename RowT>
__device__ int propose_lines(const DevNet &net, const PropArgs &pa, PropScratch *ps, const EntryEdge &E,
                             const uint64_t *code, int am, const RowT *rb, long long rs, const double u[3],
                             const double v[3], const double p0[3]) {
    const int lane = lane_id();
    float tk_s = -INFINITY;
    int tk_id = -1;
    int nbuf = 0;
    // the next pass's rows and code word are loaded before this pass's work
    RowT nz0 = 0, nz1 = 0, nz2 = 0, nz3 = 0;
    uint64_t nword = 0;
    auto load_pass = [&](int b) {
        const int g = b + lane;
        if (g < net.N) {
            const RowT *z = rb + (long long)g * rs;
            nz0 = z[0];
            nz1 = z[1];
            nz2 = z[2];
            nz3 = z[3];
        }
        nword = code[b >> 6];
    };
    if (net.N > 0) load_pass(0);
    for (int base = 0; base < net.N; base += kWave) {
        const int g = base + lane;
        bool cand = false;
        float f[kPropF];
        double sd = 0.0;
        const RowT z0 = nz0, z1 = nz1, z2 = nz2, z3 = nz3;
        const uint64_t word = nword;
        if (base + kWave < net.N) load_pass(base + kWave);
        if (g < net.N && g != E.id[0] && g != E.id[1] && g != E.id[2]) {
            const int bit = (int)((word >> lane) & 1ull);
            const double sg = bit ? -1.0 : 1.0;
            const double c0 = sg * z0, c1 = sg * z1, c2 = sg * z2, c3 = sg * z3;
            const double cu = c0 * u[0] + c1 * u[1] + c2 * u[2];
            const double cv = c0 * v[0] + c1 * v[1] + c2 * v[2];
            const double cw = c0 * p0[0] + c1 * p0[1] + c2 * p0[2] + c3;
            if (pa.mode == 2) {
                // distance order: only the midpoint's distance, in entry
                // lengths, as an FP32 rank (no features, one FP32 divide)
                const float nf = sqrtf((float)(cu * cu + cv * cv)) * (float)E.h;
                const float num = fabsf((float)(cu * E.qa + cv * E.qb + cw));
                cand = nf > 0.f && num <= pa.rho * nf;
                sd = cand ? (double)(num / nf) : 0.0;
            } else {
                const double n = sqrt(cu * cu + cv * cv);
                if (n > 0.0) {
                    sd = line_features(net, E, g, bit, cu / n, cv / n, cw / n, f);
                    cand = fabs(sd) <= (double)pa.rho;
                }
            }
        }
        if (pa.mode == 2) {
            topk_merge(cand ? (float)(-fabs(sd)) : -INFINITY, g, tk_s, tk_id, pa.k);
            continue;
        }
        const uint64_t cm = ballot(cand);
        const int nc = __popcll(cm);
        if (nc == 0) continue;
        if (nbuf + nc > kWave) {
            const float zz = prop_score(pa.net, ps->feats, ps->hs, nbuf);
            topk_merge(lane < nbuf ? zz : -INFINITY, ps->ids[lane], tk_s, tk_id, pa.k);
            nbuf = 0;
            wave_lds_sync();
        }
        if (cand) {
            const int at = nbuf + __popcll(cm & lanemask_lt());
            _Float16 *row = ps->feats + at * kPropD;
#pragma unroll
            for (int j = 0; j < kPropF; ++j) row[j] = (_Float16)f[j];
#pragma unroll
            for (int j = kPropF; j < kPropD; ++j) row[j] = (_Float16)0.f;
            ps->ids[at] = g;
        }
        nbuf += nc;
        wave_lds_sync();
    }
    if (pa.mode == 1 && nbuf > 0) {
        // rows nbuf..63 of the last 16-row group are stale: their logits are dropped
        const float zz = prop_score(pa.net, ps->feats, ps->hs, nbuf);
        topk_merge(lane < nbuf ? zz : -INFINITY, ps->ids[lane], tk_s, tk_id, pa.k);
        wave_lds_sync();
    }
    return tk_id;
}

// Training samples of one finished cell: features of its candidate lines and
// whether each carries an edge of the face (ids e of lanes < m).
template <typename RowT>
__device__ void collect_samples(const DevNet &net, const PropArgs &pa, const EntryEdge &E, const uint64_t *code,
                                int am, const RowT *rb, long long rs, const double u[3], const double v[3],
                                const double p0[3], int m, int e) {
    const int lane = lane_id();
    for (int base = 0; base < net.N; base += kWave) {
        const int g = base + lane;
        bool cand = false;
        float f[kPropF];
        if (g < net.N && g != E.id[0] && g != E.id[1] && g != E.id[2]) {
            double a, b, o;
            if (frame_line(net, g, code, am, rb, rs, u, v, p0, a, b, o)) {
                const double sd = line_features(net, E, g, code_bit(code, g), a, b, o, f);
                cand = fabs(sd) <= (double)pa.rho;
            }
        }
        bool edge = false;
        for (int k = 0; k < m; ++k) edge |= bcast(e, k) == g;
        unsigned long long basev;
        const unsigned long long idx = wave_reserve(pa.n_samples, cand, &basev);
        if (cand && idx < pa.cap) {
            float *row = pa.samples + idx * kPropD;
            for (int j = 0; j < kPropD; ++j) row[j] = j < kPropF ? f[j] : 0.f;
            pa.labels[idx] = edge ? 1 : 0;
        }
    }
}

// Clips the face of one cell (one wave) and writes it; rows of the cell's
// chain are read as rb[row * rs + q] (FP64, or FP32 from the split-BF16
// chain).  margin > 0 (FP32 rows): faces that margin_ambiguous flags, and
// empty or degenerate results, are not written but appended to fb.
// 2-D line of constraint slot l of a cell (0..N-1 hidden units, N..N+M-1
// comparisons with the other heads, then the six box planes) in the plane
// frame: cu a + cv b + cw <= 0 inside.  False for the cell's own head.
template <typename RowT>
__device__ __forceinline__ bool slot_line(const DevNet &net, int l, const uint64_t *code, int am, const RowT *rb,
                                          long long rs, const double u[3], const double v[3], const double p0[3],
                                          const double aF[4], double &cu, double &cv, double &cw, int &id) {
    double c[4];
    if (l < net.N) {
        const RowT *z = rb + (long long)(l) * rs;
        const double sg = code_bit(code, l) ? -1.0 : 1.0;
        c[0] = sg * z[0];
        c[1] = sg * z[1];
        c[2] = sg * z[2];
        c[3] = sg * z[3];
        id = l;
    } else if (l < net.N + net.M) {
        const int hd = l - net.N;
        if (hd == am) return false;
        const RowT *z = rb + (long long)(l) * rs;
        c[0] = z[0] - aF[0];
        c[1] = z[1] - aF[1];
        c[2] = z[2] - aF[2];
        c[3] = z[3] - aF[3];
        id = l;
    } else {
        const int t = l - net.N - net.M;
        const int axb = t >> 1;
        const double sg = (t & 1) ? -1.0 : 1.0;
        cu = sg * u[axb];
        cv = sg * v[axb];
        cw = sg * p0[axb] - 1.0;
        id = -1 - t;
        return true;
    }
    cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
    cv = c[0] * v[0] + c[1] * v[1] + c[2] * v[2];
    cw = c[0] * p0[0] + c[1] * p0[1] + c[2] * p0[2] + c[3];
    return true;
}

// Wave-wide minimum of (key, id), smaller id on equal keys.
__device__ __forceinline__ void wave_argmin(double &key, int &id) {
    for (int o = 32; o > 0; o >>= 1) {
        const double k2 = __shfl_xor(key, o, kWave);
        const int i2 = __shfl_xor(id, o, kWave);
        if (k2 < key || (k2 == key && i2 < id)) {
            key = k2;
            id = i2;
        }
    }
}

// Pivoting (Sec. 4.2.1): the face traced vertex by vertex from its entry
// edge.  From a point on the current boundary line the walk moves along it,
// the face on its left; the next vertex is where the first line ahead is
// met (a ratio test over every line, one wave-wide minimum per vertex, in
// place of testing candidate vertices one by one in distance order).  Where
// several lines meet that vertex (within 2^-38 relative) the face goes on
// along the one that turns furthest, the only one that leaves the face on
// its inner side.  The walk ends when the entry line is met again.  Builds P
// counter-clockwise with edge ids as the clip does; false (P unusable) when
// the walk cannot finish within max_m vertices or meets no line ahead.
template <typename RowT>
__device__ bool pivot_poly(const DevNet &net, const uint64_t *code, int am, const RowT *rb, long long rs,
                           const double u[3], const double v[3], const double p0[3], const double aF[4],
                           const EntryEdge &E, int max_m, Poly &P) {
    const int lane = lane_id();
    const int L = net.N + net.M + 6;
    const int start = E.id[0];
    double na, nb, no;
    if (!frame_line(net, start, code, am, rb, rs, u, v, p0, na, nb, no)) return false;
    int cur = start;
    double ya = E.qa, yb = E.qb;
    int m = 0;
    P.m = 0;
    for (int step = 0; step < max_m + 8; ++step) {
        const double da = -nb, db = na;   // along the line, the inside on the left
        double s1 = __builtin_inf(), s2 = __builtin_inf();
        int id1 = 0x7fffffff;
        for (int l = lane; l < L; l += kWave) {
            double cu, cv, cw;
            int id;
            if (!slot_line(net, l, code, am, rb, rs, u, v, p0, aF, cu, cv, cw, id) || id == cur) continue;
            const double den = cu * da + cv * db;
            if (!(den > 1e-13 * sqrt(cu * cu + cv * cv))) continue;   // parallel, or behind
            const double s = -(cu * ya + cv * yb + cw) / den;
            if (s < s1 || (s == s1 && id < id1)) {
                s2 = s1;
                s1 = s;
                id1 = id;
            } else if (s < s2) {
                s2 = s;
            }
        }
        double g = s1;
        int gid = id1;
        wave_argmin(g, gid);
        if (!(g < 1e300)) return false;
        const double tol = 0x1p-38 * (1.0 + fabs(ya) + fabs(yb) + fabs(g));
        const uint64_t near = ballot(s1 <= g + tol);
        const bool tie = __popcll(near) > 1 || ballot(s2 <= g + tol) != 0;
        int nid = gid;
        if (tie) {
            // the lines through the next vertex: the one turning furthest left
            double key = __builtin_inf();
            int kid = 0x7fffffff;
            for (int l = lane; l < L; l += kWave) {
                double cu, cv, cw;
                int id;
                if (!slot_line(net, l, code, am, rb, rs, u, v, p0, aF, cu, cv, cw, id) || id == cur) continue;
                const double nrm = sqrt(cu * cu + cv * cv);
                const double den = cu * da + cv * db;
                if (!(den > 1e-13 * nrm)) continue;
                const double s = -(cu * ya + cv * yb + cw) / den;
                if (!(s <= g + tol)) continue;
                // cosine between the walk and the line's own direction (-cv, cu)
                const double c = (da * -cv + db * cu) / nrm;
                if (c < key || (c == key && id < kid)) {
                    key = c;
                    kid = id;
                }
            }
            wave_argmin(key, kid);
            nid = kid;
        }
        double ma, mb, mo;
        if (!frame_line(net, nid, code, am, rb, rs, u, v, p0, ma, mb, mo)) return false;
        const double det = na * mb - nb * ma;
        if (!(fabs(det) > 1e-300)) return false;
        const double xa = (nb * mo - no * mb) / det;
        const double xb = (ma * no - na * mo) / det;
        if (m > 0 && g <= tol) {
            // no length on the current line: the last vertex's edge is the new line
            if (lane == m - 1) P.e = nid;
        } else {
            if (m >= max_m) return false;
            if (lane == m) {
                P.a = xa;
                P.b = xb;
                P.r = 1.0 + sqrt(xa * xa + xb * xb);
                P.e = nid;
            }
            ++m;
        }
        if (nid == start) {
            P.m = m;
            return m >= 3;
        }
        cur = nid;
        na = ma;
        nb = mb;
        no = mo;
        ya = xa;
        yb = xb;
    }
    return false;
}

// ---- inline insertion (persistent march).  Lane i of a face with m
// corners holds edge i (constraint e); its neighbour is the cell with unit e
// flipped (hidden unit) or with head e - N as the argmax (a max-pool edge).
// Three phases, so that no lane waits while it holds a claim:
//   1. probe from the neighbour's fingerprint: an empty slot is claimed with
//      CAS as kPending | 18-bit tag | e | this cell (the claim names its code:
//      this cell's with e flipped); a committed slot with the same tag, or a
//      claim with the same short tag, is compared on the full code;
//   2. every claim becomes the next cell id: its code, argmax, shape,
//      fingerprint and clip hints are written, then (release) the slot turns
//      into tag | id and ready[id] into the epoch;
//   3. a lane that met an equal claim of another wave waits (bounded) for it
//      to be committed and takes its id.
// Claims are committed in phase 2 without waiting on anything, so every wait
// of phase 3 ends.  The neighbour ids go to the face's nbr slots.
__device__ __forceinline__ uint64_t flip_word(const uint64_t *code, int flip, int w) {
    uint64_t x = code[w];
    if (flip >= 0 && (flip >> 6) == w) x ^= 1ull << (flip & 63);
    return x;
}

__device__ void insert_neighbours(const DevNet &net, const InlineInsert &I, long long cell, const CellRec &rec,
                                  int m, int e_out, const ClipOut &out, long long obase, Counters *ctr) {
    const uint64_t *code = rec.code;
    const int am = rec.am;
    const int lane = lane_id();
    const bool want = lane < m && e_out >= 0;
    const int e_prev = shfl(e_out, lane == 0 ? m - 1 : lane - 1);
    const int e_next = shfl(e_out, lane + 1 >= m ? 0 : lane + 1);
    const uint64_t dm = ballot(lane < m && e_out < 0);
    if (lane == 0 && dm) atomicAdd(&ctr->domain_edges, (unsigned long long)__popcll(dm));
    const uint64_t h = rec.hash;
    const int shp = rec.shape;
    uint64_t hn = 0;
    int nam = am, flip = -1;
    if (want) {
        if (e_out < net.N) {
            hn = h ^ net.zobrist[e_out];
            flip = e_out;
        } else {
            hn = h ^ net.zobrist[net.N + am] ^ net.zobrist[e_out];
            nam = e_out - net.N;
        }
    }
    const unsigned long long tag = slot_tag(hn);
    const unsigned long long ptag = (hn >> 46) & 0x3ffffull;
    const unsigned long long mine = kPending | (ptag << 45) | ((unsigned long long)e_out << 31) |
                                    (unsigned long long)cell;
    unsigned long long pos = hn & I.hmask;
    int state = want ? 0 : 3;   // 0 probing, 1 claimed, 2 equal claim met, 3 done
    long long nid = -1;
    // phase 1
    for (unsigned long long probe = 0; state == 0; ++probe) {
        if (probe > I.hmask) {
            atomicAdd(&ctr->overflow_hash, 1ull);
            st_dev(&ctr->stop, 1ull);
            state = 3;
            break;
        }
        // the record a slot names was complete before the slot was written
        // (a claim names a cell being processed; a committed id's record was
        // published before the commit), and is read after the slot.  The claim
        // is tried at once: a failed compare-exchange returns the slot's
        // value, as a load would, so an empty slot costs one round trip
        unsigned long long sv = 0;
        if (__hip_atomic_compare_exchange_strong(&I.slots[pos], &sv, mine, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
            state = 1;
            break;
        }
        int oc = -1, oflip = -1, oam_claim = -1;
        bool cmp = false;
        if (sv & kPending) {
            if (((sv >> 45) & 0x3ffffull) == ptag) {
                // a claim: the code of cell (low 31 bits) with constraint e
                // flipped; its argmax is the cell's, or the head e - N
                oc = (int)(sv & 0x7fffffffull);
                const int oe = (int)((sv >> 31) & 0x3fffull);
                oflip = oe < net.N ? oe : -1;
                oam_claim = oe < net.N ? -1 : oe - net.N;
                cmp = true;
            }
        } else if (((sv >> 32) & 0x7fffffffull) == tag) {
            oc = (int)(sv & 0xffffffffull);
            cmp = (unsigned long long)oc < I.cap_cells;
        }
        if (cmp) {
            // argmax, shape and the code words are loaded before any is
            // compared (eight words at a time), not one round trip each
            const uint64_t *ocode = I.codes + (long long)oc * net.W;
            const int oam_l = ld_dev(&I.argmax[oc]);
            const int osh = ld_dev(&I.shape[oc]);
            bool eq = true;
            for (int w0 = 0; w0 < net.W; w0 += 8) {
                uint64_t x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = ld_dev(&ocode[min(w0 + u, net.W - 1)]);
                if (w0 == 0) eq = (oam_claim >= 0 ? oam_claim : oam_l) == nam && osh == shp;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int w = min(w0 + u, net.W - 1);   // a repeated last word compares as it did
                    if (oflip >= 0 && (oflip >> 6) == w) x[u] ^= 1ull << (oflip & 63);
                    eq = eq && x[u] == flip_word(code, flip, w);
                }
                if (!eq) break;
            }
            if (eq) {
                if (sv & kPending) {
                    state = 2;
                } else {
                    nid = oc;
                    state = 3;
                }
                break;
            }
        }
        pos = (pos + 1) & I.hmask;
    }
    // phase 2
    const bool own = state == 1;
    unsigned long long base;
    const unsigned long long id = wave_reserve(&ctr->n_cells, own, &base);
    if (own) {
        if (id >= I.cap_cells) {
            atomicAdd(&ctr->overflow_cells, 1ull);
            st_dev(&ctr->stop, 1ull);
        } else {
            uint64_t *dst = I.codes + (long long)id * net.W;
            for (int w = 0; w < net.W; ++w) st_dev(&dst[w], flip_word(code, flip, w));
            st_dev(&I.argmax[id], nam);
            st_dev(&I.shape[id], shp);
            st_dev(&I.cell_hash[id], hn);
            st_dev(&I.hints[id * 3 + 0], e_out < net.N ? e_out : net.N + am);   // the crossed plane, in its ids
            st_dev(&I.hints[id * 3 + 1], e_prev);
            st_dev(&I.hints[id * 3 + 2], e_next);
            st_dev(&I.face_m[id], 0);
            nid = (long long)id;
        }
    }
    // the records are complete before any slot or flag names them
    publish_wait();
    if (own) {
        st_dev(&I.slots[pos], (tag << 32) | (nid >= 0 ? (unsigned long long)nid : 0xffffffffull));
        if (nid >= 0) st_dev(&I.ready[nid], I.epoch);
    }
    // phase 3
    if (state == 2) {
        unsigned long long sv = kPending;
        for (unsigned long long k = 0; k < (I.spin_limit >> 4); ++k) {   // polls of ~1-2 us: under a second
            sv = ld_dev(&I.slots[pos]);
            if (!(sv & kPending)) break;
            __builtin_amdgcn_s_sleep(1);
        }
        if (sv & kPending) {
            atomicAdd(&ctr->stalled, 1ull);
            st_dev(&ctr->stop, 1ull);
        } else {
            const unsigned long long oc = sv & 0xffffffffull;
            nid = oc < I.cap_cells ? (long long)oc : -1;
        }
    }
    if (want && out.nbr) out.nbr[obase + lane] = (int)nid;
}

template <typename RowT, bool Learn, bool Pivot = false>
__device__ void clip_cell(const DevNet &net, const uint64_t *codes, const int *argmax,
                          const uint64_t *cell_hash, const int *hints, long long cell,
                          long long n_seed_cells, const RowT *rb, long long rs, PolyScratch &S, const ClipOut &out,
                          const Candidates &cand, unsigned long long cand_cap, Counters *ctr, double margin,
                          double vertex_tol, const Fallback &fb, const PropArgs &pa, PropScratch *ps,
                          const InlineInsert *ins = nullptr, const CellRec *rec = nullptr) {
    const int lane = lane_id();
    const uint64_t *code = rec ? rec->code : codes + cell * net.W;
    const int am_in = rec ? rec->am : (argmax ? argmax[cell] : 0);
    const bool am_ok = am_in >= 0 && am_in < net.M;   // a bad argmax gives an empty face
    const int am = am_ok ? am_in : 0;
    const long long oi = cell - out.out_base;
    int flags = 0;
    // precision check: a hidden line that stays farther than near_tol (x |c|_1)
    // from every vertex of an intermediate polygon clears margin + est (est <=
    // vertex_tol, vertex scale <= 2 in the box) at the final vertices
    const double near_tol = margin > 0.0 ? 2.5 * (margin + vertex_tol) : 0.0;
    int n_near = 0;
    EntryEdge E;
    bool have_entry = false;
    int ncuts = 0;   // lines that cut in the every-line pass
    (void)ps;

    // rows the first cuts need, loaded with the face plane's so that their
    // latencies overlap: the three lines the parent's face says bound this
    // one (below) and the first pass's 64 hidden lines
    int hid[3] = {-1, -1, -1};
    RowT hr[3][4] = {};
    if (hints || rec) {
#pragma unroll
        for (int h = 0; h < 3; ++h) {
            hid[h] = rec ? rec->hint[h] : hints[cell * 3 + h];
            if (hid[h] < 0 || hid[h] >= net.N + net.M || hid[h] == net.N + am) hid[h] = -1;
            if (hid[h] >= 0) {
                const RowT *z = rb + (long long)hid[h] * rs;
                hr[h][0] = z[0];
                hr[h][1] = z[1];
                hr[h][2] = z[2];
                hr[h][3] = z[3];
            }
        }
    }
    RowT nz0 = 0, nz1 = 0, nz2 = 0, nz3 = 0;
    uint64_t nword = 0;
    auto load_pass = [&](int b) {
        const int g = b + lane;
        if (g < net.N) {
            const RowT *z = rb + (long long)g * rs;
            nz0 = z[0];
            nz1 = z[1];
            nz2 = z[2];
            nz3 = z[3];
        }
        nword = code[b >> 6];
    };
    if (net.N > 0) load_pass(0);

    // ---- plane frame: n = a_F[0:3], foot point p0, orthonormal u, v with u x v = n/|n|
    const RowT *aF = rb + (long long)(net.N + am) * rs;
    const double fx = aF[0], fy = aF[1], fz = aF[2], fw = aF[3];
    const double nn = fx * fx + fy * fy + fz * fz;
    Poly P;
    P.m = 0;
    double p0[3], u[3], v[3];
    if (nn > 0.0 && am_ok) {
        p0[0] = -fw * fx / nn;
        p0[1] = -fw * fy / nn;
        p0[2] = -fw * fz / nn;
        const double inl = 1.0 / sqrt(nn);
        const double n0 = fx * inl, n1 = fy * inl, n2 = fz * inl;
        int ax = 0;
        if (fabs(n1) < fabs(n0)) ax = 1;
        if (fabs(n2) < fabs(ax == 0 ? n0 : n1)) ax = 2;
        // u = normalize(n x e_ax)
        double ux = ax == 0 ? 0.0 : (ax == 1 ? -n2 : n1);
        double uy = ax == 0 ? n2 : (ax == 1 ? 0.0 : -n0);
        double uz = ax == 0 ? -n1 : (ax == 1 ? n0 : 0.0);
        const double iu = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
        u[0] = ux * iu;
        u[1] = uy * iu;
        u[2] = uz * iu;
        v[0] = n1 * u[2] - n2 * u[1];
        v[1] = n2 * u[0] - n0 * u[2];
        v[2] = n0 * u[1] - n1 * u[0];
        // starting square, counter-clockwise, edges -7..-10
        const double sa[4] = {-kSquareHalf, kSquareHalf, kSquareHalf, -kSquareHalf};
        const double sb[4] = {-kSquareHalf, -kSquareHalf, kSquareHalf, kSquareHalf};
        const int li = lane < 4 ? lane : 0;
        P.a = sa[li];
        P.b = sb[li];
        P.r = 1.0 + sqrt(P.a * P.a + P.b * P.b);
        P.e = -7 - li;
        P.m = 4;
        bool walked = false;
        if constexpr (Pivot) {
            // pivoting form: trace the face from the entry edge; seeds,
            // entry edges ending on a box plane or degenerate, and walks
            // that do not close are clipped
            EntryEdge E0;
            if (entry_edge(net, hints, cell, code, am, rb, rs, u, v, p0, E0)) {
                const double aFd[4] = {fx, fy, fz, fw};
                Poly W;
                walked = pivot_poly(net, code, am, rb, rs, u, v, p0, aFd, E0, kMaxPoly, W);
                if (walked) P = W;
            }
            if (lane == 0 && ctr) atomicAdd(walked ? &ctr->pivot_cells : &ctr->pivot_fallback, 1ull);
        }
        if (!walked) {
        // lines the parent's face says bound this one: the entry edge and the
        // parent's edges on either side of it (the cells around a cell edge
        // share both planes).  Any order gives the same polygon; these first
        // leave most later lines with nothing to cut.
        int entry_id = -1;
        if (hints || rec) {
            entry_id = hid[0];
#pragma unroll
            for (int h = 0; h < 3; ++h) {
                if (hid[h] < 0 || P.m <= 0) continue;
                // the oriented constraint row, as constraint_row forms it
                double c[4];
                if (hid[h] < net.N) {
                    const double sg = code_bit(code, hid[h]) ? -1.0 : 1.0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) c[k] = sg * hr[h][k];
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) c[k] = hr[h][k] - aF[k];
                }
                const double hu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
                const double hv = c[0] * v[0] + c[1] * v[1] + c[2] * v[2];
                const double hw = c[0] * p0[0] + c[1] * p0[1] + c[2] * p0[2] + c[3];
                sh_clip(P, hu, hv, hw, sqrt(hu * hu + hv * hv), hid[h], S, flags);
            }
        }
        // learned form: clip the proposed lines next; the pass below still
        // tests every line, so the face does not depend on the proposals
        if constexpr (Learn) {
        if ((pa.mode != 0 || pa.samples) && P.m > 0)
            have_entry = entry_edge(net, hints, cell, code, am, rb, rs, u, v, p0, E);
        if (have_entry && ((pa.mode == 1 && ps) || pa.mode == 2)) {
            const int pid = propose_lines(net, pa, ps, E, code, am, rb, rs, u, v, p0);
            // lane t holds proposal t: its line is loaded and projected by
            // all lanes at once, then the lines are clipped in rank order
            double hu = 0.0, hv = 0.0, hw = 0.0, hn = 0.0;
            if (lane < pa.k && pid >= 0) {
                double c[4];
                constraint_row(net, pid, code, am, rb, rs, c);
                hu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
                hv = c[0] * v[0] + c[1] * v[1] + c[2] * v[2];
                hw = c[0] * p0[0] + c[1] * p0[1] + c[2] * p0[2] + c[3];
                hn = sqrt(hu * hu + hv * hv);
            }
            for (int t = 0; t < pa.k && P.m > 0; ++t) {
                const int id = bcast(pid, t);
                if (id < 0) break;
                sh_clip(P, bcast(hu, t), bcast(hv, t), bcast(hw, t), bcast(hn, t), id, S, flags);
            }
        }
        }
        // hidden units, 64 lines per pass; each pass loads the next pass's
        // rows (and code word: the 64 units of a pass share one) before it
        // tests and cuts its own, so the loads' latency overlaps that work.
        // A pass's cutting lines are applied nearest first to a point of the
        // face's boundary (the entry edge's midpoint after the hint cuts,
        // else the mean of the polygon's vertices), the rest re-tested after
        // each cut: the lines near the face, which bound it, go first, and
        // fewer of the others still cut.  Every line is tested, and a line
        // that does not cut when tested never cuts later (the polygon only
        // shrinks), so the face is the same in any order.
        float qa = 0.f, qb = 0.f;
        if (P.m > 0) {
            const uint64_t em = ballot(lane < P.m && entry_id >= 0 && P.e == entry_id);
            if (em) {
                const int i = __builtin_ctzll(em);
                const int j = i + 1 >= P.m ? 0 : i + 1;
                qa = (float)(0.5 * (bcast(P.a, i) + bcast(P.a, j)));
                qb = (float)(0.5 * (bcast(P.b, i) + bcast(P.b, j)));
            } else {
                qa = (float)(wave_sum(lane < P.m ? P.a : 0.0) / P.m);
                qb = (float)(wave_sum(lane < P.m ? P.b : 0.0) / P.m);
            }
        }
        for (int base = 0; base < net.N && P.m > 0; base += kWave) {
            const int g = base + lane;
            const bool valid = g < net.N;
            const RowT z0 = nz0, z1 = nz1, z2 = nz2, z3 = nz3;
            const uint64_t word = nword;
            if (base + kWave < net.N) load_pass(base + kWave);
            double cu = 0.0, cv = 0.0, cw = 0.0, nrm = 0.0, cn = 0.0;
            bool cuts = false, close = false;
            if (valid) {
                const double sg = ((word >> lane) & 1ull) ? -1.0 : 1.0;
                const double c0 = sg * z0, c1 = sg * z1, c2 = sg * z2, c3 = sg * z3;
                cu = c0 * u[0] + c1 * u[1] + c2 * u[2];
                cv = c0 * v[0] + c1 * v[1] + c2 * v[2];
                cw = c0 * p0[0] + c1 * p0[1] + c2 * p0[2] + c3;
                nrm = sqrt(cu * cu + cv * cv);
                cn = fabs(c0) + fabs(c1) + fabs(c2) + fabs(c3);
            }
            for (int i = 0; i < P.m; ++i) {
                const double ai = bcast(P.a, i), bi = bcast(P.b, i), ri = bcast(P.r, i);
                const double d = cu * ai + cv * bi + cw;
                cuts |= d > kTau * (nrm * ri + fabs(cw));
                close |= d > -near_tol * cn;
            }
            if (near_tol > 0.0) {
                // lines that cut, or pass within near_tol of this polygon,
                // are the only hidden lines the precision check revisits
                const uint64_t nm = ballot(valid && close);
                const int at = n_near + __popcll(nm & ((1ull << lane) - 1ull));
                if (valid && close && at < kNearMax) S.near[at] = g;
                n_near += __popcll(nm);
            }
            uint64_t mask = ballot(valid && cuts);
            if (mask) {
                const float key =
                    nrm > 0.0 ? fabsf((float)cu * qa + (float)cv * qb + (float)cw) / (float)nrm : INFINITY;
                while (mask) {
                    float k = ((mask >> lane) & 1ull) ? key : INFINITY;
                    int kid = lane;
                    for (int o = 32; o > 0; o >>= 1) {
                        const float k2 = __shfl_xor(k, o, kWave);
                        const int i2 = __shfl_xor(kid, o, kWave);
                        if (k2 < k || (k2 == k && i2 < kid)) {
                            k = k2;
                            kid = i2;
                        }
                    }
                    const int t = __builtin_amdgcn_readfirstlane(kid);
                    mask &= ~(1ull << t);
                    ++ncuts;
                    if (!sh_clip(P, bcast(cu, t), bcast(cv, t), bcast(cw, t), bcast(nrm, t), base + t, S, flags)) break;
                    if (!mask) break;
                    bool c = false;
                    for (int i = 0; i < P.m; ++i) {
                        const double ai = bcast(P.a, i), bi = bcast(P.b, i), ri = bcast(P.r, i);
                        const double d = cu * ai + cv * bi + cw;
                        c |= d > kTau * (nrm * ri + fabs(cw));
                    }
                    mask = ballot(((mask >> lane) & 1ull) && c);
                }
            }
        }
        // max-pool comparisons with every other head
        if (net.M > 1 && P.m > 0) {
            const int hd = lane;
            const bool valid = hd < net.M && hd != am;
            double cu = 0.0, cv = 0.0, cw = 0.0, nrm = 0.0;
            if (valid) {
                const RowT *zi = rb + (long long)(net.N + hd) * rs;
                const double c0 = zi[0] - fx, c1 = zi[1] - fy, c2 = zi[2] - fz, c3 = zi[3] - fw;
                cu = c0 * u[0] + c1 * u[1] + c2 * u[2];
                cv = c0 * v[0] + c1 * v[1] + c2 * v[2];
                cw = c0 * p0[0] + c1 * p0[1] + c2 * p0[2] + c3;
                nrm = sqrt(cu * cu + cv * cv);
            }
            uint64_t mask = ballot(valid);
            while (mask && P.m > 0) {
                const int t = __builtin_ctzll(mask);
                mask &= mask - 1;
                if (!sh_clip(P, bcast(cu, t), bcast(cv, t), bcast(cw, t), bcast(nrm, t), net.N + t, S, flags)) break;
            }
        }

        // the six box planes, ids -1..-6.  The box section lies strictly inside
        // the starting square, so the result does not depend on when they are
        // applied; last, they rarely cut.
        // (unrolled: the axis is a constant, so u, v and p0 stay in registers)
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const int axb = t >> 1;
            const double sg = (t & 1) ? -1.0 : 1.0;
            if (P.m > 0)
                sh_clip(P, sg * u[axb], sg * v[axb], sg * p0[axb] - 1.0, sqrt(u[axb] * u[axb] + v[axb] * v[axb]),
                        -1 - t, S, flags);
        }
        }   // !walked
    }

    // ---- validity: >= 3 vertices, positive area, distinct ids, no frame edge
    int m = P.m;
    const bool act = lane < m;
    if (m >= 3) {
        // twice the area as a fan from vertex 0, so that rounding scales with
        // the polygon's own size (an absolute shoelace loses tiny faces)
        const int j = (lane + 1 >= m) ? 0 : lane + 1;
        const double ja = shfl(P.a, j), jb = shfl(P.b, j);
        const double a0 = bcast(P.a, 0), b0 = bcast(P.b, 0);
        const bool fan = lane >= 1 && lane + 1 < m;
        const double area2 = wave_sum(fan ? ((P.a - a0) * (jb - b0) - (ja - a0) * (P.b - b0)) : 0.0);
        bool dup = false;
        for (int k = 0; k < m; ++k) {
            const int ek = bcast(P.e, k);
            dup |= act && k != lane && ek == P.e;
        }
        if (ballot(dup)) flags |= kFlagDegen;
        // a starting-square edge cannot survive the box planes; if one did, the
        // face is unusable (and its id names no constraint row)
        if (ballot(act && P.e <= -7)) {
            flags |= kFlagDegen;
            m = 0;
        }
        if (!(area2 > 0.0)) m = 0;
    } else {
        m = 0;
    }
    if (m == 0) flags |= kFlagEmpty;

    if (m > out.stride) {
        flags |= kFlagTooBig;
        m = 0;
    }

    int e_out = 0;
    double x[3] = {0.0, 0.0, 0.0};
    double vsens_a = 0.0, vsens_b = 0.0, vsens_r = 0.0;
    if (m > 0) {
        // rotate so that the smallest edge id comes first
        const int minid = wave_min(lane < m ? P.e : 0x7fffffff);
        const int r0 = __builtin_ctzll(ballot(lane < m && P.e == minid));
        int src = lane + r0;
        if (src >= m) src -= m;
        if (lane >= m) src = lane;
        const int e = shfl(P.e, src);
        const int eprev = shfl(e, lane == 0 ? m - 1 : lane - 1);
        e_out = e;
        if (lane < m) {
            // vertex i = [c_{e(i-1)}; c_{e(i)}; a_F] x = -[...], in FP64
            double ca[4], cb[4];
            constraint_row(net, eprev, code, am, rb, rs, ca);
            constraint_row(net, e, code, am, rb, rs, cb);
            double A[3][3] = {{ca[0], ca[1], ca[2]}, {cb[0], cb[1], cb[2]}, {fx, fy, fz}};
            double rr[3] = {-ca[3], -cb[3], -fw};
            if (margin > 0.0) {
                // estimated vertex error from the approximate rows
                const double an = inv_norm3(A);
                const double s0 = fabs(A[0][0]) + fabs(A[0][1]) + fabs(A[0][2]);
                const double s1 = fabs(A[1][0]) + fabs(A[1][1]) + fabs(A[1][2]);
                const double s2 = fabs(A[2][0]) + fabs(A[2][1]) + fabs(A[2][2]);
                vsens_a = an;
                vsens_b = fmax(s0, fmax(s1, s2));
                vsens_r = fmax(fabs(rr[0]), fmax(fabs(rr[1]), fabs(rr[2])));
            }
            if (!solve3(A, rr, x)) {
                flags |= kFlagSingular;
                x[0] = x[1] = x[2] = __builtin_nan("");
            }
        }
        for (int o = 32; o > 0; o >>= 1) flags |= __shfl_xor(flags, o, kWave);
    }
    if (margin > 0.0) {
        // split-BF16 rows: keep the face only if FP64 could not decide otherwise
        wave_lds_sync();   // the near list was written by other lanes
        bool shaky = false;
        double est = 0.0;
        if (lane < m) {
            const double xm = fmax(fabs(x[0]), fmax(fabs(x[1]), fabs(x[2])));
            est = fb.row_eps * vsens_a * (vsens_b * xm + vsens_r) / fmax(1.0, xm);
            shaky = !(est <= vertex_tol);
        }
        const bool redo = m == 0 || flags != 0 || n_near > kNearMax || ballot(shaky) != 0 ||
                          margin_ambiguous(net, code, am, rb, rs, m, e_out, x[0], x[1], x[2], est, margin, S.near,
                                           n_near);
        if (redo) {
            if (lane == 0) {
                const unsigned long long k = atomicAdd(fb.count, 1ull);
                if (k < fb.cap) fb.list[k] = (int)cell;
                out.m[oi] = 0;
                if (ctr) atomicAdd(&ctr->escalated, 1ull);
            }
            return;
        }
    }
    long long obase = oi * out.stride;
    if (out.off) {
        // this face's corners take m consecutive slots of the shared buffer
        unsigned long long b = 0;
        if (lane == 0 && m > 0) b = atomicAdd(out.slot_n, (unsigned long long)m);
        b = (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b) |
            ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32)) << 32);
        if (m > 0 && b + (unsigned long long)m > out.slot_cap) {
            if (lane == 0 && ctr) atomicAdd(&ctr->overflow_slots, 1ull);
            m = 0;
        }
        obase = (long long)b;
        if (lane == 0) out.off[oi] = m > 0 ? obase : 0;
    }
    if (m > 0 && lane < m) {
        const long long o = obase + lane;
        out.ids[o] = e_out;
        out.verts[o * 3 + 0] = x[0];
        out.verts[o * 3 + 1] = x[1];
        out.verts[o * 3 + 2] = x[2];
        if (out.nbr) out.nbr[o] = -1;
    }
    if (lane == 0) {
        out.m[oi] = m;
        if (out.flags) out.flags[oi] = flags;
    }

    if constexpr (Learn) {
        if (pa.stats && pa.mode != 0 && have_entry && lane == 0) {
            const int slot = (int)(cell % kPropSlots);
            atomicAdd(&pa.stats[0 * kPropSlots + slot], 1ull);
            if (ncuts == 0) atomicAdd(&pa.stats[1 * kPropSlots + slot], 1ull);
            atomicAdd(&pa.stats[2 * kPropSlots + slot], (unsigned long long)ncuts);
        }
        if (pa.samples && have_entry && m > 0)
            collect_samples(net, pa, E, code, am, rb, rs, u, v, p0, m, e_out);
    }

    if (ctr && lane == 0) {
        if (m == 0) {
            if (cell >= n_seed_cells) atomicAdd(&ctr->degenerate, 1ull);
        } else if (flags & kFlagDegen) {
            atomicAdd(&ctr->degenerate, 1ull);
        }
        if (flags & kFlagTooBig) atomicAdd(&ctr->too_big, 1ull);
    }

    // ---- neighbour candidates: flip the unit (or the argmax) behind each edge
    if (ins && rec && m > 0) {
        insert_neighbours(net, *ins, cell, *rec, m, e_out, out, obase, ctr);
    } else if (cand.parent && m > 0) {
        const bool want = lane < m && e_out >= 0;
        const int e_prev = shfl(e_out, lane == 0 ? m - 1 : lane - 1);
        const int e_next = shfl(e_out, lane + 1 >= m ? 0 : lane + 1);
        // edge i runs from vertex i to vertex i + 1
        const int vn = lane + 1 >= m ? 0 : lane + 1;
        const double nx = shfl(x[0], vn), ny = shfl(x[1], vn), nz = shfl(x[2], vn);
        if (ctr) {
            const uint64_t dm = ballot(lane < m && e_out < 0);
            if (lane == 0 && dm) atomicAdd(&ctr->domain_edges, (unsigned long long)__popcll(dm));
        }
        unsigned long long basev;
        const unsigned long long idx = wave_reserve(&ctr->n_cand, want, &basev);
        if (want) {
            if (idx < cand_cap) {
                const uint64_t h = cell_hash[cell];
                uint64_t hn;
                if (e_out < net.N) hn = h ^ net.zobrist[e_out];
                else hn = h ^ net.zobrist[net.N + am] ^ net.zobrist[e_out];
                cand.parent[idx] = (int)cell;
                cand.slot[idx] = lane;
                cand.unit[idx] = e_out;
                cand.hash[idx] = hn;
                cand.hint_prev[idx] = e_prev;
                cand.hint_next[idx] = e_next;
                if (cand.key) cand.key[idx] = morton_key(0.5 * (x[0] + nx), 0.5 * (x[1] + ny), 0.5 * (x[2] + nz));
            } else {
                atomicAdd(&ctr->overflow_cand, 1ull);
            }
        }
    }
}



// ---- calibration of the split-BF16 certificate.  For cells whose faces the
// FP64 chain and clip produced (m, ids, verts), each vertex is solved again
// from the FP32 rows of its two edges and the face plane, as the split form
// does, and compared with the FP64 vertex:
//   ratio  = |x32 - x64|_inf / max(1, |x64|_inf) / sensitivity(FP32 rows),
//   margin = max over hidden and head rows of |(c32 - c64) . [x64; 1]| /
//            (|c64|_1 (1 + |x64|_inf)).
// The largest of each over all vertices goes to out[0], out[1] (non-negative
// doubles compared as integers by atomicMax); out[2] counts the vertices.
// One wave per cell.
__global__ __launch_bounds__(256) void k_calib_split(DevNet net, const uint64_t *__restrict__ codes,
                                                     const int *__restrict__ argmax, long long n,
                                                     const double *__restrict__ rows64,
                                                     const float *__restrict__ rows32, const int *__restrict__ fm,
                                                     const int *__restrict__ fids, const double *__restrict__ fverts,
                                                     const long long *__restrict__ foff, unsigned long long *out) {
    const int lane = lane_id();
    const long long cell = 4LL * blockIdx.x + (threadIdx.x >> 6);
    if (cell >= n) return;
    const int m = fm[cell];
    if (m < 3 || m > kMaxPoly) return;
    const uint64_t *code = codes + cell * net.W;
    const int am = argmax ? argmax[cell] : 0;
    if (am < 0 || am >= net.M) return;
    const double *r64 = rows64 + cell * (long long)net.R * 4;
    const float *r32 = rows32 + cell * (long long)net.R * 4;
    double ratio = 0.0, marg = 0.0;
    double x64[3] = {0.0, 0.0, 0.0};
    if (lane < m) {
        const long long o = foff[cell] + lane;
        const int e = fids[o];
        const int ep = fids[foff[cell] + (lane == 0 ? m - 1 : lane - 1)];
        for (int k = 0; k < 3; ++k) x64[k] = fverts[o * 3 + k];
        double ca[4], cb[4];
        constraint_row(net, ep, code, am, r32, 4, ca);
        constraint_row(net, e, code, am, r32, 4, cb);
        const float *aF = r32 + (long long)(net.N + am) * 4;
        double A[3][3] = {{ca[0], ca[1], ca[2]}, {cb[0], cb[1], cb[2]}, {aF[0], aF[1], aF[2]}};
        double rr[3] = {-ca[3], -cb[3], -(double)aF[3]};
        const double an = inv_norm3(A);
        const double s0 = fabs(A[0][0]) + fabs(A[0][1]) + fabs(A[0][2]);
        const double s1 = fabs(A[1][0]) + fabs(A[1][1]) + fabs(A[1][2]);
        const double s2 = fabs(A[2][0]) + fabs(A[2][1]) + fabs(A[2][2]);
        const double rmax = fmax(fabs(rr[0]), fmax(fabs(rr[1]), fabs(rr[2])));
        double x32[3];
        if (solve3(A, rr, x32)) {
            const double xm = fmax(fabs(x64[0]), fmax(fabs(x64[1]), fabs(x64[2])));
            const double sens = an * (fmax(s0, fmax(s1, s2)) * xm + rmax) / fmax(1.0, xm);
            const double err = fmax(fabs(x32[0] - x64[0]), fmax(fabs(x32[1] - x64[1]), fabs(x32[2] - x64[2])));
            if (sens > 0.0 && sens < __builtin_inf()) ratio = err / fmax(1.0, xm) / sens;
        }
    }
    // sign-test error of every hidden and head row at every vertex
    for (int i = 0; i < m; ++i) {
        const double xi = bcast(x64[0], i), yi = bcast(x64[1], i), zi = bcast(x64[2], i);
        const double sc = 1.0 + fmax(fabs(xi), fmax(fabs(yi), fabs(zi)));
        for (int g = lane; g < net.N + net.M; g += kWave) {
            const long long row = (long long)(g) * 4;
            const double *a = r64 + row;
            const float *b = r32 + row;
            const double d = ((double)b[0] - a[0]) * xi + ((double)b[1] - a[1]) * yi + ((double)b[2] - a[2]) * zi +
                             ((double)b[3] - a[3]);
            const double cn = fabs(a[0]) + fabs(a[1]) + fabs(a[2]) + fabs(a[3]);
            if (cn > 0.0) marg = fmax(marg, fabs(d) / (cn * sc));
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        ratio = fmax(ratio, __shfl_xor(ratio, o, kWave));
        marg = fmax(marg, __shfl_xor(marg, o, kWave));
    }
    if (lane == 0) {
        if (ratio == ratio) atomicMax(&out[0], (unsigned long long)__double_as_longlong(ratio));
        if (marg == marg) atomicMax(&out[1], (unsigned long long)__double_as_longlong(marg));
        atomicAdd(&out[2], (unsigned long long)m);
    }
}

void launch_calib_split(const DevNet &net, const uint64_t *codes, const int *argmax, long long n,
                        const double *rows64, const float *rows32, const int *fm, const int *fids,
                        const double *fverts, const long long *foff, unsigned long long *out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_calib_split, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, net, codes, argmax, n, rows64,
                       rows32, fm, fids, fverts, foff, out);
}

// Positions 0..count-1 of a step: cell lo + p, or list[p] (count read on the
// device from *list_count, at most cap).
// With dev set (device-driven steps), the range is cells dev[0] ..
// dev[0] + dev[1] - 1, read on the device (lo, hi unused).
struct CellRange {
    long long lo, hi;
    const int *list;
    const unsigned long long *list_count;
    unsigned long long cap;
    const unsigned long long *dev;
    __device__ long long base() const { return dev ? (long long)dev[0] : lo; }
    __device__ long long count() const {
        if (dev) return (long long)dev[1];
        if (!list || !list_count) return hi - lo;
        const unsigned long long c = *list_count;
        return (long long)(c < cap ? c : cap);
    }
    __device__ long long cell(long long p) const { return list ? (long long)list[p] : base() + p; }
    __device__ long long tile_base(long long p) const { return list ? p : base() + p; }
};

// Unfused FP64 chain, 4 G cells per workgroup: rows of position p go to
// rows[p][R][4].
template <int G, int KC>
__global__ __launch_bounds__(256) void k_chain_f64(DevNet net, const uint64_t *__restrict__ codes,
                                                   const int *__restrict__ cell_shape, CellRange rg,
                                                   double *__restrict__ rows) {
    __shared__ uint64_t code_lds[4 * G * kMaxWords];
    __shared__ int shape_lds[4 * G];
    const long long p0 = 4LL * G * blockIdx.x;
    const long long n = rg.count();
    if (p0 >= n) return;
    const int ncell = (int)min(4LL * G, n - p0);
    chain_tile<G, KC>(net, codes, cell_shape, rg.list, rg.tile_base(p0), ncell, rows + p0 * (long long)net.R * 4,
                      4, (long long)net.R * 4, code_lds, shape_lds);
}

// Dense FP64 chain, four cells per workgroup, the previous layer's rows in LDS.
template <int KC>
__global__ __launch_bounds__(256) void k_chain_f64_lds(DevNet net, const uint64_t *__restrict__ codes,
                                                       const int *__restrict__ cell_shape, CellRange rg,
                                                       double *__restrict__ rows) {
    __shared__ uint64_t code_lds[4 * kMaxWords];
    __shared__ int shape_lds[4];
    __shared__ double zl[2 * kLdsRows * 16];
    const long long p0 = 4LL * blockIdx.x;
    const long long n = rg.count();
    if (p0 >= n) return;
    const int ncell = (int)min(4LL, n - p0);
    chain_tile<1, KC>(net, codes, cell_shape, rg.list, rg.tile_base(p0), ncell, rows + p0 * (long long)net.R * 4, 4,
                      (long long)net.R * 4, code_lds, shape_lds, zl);
}

// Dense FP64 chain, four cells per workgroup, the previous hidden layer
// staged in LDS (dynamic: widest hidden layer x 16 doubles).
template <int KC>
__global__ __launch_bounds__(256) void k_chain_f64_res(DevNet net, const uint64_t *__restrict__ codes,
                                                       const int *__restrict__ cell_shape, CellRange rg,
                                                       double *__restrict__ rows) {
    __shared__ uint64_t code_lds[4 * kMaxWords];
    __shared__ int shape_lds[4];
    extern __shared__ double zr[];
    const long long p0 = 4LL * blockIdx.x;
    const long long n = rg.count();
    if (p0 >= n) return;
    const int ncell = (int)min(4LL, n - p0);
    chain_tile_res<KC>(net, codes, cell_shape, rg.list, rg.tile_base(p0), ncell, rows + p0 * (long long)net.R * 4,
                       4, (long long)net.R * 4, code_lds, shape_lds, zr);
}

// Gathered FP64 chain, four cells per workgroup.
template <int KC>
__global__ __launch_bounds__(256) void k_chain_f64_gather(DevNet net, const uint64_t *__restrict__ codes,
                                                          const int *__restrict__ cell_shape, CellRange rg,
                                                          double *__restrict__ rows) {
    __shared__ uint64_t code_lds[4 * kMaxWords];
    __shared__ int shape_lds[4];
    __shared__ short lists[kListBlocks * (kListMax + 4)];
    __shared__ int cnt_lds[kListMax / 64];
    const long long p0 = 4LL * blockIdx.x;
    const long long n = rg.count();
    if (p0 >= n) return;
    const int ncell = (int)min(4LL, n - p0);
    chain_tile_gather<KC>(net, codes, cell_shape, rg.list, rg.tile_base(p0), ncell,
                          rows + p0 * (long long)net.R * 4, 4, (long long)net.R * 4, code_lds, shape_lds, lists,
                          cnt_lds);
}

// ---- staged-B chain.  The producing layer writes its output, masked by the
// cells' codes (diag(s_l)) and zero padded, into one LDS buffer that the next
// layer reads as its B operand: the K loop has no code tests, no branches and
// no global B loads.  Weight fragments (A) stream from L2 one batch of K-steps
// ahead of the MFMAs that use them; when every weight is an FP32 number they
// stream as FP32 (half the bytes) and are widened exactly in registers.
// Wave w owns the 16-row output tiles w, w + nwaves, ... (at most MTW) for all
// 4 G cells of the workgroup and keeps their accumulators until the layer's
// barrier, so a single LDS buffer suffices.  Blocks from the input use
// Z_0 = [I | 0]; a source other than the previous layer (a shortcut between
// hidden layers) is read from the rows in global memory with code tests.
constexpr int kLbKSteps = 8;    // A fragments loaded ahead, per output tile slot x MTW

template <typename AT>
__device__ __forceinline__ const AT *lb_frags(const DevNet &net);
template <>
__device__ __forceinline__ const double *lb_frags<double>(const DevNet &net) { return net.wfrag; }
template <>
__device__ __forceinline__ const float *lb_frags<float>(const DevNet &net) { return net.wfrag32; }

template <int G, int MTW, typename AT>
__global__ __launch_bounds__(MTW == 1 ? 1024 : 512) void k_chain_lb(DevNet net, const uint64_t *__restrict__ codes,
                                                   const int *__restrict__ cell_shape, CellRange rg,
                                                   double *__restrict__ rows) {
    constexpr int NC = 4 * G;            // cells per workgroup
    constexpr int NCOL = 16 * G;         // MFMA columns
    constexpr int KC = kLbKSteps / MTW;  // K-steps per batch
    extern __shared__ double bsh[];      // [net.lb_kpad][NCOL]: masked rows of the previous layer
    __shared__ uint64_t code_lds[NC * kMaxWords];
    __shared__ int shape_lds[NC];
    const long long p0 = (long long)NC * blockIdx.x;
    const long long n = rg.count();
    if (p0 >= n) return;
    const int ncell = (int)min((long long)NC, n - p0);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int col = lane & 15;    // MFMA column (B, D) / row within the tile (A)
    const int kq = lane >> 4;     // k within the K-step (A, B) / row offset (D)
    const int q = col & 3;        // homogeneous component of this column
    const int cl = col >> 2;      // cell of this column within its group
    stage_tile(net, codes, cell_shape, rg.list, rg.tile_base(p0), ncell, code_lds, shape_lds, NC);
    for (int t = threadIdx.x; t < net.lb_kpad * NCOL; t += blockDim.x) bsh[t] = 0.0;
    __syncthreads();
    double *zb = rows + p0 * (long long)net.R * 4;
    const long long cs = (long long)net.R * 4;
    const AT *wf = lb_frags<AT>(net);

    for (int l = 1; l < net.n_layers; ++l) {
        const int nl = net.width[l];
        const int mtiles = (nl + 15) >> 4;
        int nmt = 0;   // output tiles of this wave in this layer
#pragma unroll
        for (int s = 0; s < MTW; ++s)
            if (wave + s * nwaves < mtiles) nmt = s + 1;
        v4d acc[MTW][G];
#pragma unroll
        for (int s = 0; s < MTW; ++s)
#pragma unroll
            for (int g = 0; g < G; ++g) acc[s][g] = v4d{0.0, 0.0, 0.0, 0.0};
        for (int b = 0; b < net.n_blocks; ++b) {
            if (net.blk_dst[b] != l || nmt == 0) continue;
            const int j = net.blk_src[b];
            const int ks_n = net.blk_ld[b] >> 2;
            const AT *fr[MTW];
#pragma unroll
            for (int s = 0; s < MTW; ++s)   // an idle slot reads the last tile (in bounds, unused)
                fr[s] = wf + net.blk_frag_off[b] + (long long)min(wave + s * nwaves, mtiles - 1) * ks_n * 64 + lane;
            if (j == 0) {
                // Z_0 = [I | 0]: one K-step; row k of B is e_k for k < 3
                const double bv = (kq < 3 && kq == q) ? 1.0 : 0.0;
#pragma unroll
                for (int s = 0; s < MTW; ++s) {
                    if (s >= nmt) break;
                    const double a = (double)fr[s][0];
#pragma unroll
                    for (int g = 0; g < G; ++g) acc[s][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[s][g], 0, 0, 0);
                }
                continue;
            }
            if (j == l - 1) {
                // B from LDS; rows past the source's width read as zeros, so the
                // clamped A loads of the last batch contribute nothing
                AT ac[MTW][KC], an[MTW][KC];
#pragma unroll
                for (int s = 0; s < MTW; ++s)
#pragma unroll
                    for (int u = 0; u < KC; ++u) ac[s][u] = fr[s][min(u, ks_n - 1) * 64];
                const double *bcol = bsh + kq * NCOL + col;
                for (int ks0 = 0; ks0 < ks_n; ks0 += KC) {
#pragma unroll
                    for (int s = 0; s < MTW; ++s)
#pragma unroll
                        for (int u = 0; u < KC; ++u) an[s][u] = fr[s][min(ks0 + KC + u, ks_n - 1) * 64];
                    double bv[KC][G];
#pragma unroll
                    for (int u = 0; u < KC; ++u)
#pragma unroll
                        for (int g = 0; g < G; ++g) bv[u][g] = bcol[(ks0 + u) * 4 * NCOL + g * 16];
#pragma unroll
                    for (int u = 0; u < KC; ++u)
#pragma unroll
                        for (int s = 0; s < MTW; ++s) {
                            if (s >= nmt) break;
                            const double a = (double)ac[s][u];
#pragma unroll
                            for (int g = 0; g < G; ++g)
                                acc[s][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[u][g], acc[s][g], 0, 0, 0);
                        }
#pragma unroll
                    for (int s = 0; s < MTW; ++s)
#pragma unroll
                        for (int u = 0; u < KC; ++u) ac[s][u] = an[s][u];
                }
                continue;
            }
            // a shortcut from an earlier hidden layer: its rows, written by this
            // workgroup, from global memory, masked here
            const int nj = net.width[j];
            const int uoff = net.unit_off[j];
            const long long roff = (long long)net.row_off[j] * 4;
            for (int ks = 0; ks < ks_n; ++ks) {
                const int k = ks * 4 + kq;
                double bv[G];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int c = 4 * g + cl;
                    bv[g] = (k < nj && c < ncell && code_bit(code_lds + c * net.W, uoff + k))
                                ? zb[c * cs + roff + (long long)k * 4 + q] : 0.0;
                }
#pragma unroll
                for (int s = 0; s < MTW; ++s) {
                    if (s >= nmt) break;
                    const double a = (double)fr[s][ks * 64];
#pragma unroll
                    for (int g = 0; g < G; ++g) acc[s][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[g], acc[s][g], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // every wave is done with the previous layer's B
        // rows (plus bias) to global memory; masked rows into the B buffer.
        // v_mfma_f64_16x16x4f64 leaves D[kq + 4 r][col] in register r.
        const bool hidden = l < net.n_layers - 1;
#pragma unroll
        for (int s = 0; s < MTW; ++s) {
            if (s >= nmt) break;
            const int mt = wave + s * nwaves;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int c = 4 * g + cl;
                const bool ok = c < ncell;
                const double *bias = net.bias + (long long)shape_lds[c] * net.bias_stride + net.bias_off[l];
                const uint64_t *code = code_lds + c * net.W;
                double *z0 = zb + c * cs + (long long)net.row_off[l] * 4 + q;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = mt * 16 + kq + 4 * r;
                    double v = acc[s][g][r];
                    if (i < nl) {
                        if (q == 3) v += bias[i];
                        if (ok) z0[(long long)i * 4] = v;
                    }
                    if (hidden) {
                        const bool on = ok && i < nl && code_bit(code, net.unit_off[l] + i);
                        bsh[i * NCOL + g * 16 + col] = on ? v : 0.0;
                    }
                }
            }
        }
        if (hidden) {
            // rows the next layer's batches may read past this layer's tiles
            const int r0 = mtiles * 16;
            const int r1 = min(net.lb_kpad, (nl + 31) & ~31);
            for (int t = threadIdx.x; t < (r1 - r0) * NCOL; t += blockDim.x) bsh[r0 * NCOL + t] = 0.0;
        }
        __syncthreads();
    }
}

// Split-BF16 chain: FP32 rows of position p go to rows[p][R][4].
__global__ __launch_bounds__(256) void k_chain_bf16(DevNet net, const uint64_t *__restrict__ codes,
                                                    const int *__restrict__ cell_shape, CellRange rg,
                                                    float *__restrict__ rows) {
    __shared__ uint64_t code_lds[4 * kMaxWords];
    __shared__ int shape_lds[4];
    const long long p0 = 4LL * blockIdx.x;
    const long long n = rg.count();
    if (p0 >= n) return;
    const int ncell = (int)min(4LL, n - p0);
    chain_tile_bf16(net, codes, cell_shape, rg.list, rg.tile_base(p0), ncell, rows + p0 * (long long)net.R * 4, 4,
                    (long long)net.R * 4, code_lds, shape_lds);
}

// Unfused clip: one wave per position, four per workgroup.
template <typename RowT>
__global__ __launch_bounds__(256) void k_clip(DevNet net, const uint64_t *__restrict__ codes,
                                              const int *__restrict__ argmax, const uint64_t *__restrict__ cell_hash,
                                              const int *__restrict__ hints, CellRange rg, long long n_seed_cells,
                                              const RowT *__restrict__ rows, ClipOut out, Candidates cand,
                                              unsigned long long cand_cap, Counters *ctr, double margin,
                                              double vertex_tol, Fallback fb, PropArgs pa) {
    __shared__ PolyScratch scratch[4];
    const int wave = threadIdx.x >> 6;
    const long long p = 4LL * blockIdx.x + wave;
    if (p >= rg.count()) return;
    clip_cell<RowT, false>(net, codes, argmax, cell_hash, hints, rg.cell(p), n_seed_cells,
                           rows + p * (long long)net.R * 4, 4, scratch[wave], out, cand, cand_cap, ctr, margin,
                           vertex_tol, fb, pa, nullptr);
}

// The clip with the learned form's steps (proposals, counting, sample
// collection) and the scorer's LDS.
__global__ __launch_bounds__(256) void k_clip_pivot(DevNet net, const uint64_t *__restrict__ codes,
                                                    const int *__restrict__ argmax,
                                                    const uint64_t *__restrict__ cell_hash,
                                                    const int *__restrict__ hints, CellRange rg,
                                                    long long n_seed_cells, const double *__restrict__ rows,
                                                    ClipOut out, Candidates cand, unsigned long long cand_cap,
                                                    Counters *ctr, PropArgs pa) {
    __shared__ PolyScratch scratch[4];
    const int wave = threadIdx.x >> 6;
    const long long p = 4LL * blockIdx.x + wave;
    if (p >= rg.count()) return;
    const Fallback none{nullptr, nullptr, 0, 0.0};
    clip_cell<double, false, true>(net, codes, argmax, cell_hash, hints, rg.cell(p), n_seed_cells,
                                   rows + p * (long long)net.R * 4, 4, scratch[wave], out, cand, cand_cap, ctr, 0.0,
                                   0.0, none, pa, nullptr);
}

template <typename RowT>
__global__ __launch_bounds__(256, 3) void k_clip_prop(DevNet net, const uint64_t *__restrict__ codes,
                                                   const int *__restrict__ argmax,
                                                   const uint64_t *__restrict__ cell_hash,
                                                   const int *__restrict__ hints, CellRange rg, long long n_seed_cells,
                                                   const RowT *__restrict__ rows, ClipOut out, Candidates cand,
                                                   unsigned long long cand_cap, Counters *ctr, double margin,
                                                   double vertex_tol, Fallback fb, PropArgs pa) {
    __shared__ PolyScratch scratch[4];
    __shared__ PropScratch pscr[4];
    const int wave = threadIdx.x >> 6;
    const long long p = 4LL * blockIdx.x + wave;
    if (p >= rg.count()) return;
    clip_cell<RowT, true>(net, codes, argmax, cell_hash, hints, rg.cell(p), n_seed_cells,
                          rows + p * (long long)net.R * 4, 4, scratch[wave], out, cand, cand_cap, ctr, margin,
                          vertex_tol, fb, pa, &pscr[wave]);
}

// Fused step: the chain of four cells lands in LDS as [row][cell][4]
// (16 consecutive doubles per row: conflict-free B loads and D stores), then
// wave w clips cell w straight from LDS.  No row ever goes to HBM.
__global__ __launch_bounds__(256) void k_march_fused(DevNet net, const uint64_t *__restrict__ codes,
                                                     const int *__restrict__ cell_shape,
                                                     const int *__restrict__ argmax,
                                                     const uint64_t *__restrict__ cell_hash,
                                                     const int *__restrict__ hints, long long lo,
                                                     long long hi, long long n_seed_cells, ClipOut out,
                                                     Candidates cand, unsigned long long cand_cap,
                                                     Counters *ctr) {
    extern __shared__ double zl[];
    __shared__ PolyScratch scratch[4];
    __shared__ uint64_t code_lds[4 * kMaxWords];
    __shared__ int shape_lds[4];
    const int wave = threadIdx.x >> 6;
    const long long c0 = lo + 4LL * blockIdx.x;
    const int ncell = (int)min(4LL, hi - c0);
    chain_tile<1, kKChunk>(net, codes, cell_shape, nullptr, c0, ncell, zl, 16, 4, code_lds, shape_lds);
    if (wave >= ncell) return;
    const Fallback none{nullptr, nullptr, 0, 0.0};
    const PropArgs off{};
    clip_cell<double, false>(net, codes, argmax, cell_hash, hints, c0 + wave, n_seed_cells, zl + wave * 4, 16,
                             scratch[wave], out, cand, cand_cap, ctr, 0.0, 0.0, none, off, nullptr);
}

// ---- chain of one persistent tile (four cells, four waves) with the
// staged-B scheme of k_chain_lb, but two LDS buffers used in turn by layer
// parity (bsh: 2 x lb_kpad x 16 doubles): layer l writes its masked output
// into buffer l & 1 while every wave still reads layer l - 1 from the other,
// so a wave can finish its output tiles group by group (MTW tiles at a time)
// and one barrier per layer suffices at any width.  Rows (plus bias) go to
// zb[cell * cs + row * 4 + q].  Same products in the same order as the dense
// tile (equal rows).  Ends with a barrier.
template <typename AT, int MTW>
__device__ void chain_tile_pp(const DevNet &net, const uint64_t *code_lds, const int *shape_lds, int ncell,
                              double *zb, long long cs, double *bsh) {
    // K-steps per batch: 2 x 8 MFMAs in flight per prefetch with FP32
    // fragments, 8 with FP64 ones (the register budget of three waves per SIMD)
    constexpr int KC = (sizeof(AT) == 4 ? 2 : 1) * kLbKSteps / MTW;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int col = lane & 15;
    const int kq = lane >> 4;
    const int q = col & 3;
    const int cl = col >> 2;
    const bool ok = cl < ncell;
    const int kpad = net.lb_kpad;
    const AT *wf = lb_frags<AT>(net);
    const uint64_t *code = code_lds + cl * net.W;
    const double *bias_c = net.bias + (long long)shape_lds[cl] * net.bias_stride;
    double *zc = zb + cl * cs + q;
    for (int l = 1; l < net.n_layers; ++l) {
        const int nl = net.width[l];
        const int mtiles = (nl + 15) >> 4;
        const bool hidden = l < net.n_layers - 1;
        double *ob = bsh + (l & 1) * kpad * 16;
        const double *ib = bsh + ((l - 1) & 1) * kpad * 16;
        for (int g0 = 0; g0 < mtiles; g0 += nwaves * MTW) {
            int nmt = 0;
#pragma unroll
            for (int s = 0; s < MTW; ++s)
                if (g0 + wave + s * nwaves < mtiles) nmt = s + 1;
            if (nmt == 0) break;
            v4d acc[MTW];
#pragma unroll
            for (int s = 0; s < MTW; ++s) acc[s] = v4d{0.0, 0.0, 0.0, 0.0};
            for (int b = 0; b < net.n_blocks; ++b) {
                if (net.blk_dst[b] != l) continue;
                const int j = net.blk_src[b];
                const int ks_n = net.blk_ld[b] >> 2;
                const AT *fr[MTW];
#pragma unroll
                for (int s = 0; s < MTW; ++s)
                    fr[s] = wf + net.blk_frag_off[b] + (long long)min(g0 + wave + s * nwaves, mtiles - 1) * ks_n * 64 +
                            lane;
                if (j == 0) {
                    const double bv = (kq < 3 && kq == q) ? 1.0 : 0.0;
#pragma unroll
                    for (int s = 0; s < MTW; ++s) {
                        if (s >= nmt) break;
                        acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)fr[s][0], bv, acc[s], 0, 0, 0);
                    }
                    continue;
                }
                if (j == l - 1) {
                    AT ac[MTW][KC], an[MTW][KC];
#pragma unroll
                    for (int s = 0; s < MTW; ++s)
#pragma unroll
                        for (int u = 0; u < KC; ++u) ac[s][u] = fr[s][min(u, ks_n - 1) * 64];
                    const double *bcol = ib + kq * 16 + col;
                    for (int ks0 = 0; ks0 < ks_n; ks0 += KC) {
#pragma unroll
                        for (int s = 0; s < MTW; ++s)
#pragma unroll
                            for (int u = 0; u < KC; ++u) an[s][u] = fr[s][min(ks0 + KC + u, ks_n - 1) * 64];
                        double bv[KC];
#pragma unroll
                        for (int u = 0; u < KC; ++u) bv[u] = bcol[(ks0 + u) * 64];
#pragma unroll
                        for (int u = 0; u < KC; ++u)
#pragma unroll
                            for (int s = 0; s < MTW; ++s) {
                                if (s >= nmt) break;
                                acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ac[s][u], bv[u], acc[s], 0, 0, 0);
                            }
#pragma unroll
                        for (int s = 0; s < MTW; ++s)
#pragma unroll
                            for (int u = 0; u < KC; ++u) ac[s][u] = an[s][u];
                    }
                    continue;
                }
                // a shortcut from an earlier hidden layer: its rows, written
                // by this workgroup, from global memory, masked here
                const int nj = net.width[j];
                const int uoff = net.unit_off[j];
                const long long roff = (long long)net.row_off[j] * 4;
                for (int ks = 0; ks < ks_n; ++ks) {
                    const int k = ks * 4 + kq;
                    const double bv = (k < nj && ok && code_bit(code, uoff + k)) ? zc[roff + (long long)k * 4] : 0.0;
#pragma unroll
                    for (int s = 0; s < MTW; ++s) {
                        if (s >= nmt) break;
                        acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)fr[s][ks * 64], bv, acc[s], 0, 0, 0);
                    }
                }
            }
            // rows (plus bias) to global memory, masked rows to the B buffer;
            // v_mfma_f64_16x16x4f64 leaves D[kq + 4 r][col] in register r
            const double *bias = bias_c + net.bias_off[l];
            double *z0 = zc + (long long)net.row_off[l] * 4;
#pragma unroll
            for (int s = 0; s < MTW; ++s) {
                if (s >= nmt) break;
                const int mt = g0 + wave + s * nwaves;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = mt * 16 + kq + 4 * r;
                    double v = acc[s][r];
                    if (i < nl) {
                        if (q == 3) v += bias[i];
                        if (ok) z0[(long long)i * 4] = v;
                    }
                    if (hidden) {
                        const bool on = ok && i < nl && code_bit(code, net.unit_off[l] + i);
                        ob[i * 16 + col] = on ? v : 0.0;
                    }
                }
            }
        }
        if (hidden) {
            // rows the next layer's batches may read past this layer's tiles
            const int r0 = mtiles * 16;
            const int r1 = min(kpad, (nl + 31) & ~31);
            for (int t = threadIdx.x; t < (r1 - r0) * 16; t += blockDim.x) ob[r0 * 16 + t] = 0.0;
        }
        __syncthreads();
    }
}

// ---- persistent march (plain FP64 form).  Cell ids are tickets: a
// workgroup takes the next four ids with one fetch-add on next_cell (ids not
// yet discovered included: cells are numbered in the order they are found),
// and processes each of them once it is published (its ready flag set by
// the workgroup that found it).  A round takes the published ones of its
// held ids (up to four), copies their records to LDS, computes their affine
// chain into the workgroup's rows buffer, and each wave clips one cell and
// inserts that face's neighbours into the hash set itself
// (insert_neighbours), which numbers and publishes the new cells.  All data
// another workgroup wrote is read with device-scope loads (ld_dev) and all
// data another workgroup reads is written with device-scope stores, so no
// cache-wide fence is needed.  The march ends when every discovered cell is
// finished: done_cells is read before n_cells (a cell is counted done only
// after its insertions completed), so equal counts mean no cell is in flight
// and none can appear; the ids a workgroup still holds then name no cell.
// Every wait is bounded: a workgroup that has slept spin_limit naps (about
// 64 cycles each) in its queue polls without a cell finishing anywhere stops
// the march and counts a stall, and so does a wait for another wave's claim
// that outlasts spin_limit / 16 polls; capacity overflows stop it too.  Idle
// workgroups back off to about 8k cycles between polls: their device-scope
// loads would otherwise compete with the working ones.  The
// host checks both.  At least three waves per SIMD (the register budget
// that allows, without spills): three workgroups per CU share the clip's
// latency.
template <int CH>
__global__ __launch_bounds__(256, 3) void k_march_persist(DevNet net, uint64_t *codes, int *cell_shape, int *argmax,
                                                       uint64_t *cell_hash, int *hints, double *rows_ws,
                                                       long long n_seed_cells, ClipOut out, Counters *ctr,
                                                       InlineInsert ins) {
    extern __shared__ double bsh[];   // CH > 0: 2 x lb_kpad x 16 doubles, the chain's B buffers
    __shared__ PolyScratch scratch[4];
    __shared__ uint64_t code_lds[4 * kMaxWords];
    __shared__ int shape_lds[4];
    __shared__ int am_lds[4];
    __shared__ int hint_lds[4][3];
    __shared__ uint64_t hash_lds[4];
    __shared__ long long tile_cell_id[4];
    __shared__ int tile_n;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const long long cs = (long long)net.R * 4;
    double *zb = rows_ws + (long long)blockIdx.x * 4 * cs;
    const Candidates none_c{};
    const Fallback none_f{nullptr, nullptr, 0, 0.0};
    const PropArgs off{};
    // held tickets (thread 0 only): ids not processed yet, -1 = none
    long long held[4] = {-1, -1, -1, -1};
    for (;;) {
        if (threadIdx.x == 0) {
            int n = 0;
            unsigned long long last_done = ~0ull, slept = 0;   // naps since done_cells last moved
            int nap = 1;
            for (unsigned poll = 0;; ++poll) {
                if (held[0] < 0 && held[1] < 0 && held[2] < 0 && held[3] < 0) {
                    const unsigned long long a = atomicAdd(&ctr->next_cell, 4ull);
                    for (int k = 0; k < 4; ++k) held[k] = (long long)a + k;
                }
                // the published ones of the held ids form this round's tile
                for (int k = 0; k < 4; ++k) {
                    const long long c = held[k];
                    if (c >= 0 && (unsigned long long)c < ins.cap_cells && ld_dev(&ins.ready[c]) == ins.epoch) {
                        tile_cell_id[n++] = c;
                        held[k] = -1;
                    }
                }
                if (n > 0) break;
                if ((poll & 7) == 7) {
                    if (ld_dev(&ctr->stop)) break;
                    // done_cells first: its count only includes cells whose
                    // insertions (n_cells increments) had completed
                    const unsigned long long d = ld_dev(&ctr->done_cells);
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    const unsigned long long c2 = ld_dev(&ctr->n_cells);
                    if (d >= c2) break;   // nothing in flight: the march is over
                    if (d != last_done) {
                        last_done = d;
                        slept = 0;
                    } else if (slept > ins.spin_limit) {   // spin_limit naps of ~64 cycles: ~0.2 s
                        atomicAdd(&ctr->stalled, 1ull);
                        st_dev(&ctr->stop, 1ull);
                        break;
                    }
                }
                // back off while nothing held is published (about 64 * nap
                // cycles, at most about 8k): idle workgroups' polls are
                // device-scope loads that compete with the working ones
                for (int z = 0; z < nap; ++z) __builtin_amdgcn_s_sleep(1);
                slept += nap;
                if (nap < 128) nap <<= 1;
            }
            tile_n = n;
        }
        __syncthreads();
        const int n = tile_n;
        if (n <= 0) break;
        if (threadIdx.x < n) {
            // the flag was seen before these loads are issued
            const long long c = tile_cell_id[threadIdx.x];
            const int sh = ld_dev(&cell_shape[c]);
            shape_lds[threadIdx.x] = (sh >= 0 && sh < net.S) ? sh : 0;
            am_lds[threadIdx.x] = ld_dev(&argmax[c]);
            for (int h = 0; h < 3; ++h) hint_lds[threadIdx.x][h] = ld_dev(&hints[c * 3 + h]);
            hash_lds[threadIdx.x] = ld_dev(&cell_hash[c]);
        } else if (threadIdx.x < 4) {
            shape_lds[threadIdx.x] = 0;
        }
        for (int t = threadIdx.x; t < 4 * net.W; t += blockDim.x) {
            const int c = t / net.W;
            code_lds[t] = c < n ? ld_dev(&codes[tile_cell_id[c] * net.W + (t - c * net.W)]) : 0ull;
        }
        __syncthreads();
        if constexpr (CH == 0)
            chain_tile<1, 4>(net, codes, cell_shape, nullptr, 0, n, zb, 4, cs, code_lds, shape_lds, nullptr, true);
        else
            chain_tile_pp<typename std::conditional<CH == 2, float, double>::type, 2>(net, code_lds, shape_lds, n,
                                                                                      zb, cs, bsh);
        if (wave < n) {
            CellRec rec;
            rec.code = code_lds + wave * net.W;
            rec.am = am_lds[wave];
            rec.shape = shape_lds[wave];
            rec.hint[0] = hint_lds[wave][0];
            rec.hint[1] = hint_lds[wave][1];
            rec.hint[2] = hint_lds[wave][2];
            rec.hash = hash_lds[wave];
            clip_cell<double, false>(net, codes, argmax, cell_hash, hints, tile_cell_id[wave], n_seed_cells,
                                     zb + wave * cs, 4, scratch[wave], out, none_c, 0, ctr, 0.0, 0.0, none_f, off,
                                     nullptr, &ins, &rec);
        }
        __syncthreads();
        // every wave's insertions have completed (publish_wait) before the barrier
        if (threadIdx.x == 0) atomicAdd(&ctr->done_cells, (unsigned long long)n);
    }
}

// Ready flags of the seed cells (0 .. n_cells - 1) for a persistent march.
__global__ void k_mark_ready(unsigned *ready, const Counters *ctr, unsigned epoch) {
    const unsigned long long n = ctr->n_cells;
    for (unsigned long long c = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; c < n;
         c += (unsigned long long)gridDim.x * blockDim.x)
        ready[c] = epoch;
}

// Logits of n feature rows (FP32 [n][kPropD]) by the scorer the proposing
// clip uses (FP16 operands, FP32 accumulation); one wave per 64 rows.
__global__ __launch_bounds__(256) void k_prop_score(PropNet P, const float *__restrict__ X, long long n,
                                                    float *__restrict__ z) {
    __shared__ PropScratch ps[4];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const long long r0 = (4LL * blockIdx.x + wave) * kWave;
    if (r0 >= n) return;
    const int rows = (int)min((long long)kWave, n - r0);
    for (int i = lane; i < kWave * kPropD; i += kWave) {
        const int r = i / kPropD;
        ps[wave].feats[i] = (_Float16)(r < rows ? X[(r0 + r) * kPropD + (i % kPropD)] : 0.f);
    }
    wave_lds_sync();
    const float zz = prop_score(P, ps[wave].feats, ps[wave].hs, rows);
    if (lane < rows) z[r0 + lane] = zz;
}

// Repacks padded per-cell rows into the dense [n][N+M][4] FP64 layout of am_chain.
template <typename RowT>
__global__ void k_rows_unpad(DevNet net, long long n, const RowT *__restrict__ rows, double *__restrict__ out) {
    const int G = net.N + net.M;
    const long long total = n * G;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const long long c = t / G;
        const int g = (int)(t % G);
        const RowT *src = rows + (c * net.R + (g)) * 4;
        double *dst = out + t * 4;
        dst[0] = src[0];
        dst[1] = src[1];
        dst[2] = src[2];
        dst[3] = src[3];
    }
}

size_t fused_lds_bytes(const DevNet &net) { return sizeof(double) * 16 * (size_t)net.R; }

// Static LDS of the fused kernel: four waves' clip scratch and the tile's codes.
size_t fused_static_lds_bytes() { return 4 * sizeof(PolyScratch) + 4 * kMaxWords * sizeof(uint64_t) + 64; }

// Rows the staged chain holds in LDS: the widest hidden layer padded to
// whole K-steps, or 0 when that exceeds kResMax.
static int res_rows(const DevNet &net) {
    int w = 0;
    for (int l = 1; l < net.n_layers - 1; ++l) w = max(w, net.width[l]);
    w = (w + 3) & ~3;
    return w <= kResMax ? w : 0;
}

size_t chain_res_lds_bytes(const DevNet &net) { return (size_t)res_rows(net) * 16 * sizeof(double); }

hipError_t prepare_chain_res(size_t bytes) {
    return hipFuncSetAttribute((const void *)k_chain_f64_res<kKChunk>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

hipError_t prepare_fused(size_t bytes) {
    return hipFuncSetAttribute((const void *)k_march_fused, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

static CellRange range_of(long long lo, long long hi, const int *list, const unsigned long long *count,
                          unsigned long long cap, const unsigned long long *dev = nullptr) {
    CellRange r;
    r.dev = dev;
    r.lo = lo;
    r.hi = hi;
    r.list = list;
    r.list_count = count;
    r.cap = cap;
    return r;
}

// Staged-B chain shapes: variant 6 = four cells per workgroup, 7 = eight, 8 =
// four cells with two output tiles per wave; one tile per wave otherwise.
// Tiles per wave double while the widest layer would need more waves than a
// workgroup of that kind holds (16 with one tile per wave, else 8), up to 4.
struct LbShape {
    int G, MTW, nwaves;
    bool f32;
    size_t lds;
};

static bool lb_shape(const DevNet &net, int variant, LbShape &o) {
    if (variant < 6 || variant > 8 || net.lb_kpad <= 0) return false;
    int mt_max = 0;
    for (int l = 1; l < net.n_layers; ++l) mt_max = max(mt_max, (net.width[l] + 15) / 16);
    o.G = variant == 7 ? 2 : 1;
    o.MTW = variant == 8 ? 2 : 1;
    while (o.MTW <= 4 && (mt_max + o.MTW - 1) / o.MTW > (o.MTW == 1 ? 16 : 8)) o.MTW *= 2;
    o.nwaves = (mt_max + o.MTW - 1) / o.MTW;
    o.f32 = net.wfrag32 != nullptr;
    o.lds = (size_t)net.lb_kpad * 16 * o.G * sizeof(double);
    return o.MTW <= 4;
}

template <int G, int MTW, typename AT>
static void launch_lb_t(const DevNet &net, const uint64_t *codes, const int *cell_shape, const CellRange &rg,
                        long long n, double *rows, const LbShape &o, hipStream_t st) {
    hipLaunchKernelGGL((k_chain_lb<G, MTW, AT>), dim3((unsigned)((n + 4 * G - 1) / (4 * G))), dim3(64 * o.nwaves),
                       o.lds, st, net, codes, cell_shape, rg, rows);
}

template <int G, int MTW, typename AT>
static hipError_t prepare_lb_t(size_t bytes) {
    return hipFuncSetAttribute((const void *)k_chain_lb<G, MTW, AT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

// Sets the LDS limits of the staged-B chain for `net` and returns the mask
// of variants (bit v - 6) that fit in lds_limit bytes per workgroup.
int prepare_chain_lb(const DevNet &net, size_t lds_limit) {
    int ok = 0;
    for (int v = 6; v <= 8; ++v) {
        LbShape o;
        if (!lb_shape(net, v, o)) continue;
        const size_t stat = sizeof(uint64_t) * 4 * o.G * kMaxWords + 64;
        if (o.lds + stat > lds_limit) continue;
        hipError_t e;
#define AM_LB_PREP(G_, M_) (o.f32 ? prepare_lb_t<G_, M_, float>(o.lds) : prepare_lb_t<G_, M_, double>(o.lds))
        if (o.G == 2)
            e = o.MTW == 4 ? AM_LB_PREP(2, 4) : o.MTW == 2 ? AM_LB_PREP(2, 2) : AM_LB_PREP(2, 1);
        else
            e = o.MTW == 4 ? AM_LB_PREP(1, 4) : o.MTW == 2 ? AM_LB_PREP(1, 2) : AM_LB_PREP(1, 1);
#undef AM_LB_PREP
        if (e == hipSuccess) ok |= 1 << (v - 6);
        else (void)hipGetLastError();
    }
    return ok;
}

// Launches staged-B variant `variant`; false if it cannot run on this net.
static bool launch_lb(const DevNet &net, int variant, const uint64_t *codes, const int *cell_shape,
                      const CellRange &rg, long long n, double *rows, hipStream_t st) {
    LbShape o;
    if (!((net.lb_ok >> (variant - 6)) & 1) || !lb_shape(net, variant, o)) return false;
#define AM_LB_GO(G_, M_)                                                            \
    (o.f32 ? launch_lb_t<G_, M_, float>(net, codes, cell_shape, rg, n, rows, o, st) \
           : launch_lb_t<G_, M_, double>(net, codes, cell_shape, rg, n, rows, o, st))
    if (o.G == 2)
        o.MTW == 4 ? AM_LB_GO(2, 4) : o.MTW == 2 ? AM_LB_GO(2, 2) : AM_LB_GO(2, 1);
    else
        o.MTW == 4 ? AM_LB_GO(1, 4) : o.MTW == 2 ? AM_LB_GO(1, 2) : AM_LB_GO(1, 1);
#undef AM_LB_GO
    return true;
}

// Positions [0, hi - lo) of cells lo..hi-1, or (list != NULL) the first
// *count entries of list, launched for up to hi - lo positions.
// g: tile variant: 1, 2 or 4 column groups per workgroup (4 g cells); 3: four
// cells with the previous layer's rows in LDS (kept there for layers of at
// most 128 units, staged from global memory per layer for wider ones up to
// 512); 5: four cells with the K loop over the units active in any of them;
// 6, 7, 8: the staged-B chain (4, 8 cells; 4 cells with two tiles per wave),
// or variant 1 where it cannot run.
void launch_chain(const DevNet &net, const uint64_t *codes, const int *cell_shape, long long lo, long long hi,
                  const int *list, const unsigned long long *count, double *rows, int g, hipStream_t st) {
    if (hi <= lo) return;
    const CellRange rg = range_of(lo, hi, list, count, (unsigned long long)(hi - lo));
    const long long n = hi - lo;
    if (g >= 6 && launch_lb(net, g, codes, cell_shape, rg, n, rows, st)) return;
    if (g >= 6) g = 1;
    if (g == 5)
        hipLaunchKernelGGL((k_chain_f64_gather<kKChunk>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, net,
                           codes, cell_shape, rg, rows);
    else if (g == 3 && res_rows(net) > kLdsRows)
        hipLaunchKernelGGL((k_chain_f64_res<kKChunk>), dim3((unsigned)((n + 3) / 4)), dim3(256),
                           chain_res_lds_bytes(net), st, net, codes, cell_shape, rg, rows);
    else if (g == 3)
        hipLaunchKernelGGL((k_chain_f64_lds<kKChunk>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, net, codes,
                           cell_shape, rg, rows);
    else if (g >= 4)
        hipLaunchKernelGGL((k_chain_f64<4, 4>), dim3((unsigned)((n + 15) / 16)), dim3(256), 0, st, net, codes,
                           cell_shape, rg, rows);
    else if (g == 2)
        hipLaunchKernelGGL((k_chain_f64<2, 4>), dim3((unsigned)((n + 7) / 8)), dim3(256), 0, st, net, codes,
                           cell_shape, rg, rows);
    else
        hipLaunchKernelGGL((k_chain_f64<1, kKChunk>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, net, codes,
                           cell_shape, rg, rows);
}

void launch_chain_bf16(const DevNet &net, const uint64_t *codes, const int *cell_shape, long long lo, long long hi,
                       float *rows, hipStream_t st) {
    if (hi <= lo) return;
    const long long tiles = (hi - lo + 3) / 4;
    hipLaunchKernelGGL(k_chain_bf16, dim3((unsigned)tiles), dim3(256), 0, st, net, codes, cell_shape,
                       range_of(lo, hi, nullptr, nullptr, 0), rows);
}

void launch_clip(const DevNet &net, const uint64_t *codes, const int *argmax, const uint64_t *cell_hash,
                 const int *hints, long long lo, long long hi, const int *list, const unsigned long long *count,
                 long long n_seed_cells, const double *rows, const ClipOut &out, const Candidates &cand,
                 unsigned long long cand_cap, Counters *ctr, const PropArgs &pa, hipStream_t st) {
    if (hi <= lo) return;
    const long long blocks = (hi - lo + 3) / 4;
    const Fallback none{nullptr, nullptr, 0, 0.0};
    if (pa.face_routine == 1)
        hipLaunchKernelGGL(k_clip_pivot, dim3((unsigned)blocks), dim3(256), 0, st, net, codes, argmax, cell_hash,
                           hints, range_of(lo, hi, list, count, (unsigned long long)(hi - lo)), n_seed_cells, rows,
                           out, cand, cand_cap, ctr, pa);
    else if (pa.mode != 0 || pa.samples)
        hipLaunchKernelGGL(k_clip_prop<double>, dim3((unsigned)blocks), dim3(256), 0, st, net, codes, argmax,
                           cell_hash, hints, range_of(lo, hi, list, count, (unsigned long long)(hi - lo)),
                           n_seed_cells, rows, out, cand, cand_cap, ctr, 0.0, 0.0, none, pa);
    else
        hipLaunchKernelGGL(k_clip<double>, dim3((unsigned)blocks), dim3(256), 0, st, net, codes, argmax, cell_hash,
                           hints, range_of(lo, hi, list, count, (unsigned long long)(hi - lo)), n_seed_cells, rows,
                           out, cand, cand_cap, ctr, 0.0, 0.0, none, pa);
}

void launch_clip_f32(const DevNet &net, const uint64_t *codes, const int *argmax, const uint64_t *cell_hash,
                     const int *hints, long long lo, long long hi, long long n_seed_cells, const float *rows,
                     const ClipOut &out, const Candidates &cand, unsigned long long cand_cap, Counters *ctr,
                     double margin, double vertex_tol, double row_eps, int *fb_list, unsigned long long *fb_count,
                     const PropArgs &pa, hipStream_t st) {
    if (hi <= lo) return;
    const long long blocks = (hi - lo + 3) / 4;
    const Fallback fb{fb_list, fb_count, (unsigned long long)(hi - lo), row_eps};
    if (pa.mode != 0 || pa.samples)
        hipLaunchKernelGGL(k_clip_prop<float>, dim3((unsigned)blocks), dim3(256), 0, st, net, codes, argmax,
                           cell_hash, hints, range_of(lo, hi, nullptr, nullptr, 0), n_seed_cells, rows, out, cand,
                           cand_cap, ctr, margin, vertex_tol, fb, pa);
    else
        hipLaunchKernelGGL(k_clip<float>, dim3((unsigned)blocks), dim3(256), 0, st, net, codes, argmax, cell_hash,
                           hints, range_of(lo, hi, nullptr, nullptr, 0), n_seed_cells, rows, out, cand, cand_cap,
                           ctr, margin, vertex_tol, fb, pa);
}

void launch_fused(const DevNet &net, const uint64_t *codes, const int *cell_shape, const int *argmax,
                  const uint64_t *cell_hash,
                  const int *hints, long long lo, long long hi, long long n_seed_cells, const ClipOut &out,
                  const Candidates &cand, unsigned long long cand_cap, Counters *ctr, hipStream_t st) {
    if (hi <= lo) return;
    const long long blocks = (hi - lo + 3) / 4;
    hipLaunchKernelGGL(k_march_fused, dim3((unsigned)blocks), dim3(256), fused_lds_bytes(net), st, net, codes,
                       cell_shape, argmax, cell_hash, hints, lo, hi, n_seed_cells, out, cand, cand_cap, ctr);
}

// Persistent march: the chain variant for `net` (0 dense tile; 1, 2 the
// ping-pong staged-B tile with FP64 or FP32 weight fragments, for hidden
// layers of at most 256 units, whose two B buffers (64 KB) still leave two
// or three workgroups per CU; wider, the buffers would leave one, and the
// dense tile is faster), its dynamic LDS, and the workgroups that fit on the
// device at once.
template <int CH>
static hipError_t persist_setup_t(size_t lds, int *blocks) {
    hipError_t e = hipFuncSetAttribute((const void *)k_march_persist<CH>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, per_cu = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_march_persist<CH>, 256, lds);
    if (e != hipSuccess) return e;
    *blocks = (per_cu > 0 ? per_cu : 1) * cus;
    return hipSuccess;
}

hipError_t persist_setup(const DevNet &net, size_t lds_limit, int *variant, size_t *lds, int *blocks) {
    const size_t pp = (size_t)2 * net.lb_kpad * 16 * sizeof(double);
    const size_t stat = sizeof(PolyScratch) * 4 + sizeof(uint64_t) * 4 * kMaxWords + 256;
    if (net.lb_kpad > 0 && net.lb_kpad <= 256 && pp + stat <= lds_limit) {
        *variant = net.wfrag32 ? 2 : 1;
        *lds = pp;
        return *variant == 2 ? persist_setup_t<2>(pp, blocks) : persist_setup_t<1>(pp, blocks);
    }
    *variant = 0;
    *lds = 0;
    return persist_setup_t<0>(0, blocks);
}

void launch_persist(const DevNet &net, int variant, size_t lds, uint64_t *codes, int *cell_shape, int *argmax,
                    uint64_t *cell_hash, int *hints, double *rows_ws, int blocks, long long n_seed_cells,
                    const ClipOut &out, Counters *ctr, const InlineInsert &ins, hipStream_t st) {
    hipLaunchKernelGGL(k_mark_ready, dim3(256), dim3(256), 0, st, ins.ready, ctr, ins.epoch);
#define AM_PERSIST_GO(CH_)                                                                                    \
    hipLaunchKernelGGL(k_march_persist<CH_>, dim3((unsigned)blocks), dim3(256), lds, st, net, codes, cell_shape, \
                       argmax, cell_hash, hints, rows_ws, n_seed_cells, out, ctr, ins)
    if (variant == 2) AM_PERSIST_GO(2);
    else if (variant == 1) AM_PERSIST_GO(1);
    else AM_PERSIST_GO(0);
#undef AM_PERSIST_GO
}

void launch_rows_unpad(const DevNet &net, long long n, const void *rows, bool f32, double *out, hipStream_t st) {
    if (n <= 0) return;
    const long long total = n * (net.N + net.M);
    long long blocks = (total + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    if (f32)
        hipLaunchKernelGGL(k_rows_unpad<float>, dim3((unsigned)blocks), dim3(256), 0, st, net, n,
                           (const float *)rows, out);
    else
        hipLaunchKernelGGL(k_rows_unpad<double>, dim3((unsigned)blocks), dim3(256), 0, st, net, n,
                           (const double *)rows, out);
}

void launch_prop_score(const PropNet &P, const float *X, long long n, float *z, hipStream_t st) {
    const long long blocks = (n + 4 * kWave - 1) / (4 * kWave);
    hipLaunchKernelGGL(k_prop_score, dim3((unsigned)blocks), dim3(256), 0, st, P, X, n, z);
}

// ---- device-driven steps: the step's range lives in the counters, so a fixed
// sequence of steps can be captured in a graph and replayed without the host.

// Opens a step: up to `chunk` cells from step_lo (none after an overflow),
// and clears the candidate count.
// First range of a device-driven march (later ones are taken by the resolve
// kernel that ends each step).
__global__ void k_step_begin(Counters *c, unsigned long long chunk, unsigned long long cap_cells) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
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

void launch_step_begin(Counters *ctr, long long chunk, long long cap_cells, hipStream_t st) {
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(64), 0, st, ctr, (unsigned long long)chunk,
                       (unsigned long long)cap_cells);
}

// Chain (dense variants 1, 2, 3, 4) and clip of the device-driven step; grids
// cover `chunk` cells, workgroups past the step's count exit at once.
void launch_chain_dev(const DevNet &net, const uint64_t *codes, const int *cell_shape, Counters *ctr, long long chunk,
                      double *rows, int g, hipStream_t st) {
    const CellRange rg = range_of(0, chunk, nullptr, nullptr, 0, &ctr->step_lo);
    if (g >= 6 && launch_lb(net, g, codes, cell_shape, rg, chunk, rows, st)) return;
    if (g >= 6) g = 1;
    if (g == 3 && res_rows(net) > kLdsRows)
        hipLaunchKernelGGL((k_chain_f64_res<kKChunk>), dim3((unsigned)((chunk + 3) / 4)), dim3(256),
                           chain_res_lds_bytes(net), st, net, codes, cell_shape, rg, rows);
    else if (g == 3)
        hipLaunchKernelGGL((k_chain_f64_lds<kKChunk>), dim3((unsigned)((chunk + 3) / 4)), dim3(256), 0, st, net,
                           codes, cell_shape, rg, rows);
    else if (g >= 4)
        hipLaunchKernelGGL((k_chain_f64<4, 4>), dim3((unsigned)((chunk + 15) / 16)), dim3(256), 0, st, net, codes,
                           cell_shape, rg, rows);
    else if (g == 2)
        hipLaunchKernelGGL((k_chain_f64<2, 4>), dim3((unsigned)((chunk + 7) / 8)), dim3(256), 0, st, net, codes,
                           cell_shape, rg, rows);
    else
        hipLaunchKernelGGL((k_chain_f64<1, kKChunk>), dim3((unsigned)((chunk + 3) / 4)), dim3(256), 0, st, net,
                           codes, cell_shape, rg, rows);
}

void launch_clip_dev(const DevNet &net, const uint64_t *codes, const int *argmax, const uint64_t *cell_hash,
                     const int *hints, Counters *ctr, long long chunk, long long n_seed_cells, const double *rows,
                     const ClipOut &out, const Candidates &cand, unsigned long long cand_cap, const PropArgs &pa,
                     hipStream_t st) {
    const Fallback none{nullptr, nullptr, 0, 0.0};
    const CellRange rg = range_of(0, chunk, nullptr, nullptr, 0, &ctr->step_lo);
    if (pa.mode != 0)
        hipLaunchKernelGGL(k_clip_prop<double>, dim3((unsigned)((chunk + 3) / 4)), dim3(256), 0, st, net, codes,
                           argmax, cell_hash, hints, rg, n_seed_cells, rows, out, cand, cand_cap, ctr, 0.0, 0.0, none,
                           pa);
    else
        hipLaunchKernelGGL(k_clip<double>, dim3((unsigned)((chunk + 3) / 4)), dim3(256), 0, st, net, codes, argmax,
                           cell_hash, hints, rg, n_seed_cells, rows, out, cand, cand_cap, ctr, 0.0, 0.0, none, pa);
}

// Split-BF16 form of a device-driven step: the BF16 chain and the FP32-row
// clip of the step's range; cells it cannot certify go to fb_list (count in
// ctr->fb_n, cleared when the step's range is taken) and are redone by the
// FP64 chain (variant g) and clip, all sized for `chunk` cells.
void launch_split_step_dev(const DevNet &net, const uint64_t *codes, const int *cell_shape, const int *argmax,
                           const uint64_t *cell_hash, const int *hints, Counters *ctr, long long chunk,
                           long long n_seed_cells, double *rows, const ClipOut &out, const Candidates &cand,
                           unsigned long long cand_cap, double margin, double vertex_tol, double row_eps,
                           int *fb_list, int g, const PropArgs &pa, hipStream_t st) {
    const CellRange rg = range_of(0, chunk, nullptr, nullptr, 0, &ctr->step_lo);
    const unsigned blocks = (unsigned)((chunk + 3) / 4);
    hipLaunchKernelGGL(k_chain_bf16, dim3(blocks), dim3(256), 0, st, net, codes, cell_shape, rg, (float *)rows);
    const Fallback fb{fb_list, &ctr->fb_n, (unsigned long long)chunk, row_eps};
    if (pa.mode != 0)
        hipLaunchKernelGGL(k_clip_prop<float>, dim3(blocks), dim3(256), 0, st, net, codes, argmax, cell_hash, hints, rg,
                           n_seed_cells, (const float *)rows, out, cand, cand_cap, ctr, margin, vertex_tol, fb, pa);
    else
        hipLaunchKernelGGL(k_clip<float>, dim3(blocks), dim3(256), 0, st, net, codes, argmax, cell_hash, hints, rg,
                           n_seed_cells, (const float *)rows, out, cand, cand_cap, ctr, margin, vertex_tol, fb, pa);
    launch_chain(net, codes, cell_shape, 0, chunk, fb_list, &ctr->fb_n, rows, g == 5 ? 1 : g, st);
    launch_clip(net, codes, argmax, cell_hash, hints, 0, chunk, fb_list, &ctr->fb_n, n_seed_cells, rows, out, cand,
                cand_cap, ctr, pa, st);
}

}  // namespace am
