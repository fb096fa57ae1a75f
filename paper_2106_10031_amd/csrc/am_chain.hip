// am_chain.hip -- the per-cell affine chain on FP64 matrix cores (gfx950).
//
// For a cell with activation code s, Lemma 1 and Corollary 1 of the paper give
// every pre-activation as an affine function of x inside the cell.  With the
// bias carried by the homogeneous coordinate, the rows Z_l (n_l x 4) obey
//     Z_0 = [I_3 | 0],
//     Z_l = sum over blocks (l <- j) of W_{l<-j} diag(s_j) Z_j  +  b_l e_4^T,
// where diag(s_0) = I (the input is never rectified); shortcut blocks of
// Sec. 5.1 and the max-pooled heads of Sec. 5.2 are ordinary blocks.
//
// Batched over cells this is a dense GEMM per layer: W (n_l x n_j) times the
// stacked masked rows [diag(s^(c)) Z_j^(c)]_c (n_j x 4C).  A workgroup of four
// waves owns four cells = 16 columns, the N size of v_mfma_f64_16x16x4f64;
// wave w computes the 16-row output tiles w, w+4, ...  The mask diag(s_j) is
// applied while loading the B operand.  Every layer is written to the rows
// buffer (the clip reads it); the next layer reads it back through L1/L2.
#include "am_internal.h"

namespace am {

typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_chain_f64(DevNet net, const uint64_t *__restrict__ codes,
                                                   long long lo, long long hi,
                                                   double *__restrict__ rows) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const long long c0 = lo + 4LL * blockIdx.x;
    const int col = lane & 15;       // MFMA column (B, D) / row within the tile (A)
    const int kq = lane >> 4;        // k within the K-step of 4 (A, B) / row offset (D)
    const int q = col & 3;           // homogeneous component of this column
    const long long cell = c0 + (col >> 2);
    const bool cell_ok = cell < hi;
    const long long cidx = cell_ok ? cell : c0;
    const uint64_t *code = codes + cidx * net.W;
    double *crow = rows + (cidx - lo) * (long long)net.R * 4;

    for (int l = 1; l < net.n_layers; ++l) {
        const int nl = net.width[l];
        const int mtiles = (nl + 15) >> 4;
        for (int mt = wave; mt < mtiles; mt += 4) {
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            for (int b = 0; b < net.n_blocks; ++b) {
                if (net.blk_dst[b] != l) continue;
                const int j = net.blk_src[b];
                const int ld = net.blk_ld[b];
                const int nj = net.width[j];
                const double *Wrow = net.weights + net.blk_off[b] + (long long)(mt * 16 + col) * ld;
                if (j == 0) {
                    // Z_0 = [I | 0]: one K-step (ld == 4); row k of B is e_k for k < 3.
                    const double a = Wrow[kq];
                    const double bv = (kq < 3 && kq == q) ? 1.0 : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
                    continue;
                }
                const int uoff = net.unit_off[j];
                const double *zj = crow + (long long)net.row_off[j] * 4 + q;
                for (int k0 = 0; k0 < ld; k0 += 4) {
                    const int k = k0 + kq;
                    const double a = Wrow[k];
                    double bv = 0.0;
                    if (k < nj && cell_ok && code_bit(code, uoff + k)) bv = zj[k * 4];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
                }
            }
            if (cell_ok) {
                const double *bias = net.bias + net.bias_off[l];
                double *zl = crow + (long long)net.row_off[l] * 4 + q;
                // v_mfma_f64_16x16x4f64 leaves D[kq + 4 r][col] in register r of
                // lane (kq * 16 + col)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = mt * 16 + kq + 4 * r;
                    if (i < nl) zl[i * 4] = acc[r] + (q == 3 ? bias[i] : 0.0);
                }
            }
        }
        __syncthreads();
    }
}

// Repacks padded per-cell rows into the dense [n][N+M][4] layout of am_chain.
__global__ void k_rows_unpad(DevNet net, long long n, const double *__restrict__ rows,
                             double *__restrict__ out) {
    const int G = net.N + net.M;
    const long long total = n * G;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const long long c = t / G;
        const int g = (int)(t % G);
        const double *src = rows + (c * net.R + net.row_of_unit[g]) * 4;
        double *dst = out + t * 4;
        dst[0] = src[0];
        dst[1] = src[1];
        dst[2] = src[2];
        dst[3] = src[3];
    }
}

void launch_chain(const DevNet &net, const uint64_t *codes, long long lo, long long hi, double *rows,
                  hipStream_t st) {
    if (hi <= lo) return;
    const long long tiles = (hi - lo + 3) / 4;
    hipLaunchKernelGGL(k_chain_f64, dim3((unsigned)tiles), dim3(256), 0, st, net, codes, lo, hi, rows);
}

void launch_rows_unpad(const DevNet &net, long long n, const double *rows, double *out, hipStream_t st) {
    if (n <= 0) return;
    const long long total = n * (net.N + net.M);
    long long blocks = (total + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_rows_unpad, dim3((unsigned)blocks), dim3(256), 0, st, net, n, rows, out);
}

}  // namespace am
