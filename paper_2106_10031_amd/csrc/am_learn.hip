// am_learn.hip -- training kernels of the constraint-proposal scorer.
//
// The scorer (relu(W1 x + b1) -> relu(W2 . + b2) -> w3 . + b3, see
// am_internal.h) is trained on the GPU by minimising the mean binary
// cross-entropy of its logits against labels (1: the line carries an edge of
// the face).  Parameters are kept in FP32 in the flat order
//   W1 [H][D], b1 [H], W2 [H][H], b2 [H], w3 [H], b3
// with H = kPropH, D = kPropD.  The gradient kernel works in FP32: one block of
// 128 threads (thread t = hidden unit t) takes tiles of 32 samples, keeps its
// share of the gradient in registers and writes one partial gradient per
// block; a second kernel sums the partials in FP64.
#include <hip/hip_runtime.h>

#include "am_internal.h"

namespace am {

namespace {

constexpr int H = kPropH;
constexpr int D = kPropD;
constexpr int kTile = 32;
constexpr long long kParams = (long long)H * D + H + (long long)H * H + H + H + 1;
constexpr int kGradBlocks = 1024;

struct Offsets {
    long long W1 = 0, b1 = (long long)H * D, W2 = b1 + H, b2 = W2 + (long long)H * H, w3 = b2 + H, b3 = w3 + H;
};

__device__ __forceinline__ float wave_sum_f(float x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// W2T[k][t] = W2[t][k], so that the forward pass reads it coalesced.
__global__ void k_prop_transpose(const float *__restrict__ params, float *__restrict__ w2t) {
    const Offsets O;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= H * H) return;
    const int t = i / H, k = i % H;
    w2t[k * H + t] = params[O.W2 + i];
}

__global__ __launch_bounds__(128) void k_prop_grad(const float *__restrict__ X, const unsigned char *__restrict__ y,
                                                   long long n, const float *__restrict__ params,
                                                   const float *__restrict__ w2t, float *__restrict__ partial,
                                                   double *__restrict__ partial_loss) {
    const Offsets O;
    const int t = threadIdx.x;          // hidden unit of both layers
    const int wave = t >> 6;
    __shared__ float xs[kTile][D];
    __shared__ float h1s[kTile][H];
    __shared__ float da2s[kTile][H];
    __shared__ float zred[kTile][2];
    __shared__ float dzs[kTile];

    float w1[D], gw1[D], gw2[H];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        w1[k] = params[O.W1 + (long long)t * D + k];
        gw1[k] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < H; ++k) gw2[k] = 0.f;
    const float b1 = params[O.b1 + t], b2 = params[O.b2 + t], w3 = params[O.w3 + t], b3 = params[O.b3];
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f;
    double loss = 0.0;
    const double inv_n = 1.0 / (double)n;

    for (long long s0 = (long long)blockIdx.x * kTile; s0 < n; s0 += (long long)gridDim.x * kTile) {
        const int ns = (int)min((long long)kTile, n - s0);
        for (int i = t; i < kTile * D; i += 128) {
            const int s = i / D, k = i % D;
            xs[s][k] = s < ns ? X[(s0 + s) * D + k] : 0.f;
        }
        __syncthreads();
        unsigned m1 = 0u, m2 = 0u;     // bit s: pre-activation of sample s > 0
        float a2r[kTile];
        for (int s = 0; s < kTile; ++s) {
            float a = b1;
#pragma unroll
            for (int k = 0; k < D; ++k) a += w1[k] * xs[s][k];
            if (a > 0.f) m1 |= 1u << s;
            h1s[s][t] = fmaxf(a, 0.f);
        }
        __syncthreads();
        for (int s = 0; s < kTile; ++s) {
            float a = b2;
            for (int k = 0; k < H; ++k) a += w2t[k * H + t] * h1s[s][k];
            a2r[s] = a;
            if (a > 0.f) m2 |= 1u << s;
            const float v = wave_sum_f(w3 * fmaxf(a, 0.f));
            if ((t & 63) == 0) zred[s][wave] = v;
        }
        __syncthreads();
        if (t < kTile) {
            const int s = t;
            float dz = 0.f;
            if (s < ns) {
                const double z = (double)zred[s][0] + (double)zred[s][1] + (double)b3;
                const double yy = y[s0 + s] ? 1.0 : 0.0;
                loss += fmax(z, 0.0) - z * yy + log1p(exp(-fabs(z)));
                const double sig = 0.5 * (1.0 + tanh(0.5 * z));
                dz = (float)((sig - yy) * inv_n);
            }
            dzs[s] = dz;
        }
        __syncthreads();
        for (int s = 0; s < kTile; ++s) {
            const float dz = dzs[s];
            gw3 += dz * fmaxf(a2r[s], 0.f);
            if (t == 0) gb3 += dz;
            const float d2 = (m2 >> s) & 1u ? dz * w3 : 0.f;
            da2s[s][t] = d2;
            gb2 += d2;
#pragma unroll
            for (int k = 0; k < H; ++k) gw2[k] += d2 * h1s[s][k];
        }
        __syncthreads();
        for (int s = 0; s < kTile; ++s) {
            float dh = 0.f;
            for (int j = 0; j < H; ++j) dh += da2s[s][j] * params[O.W2 + (long long)j * H + t];
            const float d1 = (m1 >> s) & 1u ? dh : 0.f;
            gb1 += d1;
#pragma unroll
            for (int k = 0; k < D; ++k) gw1[k] += d1 * xs[s][k];
        }
        __syncthreads();
    }

    float *P = partial + (long long)blockIdx.x * kParams;
#pragma unroll
    for (int k = 0; k < D; ++k) P[O.W1 + (long long)t * D + k] = gw1[k];
    P[O.b1 + t] = gb1;
#pragma unroll
    for (int k = 0; k < H; ++k) P[O.W2 + (long long)t * H + k] = gw2[k];
    P[O.b2 + t] = gb2;
    P[O.w3 + t] = gw3;
    if (t == 0) P[O.b3] = gb3;
    // loss: threads 0..31 hold sample sums
    __shared__ double lred[128];
    lred[t] = loss;
    __syncthreads();
    if (t == 0) {
        double sum = 0.0;
        for (int i = 0; i < kTile; ++i) sum += lred[i];
        partial_loss[blockIdx.x] = sum;
    }
}

__global__ void k_prop_reduce(const float *__restrict__ partial, int nblk, float *__restrict__ grad) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(long long)b * kParams + p];
    grad[p] = (float)s;
}

// omb1, omb2 = 1 - beta (formed in FP64 on the host: 1.f - 0.999f is off by 1.3e-5)
__global__ void k_prop_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, long long n, float lr, float beta1, float beta2, float omb1,
                            float omb2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + omb1 * gi;
    const float vi = beta2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

long long prop_param_count() { return kParams; }
int prop_grad_blocks() { return kGradBlocks; }

// scratch: [kGradBlocks * kParams] floats partials + [H*H] floats W2T;
// loss_scratch: [kGradBlocks] doubles.
void launch_prop_grad(const float *X, const unsigned char *y, long long n, const float *params, float *grad,
                      float *scratch, double *loss_scratch, hipStream_t st) {
    float *w2t = scratch + (long long)kGradBlocks * kParams;
    hipLaunchKernelGGL(k_prop_transpose, dim3((H * H + 255) / 256), dim3(256), 0, st, params, w2t);
    hipLaunchKernelGGL(k_prop_grad, dim3(kGradBlocks), dim3(128), 0, st, X, y, n, params, w2t, scratch,
                       loss_scratch);
    hipLaunchKernelGGL(k_prop_reduce, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, st, scratch,
                       kGradBlocks, grad);
}

void launch_prop_adam(float *p, const float *g, float *m, float *v, int step, float lr, hipStream_t st) {
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - pow(b1, step)), c2 = (float)(1.0 - pow(b2, step));
    hipLaunchKernelGGL(k_prop_adam, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, st, p, g, m, v, kParams,
                       lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
}

}  // namespace am
