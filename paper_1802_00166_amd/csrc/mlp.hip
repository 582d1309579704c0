// The cost model's multilayer perceptron, 8 -> 64 ReLU -> 64 ReLU -> 1, in
// binary32: inference, loss gradient, and training with Adam (Kingma and Ba,
// 2015), all on the device.
//
// Parameters are one flat array of MLP_NP floats: W1 [64][8], b1 [64],
// W2 [64][64], b2 [64], W3 [64], b3 (row-major, output index first).  The
// loss is the mean squared error over a batch.  Every sum runs in a fixed
// order, so results do not depend on scheduling.
//
// Training is one launch of one block: the batch (at most 256 samples, one
// per thread) is small enough that a single CU finishes all epochs in well
// under a second, and one block needs no grid-wide synchronisation between
// the forward pass, the gradient reduction and the update.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace pcot {

namespace {

constexpr int NI = 8, NH = 64;
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NH;
constexpr int NP = OB3 + 1;  // 4801
constexpr int BT = 256;      // threads per block = largest batch
constexpr int PPT = (NP + BT - 1) / BT;  // parameters per thread in the update

static_assert(NP == MLP_NP, "parameter count");

// Per-batch activations in global scratch, [sample][unit].
struct Act {
    float* h1;  // relu(z1)
    float* h2;  // relu(z2)
    float* g1;  // dL/dz1
    float* g2;  // dL/dz2
    float* gy;  // dL/dyhat
};

// Forward of one sample; returns yhat.  h1/h2 are written when `act` rows are given.
__device__ float forward1(const float* P, const float* x, float* h1row, float* h2row, float h1[NH]) {
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < NI; ++k) s += P[OW1 + i * NI + k] * x[k];
        h1[i] = fmaxf(s + P[OB1 + i], 0.f);
        if (h1row) h1row[i] = h1[i];
    }
    float yh = 0.f;
    for (int o = 0; o < NH; ++o) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < NH; ++i) s += P[OW2 + o * NH + i] * h1[i];
        const float h2 = fmaxf(s + P[OB2 + o], 0.f);
        if (h2row) h2row[o] = h2;
        yh += P[OW3 + o] * h2;
    }
    return yh + P[OB3];
}

// Forward and per-sample backward of sample `b` of a batch of `nb` (thread b).
__device__ float sample_pass(const float* P, const float* x, float y, int b, int nb, const Act& a) {
    float h1[NH];
    const float yh = forward1(P, x, a.h1 + b * NH, a.h2 + b * NH, h1);
    const float r = yh - y;
    const float gy = 2.f * r / (float)nb;
    a.gy[b] = gy;
    float g2[NH];
#pragma unroll
    for (int o = 0; o < NH; ++o) {
        g2[o] = a.h2[b * NH + o] > 0.f ? gy * P[OW3 + o] : 0.f;
        a.g2[b * NH + o] = g2[o];
    }
#pragma unroll 4
    for (int i = 0; i < NH; ++i) {
        float s = 0.f;
#pragma unroll
        for (int o = 0; o < NH; ++o) s += g2[o] * P[OW2 + o * NH + i];
        a.g1[b * NH + i] = h1[i] > 0.f ? s : 0.f;
    }
    return r * r;
}

// Gradient of parameter p over the batch (samples in order 0..nb-1).
__device__ float param_grad(int p, int nb, const Act& a, const float* X, const int* rows) {
    float g = 0.f;
    if (p < OB1) {
        const int i = p / NI, k = p % NI;
        for (int b = 0; b < nb; ++b) g += a.g1[b * NH + i] * X[rows[b] * NI + k];
    } else if (p < OW2) {
        const int i = p - OB1;
        for (int b = 0; b < nb; ++b) g += a.g1[b * NH + i];
    } else if (p < OB2) {
        const int o = (p - OW2) / NH, i = (p - OW2) % NH;
        for (int b = 0; b < nb; ++b) g += a.g2[b * NH + o] * a.h1[b * NH + i];
    } else if (p < OW3) {
        const int o = p - OB2;
        for (int b = 0; b < nb; ++b) g += a.g2[b * NH + o];
    } else if (p < OB3) {
        const int o = p - OW3;
        for (int b = 0; b < nb; ++b) g += a.gy[b] * a.h2[b * NH + o];
    } else {
        for (int b = 0; b < nb; ++b) g += a.gy[b];
    }
    return g;
}

// Sum over the block in a fixed tree; every thread gets the result.
__device__ float block_sum(float v, float* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = BT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const float r = sh[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(BT) k_mlp_forward(const float* __restrict__ params, const float* __restrict__ X,
                                                    int n, float* __restrict__ yhat) {
    __shared__ float P[NP];
    for (int p = threadIdx.x; p < NP; p += BT) P[p] = params[p];
    __syncthreads();
    const int b = blockIdx.x * BT + threadIdx.x;
    if (b >= n) return;
    float x[NI], h1[NH];
#pragma unroll
    for (int k = 0; k < NI; ++k) x[k] = X[b * NI + k];
    yhat[b] = forward1(P, x, nullptr, nullptr, h1);
}

// One batch (rows 0..n-1 of X): loss and gradient, no update.
__global__ void __launch_bounds__(BT) k_mlp_grad(const float* __restrict__ params, const float* __restrict__ X,
                                                 const float* __restrict__ y, const int* __restrict__ rows, int n,
                                                 Act a, float* __restrict__ grad, float* __restrict__ loss) {
    __shared__ float P[NP];
    __shared__ float sh[BT];
    for (int p = threadIdx.x; p < NP; p += BT) P[p] = params[p];
    __syncthreads();
    const int b = threadIdx.x;
    float l = 0.f;
    if (b < n) {
        float x[NI];
#pragma unroll
        for (int k = 0; k < NI; ++k) x[k] = X[rows[b] * NI + k];
        l = sample_pass(P, x, y[rows[b]], b, n, a);
    }
    __threadfence_block();
    const float tot = block_sum(l, sh);
    for (int p = threadIdx.x; p < NP; p += BT) grad[p] = param_grad(p, n, a, X, rows);
    if (threadIdx.x == 0) *loss = tot / (float)n;
}

// Adam training over `epochs` passes; `order` holds a permutation of 0..n-1
// per epoch (epochs x n), cut into batches of `bsz` in that order.  m, v and
// the step count continue from their inputs.  loss_out[e] = mean squared error
// over epoch e's batches (before each batch's update).
__global__ void __launch_bounds__(BT) k_mlp_train(float* __restrict__ params, float* __restrict__ mom,
                                                  float* __restrict__ vel, const float* __restrict__ X,
                                                  const float* __restrict__ y, const int* __restrict__ order, int n,
                                                  int epochs, int bsz, int step0, float lr, float beta1, float beta2,
                                                  float eps, Act a, float* __restrict__ loss_out) {
    __shared__ float P[NP];
    __shared__ float sh[BT];
    for (int p = threadIdx.x; p < NP; p += BT) P[p] = params[p];
    float m[PPT], v[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int p = threadIdx.x + j * BT;
        m[j] = p < NP ? mom[p] : 0.f;
        v[j] = p < NP ? vel[p] : 0.f;
    }
    __syncthreads();
    int step = step0;
    float b1t = 1.f, b2t = 1.f;  // beta^step, kept as running products
    for (int s = 0; s < step0; ++s) { b1t *= beta1; b2t *= beta2; }
    for (int e = 0; e < epochs; ++e) {
        const int* ord = order + (size_t)e * n;
        float esum = 0.f;
        for (int b0 = 0; b0 < n; b0 += bsz) {
            const int nb = min(bsz, n - b0);
            const int* rows = ord + b0;
            float l = 0.f;
            if ((int)threadIdx.x < nb) {
                float x[NI];
                const int r = rows[threadIdx.x];
#pragma unroll
                for (int k = 0; k < NI; ++k) x[k] = X[r * NI + k];
                l = sample_pass(P, x, y[r], threadIdx.x, nb, a);
            }
            __threadfence_block();
            esum += block_sum(l, sh);  // also orders the activation writes
            ++step;
            b1t *= beta1;
            b2t *= beta2;
            const float c1 = 1.f - b1t, c2 = 1.f - b2t;
            float g[PPT];
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int p = threadIdx.x + j * BT;
                g[j] = p < NP ? param_grad(p, nb, a, X, rows) : 0.f;
            }
            __syncthreads();  // every gradient read P before any update
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int p = threadIdx.x + j * BT;
                if (p < NP) {
                    m[j] = beta1 * m[j] + (1.f - beta1) * g[j];
                    v[j] = beta2 * v[j] + (1.f - beta2) * g[j] * g[j];
                    const float mh = m[j] / c1, vh = v[j] / c2;
                    P[p] = P[p] - lr * mh / (sqrtf(vh) + eps);
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) loss_out[e] = esum / (float)n;
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int p = threadIdx.x + j * BT;
        if (p < NP) {
            params[p] = P[p];
            mom[p] = m[j];
            vel[p] = v[j];
        }
    }
}

}  // namespace

size_t mlp_scratch_floats() { return (size_t)4 * BT * NH + BT; }

hipError_t launch_mlp_forward(const float* params, const float* X, int n, float* yhat, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + BT - 1) / BT), dim3(BT), 0, s, params, X, n, yhat);
    return hipGetLastError();
}

static Act act_of(float* scratch) {
    Act a;
    a.h1 = scratch;
    a.h2 = a.h1 + BT * NH;
    a.g1 = a.h2 + BT * NH;
    a.g2 = a.g1 + BT * NH;
    a.gy = a.g2 + BT * NH;
    return a;
}

hipError_t launch_mlp_grad(const float* params, const float* X, const float* y, const int* rows, int n,
                           float* scratch, float* grad, float* loss, hipStream_t s) {
    if (n <= 0 || n > BT) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(BT), 0, s, params, X, y, rows, n, act_of(scratch), grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_train(float* params, float* m, float* v, const float* X, const float* y, const int* order,
                            int n, int epochs, int bsz, int step0, float lr, float beta1, float beta2, float eps,
                            float* scratch, float* loss_out, hipStream_t s) {
    if (n <= 0 || bsz <= 0 || bsz > BT) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(BT), 0, s, params, m, v, X, y, order, n, epochs, bsz, step0, lr,
                       beta1, beta2, eps, act_of(scratch), loss_out);
    return hipGetLastError();
}

}  // namespace pcot
