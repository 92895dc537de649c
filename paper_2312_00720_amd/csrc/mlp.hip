// The selector network: 12 features -> 64 -> 64 (ReLU) -> 7 logits, softmax
// over the classes valid for each sample, cross-entropy loss, gradients and Adam.
// FP32. Parameters are one flat vector: W1 (64x12, row-major), b1, W2 (64x64),
// b2, W3 (7x64), b3 — 5447 floats.
//
// Every matrix product is small (batch x 64 x 64 at most), so each output element
// is one thread summing its terms in a fixed order: gradients are bit-identical
// from run to run.
#include <math.h>

#include "internal.hpp"

namespace gj {
namespace {

constexpr int F = 12, H = 64, C = 7;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * F, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + C * H, N_PARAMS = OFF_B3 + C;
static_assert(N_PARAMS == GJ_MLP_PARAMS, "parameter count");

// out[m, n] = sum_k A[m*am + k*ak] * B[k*bk + n*bn] (+ bias[n]) (then ReLU if relu),
// k summed in increasing order.
__global__ void k_mm(int M, int N, int K, const float *__restrict__ A, int am, int ak, const float *__restrict__ B,
                     int bk, int bn, const float *__restrict__ bias, int relu, float *__restrict__ out) {
    const int64_t total = (int64_t)M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(e / N), n = (int)(e % N);
        float acc = 0.f;
        for (int k = 0; k < K; ++k) acc = fmaf(A[(int64_t)m * am + (int64_t)k * ak], B[(int64_t)k * bk + (int64_t)n * bn], acc);
        if (bias) acc += bias[n];
        if (relu) acc = fmaxf(acc, 0.f);
        out[e] = acc;
    }
}

// Masked softmax and cross-entropy per sample: probabilities P, dL/dlogits D (of
// the batch-mean loss) and the per-sample loss.
__global__ void k_softmax_xent(int B, const float *__restrict__ Z, const float *__restrict__ mask,
                               const int32_t *__restrict__ y, float *__restrict__ P, float *__restrict__ D,
                               float *__restrict__ loss) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        float mx = -INFINITY;
        for (int c = 0; c < C; ++c)
            if (mask[b * C + c] > 0.f) mx = fmaxf(mx, Z[b * C + c]);
        float e[C], sum = 0.f;
        for (int c = 0; c < C; ++c) {
            e[c] = mask[b * C + c] > 0.f ? expf(Z[b * C + c] - mx) : 0.f;
            sum += e[c];
        }
        for (int c = 0; c < C; ++c) {
            const float p = e[c] / sum;
            P[b * C + c] = p;
            if (D) D[b * C + c] = (p - (y && c == y[b] ? 1.f : 0.f)) / (float)B;
        }
        if (loss && y) loss[b] = -logf(P[b * C + y[b]]);
    }
}

// D[i] *= (Z[i] > 0)
__global__ void k_relu_grad(int64_t n, float *__restrict__ D, const float *__restrict__ Z) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!(Z[i] > 0.f)) D[i] = 0.f;
}

// out[n] = sum over rows of D[:, n], rows summed in order.
__global__ void k_colsum(int rows, int cols, const float *__restrict__ D, float *__restrict__ out) {
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < cols; n += gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int r = 0; r < rows; ++r) acc += D[(int64_t)r * cols + n];
        out[n] = acc;
    }
}

__global__ void k_mean(int n, const float *__restrict__ x, float *__restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float acc = 0.f;
        for (int i = 0; i < n; ++i) acc += x[i];
        *out = acc / (float)n;
    }
}

__global__ void k_adam(int n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

uint32_t grid_for(int64_t n) { return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

void mm(hipStream_t s, int M, int N, int K, const float *A, int am, int ak, const float *B, int bk, int bn,
        const float *bias, int relu, float *out) {
    GJ_LAUNCH("k_mlp_mm", 4.0 * ((double)M * K + (double)K * N + (double)M * N), k_mm, dim3(grid_for((int64_t)M * N)),
              dim3(256), 0, s, M, N, K, A, am, ak, B, bk, bn, bias, relu, out);
}

struct Acts {
    float *z1, *z2, *z3, *p;
};

// z1 = relu-less pre-activations are kept so that the backward pass can mask.
void forward(hipStream_t s, const float *theta, const float *X, int B, Acts &a, float *h1, float *h2) {
    mm(s, B, H, F, X, F, 1, theta + OFF_W1, 1, F, theta + OFF_B1, 0, a.z1);
    mm(s, B, H, F, X, F, 1, theta + OFF_W1, 1, F, theta + OFF_B1, 1, h1);
    mm(s, B, H, H, h1, H, 1, theta + OFF_W2, 1, H, theta + OFF_B2, 0, a.z2);
    mm(s, B, H, H, h1, H, 1, theta + OFF_W2, 1, H, theta + OFF_B2, 1, h2);
    mm(s, B, C, H, h2, H, 1, theta + OFF_W3, 1, H, theta + OFF_B3, 0, a.z3);
}

}  // namespace
}  // namespace gj

extern "C" {

int gj_mlp_forward(const float *params, const float *X, const float *mask, int32_t batch, float *probs,
                   const gj_allocator *alloc, void *stream) {
    try {
        gj::require(params && X && mask && probs && batch >= 0, "bad argument");
        if (batch == 0) return GJ_OK;
        gj::Ctx ctx(alloc, (hipStream_t)stream);
        hipStream_t s = (hipStream_t)stream;
        const int B = batch;
        gj::Acts a{ctx.scratch_n<float>((size_t)B * gj::H), ctx.scratch_n<float>((size_t)B * gj::H),
                   ctx.scratch_n<float>((size_t)B * gj::C), probs};
        float *h1 = ctx.scratch_n<float>((size_t)B * gj::H), *h2 = ctx.scratch_n<float>((size_t)B * gj::H);
        gj::forward(s, params, X, B, a, h1, h2);
        GJ_LAUNCH("k_softmax_xent", 44.0 * B, gj::k_softmax_xent, dim3(gj::grid_for(B)), dim3(256), 0, s, B, a.z3,
                  mask, (const int32_t *)nullptr, probs, (float *)nullptr, (float *)nullptr);
        return GJ_OK;
    } catch (const gj::Error &e) {
        return e.code;
    } catch (...) {
        return GJ_EHIP;
    }
}

int gj_mlp_grad(const float *params, const float *X, const float *mask, const int32_t *labels, int32_t batch,
                float *grad, float *loss, const gj_allocator *alloc, void *stream) {
    try {
        gj::require(params && X && mask && labels && grad && batch > 0, "bad argument");
        gj::Ctx ctx(alloc, (hipStream_t)stream);
        hipStream_t s = (hipStream_t)stream;
        using namespace gj;
        const int B = batch;
        Acts a{ctx.scratch_n<float>((size_t)B * H), ctx.scratch_n<float>((size_t)B * H),
               ctx.scratch_n<float>((size_t)B * C), ctx.scratch_n<float>((size_t)B * C)};
        float *h1 = ctx.scratch_n<float>((size_t)B * H), *h2 = ctx.scratch_n<float>((size_t)B * H);
        float *d3 = ctx.scratch_n<float>((size_t)B * C), *d2 = ctx.scratch_n<float>((size_t)B * H),
              *d1 = ctx.scratch_n<float>((size_t)B * H), *lb = ctx.scratch_n<float>((size_t)B);
        forward(s, params, X, B, a, h1, h2);
        GJ_LAUNCH("k_softmax_xent", 48.0 * B, k_softmax_xent, dim3(grid_for(B)), dim3(256), 0, s, B, a.z3, mask,
                  labels, a.p, d3, lb);
        // gW3 = d3^T h2, gb3 = colsum d3
        mm(s, C, H, B, d3, 1, C, h2, H, 1, nullptr, 0, grad + OFF_W3);
        GJ_LAUNCH("k_colsum", 4.0 * B * C, k_colsum, dim3(1), dim3(256), 0, s, B, C, d3, grad + OFF_B3);
        // d2 = (d3 W3) * (z2 > 0)
        mm(s, B, H, C, d3, C, 1, params + OFF_W3, H, 1, nullptr, 0, d2);
        GJ_LAUNCH("k_relu_grad", 8.0 * B * H, k_relu_grad, dim3(grid_for((int64_t)B * H)), dim3(256), 0, s,
                  (int64_t)B * H, d2, a.z2);
        mm(s, H, H, B, d2, 1, H, h1, H, 1, nullptr, 0, grad + OFF_W2);
        GJ_LAUNCH("k_colsum", 4.0 * B * H, k_colsum, dim3(1), dim3(256), 0, s, B, H, d2, grad + OFF_B2);
        // d1 = (d2 W2) * (z1 > 0)
        mm(s, B, H, H, d2, H, 1, params + OFF_W2, H, 1, nullptr, 0, d1);
        GJ_LAUNCH("k_relu_grad", 8.0 * B * H, k_relu_grad, dim3(grid_for((int64_t)B * H)), dim3(256), 0, s,
                  (int64_t)B * H, d1, a.z1);
        mm(s, H, F, B, d1, 1, H, X, F, 1, nullptr, 0, grad + OFF_W1);
        GJ_LAUNCH("k_colsum", 4.0 * B * H, k_colsum, dim3(1), dim3(256), 0, s, B, H, d1, grad + OFF_B1);
        if (loss) GJ_LAUNCH("k_mean", 4.0 * B, k_mean, dim3(1), dim3(64), 0, s, B, lb, loss);
        return GJ_OK;
    } catch (const gj::Error &e) {
        return e.code;
    } catch (...) {
        return GJ_EHIP;
    }
}

int gj_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t t, float lr, float beta1, float beta2,
                float eps, void *stream) {
    try {
        gj::require(params && grad && m && v && t >= 1, "bad argument");
        const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
        hipStream_t s = (hipStream_t)stream;
        GJ_LAUNCH("k_adam", 20.0 * gj::N_PARAMS, gj::k_adam, dim3(gj::grid_for(gj::N_PARAMS)), dim3(256), 0, s,
                  gj::N_PARAMS, params, grad, m, v, lr, beta1, beta2, eps, c1, c2);
        return GJ_OK;
    } catch (const gj::Error &e) {
        return e.code;
    } catch (...) {
        return GJ_EHIP;
    }
}

}  // extern "C"
