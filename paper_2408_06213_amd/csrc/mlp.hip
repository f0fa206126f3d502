// Learned plan-cost model: a small multilayer perceptron that predicts the
// log-time of a batch under a candidate schedule and size-class mapping,
// from plan features. The autotuner ranks candidates with it and times only
// the best few; it never touches a random word, a roll or a swap, so every
// choice it makes stays exactly uniform.
//
// Network: y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3, inputs n_in,
// two hidden layers of `hidden`, one output, FP32. Training minimizes the
// mean squared error with Adam. Forward, backward and update are the kernels
// below (VALU; the layers are far too small for matrix cores to matter).
// Reductions over the batch run in a fixed order, so results are
// reproducible run to run.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "brr.h"
#include "internal.hpp"

using namespace brr;

namespace {

// Z[b, o] = sum_i X[b, i] W[i, o] + c[o]; A = tanh(Z) when act.
__global__ void k_fwd(const float *X, const float *W, const float *c, float *A, uint32_t B,
                      uint32_t I, uint32_t O, int act)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * O) return;
    const uint32_t b = t / O, o = t % O;
    float z = c[o];
    for (uint32_t i = 0; i < I; ++i) z += X[b * I + i] * W[i * O + o];
    A[t] = act ? tanhf(z) : z;
}

// dW[i, o] = sum_b X[b, i] dZ[b, o]; row i = I holds dc[o] = sum_b dZ[b, o].
__global__ void k_bwd_w(const float *X, const float *dZ, float *dW, float *dc, uint32_t B,
                        uint32_t I, uint32_t O)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (I + 1) * O) return;
    const uint32_t i = t / O, o = t % O;
    float s = 0;
    if (i < I)
        for (uint32_t b = 0; b < B; ++b) s += X[b * I + i] * dZ[b * O + o];
    else
        for (uint32_t b = 0; b < B; ++b) s += dZ[b * O + o];
    if (i < I)
        dW[i * O + o] = s;
    else
        dc[o] = s;
}

// dZp[b, i] = (sum_o dZ[b, o] W[i, o]) * (1 - A[b, i]^2): the gradient at the
// previous layer's pre-activation through tanh.
__global__ void k_bwd_x(const float *dZ, const float *W, const float *A, float *dZp, uint32_t B,
                        uint32_t I, uint32_t O)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * I) return;
    const uint32_t b = t / I, i = t % I;
    float s = 0;
    for (uint32_t o = 0; o < O; ++o) s += dZ[b * O + o] * W[i * O + o];
    const float a = A[t];
    dZp[t] = s * (1.0f - a * a);
}

// dY = 2 (Y - T) / B; loss = mean (Y - T)^2 (one thread, fixed order).
__global__ void k_mse(const float *Y, const float *T, float *dY, float *loss, uint32_t B)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < B) dY[t] = 2.0f * (Y[t] - T[t]) / (float)B;
    if (t == 0 && loss) {
        float s = 0;
        for (uint32_t b = 0; b < B; ++b) s += (Y[b] - T[b]) * (Y[b] - T[b]);
        *loss = s / (float)B;
    }
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, uint32_t n, float lr,
                       float c1, float c2)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    m[t] = beta1 * m[t] + (1 - beta1) * g[t];
    v[t] = beta2 * v[t] + (1 - beta2) * g[t] * g[t];
    p[t] -= lr * (m[t] / c1) / (sqrtf(v[t] / c2) + eps);
}

uint32_t blocks(uint64_t n) { return (uint32_t)((n + 255) / 256); }

} // namespace

struct brr_mlp {
    uint32_t n_in, hidden;
    uint64_t nparams;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr; // parameters, gradients, Adam
    uint32_t cap = 0; // batch capacity of the activation buffers
    float *a1 = nullptr, *a2 = nullptr, *y = nullptr, *dy = nullptr, *d2 = nullptr, *d1 = nullptr;
    uint64_t t = 0;   // Adam steps
    // views into p/g: W1 [n_in x h], b1 [h], W2 [h x h], b2 [h], W3 [h x 1], b3 [1]
    float *W1(float *base) const { return base; }
    float *b1(float *base) const { return base + (uint64_t)n_in * hidden; }
    float *W2(float *base) const { return b1(base) + hidden; }
    float *b2(float *base) const { return W2(base) + (uint64_t)hidden * hidden; }
    float *W3(float *base) const { return b2(base) + hidden; }
    float *b3(float *base) const { return W3(base) + hidden; }
};

namespace {

brr_status ensure_cap(brr_mlp *net, uint32_t B)
{
    if (B <= net->cap) return BRR_OK;
    for (float **buf : {&net->a1, &net->a2, &net->y, &net->dy, &net->d2, &net->d1})
        if (*buf) (void)hipFree(*buf), *buf = nullptr;
    const uint64_t h = net->hidden;
    if (hipMalloc(reinterpret_cast<void **>(&net->a1), B * h * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&net->a2), B * h * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&net->d2), B * h * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&net->d1), B * h * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&net->y), B * 4ull) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&net->dy), B * 4ull) != hipSuccess)
        return BRR_ENOMEM;
    net->cap = B;
    return BRR_OK;
}

hipError_t forward(brr_mlp *net, const float *x, uint32_t B, hipStream_t s)
{
    const uint32_t I = net->n_in, H = net->hidden;
    float *p = net->p;
    k_fwd<<<blocks((uint64_t)B * H), 256, 0, s>>>(x, net->W1(p), net->b1(p), net->a1, B, I, H, 1);
    k_fwd<<<blocks((uint64_t)B * H), 256, 0, s>>>(net->a1, net->W2(p), net->b2(p), net->a2, B, H, H,
                                                1);
    k_fwd<<<blocks(B), 256, 0, s>>>(net->a2, net->W3(p), net->b3(p), net->y, B, H, 1, 0);
    return hipGetLastError();
}

// SplitMix64 (Steele, Lea, Flood 2014) for the initial weights.
uint64_t splitmix(uint64_t &x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

} // namespace

extern "C" {

brr_status brr_mlp_create(brr_mlp **out, uint32_t n_in, uint32_t hidden, uint64_t seed)
{
    if (!out || n_in == 0 || n_in > 256 || hidden == 0 || hidden > 256) return BRR_EINVAL;
    *out = nullptr;
    brr_status st = ensure_device();
    if (st != BRR_OK) return st;
    brr_mlp *net = new (std::nothrow) brr_mlp();
    if (!net) return BRR_ENOMEM;
    net->n_in = n_in;
    net->hidden = hidden;
    net->nparams = (uint64_t)n_in * hidden + hidden + (uint64_t)hidden * hidden + hidden + hidden + 1;
    const uint64_t bytes = net->nparams * 4;
    for (float **buf : {&net->p, &net->g, &net->m, &net->v})
        if (hipMalloc(reinterpret_cast<void **>(buf), bytes) != hipSuccess) {
            brr_mlp_destroy(net);
            return BRR_ENOMEM;
        }
    // Glorot-uniform weights, zero biases
    std::vector<float> h(net->nparams, 0.0f);
    uint64_t x = seed;
    auto fill = [&](float *dst, uint32_t fan_in, uint32_t fan_out) {
        const double lim = std::sqrt(6.0 / (fan_in + fan_out));
        for (uint64_t k = 0; k < (uint64_t)fan_in * fan_out; ++k)
            dst[k] = (float)((splitmix(x) >> 11) * 0x1.0p-53 * 2 * lim - lim);
    };
    fill(net->W1(h.data()), n_in, hidden);
    fill(net->W2(h.data()), hidden, hidden);
    fill(net->W3(h.data()), hidden, 1);
    if (hipMemcpy(net->p, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(net->m, 0, bytes) != hipSuccess || hipMemset(net->v, 0, bytes) != hipSuccess ||
        hipMemset(net->g, 0, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        brr_mlp_destroy(net);
        return BRR_EHIP;
    }
    *out = net;
    return BRR_OK;
}

void brr_mlp_destroy(brr_mlp *net)
{
    if (!net) return;
    for (float *buf : {net->p, net->g, net->m, net->v, net->a1, net->a2, net->y, net->dy, net->d2,
                       net->d1})
        if (buf) (void)hipFree(buf);
    delete net;
}

uint64_t brr_mlp_num_params(const brr_mlp *net) { return net ? net->nparams : 0; }

brr_status brr_mlp_get_params(const brr_mlp *net, float *h_out)
{
    if (!net || !h_out) return BRR_EINVAL;
    return hipMemcpy(h_out, net->p, net->nparams * 4, hipMemcpyDeviceToHost) == hipSuccess ? BRR_OK
                                                                                          : BRR_EHIP;
}

brr_status brr_mlp_set_params(brr_mlp *net, const float *h_in)
{
    if (!net || !h_in) return BRR_EINVAL;
    return hipMemcpy(net->p, h_in, net->nparams * 4, hipMemcpyHostToDevice) == hipSuccess ? BRR_OK
                                                                                         : BRR_EHIP;
}

brr_status brr_mlp_get_grads(const brr_mlp *net, float *h_out)
{
    if (!net || !h_out) return BRR_EINVAL;
    return hipMemcpy(h_out, net->g, net->nparams * 4, hipMemcpyDeviceToHost) == hipSuccess ? BRR_OK
                                                                                          : BRR_EHIP;
}

brr_status brr_mlp_forward(brr_mlp *net, const float *d_x, uint32_t batch, float *d_y, void *stream)
{
    if (!net || (batch && (!d_x || !d_y))) return BRR_EINVAL;
    if (batch == 0) return BRR_OK;
    brr_status st = ensure_cap(net, batch);
    if (st != BRR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (forward(net, d_x, batch, s) != hipSuccess) return BRR_EHIP;
    return hipMemcpyAsync(d_y, net->y, batch * 4ull, hipMemcpyDeviceToDevice, s) == hipSuccess
               ? BRR_OK
               : BRR_EHIP;
}

brr_status brr_mlp_backward(brr_mlp *net, const float *d_x, const float *d_t, uint32_t batch,
                            float *d_loss, void *stream)
{
    if (!net || !d_x || !d_t || batch == 0) return BRR_EINVAL;
    brr_status st = ensure_cap(net, batch);
    if (st != BRR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint32_t I = net->n_in, H = net->hidden, B = batch;
    float *p = net->p, *g = net->g;
    if (forward(net, d_x, B, s) != hipSuccess) return BRR_EHIP;
    k_mse<<<blocks(B), 256, 0, s>>>(net->y, d_t, net->dy, d_loss, B);
    k_bwd_w<<<blocks((uint64_t)(H + 1) * 1), 256, 0, s>>>(net->a2, net->dy, net->W3(g), net->b3(g), B,
                                                          H, 1);
    k_bwd_x<<<blocks((uint64_t)B * H), 256, 0, s>>>(net->dy, net->W3(p), net->a2, net->d2, B, H, 1);
    k_bwd_w<<<blocks((uint64_t)(H + 1) * H), 256, 0, s>>>(net->a1, net->d2, net->W2(g), net->b2(g),
                                                          B, H, H);
    k_bwd_x<<<blocks((uint64_t)B * H), 256, 0, s>>>(net->d2, net->W2(p), net->a1, net->d1, B, H, H);
    k_bwd_w<<<blocks((uint64_t)(I + 1) * H), 256, 0, s>>>(d_x, net->d1, net->W1(g), net->b1(g), B, I,
                                                          H);
    return hipGetLastError() == hipSuccess ? BRR_OK : BRR_EHIP;
}

brr_status brr_mlp_adam_step(brr_mlp *net, float lr, void *stream)
{
    if (!net || !(lr > 0)) return BRR_EINVAL;
    ++net->t;
    const float c1 = 1.0f - std::pow(0.9f, (float)net->t);
    const float c2 = 1.0f - std::pow(0.999f, (float)net->t);
    k_adam<<<blocks(net->nparams), 256, 0, static_cast<hipStream_t>(stream)>>>(
        net->p, net->g, net->m, net->v, (uint32_t)net->nparams, lr, c1, c2);
    return hipGetLastError() == hipSuccess ? BRR_OK : BRR_EHIP;
}

brr_status brr_mlp_train(brr_mlp *net, const float *d_x, const float *d_t, uint32_t batch,
                         uint32_t steps, float lr, float *h_final_loss, void *stream)
{
    if (!net || !d_x || !d_t || batch == 0) return BRR_EINVAL;
    float *d_loss = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMallocAsync(reinterpret_cast<void **>(&d_loss), 4, s) != hipSuccess) return BRR_ENOMEM;
    brr_status st = BRR_OK;
    for (uint32_t k = 0; k < steps && st == BRR_OK; ++k) {
        st = brr_mlp_backward(net, d_x, d_t, batch, (k + 1 == steps) ? d_loss : nullptr, stream);
        if (st == BRR_OK) st = brr_mlp_adam_step(net, lr, stream);
    }
    if (st == BRR_OK && steps && h_final_loss &&
        hipMemcpyAsync(h_final_loss, d_loss, 4, hipMemcpyDeviceToHost, s) != hipSuccess)
        st = BRR_EHIP;
    (void)hipFreeAsync(d_loss, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == BRR_OK) st = BRR_EHIP;
    return st;
}

} // extern "C"
