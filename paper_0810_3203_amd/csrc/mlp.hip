// A small fp32 multilayer perceptron used as the cost model of the batch
// planner: inputs are features of a (request, schedule candidate) pair, the
// output is the predicted log of its run time.  Forward pass, backward pass
// (mean squared error) and Adam updates are the kernels below; layers are
// tiny (<= 64 wide), so each kernel maps one thread to one output value.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/tft.h"

namespace {

// Z[b][o] = sum_i X[b][i] W[o][i] + bias[o]; A = relu(Z) when relu
__global__ void linear_fwd(const float *__restrict__ X, const float *__restrict__ Wt, const float *__restrict__ bias,
                           float *__restrict__ Z, float *__restrict__ A, uint32_t B, uint32_t I, uint32_t O,
                           int relu) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * O) return;
    const uint32_t b = t / O, o = t % O;
    float acc = bias[o];
    for (uint32_t i = 0; i < I; ++i) acc += X[b * I + i] * Wt[o * I + i];
    Z[t] = acc;
    if (A) A[t] = relu ? fmaxf(acc, 0.0f) : acc;
}

// dX[b][i] = sum_o dZ[b][o] W[o][i]; then dX *= (Zprev > 0) when Zprev (relu of the previous layer)
__global__ void linear_bwd_x(const float *__restrict__ dZ, const float *__restrict__ Wt,
                             const float *__restrict__ Zprev, float *__restrict__ dX, uint32_t B, uint32_t I,
                             uint32_t O) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * I) return;
    const uint32_t b = t / I, i = t % I;
    float acc = 0.0f;
    for (uint32_t o = 0; o < O; ++o) acc += dZ[b * O + o] * Wt[o * I + i];
    if (Zprev && !(Zprev[t] > 0.0f)) acc = 0.0f;
    dX[t] = acc;
}

// dW[o][i] = sum_b dZ[b][o] X[b][i]; db[o] = sum_b dZ[b][o]
__global__ void linear_bwd_w(const float *__restrict__ dZ, const float *__restrict__ X, float *__restrict__ dW,
                             float *__restrict__ db, uint32_t B, uint32_t I, uint32_t O) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < O * I) {
        const uint32_t o = t / I, i = t % I;
        float acc = 0.0f;
        for (uint32_t b = 0; b < B; ++b) acc += dZ[b * O + o] * X[b * I + i];
        dW[t] = acc;
    } else if (t < O * I + O) {
        const uint32_t o = t - O * I;
        float acc = 0.0f;
        for (uint32_t b = 0; b < B; ++b) acc += dZ[b * O + o];
        db[o] = acc;
    }
}

// loss = sum_b (y_b - t_b)^2 / (2B); dy_b = (y_b - t_b) / B.  One workgroup.
__global__ void mse(const float *__restrict__ y, const float *__restrict__ tgt, float *__restrict__ dy,
                    float *__restrict__ loss, uint32_t B) {
    __shared__ float part[256];
    float acc = 0.0f;
    for (uint32_t b = threadIdx.x; b < B; b += blockDim.x) {
        const float d = y[b] - tgt[b];
        dy[b] = d / (float)B;
        acc += d * d;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] / (2.0f * (float)B);
}

__global__ void adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                     uint32_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.0f - b1) * gt;
    const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

inline uint32_t blocks(uint64_t n) { return (uint32_t)((n + 255) / 256); }

uint64_t mix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

struct tft_mlp {
    uint32_t in, hidden, depth;
    std::vector<uint32_t> dims;       // layer widths: in, hidden x depth, 1
    std::vector<uint64_t> woff, boff; // parameter offsets per layer
    uint64_t nparam = 0;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
    float *act = nullptr;  // Z and A per layer, plus dZ buffers, for `cap` rows
    uint32_t cap = 0;
    uint64_t step = 0;
    std::vector<uint64_t> zoff, aoff;
    uint64_t dz0 = 0, dz1 = 0, dy = 0, act_total = 0;
};

namespace {

int ensure_cap(tft_mlp *M, uint32_t B) {
    if (B <= M->cap) return TFT_OK;
    const size_t L = M->dims.size() - 1;
    M->zoff.assign(L, 0);
    M->aoff.assign(L, 0);
    uint64_t off = 0;
    uint32_t widest = 1;
    for (size_t k = 0; k < L; k++) {
        const uint32_t o = M->dims[k + 1];
        widest = std::max(widest, std::max(o, M->dims[k]));
        M->zoff[k] = off;
        off += (uint64_t)B * o;
        M->aoff[k] = off;
        off += (uint64_t)B * o;
    }
    M->dz0 = off;
    off += (uint64_t)B * widest;
    M->dz1 = off;
    off += (uint64_t)B * widest;
    M->dy = off;
    off += B;
    if (M->act) (void)hipFree(M->act);
    M->act = nullptr;
    if (hipMalloc(&M->act, off * sizeof(float)) != hipSuccess) return TFT_E_DEVICE;
    M->cap = B;
    M->act_total = off;
    return TFT_OK;
}

// forward pass for B rows of x; returns the device pointer of the outputs (B floats)
float *forward(tft_mlp *M, const float *x, uint32_t B, hipStream_t st) {
    const size_t L = M->dims.size() - 1;
    const float *in = x;
    for (size_t k = 0; k < L; k++) {
        const uint32_t I = M->dims[k], O = M->dims[k + 1];
        float *Z = M->act + M->zoff[k], *A = M->act + M->aoff[k];
        hipLaunchKernelGGL(linear_fwd, dim3(blocks((uint64_t)B * O)), dim3(256), 0, st, in, M->params + M->woff[k],
                           M->params + M->boff[k], Z, A, B, I, O, k + 1 < L ? 1 : 0);
        in = A;
    }
    return M->act + M->aoff[L - 1];
}

int gradient(tft_mlp *M, const float *x, const float *tgt, uint32_t B, hipStream_t st) {
    int rc = ensure_cap(M, B);
    if (rc) return rc;
    const size_t L = M->dims.size() - 1;
    float *y = forward(M, x, B, st);
    float *dZ = M->act + M->dy;
    hipLaunchKernelGGL(mse, dim3(1), dim3(256), 0, st, y, tgt, dZ, M->loss, B);
    float *bufs[2] = {M->act + M->dz0, M->act + M->dz1};
    int cur = 0;
    for (size_t kk = L; kk-- > 0;) {
        const uint32_t I = M->dims[kk], O = M->dims[kk + 1];
        const float *X = kk ? M->act + M->aoff[kk - 1] : x;
        hipLaunchKernelGGL(linear_bwd_w, dim3(blocks((uint64_t)O * I + O)), dim3(256), 0, st, dZ, X,
                           M->grads + M->woff[kk], M->grads + M->boff[kk], B, I, O);
        if (kk) {
            float *dX = bufs[cur];
            hipLaunchKernelGGL(linear_bwd_x, dim3(blocks((uint64_t)B * I)), dim3(256), 0, st, dZ,
                               M->params + M->woff[kk], M->act + M->zoff[kk - 1], dX, B, I, O);
            dZ = dX;
            cur ^= 1;
        }
    }
    return hipGetLastError() == hipSuccess ? TFT_OK : TFT_E_DEVICE;
}

int adam_step(tft_mlp *M, float lr, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    M->step++;
    const float c1 = 1.0f - std::pow(b1, (float)M->step), c2 = 1.0f - std::pow(b2, (float)M->step);
    hipLaunchKernelGGL(adam, dim3(blocks(M->nparam)), dim3(256), 0, st, M->params, M->grads, M->m, M->v,
                       (uint32_t)M->nparam, lr, b1, b2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? TFT_OK : TFT_E_DEVICE;
}

}  // namespace

extern "C" {

int tft_mlp_create(uint32_t in_features, uint32_t hidden, uint32_t depth, uint64_t seed, tft_mlp **out) {
    if (!out || in_features < 1 || in_features > 256 || hidden < 1 || hidden > 256 || depth < 1 || depth > 8)
        return TFT_E_ARG;
    tft_mlp *M = new tft_mlp();
    M->in = in_features;
    M->hidden = hidden;
    M->depth = depth;
    M->dims.push_back(in_features);
    for (uint32_t k = 0; k < depth; k++) M->dims.push_back(hidden);
    M->dims.push_back(1);
    std::vector<float> host;
    uint64_t ctr = seed;
    for (size_t k = 0; k + 1 < M->dims.size(); k++) {
        const uint32_t I = M->dims[k], O = M->dims[k + 1];
        M->woff.push_back(host.size());
        const float lim = std::sqrt(6.0f / (float)I);  // He-uniform
        for (uint64_t q = 0; q < (uint64_t)O * I; q++) {
            const double u = (double)(mix(ctr++) >> 11) / 9007199254740992.0;  // [0, 1)
            host.push_back((float)((2.0 * u - 1.0) * lim));
        }
        M->boff.push_back(host.size());
        for (uint32_t o = 0; o < O; o++) host.push_back(0.0f);
    }
    M->nparam = host.size();
    const size_t bytes = M->nparam * sizeof(float);
    bool ok = hipMalloc(&M->params, bytes) == hipSuccess && hipMalloc(&M->grads, bytes) == hipSuccess &&
              hipMalloc(&M->m, bytes) == hipSuccess && hipMalloc(&M->v, bytes) == hipSuccess &&
              hipMalloc(&M->loss, sizeof(float)) == hipSuccess;
    ok = ok && hipMemcpy(M->params, host.data(), bytes, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemset(M->grads, 0, bytes) == hipSuccess && hipMemset(M->m, 0, bytes) == hipSuccess &&
         hipMemset(M->v, 0, bytes) == hipSuccess;
    if (!ok) {
        tft_mlp_destroy(M);
        return TFT_E_DEVICE;
    }
    *out = M;
    return TFT_OK;
}

uint64_t tft_mlp_param_count(const tft_mlp *M) { return M ? M->nparam : 0; }

int tft_mlp_get_params(const tft_mlp *M, float *host, uint64_t n) {
    if (!M || !host || n != M->nparam) return TFT_E_ARG;
    return hipMemcpy(host, M->params, n * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess ? TFT_OK
                                                                                              : TFT_E_DEVICE;
}

int tft_mlp_set_params(tft_mlp *M, const float *host, uint64_t n) {
    if (!M || !host || n != M->nparam) return TFT_E_ARG;
    return hipMemcpy(M->params, host, n * sizeof(float), hipMemcpyHostToDevice) == hipSuccess ? TFT_OK
                                                                                              : TFT_E_DEVICE;
}

int tft_mlp_forward(tft_mlp *M, const float *x, uint32_t batch, float *y, void *stream) {
    if (!M || !x || !y || batch == 0) return TFT_E_ARG;
    int rc = ensure_cap(M, batch);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *o = forward(M, x, batch, st);
    if (hipMemcpyAsync(y, o, batch * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess) return TFT_E_DEVICE;
    return hipGetLastError() == hipSuccess ? TFT_OK : TFT_E_DEVICE;
}

int tft_mlp_gradient(tft_mlp *M, const float *x, const float *target, uint32_t batch, float *grad, float *loss,
                     void *stream) {
    if (!M || !x || !target || batch == 0) return TFT_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = gradient(M, x, target, batch, st);
    if (rc) return rc;
    if (grad && hipMemcpyAsync(grad, M->grads, M->nparam * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return TFT_E_DEVICE;
    if (loss && hipMemcpyAsync(loss, M->loss, sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return TFT_E_DEVICE;
    return TFT_OK;
}

int tft_mlp_train(tft_mlp *M, const float *x, const float *target, uint32_t batch, uint32_t iters, float lr,
                  float *final_loss, void *stream) {
    if (!M || !x || !target || batch == 0) return TFT_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (uint32_t it = 0; it < iters; it++) {
        int rc = gradient(M, x, target, batch, st);
        if (!rc) rc = adam_step(M, lr, st);
        if (rc) return rc;
    }
    if (final_loss) {
        int rc = gradient(M, x, target, batch, st);
        if (rc) return rc;
        if (hipMemcpyAsync(final_loss, M->loss, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return TFT_E_DEVICE;
    }
    return TFT_OK;
}

void tft_mlp_destroy(tft_mlp *M) {
    if (!M) return;
    for (float *p : {M->params, M->grads, M->m, M->v, M->loss, M->act})
        if (p) (void)hipFree(p);
    delete M;
}

}  // extern "C"
