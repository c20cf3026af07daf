// mlp.hip -- the work-item cost model: a 4 -> 64 -> 64 -> 64 -> 1 FP32
// multilayer perceptron with ReLU activations, trained on the GPU by the
// kernels below (forward, backward, Adam) on per-item kernel timings, and
// used to predict item costs for scheduling.  It never affects the counts.
//
// Parameter layout (one packed float array):
//   W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4
// Inputs are standardised with per-feature mean/std and the target (log2 of
// the item time) with its own mean/std; both are part of the model.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <random>
#include <vector>

#include "internal.h"

namespace fcfc {

constexpr int NF = 4, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NH, OFF_W4 = OFF_B3 + NH, OFF_B4 = OFF_W4 + NH,
              NPARAM = OFF_B4 + 1;
constexpr int MB = 64;  // samples per workgroup in the gradient kernel

struct Model {
    float* params = nullptr;  // device NPARAM
    float* grad = nullptr;    // device NPARAM (+1 loss accumulator)
    float* m1 = nullptr;      // Adam moments
    float* m2 = nullptr;
    float norm[10] = {0, 0, 0, 0, 1, 1, 1, 1, 0, 1};  // x mean[4], x std[4], y mean, y std
    int step = 0;
};

// forward pass of one sample held in registers; params in LDS
__device__ inline float mlp_one(const float* __restrict__ P, const float x[NF]) {
    float h1[NH], h2[NH];
#pragma unroll
    for (int o = 0; o < NH; o++) {
        float acc = P[OFF_B1 + o];
#pragma unroll
        for (int i = 0; i < NF; i++) acc = __builtin_fmaf(P[OFF_W1 + o * NF + i], x[i], acc);
        h1[o] = fmaxf(acc, 0.f);
    }
#pragma unroll
    for (int o = 0; o < NH; o++) {
        float acc = P[OFF_B2 + o];
#pragma unroll
        for (int i = 0; i < NH; i++) acc = __builtin_fmaf(P[OFF_W2 + o * NH + i], h1[i], acc);
        h2[o] = fmaxf(acc, 0.f);
    }
    float y = P[OFF_B4];
#pragma unroll
    for (int o = 0; o < NH; o++) {
        float acc = P[OFF_B3 + o];
#pragma unroll
        for (int i = 0; i < NH; i++) acc = __builtin_fmaf(P[OFF_W3 + o * NH + i], h2[i], acc);
        y = __builtin_fmaf(P[OFF_W4 + o], fmaxf(acc, 0.f), y);
    }
    return y;
}

struct NormArgs {
    float xm[NF], xs[NF], ym, ys;
};

// y[i] = ys * mlp((x[i] - xm) / xs) + ym
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ X,
                                                     int64_t m, NormArgs nrm, float* __restrict__ Y) {
    __shared__ float P[NPARAM];
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) P[i] = params[i];
    __syncthreads();
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    float x[NF];
#pragma unroll
    for (int i = 0; i < NF; i++) x[i] = (X[s * NF + i] - nrm.xm[i]) / nrm.xs[i];
    Y[s] = mlp_one(P, x) * nrm.ys + nrm.ym;
}

// Gradient of 0.5 * sum_s (y_s - t_s)^2 (standardised units) over samples
// [s0, s0 + count) taken through the permutation `perm` (or identity), added
// to grad[]; grad[NPARAM] accumulates the loss.  One workgroup of 256 threads
// handles MB samples: layers are 64 x 64 products spread over the threads.
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ params, const float* __restrict__ X,
                                                  const float* __restrict__ T, const uint32_t* __restrict__ perm,
                                                  int64_t s0, int64_t count, NormArgs nrm,
                                                  float* __restrict__ grad) {
    __shared__ float xin[MB][NF];
    __shared__ float H1[MB][NH], H2[MB][NH], H3[MB][NH];
    __shared__ float D[MB][NH], E[MB][NH];
    __shared__ float dy[MB];
    const int t = threadIdx.x;
    const int64_t base = s0 + (int64_t)blockIdx.x * MB;
    const int nloc = (int)min<int64_t>(MB, count - (int64_t)blockIdx.x * MB);
    if (nloc <= 0) return;
    for (int i = t; i < MB * NF; i += 256) {
        int s = i / NF, f = i % NF;
        float v = 0.f;
        if (s < nloc) {
            int64_t idx = base + s;
            if (perm) idx = perm[idx];
            v = (X[idx * NF + f] - nrm.xm[f]) / nrm.xs[f];
        }
        xin[s][f] = v;
    }
    __syncthreads();
    const int s = t >> 2;          // sample (forward/backward on activations)
    const int c0 = (t & 3) * 16;   // 16 columns per thread
    // layer 1
    for (int c = c0; c < c0 + 16; c++) {
        float acc = params[OFF_B1 + c];
        for (int i = 0; i < NF; i++) acc = __builtin_fmaf(params[OFF_W1 + c * NF + i], xin[s][i], acc);
        H1[s][c] = fmaxf(acc, 0.f);
    }
    __syncthreads();
    for (int c = c0; c < c0 + 16; c++) {
        float acc = params[OFF_B2 + c];
        for (int i = 0; i < NH; i++) acc = __builtin_fmaf(params[OFF_W2 + c * NH + i], H1[s][i], acc);
        H2[s][c] = fmaxf(acc, 0.f);
    }
    __syncthreads();
    for (int c = c0; c < c0 + 16; c++) {
        float acc = params[OFF_B3 + c];
        for (int i = 0; i < NH; i++) acc = __builtin_fmaf(params[OFF_W3 + c * NH + i], H2[s][i], acc);
        H3[s][c] = fmaxf(acc, 0.f);
    }
    __syncthreads();
    if (t < MB) {
        float y = params[OFF_B4];
        for (int i = 0; i < NH; i++) y = __builtin_fmaf(params[OFF_W4 + i], H3[t][i], y);
        float d = 0.f;
        if (t < nloc) {
            int64_t idx = base + t;
            if (perm) idx = perm[idx];
            const float target = (T[idx] - nrm.ym) / nrm.ys;
            d = y - target;
        }
        dy[t] = d;
        atomicAdd(&grad[NPARAM], 0.5f * d * d);
    }
    __syncthreads();
    // output layer: dW4[i] = sum_s dy_s H3[s][i]; db4 = sum dy; dZ3 = dy W4 (H3 > 0)
    if (t < NH) {
        float g = 0.f;
        for (int q = 0; q < MB; q++) g = __builtin_fmaf(dy[q], H3[q][t], g);
        atomicAdd(&grad[OFF_W4 + t], g);
    }
    if (t == NH) {
        float g = 0.f;
        for (int q = 0; q < MB; q++) g += dy[q];
        atomicAdd(&grad[OFF_B4], g);
    }
    for (int c = c0; c < c0 + 16; c++) D[s][c] = (H3[s][c] > 0.f) ? dy[s] * params[OFF_W4 + c] : 0.f;
    __syncthreads();
    // layer 3: dW3[o][i] = sum_s D[s][o] H2[s][i]; db3[o] = sum_s D[s][o]; E = (D W3) (H2 > 0)
    {
        const int o = t >> 2, i0 = (t & 3) * 16;
        for (int i = i0; i < i0 + 16; i++) {
            float g = 0.f;
            for (int q = 0; q < MB; q++) g = __builtin_fmaf(D[q][o], H2[q][i], g);
            atomicAdd(&grad[OFF_W3 + o * NH + i], g);
        }
        if ((t & 3) == 0) {
            float g = 0.f;
            for (int q = 0; q < MB; q++) g += D[q][o];
            atomicAdd(&grad[OFF_B3 + o], g);
        }
    }
    for (int c = c0; c < c0 + 16; c++) {
        float acc = 0.f;
        for (int o = 0; o < NH; o++) acc = __builtin_fmaf(D[s][o], params[OFF_W3 + o * NH + c], acc);
        E[s][c] = (H2[s][c] > 0.f) ? acc : 0.f;
    }
    __syncthreads();
    // layer 2: dW2 = E^T H1; db2 = sum E; D = (E W2) (H1 > 0)
    {
        const int o = t >> 2, i0 = (t & 3) * 16;
        for (int i = i0; i < i0 + 16; i++) {
            float g = 0.f;
            for (int q = 0; q < MB; q++) g = __builtin_fmaf(E[q][o], H1[q][i], g);
            atomicAdd(&grad[OFF_W2 + o * NH + i], g);
        }
        if ((t & 3) == 0) {
            float g = 0.f;
            for (int q = 0; q < MB; q++) g += E[q][o];
            atomicAdd(&grad[OFF_B2 + o], g);
        }
    }
    __syncthreads();
    for (int c = c0; c < c0 + 16; c++) {
        float acc = 0.f;
        for (int o = 0; o < NH; o++) acc = __builtin_fmaf(E[s][o], params[OFF_W2 + o * NH + c], acc);
        D[s][c] = (H1[s][c] > 0.f) ? acc : 0.f;
    }
    __syncthreads();
    // layer 1: dW1 = D^T x; db1 = sum D
    if (t < NH * NF) {
        const int o = t / NF, i = t % NF;
        float g = 0.f;
        for (int q = 0; q < MB; q++) g = __builtin_fmaf(D[q][o], xin[q][i], g);
        atomicAdd(&grad[OFF_W1 + o * NF + i], g);
    }
    if (t < NH) {
        float g = 0.f;
        for (int q = 0; q < MB; q++) g += D[q][t];
        atomicAdd(&grad[OFF_B1 + t], g);
    }
}

// Adam step on the gradient averaged over `count` samples; clears the gradient.
__global__ void k_adam(float* __restrict__ params, float* __restrict__ grad, float* __restrict__ m1,
                       float* __restrict__ m2, float inv_count, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > NPARAM) return;
    if (i == NPARAM) {
        grad[i] = 0.f;
        return;
    }
    const float g = grad[i] * inv_count;
    const float a = b1 * m1[i] + (1.f - b1) * g;
    const float v = b2 * m2[i] + (1.f - b2) * g * g;
    m1[i] = a;
    m2[i] = v;
    params[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
    grad[i] = 0.f;
}

// per-item features (log2(1 + A points), log2(1 + B points), transverse row
// separation in cells, cells per prune radius) and log2 of the recorded time
__global__ void k_item_features(const Item* __restrict__ items, const uint32_t* __restrict__ times, uint32_t n,
                                float kcells, float* __restrict__ X, float* __restrict__ logt) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Item it = items[i];
    const float na = (float)(it.acnt_xb0 & 0xffffu);
    const float nb = (float)(it.b_end - it.b_begin);
    const float dy = (float)(int8_t)(it.meta & 0xffu), dz = (float)(int8_t)((it.meta >> 8) & 0xffu);
    X[4 * (size_t)i + 0] = log2f(1.f + na);
    X[4 * (size_t)i + 1] = log2f(1.f + nb);
    X[4 * (size_t)i + 2] = sqrtf(dy * dy + dz * dz);
    X[4 * (size_t)i + 3] = kcells;
    if (logt) logt[i] = log2f(1.f + (float)(times ? times[i] : 0u));
}

static void norm_args(const Model* md, NormArgs& n) {
    for (int i = 0; i < NF; i++) {
        n.xm[i] = md->norm[i];
        n.xs[i] = md->norm[NF + i];
    }
    n.ym = md->norm[8];
    n.ys = md->norm[9];
}

void model_item_costs(const Model* md, const Item* items, uint32_t n, float kcells, float* feat, float* pred,
                      hipStream_t st) {
    if (n == 0) return;
    NormArgs nrm;
    norm_args(md, nrm);
    hipLaunchKernelGGL(k_item_features, dim3((n + 255) / 256), dim3(256), 0, st, items, (const uint32_t*)nullptr, n,
                       kcells, feat, (float*)nullptr);
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, st, md->params, (const float*)feat,
                       (int64_t)n, nrm, pred);
}

size_t model_param_bytes() { return sizeof(float) * (NPARAM + 1); }

Model* model_snapshot(const Model* src, float* params, hipStream_t st) {
    Model* m = new (std::nothrow) Model();
    if (!m) return nullptr;
    if (hipMemcpyAsync(params, src->params, model_param_bytes(), hipMemcpyDeviceToDevice, st) != hipSuccess) {
        delete m;
        return nullptr;
    }
    m->params = params;
    for (int i = 0; i < 10; i++) m->norm[i] = src->norm[i];
    m->step = src->step;
    return m;
}

void model_snapshot_free(Model* m) { delete m; }

static fcfc_status model_alloc(Model* md) {
    float* blk = nullptr;
    if (hipMalloc((void**)&blk, sizeof(float) * (4 * (NPARAM + 1) + 64)) != hipSuccess) {
        set_error("model: cannot allocate parameters");
        return FCFC_ENOMEM;
    }
    md->params = blk;
    md->grad = blk + (NPARAM + 1);
    md->m1 = blk + 2 * (NPARAM + 1);
    md->m2 = blk + 3 * (NPARAM + 1);
    FCFC_HIP(hipMemset(blk, 0, sizeof(float) * 4 * (NPARAM + 1)));
    return FCFC_OK;
}

}  // namespace fcfc

using namespace fcfc;

extern "C" int32_t fcfc_model_nparams(void) { return NPARAM; }

extern "C" fcfc_status fcfc_model_create(uint64_t seed, fcfc_model_t* out) {
    clear_error();
    if (!out) return FCFC_EINVAL;
    Model* md = new (std::nothrow) Model();
    if (!md) return FCFC_ENOMEM;
    fcfc_status s = model_alloc(md);
    if (s != FCFC_OK) {
        delete md;
        return s;
    }
    // He-uniform initialisation (host, seeded)
    std::vector<float> h(NPARAM, 0.f);
    std::mt19937_64 rng(seed);
    auto fill = [&](int off, int nout, int nin) {
        float lim = sqrtf(6.f / (float)nin);
        std::uniform_real_distribution<float> u(-lim, lim);
        for (int i = 0; i < nout * nin; i++) h[off + i] = u(rng);
    };
    fill(OFF_W1, NH, NF);
    fill(OFF_W2, NH, NH);
    fill(OFF_W3, NH, NH);
    fill(OFF_W4, 1, NH);
    FCFC_HIP(hipMemcpy(md->params, h.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice));
    *out = (fcfc_model_t)md;
    return FCFC_OK;
}

extern "C" void fcfc_model_free(fcfc_model_t model) {
    Model* md = (Model*)model;
    if (!md) return;
    if (md->params) (void)hipFree(md->params);
    delete md;
}

extern "C" fcfc_status fcfc_model_get(fcfc_model_t model, float* params, float* norm) {
    Model* md = (Model*)model;
    if (!md) return FCFC_EINVAL;
    if (params) FCFC_HIP(hipMemcpy(params, md->params, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    if (norm) memcpy(norm, md->norm, sizeof(md->norm));
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_model_set(fcfc_model_t model, const float* params, const float* norm) {
    Model* md = (Model*)model;
    if (!md) return FCFC_EINVAL;
    if (params) FCFC_HIP(hipMemcpy(md->params, params, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
    if (norm) {
        for (int i = 0; i < 10; i++)
            if (!isfinite(norm[i]) || (i >= NF && i < 2 * NF && !(norm[i] > 0)) || (i == 9 && !(norm[i] > 0))) {
                set_error("model_set: normalisation must be finite with positive scales");
                return FCFC_EINVAL;
            }
        memcpy(md->norm, norm, sizeof(md->norm));
    }
    md->step = 0;
    FCFC_HIP(hipMemset(md->m1, 0, sizeof(float) * 2 * (NPARAM + 1)));
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_model_predict(fcfc_model_t model, const float* d_feat, int64_t m, float* d_out,
                                          void* stream) {
    clear_error();
    Model* md = (Model*)model;
    if (!md || (m > 0 && (!d_feat || !d_out)) || m < 0) return FCFC_EINVAL;
    if (m == 0) return FCFC_OK;
    NormArgs n;
    norm_args(md, n);
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       md->params, d_feat, m, n, d_out);
    FCFC_HIP(hipGetLastError());
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_model_grad(fcfc_model_t model, const float* d_feat, const float* d_target, int64_t m,
                                       float* grad_host, float* loss_host, void* stream) {
    clear_error();
    Model* md = (Model*)model;
    if (!md || m <= 0 || !d_feat || !d_target) return FCFC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    NormArgs n;
    norm_args(md, n);
    FCFC_HIP(hipMemsetAsync(md->grad, 0, sizeof(float) * (NPARAM + 1), st));
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((m + MB - 1) / MB)), dim3(256), 0, st, md->params, d_feat, d_target,
                       (const uint32_t*)nullptr, (int64_t)0, m, n, md->grad);
    std::vector<float> h(NPARAM + 1);
    FCFC_HIP(hipMemcpyAsync(h.data(), md->grad, sizeof(float) * (NPARAM + 1), hipMemcpyDeviceToHost, st));
    FCFC_HIP(hipStreamSynchronize(st));
    if (grad_host) memcpy(grad_host, h.data(), sizeof(float) * NPARAM);
    if (loss_host) *loss_host = h[NPARAM];
    FCFC_HIP(hipMemsetAsync(md->grad, 0, sizeof(float) * (NPARAM + 1), st));
    return FCFC_OK;
}

// Standardisation from the training set (host copies), then `epochs` passes of
// Adam over shuffled minibatches of `batch` samples.  Returns the mean loss of
// the last epoch (standardised units).
extern "C" fcfc_status fcfc_model_train(fcfc_model_t model, const float* d_feat, const float* d_target, int64_t m,
                                        int32_t epochs, int32_t batch, float lr, uint64_t seed, void* stream,
                                        float* final_loss) {
    clear_error();
    Model* md = (Model*)model;
    if (!md || m < 2 || !d_feat || !d_target || epochs < 1 || batch < MB || !(lr > 0)) {
        set_error("model_train: need m >= 2 samples, epochs >= 1, batch >= %d, lr > 0", MB);
        return FCFC_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    std::vector<float> hx((size_t)m * NF), ht((size_t)m);
    FCFC_HIP(hipMemcpyAsync(hx.data(), d_feat, hx.size() * 4, hipMemcpyDeviceToHost, st));
    FCFC_HIP(hipMemcpyAsync(ht.data(), d_target, ht.size() * 4, hipMemcpyDeviceToHost, st));
    FCFC_HIP(hipStreamSynchronize(st));
    for (int f = 0; f < NF; f++) {
        double s = 0, s2 = 0;
        for (int64_t i = 0; i < m; i++) {
            double v = hx[i * NF + f];
            s += v;
            s2 += v * v;
        }
        double mu = s / m, var = s2 / m - mu * mu;
        md->norm[f] = (float)mu;
        md->norm[NF + f] = (float)std::max(sqrt(std::max(var, 0.0)), 1e-3);
    }
    {
        double s = 0, s2 = 0;
        for (int64_t i = 0; i < m; i++) {
            s += ht[i];
            s2 += (double)ht[i] * ht[i];
        }
        double mu = s / m, var = s2 / m - mu * mu;
        md->norm[8] = (float)mu;
        md->norm[9] = (float)std::max(sqrt(std::max(var, 0.0)), 1e-3);
    }
    NormArgs n;
    norm_args(md, n);
    uint32_t* perm = nullptr;
    FCFC_HIP(hipMalloc((void**)&perm, sizeof(uint32_t) * (size_t)m));
    std::vector<uint32_t> hp((size_t)m);
    for (int64_t i = 0; i < m; i++) hp[i] = (uint32_t)i;
    std::mt19937_64 rng(seed);
    FCFC_HIP(hipMemsetAsync(md->grad, 0, sizeof(float) * (NPARAM + 1), st));
    float last = 0.f;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int e = 0; e < epochs; e++) {
        std::shuffle(hp.begin(), hp.end(), rng);
        FCFC_HIP(hipMemcpyAsync(perm, hp.data(), sizeof(uint32_t) * (size_t)m, hipMemcpyHostToDevice, st));
        double eloss = 0;
        for (int64_t s0 = 0; s0 < m; s0 += batch) {
            const int64_t cnt = std::min<int64_t>(batch, m - s0);
            hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((cnt + MB - 1) / MB)), dim3(256), 0, st, md->params, d_feat,
                               d_target, perm, s0, cnt, n, md->grad);
            md->step++;
            const float c1 = 1.f - powf(b1, (float)md->step), c2 = 1.f - powf(b2, (float)md->step);
            if (e == epochs - 1) {
                float l = 0.f;
                FCFC_HIP(hipMemcpyAsync(&l, md->grad + NPARAM, 4, hipMemcpyDeviceToHost, st));
                FCFC_HIP(hipStreamSynchronize(st));
                eloss += l;
            }
            hipLaunchKernelGGL(k_adam, dim3((NPARAM + 256) / 256), dim3(256), 0, st, md->params, md->grad, md->m1, md->m2,
                               1.f / (float)cnt, lr, b1, b2, eps, c1, c2);
        }
        if (e == epochs - 1) last = (float)(eloss / m);
    }
    FCFC_HIP(hipStreamSynchronize(st));
    (void)hipFree(perm);
    if (final_loss) *final_loss = last;
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_model_save(fcfc_model_t model, const char* path) {
    clear_error();
    Model* md = (Model*)model;
    if (!md || !path) return FCFC_EINVAL;
    std::vector<float> h(NPARAM);
    FCFC_HIP(hipMemcpy(h.data(), md->params, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    FILE* f = fopen(path, "wb");
    if (!f) {
        set_error("model_save: cannot open %s", path);
        return FCFC_EINVAL;
    }
    const char magic[8] = {'F', 'C', 'F', 'C', 'M', 'L', 'P', '1'};
    int32_t np = NPARAM;
    bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&np, 4, 1, f) == 1 && fwrite(md->norm, 4, 10, f) == 10 &&
              fwrite(h.data(), 4, NPARAM, f) == (size_t)NPARAM;
    fclose(f);
    if (!ok) {
        set_error("model_save: write failed");
        return FCFC_EINVAL;
    }
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_model_load(const char* path, fcfc_model_t* out) {
    clear_error();
    if (!path || !out) return FCFC_EINVAL;
    FILE* f = fopen(path, "rb");
    if (!f) {
        set_error("model_load: cannot open %s", path);
        return FCFC_EMODEL;
    }
    char magic[8];
    int32_t np = 0;
    float norm[10];
    std::vector<float> h(NPARAM);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "FCFCMLP1", 8) == 0 && fread(&np, 4, 1, f) == 1 &&
              np == NPARAM && fread(norm, 4, 10, f) == 10 && fread(h.data(), 4, NPARAM, f) == (size_t)NPARAM;
    fclose(f);
    for (int i = 0; ok && i < NPARAM; i++) ok = isfinite(h[i]);
    if (!ok) {
        set_error("model_load: %s is not a valid model file", path);
        return FCFC_EMODEL;
    }
    fcfc_model_t m = nullptr;
    FCFC_TRY(fcfc_model_create(0, &m));
    fcfc_status s = fcfc_model_set(m, h.data(), norm);
    if (s != FCFC_OK) {
        fcfc_model_free(m);
        set_error("model_load: invalid normalisation in %s", path);
        return FCFC_EMODEL;
    }
    *out = m;
    return FCFC_OK;
}

// Features (and log2 time) of the work items of the last count recorded with
// record_timing = 1 on this plan.  d_feat: cap x 4 floats, d_logt: cap floats.
extern "C" fcfc_status fcfc_plan_timings(fcfc_plan_t plan, float* d_feat, float* d_logt, int64_t cap, int64_t* n,
                                         void* stream) {
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p || !n) return FCFC_EINVAL;
    if (!p->timing_dev || p->timing_n == 0) {
        set_error("plan_timings: no count with record_timing = 1 has run on this plan");
        return FCFC_ESTATE;
    }
    *n = p->timing_n;
    if (!d_feat) return FCFC_OK;
    if (cap < (int64_t)p->timing_n) {
        set_error("plan_timings: capacity %lld < %u items", (long long)cap, p->timing_n);
        return FCFC_EINVAL;
    }
    const uint32_t* times = (const uint32_t*)p->timing_dev;
    const Item* items = (const Item*)((const char*)p->timing_dev + (size_t)p->timing_n * 4);
    const float kc = (float)(p->rprune / p->grid.side);
    hipLaunchKernelGGL(k_item_features, dim3((p->timing_n + 255) / 256), dim3(256), 0, (hipStream_t)stream, items,
                       times, p->timing_n, kc, d_feat, d_logt);
    FCFC_HIP(hipGetLastError());
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_plan_set_model(fcfc_plan_t plan, fcfc_model_t model) {
    clear_error();
    Plan* p = (Plan*)plan;
    if (!p) return FCFC_EINVAL;
    p->model = (Model*)model;
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_plan_predict(fcfc_plan_t plan, fcfc_cells_t c1, fcfc_cells_t c2, fcfc_model_t model,
                                         void* stream, double* pred_ms, int64_t* n_items) {
    clear_error();
    Plan* p = (Plan*)plan;
    Cells* a = (Cells*)c1;
    Cells* b = (Cells*)c2;
    if (!p || !a || !model || !pred_ms) {
        set_error("plan_predict: null plan, cells, model or output");
        return FCFC_EINVAL;
    }
    if (a->plan_id != p->id || (b && b->plan_id != p->id)) {
        set_error("plan_predict: cell sets were built on a different plan");
        return FCFC_EGRID;
    }
    PredictReq pr;
    pr.model = (const Model*)model;
    FCFC_TRY(count_pairs(p, a, b, nullptr, nullptr, (hipStream_t)stream, &pr));
    *pred_ms = pr.pred_ms;
    if (n_items) *n_items = pr.items;
    return FCFC_OK;
}

extern "C" fcfc_status fcfc_choose_cells(fcfc_model_t model, int32_t kind, int32_t los, const double* edges1,
                                         int32_t n1, const double* edges2, int32_t n2, double box_L,
                                         const fcfc_tuning* tune, const fcfc_catalog* c1, const fcfc_catalog* c2,
                                         void* stream, int32_t* best_k, double pred_ms[6]) {
    clear_error();
    if (!c1 || !best_k) {
        set_error("choose_cells: null catalogue or output");
        return FCFC_EINVAL;
    }
    fcfc_tuning t{};
    if (tune) t = *tune;
    if (t.n_hint <= 0) t.n_hint = (int32_t)std::min<int64_t>(c1->n, 0x7fffffff);
    t.record_timing = 0;
    for (int k = 0; k < 6; k++)
        if (pred_ms) pred_ms[k] = NAN;
    const fcfc_catalog a{c1->xyz, nullptr, c1->n};
    const fcfc_catalog b{c2 ? c2->xyz : nullptr, nullptr, c2 ? c2->n : 0};
    fcfc_catalog both[2] = {a, b};
    auto make = [&](int k, fcfc_plan_t* pl) -> fcfc_status {
        t.cells_per_rmax = k;
        FCFC_TRY(fcfc_plan_create(kind, los, edges1, n1, edges2, n2, box_L, &t, pl));
        if (box_L <= 0) {
            fcfc_status s = fcfc_plan_fit_bounds(*pl, both, c2 ? 2 : 1, stream);
            if (s != FCFC_OK) {
                fcfc_plan_free(*pl);
                return s;
            }
        }
        return FCFC_OK;
    };
    if (!model) {
        fcfc_plan_t pl = nullptr;
        FCFC_TRY(make(tune ? tune->cells_per_rmax : 0, &pl));
        *best_k = ((Plan*)pl)->grid.k;
        fcfc_plan_free(pl);
        return FCFC_OK;
    }
    double best = INFINITY;
    int bk = 0;
    for (int k = 1; k <= 6; k++) {
        fcfc_plan_t pl = nullptr;
        fcfc_status s = make(k, &pl);
        if (s == FCFC_ERANGE) continue;  // grid too fine for this box
        FCFC_TRY(s);
        if (((Plan*)pl)->grid.k != k) {
            fcfc_plan_free(pl);
            continue;
        }
        fcfc_cells_t ca = nullptr, cb = nullptr;
        s = fcfc_build_cells(pl, &a, stream, &ca);
        if (s == FCFC_OK && c2) s = fcfc_build_cells(pl, &b, stream, &cb);
        double ms = NAN;
        if (s == FCFC_OK) s = fcfc_plan_predict(pl, ca, cb, model, stream, &ms, nullptr);
        fcfc_cells_free(ca);
        fcfc_cells_free(cb);
        fcfc_plan_free(pl);
        FCFC_TRY(s);
        if (pred_ms) pred_ms[k - 1] = ms;
        if (isfinite(ms) && ms < best) {
            best = ms;
            bk = k;
        }
    }
    if (bk == 0) {
        // no usable prediction: the analytic choice
        fcfc_plan_t pl = nullptr;
        FCFC_TRY(make(0, &pl));
        bk = ((Plan*)pl)->grid.k;
        fcfc_plan_free(pl);
    }
    *best_k = bk;
    return FCFC_OK;
}
