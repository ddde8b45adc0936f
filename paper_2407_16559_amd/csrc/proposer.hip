// Learned step proposer: dataset assembly from run logs, FP32 forward /
// backward / Adam training kernels, and the per-device weight copy used by
// the controller.  Every reduction sums in a fixed order (deterministic).
#include <cstring>
#include <map>
#include <vector>

#include "host.h"

// weights used by smol_integrate* in learned mode, one copy per device
static std::map<int, float *> g_mlp;

SMOL_HIDDEN const float *proposer_weights(int dev)
{
    auto it = g_mlp.find(dev);
    return it == g_mlp.end() ? nullptr : it->second;
}

// ---- dataset: features of the decision after each accepted attempt and
// the hindsight target: the step that would have given err = err_target on
// the next attempt, log(h_{j+1}/h_j) + (1/k) log(err_target / err_{j+1}),
// clamped, less the PI controller's log factor at that decision (default
// exponents): the network learns a correction to PI.
// Log rows: (t, h, err, accepted, t_after, M0, M1, M2, M3).
__global__ void k_dataset_flags(const double *rec, int64_t rows, int *flag, int *count)
{
    __shared__ int sc[SMOL_WG];
    const int64_t j = blockIdx.x * (int64_t)SMOL_WG + threadIdx.x;
    int ok = 0;
    if (j + 1 < rows) {
        const double *r = rec + j * 9, *n = r + 9;
        // the network decides only after an accepted attempt that did not
        // follow a rejection
        const bool after_reject = j > 0 && rec[(j - 1) * 9 + 3] != 1.0;
        ok = r[3] == 1.0 && !after_reject && n[2] > 0.0 && isfinite(n[2]) && r[1] > 0.0 &&
             n[1] > 0.0;
    }
    if (j < rows) flag[j] = ok;
    sc[threadIdx.x] = ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        for (int i = 0; i < SMOL_WG; ++i) c += sc[i];
        count[blockIdx.x] = c;
    }
}

__global__ void k_dataset_rows(const double *rec, int64_t rows, int k, double err_target,
                               const int *flag, const int64_t *offset, float *X, float *target)
{
    __shared__ int sf[SMOL_WG];
    const int64_t j = blockIdx.x * (int64_t)SMOL_WG + threadIdx.x;
    sf[threadIdx.x] = j < rows ? flag[j] : 0;
    __syncthreads();
    if (j >= rows || !sf[threadIdx.x]) return;
    int64_t o = offset[blockIdx.x];
    for (int i = 0; i < (int)threadIdx.x; ++i) o += sf[i];
    const double *r = rec + j * 9, *n = r + 9;
    double hist[4];
    int nh = 0;
    for (int q = 0; q < 4 && j - q >= 0; ++q) hist[nh++] = rec[(j - q) * 9 + 2];
    float x[MLP_NIN];
    proposer_features(r + 5, r[1], hist, nh, x);
    for (int q = 0; q < MLP_NIN; ++q) X[o * MLP_NIN + q] = x[q];
    double d = log(n[1] / r[1]) + log(err_target / n[2]) / (double)k;
    d = fmin(fmax(d, MLP_LOG_FMIN), MLP_LOG_FMAX);
    // the network corrects the PI step the run took: err_prev is the last
    // accepted attempt's err before j (floored at 1e-4; 1 before the first)
    double err_prev = 1.0;
    for (int64_t i = j - 1; i >= 0; --i)
        if (rec[i * 9 + 3] == 1.0) {
            err_prev = fmax(rec[i * 9 + 2], 1e-4);
            break;
        }
    target[o] = (float)(d - pi_log_factor(r[2], err_prev, 0.7 / k, 0.4 / k));
}

// ---- training -----------------------------------------------------------
// Per row of the minibatch: forward, then the backpropagated signals
//   dy = 2 w (y - t) / B  (w = over_w when y > t),
//   d2 = dy W3 (1 - h2^2),  d1 = (W2^T d2) (1 - h1^2).
// act row layout: h1[64], h2[64], d1[64], d2[64], dy, loss term.
#define ACT 258

__global__ void k_mlp_rows(const float *p, const float *X, const float *target, const int *idx,
                           int B, float over_w, float *act, float *Y)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int64_t row = idx ? idx[b] : b;
    const float *x = X + row * MLP_NIN;
    float h1[MLP_NH], h2[MLP_NH];
    for (int u = 0; u < MLP_NH; ++u) {
        float z = p[MLP_OFF_B1 + u];
        for (int i = 0; i < MLP_NIN; ++i) z = fmaf(p[u * MLP_NIN + i], x[i], z);
        h1[u] = tanhf(z);
    }
    for (int u = 0; u < MLP_NH; ++u) {
        float z = p[MLP_OFF_B2 + u];
        for (int i = 0; i < MLP_NH; ++i) z = fmaf(p[MLP_OFF_W2 + u * MLP_NH + i], h1[i], z);
        h2[u] = tanhf(z);
    }
    float y = p[MLP_OFF_B3];
    for (int i = 0; i < MLP_NH; ++i) y = fmaf(p[MLP_OFF_W3 + i], h2[i], y);
    if (Y) Y[b] = y;
    if (!act) return;
    float *a = act + (int64_t)b * ACT;
    const float r = y - target[row];
    const float w = r > 0.0f ? over_w : 1.0f;
    const float dy = 2.0f * w * r / (float)B;
    float d2[MLP_NH];
    for (int u = 0; u < MLP_NH; ++u) {
        d2[u] = dy * p[MLP_OFF_W3 + u] * (1.0f - h2[u] * h2[u]);
        a[u] = h1[u];
        a[MLP_NH + u] = h2[u];
        a[3 * MLP_NH + u] = d2[u];
    }
    for (int i = 0; i < MLP_NH; ++i) {
        float s = 0.0f;
        for (int u = 0; u < MLP_NH; ++u) s = fmaf(p[MLP_OFF_W2 + u * MLP_NH + i], d2[u], s);
        a[2 * MLP_NH + i] = s * (1.0f - h1[i] * h1[i]);
    }
    a[4 * MLP_NH] = dy;
    a[4 * MLP_NH + 1] = w * r * r;
}

// One thread per parameter: its gradient summed over the minibatch rows in
// order; thread 0 of block 0 also sums the loss.
__global__ void k_mlp_grad(const float *X, const int *idx, int B, const float *act, float *grad,
                           float *loss)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_NPARAM) return;
    float g = 0.0f;
    if (k < MLP_OFF_B1) {
        const int u = k / MLP_NIN, i = k % MLP_NIN;
        for (int b = 0; b < B; ++b) {
            const int64_t row = idx ? idx[b] : b;
            g = fmaf(act[(int64_t)b * ACT + 2 * MLP_NH + u], X[row * MLP_NIN + i], g);
        }
    } else if (k < MLP_OFF_W2) {
        const int u = k - MLP_OFF_B1;
        for (int b = 0; b < B; ++b) g += act[(int64_t)b * ACT + 2 * MLP_NH + u];
    } else if (k < MLP_OFF_B2) {
        const int u = (k - MLP_OFF_W2) / MLP_NH, i = (k - MLP_OFF_W2) % MLP_NH;
        for (int b = 0; b < B; ++b)
            g = fmaf(act[(int64_t)b * ACT + 3 * MLP_NH + u], act[(int64_t)b * ACT + i], g);
    } else if (k < MLP_OFF_W3) {
        const int u = k - MLP_OFF_B2;
        for (int b = 0; b < B; ++b) g += act[(int64_t)b * ACT + 3 * MLP_NH + u];
    } else if (k < MLP_OFF_B3) {
        const int i = k - MLP_OFF_W3;
        for (int b = 0; b < B; ++b)
            g = fmaf(act[(int64_t)b * ACT + 4 * MLP_NH], act[(int64_t)b * ACT + MLP_NH + i], g);
    } else {
        for (int b = 0; b < B; ++b) g += act[(int64_t)b * ACT + 4 * MLP_NH];
    }
    grad[k] = g;
    if (k == 0 && loss) {
        float l = 0.0f;
        for (int b = 0; b < B; ++b) l += act[(int64_t)b * ACT + 4 * MLP_NH + 1];
        *loss = l / (float)B;
    }
}

// Adam (Kingma & Ba 2015, Algorithm 1), step t >= 1; accumulates the
// minibatch loss into *epoch_loss with weight 1/nb.
__global__ void k_adam(float *p, const float *g, float *m, float *v, int t, float lr, float b1,
                       float b2, float eps, const float *loss, float *epoch_loss, float inv_nb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0 && epoch_loss) *epoch_loss += *loss * inv_nb;
    if (k >= MLP_NPARAM) return;
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    const float mk = b1 * m[k] + (1.0f - b1) * g[k];
    const float vk = b2 * v[k] + (1.0f - b2) * g[k] * g[k];
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ void k_zero_f(float *x, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 0.0f;
}

namespace {
uint64_t splitmix_next(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }
}  // namespace

extern "C" int smol_proposer_set(const float *params, int32_t n_params, void *stream)
{
    if (!params || n_params != MLP_NPARAM) return SMOL_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    float *&w = g_mlp[dev];
    if (!w && hipMalloc(&w, sizeof(float) * MLP_NPARAM) != hipSuccess) {
        w = nullptr;
        return SMOL_ENOMEM;
    }
    HIP_TRY(hipMemcpyAsync(w, params, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    return SMOL_OK;
}

extern "C" int smol_proposer_forward(const float *params, const float *X, int64_t n_rows, float *Y,
                                     void *stream)
{
    if (!params || !X || !Y || n_rows < 0 || n_rows > (1LL << 30)) return SMOL_EINVAL;
    if (n_rows == 0) return SMOL_OK;
    hipLaunchKernelGGL(k_mlp_rows, dim3(blocks_for(n_rows, 64)), dim3(64), 0, (hipStream_t)stream,
                       params, X, (const float *)nullptr, (const int *)nullptr, (int)n_rows, 1.0f,
                       (float *)nullptr, Y);
    HIP_TRY(hipGetLastError());
    return SMOL_OK;
}

extern "C" int smol_proposer_loss_grad(const float *params, const float *X, const float *target,
                                       int64_t n_rows, float over_weight, float *loss, float *grad,
                                       void *stream)
{
    if (!params || !X || !target || !loss || !grad || n_rows < 1 || n_rows > (1LL << 24))
        return SMOL_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    float *act;
    if (hipMalloc(&act, sizeof(float) * ACT * n_rows) != hipSuccess) return SMOL_ENOMEM;
    hipLaunchKernelGGL(k_mlp_rows, dim3(blocks_for(n_rows, 64)), dim3(64), 0, s, params, X, target,
                       (const int *)nullptr, (int)n_rows, over_weight, act, (float *)nullptr);
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks_for(MLP_NPARAM, 256)), dim3(256), 0, s, X,
                       (const int *)nullptr, (int)n_rows, act, grad, loss);
    hipError_t e = hipGetLastError();
    (void)hipStreamSynchronize(s);
    (void)hipFree(act);
    if (e != hipSuccess) return hip_fail(e, "proposer_loss_grad");
    return SMOL_OK;
}

extern "C" int smol_proposer_train(const float *X, const float *target, int64_t n_rows,
                                   float *params, int32_t epochs, int32_t batch, float lr,
                                   float over_weight, uint64_t seed, float *loss_out, void *stream)
{
    if (!X || !target || !params || !loss_out || n_rows < 1 || epochs < 1 || batch < 1 ||
        n_rows > (1LL << 30) || !(lr > 0))
        return SMOL_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int B = (int)(batch < n_rows ? batch : n_rows);
    const int64_t nb = n_rows / B;  // full minibatches per epoch
    float *work = nullptr;
    int *idx = nullptr;
    const size_t nf = (size_t)ACT * B + 3 * MLP_NPARAM + 1;
    if (hipMalloc(&work, sizeof(float) * nf) != hipSuccess) return SMOL_ENOMEM;
    if (hipMalloc(&idx, sizeof(int) * n_rows) != hipSuccess) {
        (void)hipFree(work);
        return SMOL_ENOMEM;
    }
    float *act = work, *grad = act + (size_t)ACT * B, *m = grad + MLP_NPARAM, *v = m + MLP_NPARAM;
    float *loss = v + MLP_NPARAM;
    hipLaunchKernelGGL(k_zero_f, dim3(64), dim3(256), 0, s, m, (int64_t)2 * MLP_NPARAM);
    hipLaunchKernelGGL(k_zero_f, dim3(1), dim3(256), 0, s, loss_out, (int64_t)epochs);
    std::vector<int> perm(n_rows);
    uint64_t st = seed;
    int t = 0, rc = SMOL_OK;
    for (int ep = 0; ep < epochs && rc == SMOL_OK; ++ep) {
        for (int64_t i = 0; i < n_rows; ++i) perm[i] = (int)i;
        for (int64_t i = n_rows - 1; i > 0; --i) {  // Fisher-Yates with SplitMix64
            const int64_t j = (int64_t)(splitmix_next(st) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        if (hipMemcpyAsync(idx, perm.data(), sizeof(int) * n_rows, hipMemcpyHostToDevice, s) ||
            hipStreamSynchronize(s)) {
            rc = SMOL_EDEVICE;
            break;
        }
        for (int64_t q = 0; q < nb; ++q) {
            const int *bi = idx + q * B;
            hipLaunchKernelGGL(k_mlp_rows, dim3(blocks_for(B, 64)), dim3(64), 0, s, params, X, target,
                               bi, B, over_weight, act, (float *)nullptr);
            hipLaunchKernelGGL(k_mlp_grad, dim3(blocks_for(MLP_NPARAM, 256)), dim3(256), 0, s, X, bi,
                               B, act, grad, loss);
            hipLaunchKernelGGL(k_adam, dim3(blocks_for(MLP_NPARAM, 256)), dim3(256), 0, s, params,
                               grad, m, v, ++t, lr, 0.9f, 0.999f, 1e-8f, loss, loss_out + ep,
                               1.0f / (float)nb);
        }
        if (hipGetLastError() != hipSuccess) rc = SMOL_EDEVICE;
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(work);
    (void)hipFree(idx);
    return rc;
}

extern "C" int smol_proposer_dataset(const double *log, int64_t rows, int32_t method,
                                     double err_target, float *X, float *target, int64_t *n_out,
                                     void *stream)
{
    if (!log || !X || !target || !n_out || rows < 0 || rows > (1LL << 30)) return SMOL_EINVAL;
    if (!(err_target > 0.0) || !(err_target <= 1.0)) return SMOL_EINVAL;
    if (check_method(method)) return SMOL_EINVAL;
    *n_out = 0;
    if (rows < 2) return SMOL_OK;
    hipStream_t s = (hipStream_t)stream;
    const int nb = blocks_for(rows, SMOL_WG);
    int *flag = nullptr;
    int64_t *off = nullptr;
    if (hipMalloc(&flag, sizeof(int) * (rows + nb)) != hipSuccess) return SMOL_ENOMEM;
    if (hipMalloc(&off, sizeof(int64_t) * nb) != hipSuccess) {
        (void)hipFree(flag);
        return SMOL_ENOMEM;
    }
    int *count = flag + rows;
    std::vector<int> hc(nb);
    std::vector<int64_t> ho(nb);
    int rc = SMOL_OK;
    hipLaunchKernelGGL(k_dataset_flags, dim3(nb), dim3(SMOL_WG), 0, s, log, rows, flag, count);
    if (hipMemcpyAsync(hc.data(), count, sizeof(int) * nb, hipMemcpyDeviceToHost, s) ||
        hipStreamSynchronize(s)) {
        rc = SMOL_EDEVICE;
    } else {
        int64_t o = 0;
        for (int b = 0; b < nb; ++b) {
            ho[b] = o;
            o += hc[b];
        }
        *n_out = o;
        if (hipMemcpyAsync(off, ho.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, s)) rc = SMOL_EDEVICE;
        const int k = k_scheme_q[method] + 1;
        hipLaunchKernelGGL(k_dataset_rows, dim3(nb), dim3(SMOL_WG), 0, s, log, rows, k, err_target,
                           flag, off, X, target);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s)) rc = SMOL_EDEVICE;
    }
    (void)hipFree(flag);
    (void)hipFree(off);
    return rc;
}
