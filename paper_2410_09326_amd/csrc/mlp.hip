// Learned cost model: a 3-layer perceptron (64 -> 128 -> 128 -> 1, ReLU)
// that predicts the log run time of a fused pass from its 64 features.  The
// network is trained on the GPU by the kernels below (forward, backward of an
// MSE loss, Adam), all with fixed summation orders, so a training run is
// bitwise reproducible.  Used to price candidate plans (profile-guided
// activation of an optimisation, paper Sec. III-D).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <random>
#include <string>
#include <vector>

#include "mlp.hpp"
#include "runtime.hpp"

using namespace qops;

namespace qops {

// C[M x N] = A' B' (+ bias[N]) where A' = A (M x K, lda) or A^T (A is K x M),
// B' = B (K x N) or B^T (B is N x K).  16 x 16 output tiles, K staged through
// LDS in chunks of 16; every output is summed in k order.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_kernel(const float* __restrict__ A, const float* __restrict__ B,
                                                    const float* __restrict__ bias, float* __restrict__ C, int M,
                                                    int N, int K, int lda, int ldb, int ldc, int accumulate)
{
    __shared__ float As[16][17];
    __shared__ float Bs[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
    float acc = 0.f;
    for (int k0 = 0; k0 < K; k0 += 16) {
        // As[ty][tx] = A'(row, k0 + tx); Bs[ty][tx] = B'(k0 + ty, col)
        {
            const int r = blockIdx.y * 16 + ty, kk = k0 + tx;
            float v = 0.f;
            if (r < M && kk < K) v = TA ? A[(size_t)kk * lda + r] : A[(size_t)r * lda + kk];
            As[ty][tx] = v;
        }
        {
            const int kk = k0 + ty, c = blockIdx.x * 16 + tx;
            float v = 0.f;
            if (kk < K && c < N) v = TB ? B[(size_t)c * ldb + kk] : B[(size_t)kk * ldb + c];
            Bs[ty][tx] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) acc = fmaf(As[ty][kk], Bs[kk][tx], acc);
        __syncthreads();
    }
    if (row < M && col < N) {
        float v = acc + (bias ? bias[col] : 0.f);
        if (accumulate) v += C[(size_t)row * ldc + col];
        C[(size_t)row * ldc + col] = v;
    }
}

__global__ void relu_kernel(const float* __restrict__ z, float* __restrict__ h, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) h[i] = z[i] > 0.f ? z[i] : 0.f;
}

// d <- d * (z > 0)
__global__ void relu_back_kernel(const float* __restrict__ z, float* __restrict__ d, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (!(z[i] > 0.f)) d[i] = 0.f;
}

// dy[i] = 2 (y[i] - t[i]) / B; loss = (1/B) sum (y - t)^2 (single block, fixed order)
__global__ void __launch_bounds__(256) mse_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                   float* __restrict__ dy, float* __restrict__ loss, int B)
{
    __shared__ float sh[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < B; i += 256) {
        const float e = y[i] - t[i];
        dy[i] = 2.f * e / (float)B;
        s += e * e;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = sh[0] / (float)B;
}

// out[c] = sum_r D[r * ld + c] (column sums in row order)
__global__ void colsum_kernel(const float* __restrict__ D, float* __restrict__ out, int rows, int cols, int ld)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += D[(size_t)r * ld + c];
    out[c] = s;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// dst[r, :] = (src[idx[r], :] - mu) / sd   (feature standardisation + batch gather)
__global__ void gather_norm_kernel(const float* __restrict__ src, const int* __restrict__ idx,
                                   const float* __restrict__ mu, const float* __restrict__ sd, float* __restrict__ dst,
                                   int rows, int f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * f) return;
    const int r = i / f, c = i % f;
    const int s = idx ? idx[r] : r;
    dst[i] = (src[(size_t)s * f + c] - mu[c]) / sd[c];
}

__global__ void gather_kernel(const float* __restrict__ src, const int* __restrict__ idx, float* __restrict__ dst,
                              int rows)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < rows) dst[i] = src[idx[i]];
}

static unsigned blocks_for(int n) { return (unsigned)std::min(4096, (n + 255) / 256); }

template <bool TA, bool TB>
static void gemm(const float* A, const float* B, const float* bias, float* C, int M, int N, int K, int lda, int ldb,
                 int ldc, bool acc, hipStream_t s)
{
    dim3 grid((N + 15) / 16, (M + 15) / 16);
    hipLaunchKernelGGL((gemm_kernel<TA, TB>), grid, dim3(256), 0, s, A, B, bias, C, M, N, K, lda, ldb, ldc, acc ? 1 : 0);
}

}  // namespace qops

// Parameter layout (float): W1 [128 x 64], b1 [128], W2 [128 x 128], b2 [128],
// W3 [1 x 128], b3 [1].
static constexpr int F = qops::kNumFeatures, H = 128;
static constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * F, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
                     OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H, NPARAM = OFF_B3 + 1;

struct MlpWork {
    int cap = 0;
    float *X = nullptr, *t = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *y = nullptr,
          *dy = nullptr, *D2 = nullptr, *D1 = nullptr, *loss = nullptr;
};

struct qops_model {
    std::vector<float> params;          // host copy
    float mu[F], sd[F];                 // feature standardisation
    float* d_p = nullptr;               // device parameters
    float* d_g = nullptr;               // gradients
    float* d_m = nullptr;               // Adam moments
    float* d_v = nullptr;
    float* d_mu = nullptr;
    float* d_sd = nullptr;
    MlpWork w;
    int adam_step = 0;
};

namespace qops {

static hipError_t mlp_alloc(qops_model* m)
{
    hipError_t e = hipSuccess;
    auto a = [&](float*& p, size_t n) {
        if (e == hipSuccess && !p) e = hipMalloc(&p, n * sizeof(float));
    };
    a(m->d_p, NPARAM);
    a(m->d_g, NPARAM);
    a(m->d_m, NPARAM);
    a(m->d_v, NPARAM);
    a(m->d_mu, F);
    a(m->d_sd, F);
    return e;
}

static hipError_t mlp_work(qops_model* m, int rows)
{
    if (m->w.cap >= rows) return hipSuccess;
    MlpWork& w = m->w;
    float** bufs[] = {&w.X, &w.t, &w.Z1, &w.H1, &w.Z2, &w.H2, &w.y, &w.dy, &w.D2, &w.D1, &w.loss};
    for (float** b : bufs)
        if (*b) {
            (void)hipFree(*b);
            *b = nullptr;
        }
    hipError_t e = hipSuccess;
    auto a = [&](float*& p, size_t n) {
        if (e == hipSuccess) e = hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(float));
    };
    a(w.X, (size_t)rows * F);
    a(w.t, rows);
    a(w.Z1, (size_t)rows * H);
    a(w.H1, (size_t)rows * H);
    a(w.Z2, (size_t)rows * H);
    a(w.H2, (size_t)rows * H);
    a(w.y, rows);
    a(w.dy, rows);
    a(w.D2, (size_t)rows * H);
    a(w.D1, (size_t)rows * H);
    a(w.loss, 1);
    if (e == hipSuccess) w.cap = rows;
    return e;
}

static hipError_t upload_params(qops_model* m)
{
    hipError_t e = hipMemcpy(m->d_p, m->params.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_mu, m->mu, F * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_sd, m->sd, F * sizeof(float), hipMemcpyHostToDevice);
    return e;
}

// Forward on the standardised batch in w.X (rows x F); output in w.y.
static void forward(qops_model* m, int rows, hipStream_t s)
{
    MlpWork& w = m->w;
    const float* P = m->d_p;
    gemm<false, true>(w.X, P + OFF_W1, P + OFF_B1, w.Z1, rows, H, F, F, F, H, false, s);
    hipLaunchKernelGGL(relu_kernel, dim3(blocks_for(rows * H)), dim3(256), 0, s, w.Z1, w.H1, rows * H);
    gemm<false, true>(w.H1, P + OFF_W2, P + OFF_B2, w.Z2, rows, H, H, H, H, H, false, s);
    hipLaunchKernelGGL(relu_kernel, dim3(blocks_for(rows * H)), dim3(256), 0, s, w.Z2, w.H2, rows * H);
    gemm<false, true>(w.H2, P + OFF_W3, P + OFF_B3, w.y, rows, 1, H, H, H, 1, false, s);
}

// Loss and gradients (into d_g) for targets in w.t.
static void backward(qops_model* m, int rows, hipStream_t s)
{
    MlpWork& w = m->w;
    const float* P = m->d_p;
    float* G = m->d_g;
    hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(256), 0, s, w.y, w.t, w.dy, w.loss, rows);
    // layer 3: gW3 = dy^T H2 (1 x H), gb3 = sum dy
    gemm<true, false>(w.dy, w.H2, nullptr, G + OFF_W3, 1, H, rows, 1, H, H, false, s);
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(64), 0, s, w.dy, G + OFF_B3, rows, 1, 1);
    // dH2 = dy W3 (rows x H), masked by Z2 > 0
    gemm<false, false>(w.dy, P + OFF_W3, nullptr, w.D2, rows, H, 1, 1, H, H, false, s);
    hipLaunchKernelGGL(relu_back_kernel, dim3(blocks_for(rows * H)), dim3(256), 0, s, w.Z2, w.D2, rows * H);
    // layer 2: gW2 = D2^T H1, gb2 = colsum D2, dH1 = D2 W2 masked by Z1 > 0
    gemm<true, false>(w.D2, w.H1, nullptr, G + OFF_W2, H, H, rows, H, H, H, false, s);
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(H), 0, s, w.D2, G + OFF_B2, rows, H, H);
    gemm<false, false>(w.D2, P + OFF_W2, nullptr, w.D1, rows, H, H, H, H, H, false, s);
    hipLaunchKernelGGL(relu_back_kernel, dim3(blocks_for(rows * H)), dim3(256), 0, s, w.Z1, w.D1, rows * H);
    // layer 1: gW1 = D1^T X, gb1 = colsum D1
    gemm<true, false>(w.D1, w.X, nullptr, G + OFF_W1, H, F, rows, H, F, F, false, s);
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(H), 0, s, w.D1, G + OFF_B1, rows, H, H);
}

}  // namespace qops

#define MLP_HIP(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return hip_fail(_e, #expr); \
    } while (0)

extern "C" {

int32_t qops_mlp_create(const float* params, size_t n, qops_model** out)
{
    if (!out) return set_error(QOPS_INVALID_ARG, "out is null");
    *out = nullptr;
    if (params && n != (size_t)NPARAM)
        return set_error(QOPS_INVALID_ARG, "expected " + std::to_string(NPARAM) + " parameters");
    std::unique_ptr<qops_model> m(new qops_model());
    m->params.assign(NPARAM, 0.f);
    if (params) std::memcpy(m->params.data(), params, NPARAM * sizeof(float));
    for (int i = 0; i < F; ++i) {
        m->mu[i] = 0.f;
        m->sd[i] = 1.f;
    }
    *out = m.release();
    return QOPS_OK;
}

int32_t qops_mlp_num_params(size_t* n)
{
    if (!n) return set_error(QOPS_INVALID_ARG, "null argument");
    *n = NPARAM;
    return QOPS_OK;
}

int32_t qops_mlp_get_params(const qops_model* m, float* params, float* mu, float* sd)
{
    if (!m) return set_error(QOPS_INVALID_ARG, "null model");
    if (params) std::memcpy(params, m->params.data(), NPARAM * sizeof(float));
    if (mu) std::memcpy(mu, m->mu, F * sizeof(float));
    if (sd) std::memcpy(sd, m->sd, F * sizeof(float));
    return QOPS_OK;
}

int32_t qops_mlp_set_normalization(qops_model* m, const float* mu, const float* sd)
{
    if (!m || !mu || !sd) return set_error(QOPS_INVALID_ARG, "null argument");
    for (int i = 0; i < F; ++i) {
        if (!(sd[i] > 0.f)) return set_error(QOPS_INVALID_ARG, "standard deviations must be positive");
        m->mu[i] = mu[i];
        m->sd[i] = sd[i];
    }
    return QOPS_OK;
}

int32_t qops_mlp_grad(qops_model* m, const float* X, const float* t, int32_t rows, float* grads, float* loss)
{
    if (!m || !X || !t || rows < 1) return set_error(QOPS_INVALID_ARG, "bad arguments");
    MLP_HIP(mlp_alloc(m));
    MLP_HIP(mlp_work(m, rows));
    MLP_HIP(upload_params(m));
    MlpWork& w = m->w;
    std::vector<float> Xs((size_t)rows * F);
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < F; ++c) Xs[(size_t)r * F + c] = (X[(size_t)r * F + c] - m->mu[c]) / m->sd[c];
    MLP_HIP(hipMemcpy(w.X, Xs.data(), Xs.size() * sizeof(float), hipMemcpyHostToDevice));
    MLP_HIP(hipMemcpy(w.t, t, rows * sizeof(float), hipMemcpyHostToDevice));
    forward(m, rows, nullptr);
    backward(m, rows, nullptr);
    MLP_HIP(hipGetLastError());
    MLP_HIP(hipDeviceSynchronize());
    if (grads) MLP_HIP(hipMemcpy(grads, m->d_g, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    if (loss) MLP_HIP(hipMemcpy(loss, w.loss, sizeof(float), hipMemcpyDeviceToHost));
    return QOPS_OK;
}

int32_t qops_mlp_predict(qops_model* m, const float* X, int32_t rows, float* out)
{
    if (!m || !X || !out || rows < 0) return set_error(QOPS_INVALID_ARG, "bad arguments");
    if (rows == 0) return QOPS_OK;
    MLP_HIP(mlp_alloc(m));
    MLP_HIP(mlp_work(m, rows));
    MLP_HIP(upload_params(m));
    MlpWork& w = m->w;
    std::vector<float> Xs((size_t)rows * F);
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < F; ++c) Xs[(size_t)r * F + c] = (X[(size_t)r * F + c] - m->mu[c]) / m->sd[c];
    MLP_HIP(hipMemcpy(w.X, Xs.data(), Xs.size() * sizeof(float), hipMemcpyHostToDevice));
    forward(m, rows, nullptr);
    MLP_HIP(hipGetLastError());
    MLP_HIP(hipMemcpy(out, w.y, rows * sizeof(float), hipMemcpyDeviceToHost));
    return QOPS_OK;
}

int32_t qops_mlp_train(qops_model* m, const float* X, const float* t, int32_t rows, int32_t epochs, int32_t batch,
                       float lr, uint64_t seed, float* final_loss)
{
    if (!m || !X || !t || rows < 1 || epochs < 1 || batch < 1) return set_error(QOPS_INVALID_ARG, "bad arguments");
    batch = std::min(batch, (int)rows);
    MLP_HIP(mlp_alloc(m));
    MLP_HIP(mlp_work(m, batch));
    MLP_HIP(upload_params(m));
    MLP_HIP(hipMemset(m->d_m, 0, NPARAM * sizeof(float)));
    MLP_HIP(hipMemset(m->d_v, 0, NPARAM * sizeof(float)));
    m->adam_step = 0;
    float *dX = nullptr, *dT = nullptr;
    int* didx = nullptr;
    MLP_HIP(hipMalloc(&dX, (size_t)rows * F * sizeof(float)));
    MLP_HIP(hipMalloc(&dT, (size_t)rows * sizeof(float)));
    MLP_HIP(hipMalloc(&didx, (size_t)rows * sizeof(int)));
    MLP_HIP(hipMemcpy(dX, X, (size_t)rows * F * sizeof(float), hipMemcpyHostToDevice));
    MLP_HIP(hipMemcpy(dT, t, (size_t)rows * sizeof(float), hipMemcpyHostToDevice));
    std::vector<int> idx(rows);
    for (int i = 0; i < rows; ++i) idx[i] = i;
    std::mt19937_64 rng(seed);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    MlpWork& w = m->w;
    float last = 0.f;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = rows - 1; i > 0; --i) std::swap(idx[i], idx[(size_t)(rng() % (uint64_t)(i + 1))]);
        MLP_HIP(hipMemcpy(didx, idx.data(), rows * sizeof(int), hipMemcpyHostToDevice));
        for (int b0 = 0; b0 + batch <= rows; b0 += batch) {
            hipLaunchKernelGGL(gather_norm_kernel, dim3((batch * F + 255) / 256), dim3(256), 0, nullptr, dX, didx + b0,
                               m->d_mu, m->d_sd, w.X, batch, F);
            hipLaunchKernelGGL(gather_kernel, dim3((batch + 255) / 256), dim3(256), 0, nullptr, dT, didx + b0, w.t,
                               batch);
            forward(m, batch, nullptr);
            backward(m, batch, nullptr);
            ++m->adam_step;
            const float c1 = 1.f - std::pow(b1, (float)m->adam_step), c2 = 1.f - std::pow(b2, (float)m->adam_step);
            hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(NPARAM)), dim3(256), 0, nullptr, m->d_p, m->d_g, m->d_m,
                               m->d_v, NPARAM, lr, b1, b2, eps, c1, c2);
        }
        MLP_HIP(hipGetLastError());
        MLP_HIP(hipMemcpy(&last, w.loss, sizeof(float), hipMemcpyDeviceToHost));
    }
    MLP_HIP(hipDeviceSynchronize());
    MLP_HIP(hipMemcpy(m->params.data(), m->d_p, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    (void)hipFree(dX);
    (void)hipFree(dT);
    (void)hipFree(didx);
    if (final_loss) *final_loss = last;
    return QOPS_OK;
}

int32_t qops_model_save(const qops_model* m, const char* path)
{
    if (!m || !path) return set_error(QOPS_INVALID_ARG, "null argument");
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(QOPS_INVALID_ARG, std::string("cannot open ") + path);
    const char magic[8] = {'Q', 'O', 'P', 'S', 'M', 'L', 'P', '1'};
    const int32_t np = NPARAM, nf = F;
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&np, 4, 1, f) == 1 && std::fwrite(&nf, 4, 1, f) == 1 &&
              std::fwrite(m->mu, 4, F, f) == (size_t)F && std::fwrite(m->sd, 4, F, f) == (size_t)F &&
              std::fwrite(m->params.data(), 4, NPARAM, f) == (size_t)NPARAM;
    std::fclose(f);
    return ok ? QOPS_OK : set_error(QOPS_INVALID_ARG, "write failed");
}

int32_t qops_model_load(const char* path, qops_model** out)
{
    if (!path || !out) return set_error(QOPS_INVALID_ARG, "null argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(QOPS_INVALID_ARG, std::string("cannot open ") + path);
    char magic[8];
    int32_t np = 0, nf = 0;
    std::unique_ptr<qops_model> m(new qops_model());
    m->params.assign(NPARAM, 0.f);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "QOPSMLP1", 8) == 0 && std::fread(&np, 4, 1, f) == 1 &&
              std::fread(&nf, 4, 1, f) == 1 && np == NPARAM && nf == F && std::fread(m->mu, 4, F, f) == (size_t)F &&
              std::fread(m->sd, 4, F, f) == (size_t)F && std::fread(m->params.data(), 4, NPARAM, f) == (size_t)NPARAM;
    std::fclose(f);
    if (!ok) return set_error(QOPS_INVALID_ARG, "not a qops model file");
    *out = m.release();
    return QOPS_OK;
}

int32_t qops_model_free(qops_model* m)
{
    if (!m) return QOPS_OK;
    float* ptrs[] = {m->d_p, m->d_g, m->d_m, m->d_v, m->d_mu, m->d_sd, m->w.X, m->w.t, m->w.Z1, m->w.H1, m->w.Z2,
                     m->w.H2, m->w.y, m->w.dy, m->w.D2, m->w.D1, m->w.loss};
    for (float* p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
    return QOPS_OK;
}

}  // extern "C"

namespace qops {

// Host-side prediction for plan pricing (no GPU round trip): the same
// network evaluated in FP32 on the CPU of the planner.
void mlp_predict_host(const qops_model* m, const float* f, int rows, float* out)
{
    const float* P = m->params.data();
    std::vector<float> x(F), h1(H), h2(H);
    for (int r = 0; r < rows; ++r) {
        for (int c = 0; c < F; ++c) x[c] = (f[(size_t)r * F + c] - m->mu[c]) / m->sd[c];
        for (int i = 0; i < H; ++i) {
            float s = 0.f;
            for (int c = 0; c < F; ++c) s = fmaf(x[c], P[OFF_W1 + i * F + c], s);
            s += P[OFF_B1 + i];
            h1[i] = s > 0.f ? s : 0.f;
        }
        for (int i = 0; i < H; ++i) {
            float s = 0.f;
            for (int c = 0; c < H; ++c) s = fmaf(h1[c], P[OFF_W2 + i * H + c], s);
            s += P[OFF_B2 + i];
            h2[i] = s > 0.f ? s : 0.f;
        }
        float y = 0.f;
        for (int c = 0; c < H; ++c) y = fmaf(h2[c], P[OFF_W3 + c], y);
        out[r] = y + P[OFF_B3];
    }
}

}  // namespace qops
