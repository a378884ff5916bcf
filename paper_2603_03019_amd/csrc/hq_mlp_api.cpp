// Host side of the learned warm start: feature extraction, the MLP handle,
// GPU training (forward, backward and Adam in HIP kernels) and inference.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "hq.h"

namespace hqk {
hipError_t mlp_gemm(bool ta, bool tb, const uint16_t* A, const uint16_t* B, float* C, int M, int N, int K, int lda,
                    int ldb, int ldc, bool accumulate, hipStream_t s);
hipError_t mlp_bias_relu(const float* z, const float* bias, float* pre, uint16_t* hb, int rows, int cols,
                         hipStream_t s);
hipError_t mlp_head_forward(const uint16_t* h2, const float* w3, const float* b3, const float* target, float* y,
                            float* dz, float* loss_terms, int rows, int valid, int cols, hipStream_t s);
hipError_t mlp_head_backward(const uint16_t* h2, const float* dz, float* dw3, float* db3, int rows, int cols,
                             hipStream_t s);
hipError_t mlp_head_to_hidden(const float* dz, const float* w3, const float* pre, uint16_t* dhb, float* dh, int rows,
                              int cols, hipStream_t s);
hipError_t mlp_relu_backward(const float* gin, const float* pre, float* g, uint16_t* gb, int n, hipStream_t s);
hipError_t mlp_col_sum(const float* g, float* db, int rows, int cols, hipStream_t s);
hipError_t mlp_adam(float* p, const float* g, float* m1, float* m2, uint16_t* pb, int n, float lr, float b1,
                    float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t mlp_to_bf16(const float* src, uint16_t* dst, int n, hipStream_t s);
}  // namespace hqk

// set by the solver translation unit (thread-local last error)
void hq_set_error(const std::string& msg);

namespace {

constexpr int IN = HQ_MLP_IN, HID = HQ_MLP_HIDDEN;
// packed parameter vector: W1 [IN x HID], b1 [HID], W2 [HID x HID], b2 [HID], w3 [HID], b3 [1]
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + IN * HID, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == HQ_MLP_PARAMS, "parameter count");

struct HipErr {
    hipError_t e;
    const char* what;
};
#define MLP_HIP(call)                                  \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) throw HipErr{_e, #call}; \
    } while (0)

template <typename T>
T* dal(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    return (T*)p;
}

hq_status err(hq_status s, const std::string& m) {
    hq_set_error(m);
    return s;
}

}  // namespace

struct hq_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    float *p = nullptr, *m1 = nullptr, *m2 = nullptr, *g = nullptr;
    uint16_t* pb = nullptr;  // BF16 mirror of the packed parameters
    long step = 0;
    // per-batch workspace (capacity rows)
    int cap = 0;
    float *xf = nullptr, *t = nullptr, *z = nullptr, *pre1 = nullptr, *pre2 = nullptr, *y = nullptr, *dz = nullptr,
          *lt = nullptr, *dh2 = nullptr, *dh1 = nullptr;
    uint16_t *xb = nullptr, *h1b = nullptr, *h2b = nullptr, *dh2b = nullptr, *dh1b = nullptr;

    ~hq_mlp() {
        void* ptrs[] = {p, m1, m2, g, pb, xf, t, z, pre1, pre2, y, dz, lt, dh2, dh1, xb, h1b, h2b, dh2b, dh1b};
        for (void* q : ptrs)
            if (q) (void)hipFree(q);
        if (stream) (void)hipStreamDestroy(stream);
    }
    void reserve(int rows) {
        if (rows <= cap) return;
        void* ptrs[] = {xf, t, z, pre1, pre2, y, dz, lt, dh2, dh1, xb, h1b, h2b, dh2b, dh1b};
        for (void* q : ptrs)
            if (q) (void)hipFree(q);
        cap = rows;
        xf = dal<float>((size_t)rows * IN);
        t = dal<float>(rows);
        z = dal<float>((size_t)rows * HID);
        pre1 = dal<float>((size_t)rows * HID);
        pre2 = dal<float>((size_t)rows * HID);
        y = dal<float>(rows);
        dz = dal<float>(rows);
        lt = dal<float>(rows);
        dh2 = dal<float>((size_t)rows * HID);
        dh1 = dal<float>((size_t)rows * HID);
        xb = dal<uint16_t>((size_t)rows * IN);
        h1b = dal<uint16_t>((size_t)rows * HID);
        h2b = dal<uint16_t>((size_t)rows * HID);
        dh2b = dal<uint16_t>((size_t)rows * HID);
        dh1b = dal<uint16_t>((size_t)rows * HID);
    }
};

namespace {

// Forward pass of `rows` (multiple of 32) rows already in m->xf; with
// targets (valid rows < rows are padding) also the loss terms and dL/dz.
void forward(hq_mlp* m, int rows, const float* target, int valid) {
    hipStream_t s = m->stream;
    MLP_HIP(hqk::mlp_to_bf16(m->xf, m->xb, rows * IN, s));
    MLP_HIP(hqk::mlp_gemm(false, false, m->xb, m->pb + OFF_W1, m->z, rows, HID, IN, IN, HID, HID, false, s));
    MLP_HIP(hqk::mlp_bias_relu(m->z, m->p + OFF_B1, m->pre1, m->h1b, rows, HID, s));
    MLP_HIP(hqk::mlp_gemm(false, false, m->h1b, m->pb + OFF_W2, m->z, rows, HID, HID, HID, HID, HID, false, s));
    MLP_HIP(hqk::mlp_bias_relu(m->z, m->p + OFF_B2, m->pre2, m->h2b, rows, HID, s));
    MLP_HIP(hqk::mlp_head_forward(m->h2b, m->p + OFF_W3, m->p + OFF_B3, target, m->y, m->dz, m->lt, rows, valid,
                                  HID, s));
}

// Backward pass into the packed gradient m->g (after forward with targets).
void backward(hq_mlp* m, int rows) {
    hipStream_t s = m->stream;
    float* g = m->g;
    MLP_HIP(hqk::mlp_head_backward(m->h2b, m->dz, g + OFF_W3, g + OFF_B3, rows, HID, s));
    MLP_HIP(hqk::mlp_head_to_hidden(m->dz, m->p + OFF_W3, m->pre2, m->dh2b, m->dh2, rows, HID, s));
    // dW2 = H1^T dH2 ; db2 = colsum dH2
    MLP_HIP(hqk::mlp_gemm(true, false, m->h1b, m->dh2b, g + OFF_W2, HID, HID, rows, HID, HID, HID, false, s));
    MLP_HIP(hqk::mlp_col_sum(m->dh2, g + OFF_B2, rows, HID, s));
    // dH1 = (dH2 W2^T) [pre1 > 0]
    MLP_HIP(hqk::mlp_gemm(false, true, m->dh2b, m->pb + OFF_W2, m->z, rows, HID, HID, HID, HID, HID, false, s));
    MLP_HIP(hqk::mlp_relu_backward(m->z, m->pre1, m->dh1, m->dh1b, rows * HID, s));
    // dW1 = X^T dH1 ; db1 = colsum dH1
    MLP_HIP(hqk::mlp_gemm(true, false, m->xb, m->dh1b, g + OFF_W1, IN, HID, rows, IN, HID, HID, false, s));
    MLP_HIP(hqk::mlp_col_sum(m->dh1, g + OFF_B1, rows, HID, s));
}

int pad32(int r) { return (r + 31) / 32 * 32; }

}  // namespace

// Features of each unit of an instance (scale-free; original unit order).
void hq_mlp_features_impl(int N, int J, const double* lam, const double* mu, const int32_t* pref, float* f) {
    double Lam = 0.0, M = 0.0, mx = 0.0;
    for (int j = 0; j < J; ++j) Lam += lam[j];
    for (int u = 0; u < N; ++u) {
        M += mu[u];
        mx = std::max(mx, mu[u]);
    }
    const double load = M > 0.0 ? Lam / M : 0.0;
    std::vector<double> share((size_t)N * 9, 0.0), expo(N, 0.0);
    if (Lam > 0.0)
        for (int j = 0; j < J; ++j) {
            const double w = lam[j] / Lam;
            double r = 1.0;
            for (int h = 0; h < N; ++h) {
                const int u = pref[(size_t)j * N + h];
                share[(size_t)u * 9 + std::min(h, 8)] += w;
                expo[u] += w * r;
                r *= load;
            }
        }
    // The independence approximation of the loss system's utilisations (in
    // the spirit of Larson's approximate hypercube): a call from node j
    // reaches its h-th unit when the units ranked before it are busy, taken
    // as independent with probabilities rho; unit u then receives
    // r_u = sum_j lambda_j prod_{i<h} rho_{pi_j[i]} while idle and is busy
    // with probability r_u / (r_u + nu_u).  60 plain fixed-point steps from
    // rho = min(load, 0.99).
    std::vector<double> rho(N, std::min(load, 0.99)), r(N, 0.0);
    for (int it = 0; it < 60; ++it) {
        std::fill(r.begin(), r.end(), 0.0);
        for (int j = 0; j < J; ++j) {
            double pr = 1.0;
            for (int h = 0; h < N; ++h) {
                const int u = pref[(size_t)j * N + h];
                r[u] += lam[j] * pr;
                pr *= rho[u];
            }
        }
        for (int u = 0; u < N; ++u) rho[u] = r[u] + mu[u] > 0.0 ? r[u] / (r[u] + mu[u]) : 0.0;
    }
    for (int u = 0; u < N; ++u) {
        float* x = f + (size_t)u * IN;
        for (int i = 0; i < IN; ++i) x[i] = 0.0f;
        x[0] = (float)(mu[u] / (M / N));
        for (int r = 0; r < 9; ++r) x[1 + r] = (float)share[(size_t)u * 9 + r];
        x[10] = (float)load;
        x[11] = (float)expo[u];
        x[12] = (float)(N / 32.0);
        x[13] = (float)(mu[u] / mx);
        x[14] = (float)(N * share[(size_t)u * 9 + 0]);
        x[15] = 1.0f;
        x[16] = (float)rho[u];
        x[17] = (float)(Lam > 0.0 ? r[u] / Lam : 0.0);
        const double lo = std::log(rho[u] / (1.0 - rho[u]));
        x[18] = (float)(std::min(8.0, std::max(-8.0, lo)) / 8.0);
    }
}

// Predicted utilisations for an instance (used by hq_create with HQ_INIT_LEARNED).
hq_status hq_mlp_predict_instance(const hq_mlp* mc, int N, int J, const double* lam, const double* mu,
                                  const int32_t* pref, std::vector<double>& rho) {
    std::vector<float> f((size_t)N * IN), y(N);
    hq_mlp_features_impl(N, J, lam, mu, pref, f.data());
    hq_status s = hq_mlp_forward(const_cast<hq_mlp*>(mc), f.data(), N, y.data());
    if (s != HQ_OK) return s;
    rho.resize(N);
    for (int u = 0; u < N; ++u) rho[u] = std::isfinite(y[u]) ? (double)y[u] : 0.5;
    return HQ_OK;
}

extern "C" {

hq_status hq_mlp_features(int N, int J, const double* lambda_j, const double* mu_i, const int32_t* pref_lists,
                          float* features) {
    if (N < 1 || N > HQ_MAX_N || J < 1 || !lambda_j || !mu_i || !pref_lists || !features)
        return err(HQ_ERR_INVALID_ARG, "bad arguments to hq_mlp_features");
    hq_mlp_features_impl(N, J, lambda_j, mu_i, pref_lists, features);
    return HQ_OK;
}

hq_status hq_mlp_create(int device, unsigned long long seed, hq_mlp** out) {
    if (!out) return err(HQ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    try {
        std::unique_ptr<hq_mlp> m(new hq_mlp());
        if (device >= 0) MLP_HIP(hipSetDevice(device));
        MLP_HIP(hipGetDevice(&m->device));
        MLP_HIP(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
        m->p = dal<float>(NPARAM);
        m->m1 = dal<float>(NPARAM);
        m->m2 = dal<float>(NPARAM);
        m->g = dal<float>(NPARAM);
        m->pb = dal<uint16_t>(NPARAM);
        // Glorot-uniform weights, zero biases
        std::mt19937_64 rng(seed);
        std::vector<float> p(NPARAM, 0.0f);
        auto fill = [&](int off, int fan_in, int fan_out, int n) {
            const double a = std::sqrt(6.0 / (fan_in + fan_out));
            std::uniform_real_distribution<double> U(-a, a);
            for (int i = 0; i < n; ++i) p[off + i] = (float)U(rng);
        };
        fill(OFF_W1, 16, HID, IN * HID);
        for (int r = 16; r < IN; ++r)
            for (int c = 0; c < HID; ++c) p[OFF_W1 + r * HID + c] = 0.0f;  // unused feature slots
        fill(OFF_W2, HID, HID, HID * HID);
        fill(OFF_W3, HID, 1, HID);
        MLP_HIP(hipMemcpyAsync(m->p, p.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice, m->stream));
        MLP_HIP(hipMemsetAsync(m->m1, 0, NPARAM * sizeof(float), m->stream));
        MLP_HIP(hipMemsetAsync(m->m2, 0, NPARAM * sizeof(float), m->stream));
        MLP_HIP(hqk::mlp_to_bf16(m->p, m->pb, NPARAM, m->stream));
        MLP_HIP(hipStreamSynchronize(m->stream));
        *out = m.release();
    } catch (const std::bad_alloc&) {
        return err(HQ_ERR_OUT_OF_MEMORY, "device allocation failed");
    } catch (const HipErr& e) {
        return err(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

void hq_mlp_destroy(hq_mlp* m) { delete m; }

hq_status hq_mlp_get_params(const hq_mlp* m, float* params) {
    if (!m || !params) return err(HQ_ERR_INVALID_ARG, "null argument");
    try {
        MLP_HIP(hipMemcpyAsync(params, m->p, NPARAM * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MLP_HIP(hipStreamSynchronize(m->stream));
    } catch (const HipErr& e) {
        return err(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

hq_status hq_mlp_set_params(hq_mlp* m, const float* params) {
    if (!m || !params) return err(HQ_ERR_INVALID_ARG, "null argument");
    for (int i = 0; i < NPARAM; ++i)
        if (!std::isfinite(params[i])) return err(HQ_ERR_INVALID_ARG, "parameters must be finite");
    try {
        MLP_HIP(hipMemcpyAsync(m->p, params, NPARAM * sizeof(float), hipMemcpyHostToDevice, m->stream));
        MLP_HIP(hqk::mlp_to_bf16(m->p, m->pb, NPARAM, m->stream));
        MLP_HIP(hipStreamSynchronize(m->stream));
    } catch (const HipErr& e) {
        return err(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

hq_status hq_mlp_forward(hq_mlp* m, const float* X, int rows, float* y) {
    if (!m || !X || !y || rows < 1) return err(HQ_ERR_INVALID_ARG, "bad arguments to hq_mlp_forward");
    try {
        MLP_HIP(hipSetDevice(m->device));
        const int R = pad32(rows);
        m->reserve(std::max(R, 32));
        MLP_HIP(hipMemsetAsync(m->xf, 0, (size_t)R * IN * sizeof(float), m->stream));
        MLP_HIP(hipMemcpyAsync(m->xf, X, (size_t)rows * IN * sizeof(float), hipMemcpyHostToDevice, m->stream));
        forward(m, R, nullptr, rows);
        MLP_HIP(hipMemcpyAsync(y, m->y, rows * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MLP_HIP(hipStreamSynchronize(m->stream));
    } catch (const std::bad_alloc&) {
        return err(HQ_ERR_OUT_OF_MEMORY, "device allocation failed");
    } catch (const HipErr& e) {
        return err(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

hq_status hq_mlp_gradient(hq_mlp* m, const float* X, const float* t, int rows, float* grad, float* loss) {
    if (!m || !X || !t || !grad || rows < 1) return err(HQ_ERR_INVALID_ARG, "bad arguments to hq_mlp_gradient");
    try {
        MLP_HIP(hipSetDevice(m->device));
        const int R = pad32(rows);
        m->reserve(std::max(R, 32));
        MLP_HIP(hipMemsetAsync(m->xf, 0, (size_t)R * IN * sizeof(float), m->stream));
        MLP_HIP(hipMemsetAsync(m->t, 0, (size_t)R * sizeof(float), m->stream));
        MLP_HIP(hipMemcpyAsync(m->xf, X, (size_t)rows * IN * sizeof(float), hipMemcpyHostToDevice, m->stream));
        MLP_HIP(hipMemcpyAsync(m->t, t, (size_t)rows * sizeof(float), hipMemcpyHostToDevice, m->stream));
        forward(m, R, m->t, rows);
        backward(m, R);
        std::vector<float> lt(R);
        MLP_HIP(hipMemcpyAsync(grad, m->g, NPARAM * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MLP_HIP(hipMemcpyAsync(lt.data(), m->lt, R * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MLP_HIP(hipStreamSynchronize(m->stream));
        if (loss) {
            double s = 0.0;
            for (int i = 0; i < rows; ++i) s += lt[i];
            *loss = (float)(s / rows);
        }
    } catch (const std::bad_alloc&) {
        return err(HQ_ERR_OUT_OF_MEMORY, "device allocation failed");
    } catch (const HipErr& e) {
        return err(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

hq_status hq_mlp_train(hq_mlp* m, const float* X, const float* t, int rows, int epochs, int batch, float lr,
                       unsigned long long seed, float* epoch_loss) {
    if (!m || !X || !t || rows < 1 || epochs < 0 || batch < 32 || batch % 32 || !(lr > 0.0f))
        return err(HQ_ERR_INVALID_ARG, "bad arguments to hq_mlp_train (batch must be a positive multiple of 32)");
    try {
        MLP_HIP(hipSetDevice(m->device));
        m->reserve(batch);
        std::mt19937_64 rng(seed);
        std::vector<int> perm(rows);
        for (int i = 0; i < rows; ++i) perm[i] = i;
        std::vector<float> xb((size_t)batch * IN), tb(batch), lt(batch);
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        for (int ep = 0; ep < epochs; ++ep) {
            std::shuffle(perm.begin(), perm.end(), rng);
            double lsum = 0.0;
            for (int s0 = 0; s0 < rows; s0 += batch) {
                const int valid = std::min(batch, rows - s0);
                std::fill(xb.begin(), xb.end(), 0.0f);
                std::fill(tb.begin(), tb.end(), 0.0f);
                for (int i = 0; i < valid; ++i) {
                    std::memcpy(&xb[(size_t)i * IN], X + (size_t)perm[s0 + i] * IN, IN * sizeof(float));
                    tb[i] = t[perm[s0 + i]];
                }
                const int R = pad32(valid);
                MLP_HIP(hipMemcpyAsync(m->xf, xb.data(), (size_t)R * IN * sizeof(float), hipMemcpyHostToDevice,
                                       m->stream));
                MLP_HIP(hipMemcpyAsync(m->t, tb.data(), (size_t)R * sizeof(float), hipMemcpyHostToDevice, m->stream));
                forward(m, R, m->t, valid);
                backward(m, R);
                ++m->step;
                const float c1 = 1.0f - std::pow(b1, (float)m->step), c2 = 1.0f - std::pow(b2, (float)m->step);
                MLP_HIP(hqk::mlp_adam(m->p, m->g, m->m1, m->m2, m->pb, NPARAM, lr, b1, b2, eps, c1, c2, m->stream));
                MLP_HIP(hipMemcpyAsync(lt.data(), m->lt, R * sizeof(float), hipMemcpyDeviceToHost, m->stream));
                MLP_HIP(hipStreamSynchronize(m->stream));
                for (int i = 0; i < valid; ++i) lsum += lt[i];
            }
            if (epoch_loss) epoch_loss[ep] = (float)(lsum / rows);
        }
    } catch (const std::bad_alloc&) {
        return err(HQ_ERR_OUT_OF_MEMORY, "device allocation failed");
    } catch (const HipErr& e) {
        return err(HQ_ERR_DEVICE, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
    }
    return HQ_OK;
}

}  // extern "C"
