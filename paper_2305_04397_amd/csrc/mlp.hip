// Learned weight proposer: a small MLP that maps a threshold point and
// instance features [t; phi] to a weight vector on the simplex, used as the
// first weight vector of a query in place of e_1 (Alg. 1).  It is not part of
// the paper; the plain loop still decides every answer.
//
// Network: input standardisation (x - mu) / sd (fixed, set by the caller),
// then n_in -> 256 -> 256 -> 256 -> d, ReLU, softmax output; loss is the
// cross-entropy between a target weight vector and the softmax, averaged over
// the batch; optimiser Adam with bias correction.
//
// Precision: BF16 weights, inputs, activations and back-propagated gradients,
// FP32 accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16), FP32
// biases, logits, softmax, weight gradients and Adam state, FP32 master
// weights (the BF16 copies are refreshed by every Adam step).
//
// Kernels:
//   * gemm_bf16: C[M][N] = sum_k A(m, k) B(k, n) for strided BF16 operands,
//     one wave per 16 x 64 output strip (4 MFMA accumulators), with the
//     epilogue of the layer: +bias and ReLU to BF16 (hidden forward), +bias to
//     FP32 (logits), ReLU-derivative mask to BF16 (backward data), FP32 store
//     (weight gradients);
//   * softmax_xent: per row softmax, cross-entropy and (P - T) / B;
//   * bias_grad: column sums of a BF16 gradient;
//   * adam: the update of every parameter and its BF16 copy.
#include "common.h"

#include <mutex>

#include <cmath>
#include <cstdio>
#include <numeric>

namespace morap {

namespace {

typedef short s16x8 __attribute__((ext_vector_type(8)));          // BF16 bits
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int HID = 256;
constexpr int NLAYER = 4;

__host__ __device__ inline uint16_t f2bf(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even (finite inputs)
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf2f(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

enum Epilogue { EP_HIDDEN = 0, EP_LOGITS = 1, EP_BWD_DATA = 2, EP_WGRAD = 3 };

struct GemmArgs {
    const uint16_t* A;
    int64_t sam, sak;        // A(m, k) = A[m * sam + k * sak]
    const uint16_t* B;
    int64_t sbk, sbn;        // B(k, n) = B[k * sbk + n * sbn]
    int M, N, K;
    int mode;
    float* Cf;               // FP32 output (logits, weight gradients)
    uint16_t* Cb;            // BF16 output (activations, gradients)
    int64_t ldc;
    const float* bias;       // [N] (forward)
    const uint16_t* mask;    // ReLU-derivative source (backward data)
    int64_t ldm;
};

__global__ void __launch_bounds__(256) gemm_bf16(GemmArgs g) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tiles_n = (g.N + 63) / 64;
    const int tm = wave / tiles_n, tn = wave - tm * tiles_n;
    if (tm * 16 >= g.M) return;
    // operand layout of gfx950's 16x16x32 BF16 MFMA: lane l holds
    // A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16] for e = 0..7;
    // the result D[4 (l / 16) + e][l % 16] for e = 0..3
    const int r = lane & 15, kg = lane >> 4;
    const int m = tm * 16 + r;
    f32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += 32) {
        s16x8 a;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + 8 * kg + e;
            a[e] = (m < g.M && k < g.K) ? (short)g.A[m * g.sam + k * g.sak] : (short)0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = tn * 64 + j * 16 + r;
            s16x8 b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + 8 * kg + e;
                b[e] = (n < g.N && k < g.K) ? (short)g.B[k * g.sbk + n * g.sbn] : (short)0;
            }
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                             __builtin_bit_cast(bf16x8, b), acc[j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n = tn * 64 + j * 16 + r;
        if (n >= g.N) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int mm = tm * 16 + 4 * kg + e;
            if (mm >= g.M) continue;
            const float v = acc[j][e];
            const int64_t o = (int64_t)mm * g.ldc + n;
            switch (g.mode) {
                case EP_HIDDEN: g.Cb[o] = f2bf(fmaxf(v + g.bias[n], 0.f)); break;
                case EP_LOGITS: g.Cf[o] = v + g.bias[n]; break;
                case EP_BWD_DATA:
                    g.Cb[o] = f2bf(bf2f(g.mask[(int64_t)mm * g.ldm + n]) > 0.f ? v : 0.f);
                    break;
                default: g.Cf[o] = v; break;
            }
        }
    }
}

void gemm(hipStream_t s, const GemmArgs& g) {
    const int64_t waves = (int64_t)((g.M + 15) / 16) * ((g.N + 63) / 64);
    if (waves <= 0) return;
    hipLaunchKernelGGL(gemm_bf16, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, g);
    MORAP_HIP(hipGetLastError());
}

// per row: P = softmax(z), loss = -sum_k T_k log P_k, G = (P - T) / B (BF16)
__global__ void softmax_xent(const float* z, const float* T, float* P, uint16_t* G, float* loss, int n, int d,
                             float inv_b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* zi = z + (int64_t)i * d;
    float mx = -INFINITY;
    for (int k = 0; k < d; ++k) mx = fmaxf(mx, zi[k]);
    float sum = 0.f;
    for (int k = 0; k < d; ++k) sum += expf(zi[k] - mx);
    const float lse = logf(sum);
    float l = 0.f;
    for (int k = 0; k < d; ++k) {
        const float p = expf(zi[k] - mx) / sum;
        P[(int64_t)i * d + k] = p;
        if (T) {
            const float t = T[(int64_t)i * d + k];
            if (t != 0.f) l -= t * (zi[k] - mx - lse);
            G[(int64_t)i * d + k] = f2bf((p - t) * inv_b);
        }
    }
    if (loss) loss[i] = l;
}

// db[c] = sum_r G[r][c]
__global__ void bias_grad(const uint16_t* G, float* db, int n, int cols) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < n; ++r) s += bf2f(G[(int64_t)r * cols + c]);
    db[c] = s;
}

__global__ void to_bf16_kernel(const float* in, uint16_t* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(in[i]);
}

// network input: (x - mu) / sd per column, rounded to BF16
__global__ void input_kernel(const float* x, const float* mu, const float* sd, uint16_t* out, int64_t n,
                             int cols) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % cols);
    out[i] = f2bf((x[i] - mu[c]) / sd[c]);
}

// Adam with bias correction (c1 = 1 - beta1^t, c2 = 1 - beta2^t); weights
// (is_w != 0) refresh their BF16 copy
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, uint16_t* pb, const uint8_t* is_w,
                            int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (is_w[i]) pb[i] = f2bf(pi);
}

unsigned blocks_for(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

}  // namespace

struct Proposer {
    int n_in = 0, d = 0;
    int fan_in[NLAYER], fan_out[NLAYER];
    int64_t w_off[NLAYER], b_off[NLAYER], n_params = 0;
    int64_t t = 0;                    // Adam steps taken
    DevBuf p32, pb16, grad, m, v, is_w;
    std::vector<float> h_mu, h_sd;    // input standardisation (x - mu) / sd
    DevBuf mu, sd;
    int rows = 0;                     // capacity of the activation buffers
    DevBuf xb, h[NLAYER - 1], g[NLAYER - 1], logits, prob, target, gout, loss, xf;

    Proposer(int n_in_, int d_) : n_in(n_in_), d(d_) {
        const int sizes[NLAYER + 1] = {n_in, HID, HID, HID, d};
        for (int l = 0; l < NLAYER; ++l) {
            fan_in[l] = sizes[l];
            fan_out[l] = sizes[l + 1];
            w_off[l] = n_params;
            n_params += (int64_t)fan_out[l] * fan_in[l];
            b_off[l] = n_params;
            n_params += fan_out[l];
        }
        p32.ensure(n_params * 4);
        pb16.ensure(n_params * 2);
        grad.ensure(n_params * 4);
        m.ensure(n_params * 4);
        v.ensure(n_params * 4);
        is_w.ensure(n_params);
        mu.ensure((size_t)n_in * 4);
        sd.ensure((size_t)n_in * 4);
        h_mu.assign(n_in, 0.f);
        h_sd.assign(n_in, 1.f);
    }

    void set_norm(hipStream_t s, const float* m_, const float* s_) {
        h_mu.assign(m_, m_ + n_in);
        h_sd.assign(s_, s_ + n_in);
        MORAP_HIP(hipMemcpyAsync(mu.p, h_mu.data(), (size_t)n_in * 4, hipMemcpyHostToDevice, s));
        MORAP_HIP(hipMemcpyAsync(sd.p, h_sd.data(), (size_t)n_in * 4, hipMemcpyHostToDevice, s));
        MORAP_HIP(hipStreamSynchronize(s));
    }

    void ensure_rows(int n) {
        if (n <= rows) return;
        xb.ensure((size_t)n * n_in * 2);
        xf.ensure((size_t)n * n_in * 4);
        for (int l = 0; l < NLAYER - 1; ++l) {
            h[l].ensure((size_t)n * HID * 2);
            g[l].ensure((size_t)n * HID * 2);
        }
        logits.ensure((size_t)n * d * 4);
        prob.ensure((size_t)n * d * 4);
        target.ensure((size_t)n * d * 4);
        gout.ensure((size_t)n * d * 2);
        loss.ensure((size_t)n * 4);
        rows = n;
    }

    // upload FP32 parameters, reset Adam state, refresh BF16 copies
    void set(hipStream_t s, const float* host) {
        MORAP_HIP(hipMemcpyAsync(p32.p, host, n_params * 4, hipMemcpyHostToDevice, s));
        std::vector<uint8_t> w(n_params, 0);
        for (int l = 0; l < NLAYER; ++l)
            std::fill(w.begin() + w_off[l], w.begin() + b_off[l], (uint8_t)1);
        MORAP_HIP(hipMemcpyAsync(is_w.p, w.data(), n_params, hipMemcpyHostToDevice, s));
        MORAP_HIP(hipMemsetAsync(m.p, 0, n_params * 4, s));
        MORAP_HIP(hipMemsetAsync(v.p, 0, n_params * 4, s));
        hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n_params)), dim3(256), 0, s, p32.as<float>(),
                           pb16.as<uint16_t>(), n_params);
        MORAP_HIP(hipGetLastError());
        MORAP_HIP(hipStreamSynchronize(s));
        t = 0;
    }

    const uint16_t* act(int l) const {   // input of layer l
        return l == 0 ? xb.as<uint16_t>() : h[l - 1].as<uint16_t>();
    }

    // activation buffers of one forward pass
    struct Acts {
        const float* xf;       // [n][n_in] FP32 input
        uint16_t* xb;          // [n][n_in] BF16 standardised input
        uint16_t* h[NLAYER - 1];
        float* logits;         // [n][d]
        float* prob;           // [n][d]
    };
    Acts own_acts() {
        Acts a{xf.as<float>(), xb.as<uint16_t>(), {}, logits.as<float>(), prob.as<float>()};
        for (int l = 0; l < NLAYER - 1; ++l) a.h[l] = h[l].as<uint16_t>();
        return a;
    }

    // forward of n rows already in xf (FP32); logits then softmax into prob
    void forward(hipStream_t s, int n, const float* T_dev) { forward_into(s, n, own_acts(), T_dev); }

    // the same into the buffers of `b` (T_dev, when given, also fills the
    // loss and the output gradient of the context's own buffers)
    void forward_into(hipStream_t s, int n, const Acts& b, const float* T_dev) {
        hipLaunchKernelGGL(input_kernel, dim3(blocks_for((int64_t)n * n_in)), dim3(256), 0, s, b.xf, mu.as<float>(),
                           sd.as<float>(), b.xb, (int64_t)n * n_in, n_in);
        MORAP_HIP(hipGetLastError());
        for (int l = 0; l < NLAYER; ++l) {
            GemmArgs a{};
            a.A = l == 0 ? b.xb : b.h[l - 1];
            a.sam = fan_in[l];
            a.sak = 1;
            a.B = pb16.as<uint16_t>() + w_off[l];
            a.sbk = 1;
            a.sbn = fan_in[l];
            a.M = n;
            a.N = fan_out[l];
            a.K = fan_in[l];
            a.ldc = fan_out[l];
            a.bias = p32.as<float>() + b_off[l];
            if (l < NLAYER - 1) {
                a.mode = EP_HIDDEN;
                a.Cb = b.h[l];
            } else {
                a.mode = EP_LOGITS;
                a.Cf = b.logits;
            }
            gemm(s, a);
        }
        hipLaunchKernelGGL(softmax_xent, dim3(blocks_for(n, 64)), dim3(64), 0, s, b.logits, T_dev, b.prob,
                           T_dev ? gout.as<uint16_t>() : nullptr, T_dev ? loss.as<float>() : nullptr, n, d,
                           1.f / (float)n);
        MORAP_HIP(hipGetLastError());
    }

    // gradients of the mean cross-entropy into grad (after forward with T)
    void backward(hipStream_t s, int n) {
        for (int l = NLAYER - 1; l >= 0; --l) {
            const uint16_t* G = l == NLAYER - 1 ? gout.as<uint16_t>() : g[l].as<uint16_t>();
            const int N = fan_out[l], K = fan_in[l];
            // dW[N][K] = G^T H: A(i, r) = G[r][i], B(r, k) = H[r][k]
            GemmArgs w{};
            w.A = G;
            w.sam = 1;
            w.sak = N;
            w.B = act(l);
            w.sbk = K;
            w.sbn = 1;
            w.M = N;
            w.N = K;
            w.K = n;
            w.mode = EP_WGRAD;
            w.Cf = grad.as<float>() + w_off[l];
            w.ldc = K;
            gemm(s, w);
            hipLaunchKernelGGL(bias_grad, dim3(blocks_for(N)), dim3(256), 0, s, G, grad.as<float>() + b_off[l], n,
                               N);
            MORAP_HIP(hipGetLastError());
            if (l == 0) break;
            // G_{l-1}[n][K] = (G W) masked by H_{l-1} > 0: A(r, i) = G[r][i], B(i, k) = W[i][k]
            GemmArgs b{};
            b.A = G;
            b.sam = N;
            b.sak = 1;
            b.B = pb16.as<uint16_t>() + w_off[l];
            b.sbk = K;
            b.sbn = 1;
            b.M = n;
            b.N = K;
            b.K = N;
            b.mode = EP_BWD_DATA;
            b.Cb = g[l - 1].as<uint16_t>();
            b.ldc = K;
            b.mask = h[l - 1].as<uint16_t>();
            b.ldm = K;
            gemm(s, b);
        }
    }

    void adam(hipStream_t s, const morap_train_opts& o) {
        ++t;
        const float c1 = (float)(1.0 - std::pow((double)o.beta1, (double)t));
        const float c2 = (float)(1.0 - std::pow((double)o.beta2, (double)t));
        hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n_params)), dim3(256), 0, s, p32.as<float>(),
                           grad.as<float>(), m.as<float>(), v.as<float>(), pb16.as<uint16_t>(), is_w.as<uint8_t>(),
                           n_params, o.lr, o.beta1, o.beta2, o.adam_eps, c1, c2);
        MORAP_HIP(hipGetLastError());
    }

    // one step on n host rows; returns the mean loss
    double step(hipStream_t s, const float* X, const float* T, int n, const morap_train_opts* o, bool apply,
                float* grads_out) {
        ensure_rows(n);
        MORAP_HIP(hipMemcpyAsync(xf.p, X, (size_t)n * n_in * 4, hipMemcpyHostToDevice, s));
        MORAP_HIP(hipMemcpyAsync(target.p, T, (size_t)n * d * 4, hipMemcpyHostToDevice, s));
        forward(s, n, target.as<float>());
        backward(s, n);
        if (apply) adam(s, *o);
        std::vector<float> l(n);
        MORAP_HIP(hipMemcpyAsync(l.data(), loss.p, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        if (grads_out) MORAP_HIP(hipMemcpyAsync(grads_out, grad.p, n_params * 4, hipMemcpyDeviceToHost, s));
        MORAP_HIP(hipStreamSynchronize(s));
        double sum = 0;
        for (float x : l) sum += x;
        return sum / n;
    }

    void infer(hipStream_t s, const float* X, int n, float* out) {
        ensure_rows(n);
        MORAP_HIP(hipMemcpyAsync(xf.p, X, (size_t)n * n_in * 4, hipMemcpyHostToDevice, s));
        forward(s, n, nullptr);
        MORAP_HIP(hipMemcpyAsync(out, prob.p, (size_t)n * d * 4, hipMemcpyDeviceToHost, s));
        MORAP_HIP(hipStreamSynchronize(s));
    }
};

void proposer_destroy(Proposer* p) { delete p; }

// ---------------------------------------------------------------------------
// allocation-free inference: the activations of morap_proposer_infer_noalloc
// live in this fixed array (one copy per device, held until the process
// ends).  Its device address is taken once per device when a context is
// created there; host code uses that address, never the array's name.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static std::vector<unsigned char*> g_scratch;   // per device

void proposer_scratch_init(int device) {   // with `device` current
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch.size() <= device) g_scratch.resize((size_t)device + 1, nullptr);
    if (g_scratch[(size_t)device]) return;
    void* p = nullptr;
    MORAP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    MORAP_CHECK(p != nullptr, MORAP_E_HIP, "no device address for the inference scratch");
    g_scratch[(size_t)device] = static_cast<unsigned char*>(p);
}

static unsigned char* scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    MORAP_CHECK(device >= 0 && device < (int)g_scratch.size() && g_scratch[(size_t)device], MORAP_E_STATE,
                "the inference scratch of this device was not set up (no context created on it)");
    return g_scratch[(size_t)device];
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// scratch bytes of an n-row forward pass: BF16 input, three BF16 hidden
// layers, FP32 logits
static size_t scratch_need(int64_t n, int n_in, int d) {
    return round256((size_t)n * n_in * 2) + 3 * round256((size_t)n * HID * 2) + round256((size_t)n * d * 4);
}

bool proposer_ready(const morap_ctx* c, int n_in, int d) {
    return c->prop_mlp && c->prop_mlp->n_in == n_in && c->prop_mlp->d == d;
}

void proposer_infer_host(morap_ctx* c, const float* X, int n, float* out) {
    MORAP_CHECK(c->prop_mlp, MORAP_E_STATE, "no proposer");
    c->prop_mlp->infer(c->stream, X, n, out);
}

static Proposer& need(morap_ctx* c) {
    MORAP_CHECK(c->prop_mlp, MORAP_E_STATE, "no proposer: call morap_proposer_init or morap_proposer_load");
    return *c->prop_mlp;
}

static void check_rows(const float* X, const float* T, int n, int n_in, int d) {
    MORAP_CHECK(X && n >= 1, MORAP_E_INVALID, "need X and n >= 1");
    for (int64_t i = 0; i < (int64_t)n * n_in; ++i) MORAP_CHECK(std::isfinite(X[i]), MORAP_E_INVALID, "X must be finite");
    if (!T) return;
    for (int r = 0; r < n; ++r) {
        double sum = 0;
        for (int k = 0; k < d; ++k) {
            const float t = T[(int64_t)r * d + k];
            MORAP_CHECK(std::isfinite(t) && t >= 0.f, MORAP_E_INVALID, "targets must be finite and >= 0");
            sum += t;
        }
        MORAP_CHECK(std::fabs(sum - 1.0) <= 1e-4, MORAP_E_INVALID, "target rows must sum to 1");
    }
}

static void check_opts(const morap_train_opts* o) {
    MORAP_CHECK(o && o->batch >= 1 && o->epochs >= 0 && o->lr > 0 && o->beta1 >= 0 && o->beta1 < 1 &&
                    o->beta2 >= 0 && o->beta2 < 1 && o->adam_eps > 0,
                MORAP_E_INVALID, "bad training options");
}

static void init_params(morap_ctx* c, int n_in, int d, uint64_t seed) {
    MORAP_CHECK(n_in >= 1 && n_in <= 4096 && d >= 1 && d <= 4096, MORAP_E_INVALID, "bad proposer sizes");
    auto p = std::make_unique<Proposer>(n_in, d);
    std::vector<float> host(p->n_params, 0.f);
    for (int l = 0; l < NLAYER; ++l) {
        const double lim = std::sqrt(6.0 / p->fan_in[l]);   // He-uniform
        for (int64_t i = p->w_off[l]; i < p->b_off[l]; ++i) {
            const double u = (double)(splitmix64(seed + (uint64_t)i) >> 11) * 0x1.0p-53;
            host[i] = (float)(lim * (2.0 * u - 1.0));
        }
    }
    p->set(c->stream, host.data());
    p->set_norm(c->stream, p->h_mu.data(), p->h_sd.data());
    if (c->prop_mlp) proposer_destroy(c->prop_mlp);
    c->prop_mlp = p.release();
}

}  // namespace morap

using namespace morap;

extern "C" {

int morap_proposer_init(morap_ctx* ctx, int n_in, int d, uint64_t seed) {
    return guarded(ctx, [&] { init_params(ctx, n_in, d, seed); });
}

int64_t morap_proposer_num_params(const morap_ctx* ctx) {
    return ctx && ctx->prop_mlp ? ctx->prop_mlp->n_params : 0;
}

int morap_proposer_get_params(const morap_ctx* ctx, float* out) {
    auto* c = const_cast<morap_ctx*>(ctx);
    return guarded(c, [&] {
        Proposer& p = need(c);
        MORAP_CHECK(out, MORAP_E_INVALID, "NULL output");
        MORAP_HIP(hipMemcpyAsync(out, p.p32.p, p.n_params * 4, hipMemcpyDeviceToHost, c->stream));
        MORAP_HIP(hipStreamSynchronize(c->stream));
    });
}

int morap_proposer_set_params(morap_ctx* ctx, const float* in) {
    return guarded(ctx, [&] {
        Proposer& p = need(ctx);
        MORAP_CHECK(in, MORAP_E_INVALID, "NULL input");
        for (int64_t i = 0; i < p.n_params; ++i) MORAP_CHECK(std::isfinite(in[i]), MORAP_E_INVALID, "non-finite parameter");
        p.set(ctx->stream, in);
    });
}

int morap_proposer_set_input_norm(morap_ctx* ctx, const float* mu, const float* sd) {
    return guarded(ctx, [&] {
        Proposer& p = need(ctx);
        MORAP_CHECK(mu && sd, MORAP_E_INVALID, "NULL arguments");
        for (int i = 0; i < p.n_in; ++i)
            MORAP_CHECK(std::isfinite(mu[i]) && std::isfinite(sd[i]) && sd[i] > 0, MORAP_E_INVALID,
                        "need finite mu and sd > 0");
        p.set_norm(ctx->stream, mu, sd);
    });
}

int morap_proposer_infer(morap_ctx* ctx, const float* X, int n, float* W_out) {
    return guarded(ctx, [&] {
        Proposer& p = need(ctx);
        check_rows(X, nullptr, n, p.n_in, p.d);
        MORAP_CHECK(W_out, MORAP_E_INVALID, "NULL output");
        p.infer(ctx->stream, X, n, W_out);
    });
}

int morap_proposer_infer_noalloc(morap_ctx* ctx, const float* X_dev, int n, float* W_out_dev) {
    return guarded(ctx, [&] {
        Proposer& p = need(ctx);
        MORAP_CHECK(X_dev && W_out_dev && n >= 1, MORAP_E_INVALID, "need device X, device W_out and n >= 1");
        const size_t need_b = scratch_need(n, p.n_in, p.d);
        if (need_b > kScratchBytes) {
            int64_t max_rows = 0;
            while (scratch_need(max_rows + 1, p.n_in, p.d) <= kScratchBytes) ++max_rows;
            fail(MORAP_E_UNSUPPORTED, std::to_string(n) + " rows need " + std::to_string(need_b) +
                                          " bytes of inference scratch; the fixed scratch holds " +
                                          std::to_string(kScratchBytes) + " bytes (at most " +
                                          std::to_string(max_rows) + " rows for this network)");
        }
        unsigned char* base = scratch_of(ctx->device);
        Proposer::Acts a{};
        a.xf = X_dev;
        size_t off = 0;
        a.xb = reinterpret_cast<uint16_t*>(base + off);
        off += round256((size_t)n * p.n_in * 2);
        for (int l = 0; l < NLAYER - 1; ++l) {
            a.h[l] = reinterpret_cast<uint16_t*>(base + off);
            off += round256((size_t)n * HID * 2);
        }
        a.logits = reinterpret_cast<float*>(base + off);
        a.prob = W_out_dev;
        p.forward_into(ctx->stream, n, a, nullptr);
    });
}

int morap_proposer_step(morap_ctx* ctx, const float* X, const float* T, int n, const morap_train_opts* opts,
                        int apply, float* loss_out, float* grads_out) {
    return guarded(ctx, [&] {
        Proposer& p = need(ctx);
        MORAP_CHECK(T, MORAP_E_INVALID, "NULL targets");
        check_rows(X, T, n, p.n_in, p.d);
        if (apply) check_opts(opts);
        const double l = p.step(ctx->stream, X, T, n, opts, apply != 0, grads_out);
        if (loss_out) *loss_out = (float)l;
    });
}

int morap_proposer_train(morap_ctx* ctx, const float* X, const float* T, int n, const morap_train_opts* opts,
                         float* loss_out) {
    return guarded(ctx, [&] {
        Proposer& p = need(ctx);
        check_opts(opts);
        check_rows(X, T, n, p.n_in, p.d);
        std::vector<int> order(n);
        std::iota(order.begin(), order.end(), 0);
        const int B = std::min(opts->batch, n);
        std::vector<float> xb((size_t)B * p.n_in), tb((size_t)B * p.d);
        uint64_t ctr = 0;
        for (int ep = 0; ep < opts->epochs; ++ep) {
            for (int i = n - 1; i > 0; --i) {   // Fisher-Yates from SplitMix64(seed, counter)
                const int j = (int)(splitmix64(opts->seed ^ (0x5851F42D4C957F2Dull * ++ctr)) % (uint64_t)(i + 1));
                std::swap(order[i], order[j]);
            }
            double sum = 0;
            int batches = 0;
            for (int b0 = 0; b0 + B <= n; b0 += B) {   // full batches only
                for (int r = 0; r < B; ++r) {
                    std::copy(X + (size_t)order[b0 + r] * p.n_in, X + (size_t)(order[b0 + r] + 1) * p.n_in,
                              xb.begin() + (size_t)r * p.n_in);
                    std::copy(T + (size_t)order[b0 + r] * p.d, T + (size_t)(order[b0 + r] + 1) * p.d,
                              tb.begin() + (size_t)r * p.d);
                }
                sum += p.step(ctx->stream, xb.data(), tb.data(), B, opts, true, nullptr);
                ++batches;
            }
            if (loss_out) loss_out[ep] = (float)(sum / std::max(1, batches));
        }
    });
}

int morap_proposer_save(const morap_ctx* ctx, const char* path) {
    auto* c = const_cast<morap_ctx*>(ctx);
    return guarded(c, [&] {
        Proposer& p = need(c);
        MORAP_CHECK(path, MORAP_E_INVALID, "NULL path");
        std::vector<float> host(p.n_params);
        MORAP_HIP(hipMemcpyAsync(host.data(), p.p32.p, p.n_params * 4, hipMemcpyDeviceToHost, c->stream));
        MORAP_HIP(hipStreamSynchronize(c->stream));
        FILE* f = std::fopen(path, "wb");
        MORAP_CHECK(f, MORAP_E_INVALID, std::string("cannot write ") + path);
        const int32_t hdr[4] = {0x504C4D4D /* "MMLP" */, 1, p.n_in, p.d};
        bool ok = std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
                  std::fwrite(p.h_mu.data(), 4, p.n_in, f) == (size_t)p.n_in &&
                  std::fwrite(p.h_sd.data(), 4, p.n_in, f) == (size_t)p.n_in &&
                  std::fwrite(host.data(), 4, host.size(), f) == host.size();
        ok &= std::fclose(f) == 0;
        MORAP_CHECK(ok, MORAP_E_INVALID, std::string("write failed: ") + path);
    });
}

int morap_proposer_load(morap_ctx* ctx, const char* path) {
    return guarded(ctx, [&] {
        MORAP_CHECK(path, MORAP_E_INVALID, "NULL path");
        FILE* f = std::fopen(path, "rb");
        MORAP_CHECK(f, MORAP_E_INVALID, std::string("cannot read ") + path);
        int32_t hdr[4] = {0, 0, 0, 0};
        const bool hok = std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == 0x504C4D4D && hdr[1] == 1 &&
                         hdr[2] >= 1 && hdr[2] <= 4096 && hdr[3] >= 1 && hdr[3] <= 4096;
        if (!hok) std::fclose(f);
        MORAP_CHECK(hok, MORAP_E_INVALID, std::string("not a proposer file: ") + path);
        auto p = std::make_unique<Proposer>(hdr[2], hdr[3]);
        std::vector<float> host(p->n_params), nm(p->n_in), ns(p->n_in);
        const bool ok = std::fread(nm.data(), 4, nm.size(), f) == nm.size() &&
                        std::fread(ns.data(), 4, ns.size(), f) == ns.size() &&
                        std::fread(host.data(), 4, host.size(), f) == host.size();
        std::fclose(f);
        MORAP_CHECK(ok, MORAP_E_INVALID, std::string("truncated proposer file: ") + path);
        for (float x : host) MORAP_CHECK(std::isfinite(x), MORAP_E_INVALID, "non-finite parameter in file");
        for (int i = 0; i < p->n_in; ++i)
            MORAP_CHECK(std::isfinite(nm[i]) && std::isfinite(ns[i]) && ns[i] > 0, MORAP_E_INVALID,
                        "bad input standardisation in file");
        p->set(ctx->stream, host.data());
        p->set_norm(ctx->stream, nm.data(), ns.data());
        if (ctx->prop_mlp) proposer_destroy(ctx->prop_mlp);
        ctx->prop_mlp = p.release();
    });
}

}  // extern "C"
