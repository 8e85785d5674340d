// Surrogate network for the MDLG equilibrium distribution on gfx950:
// 6 -> 256 -> 256 -> 256 -> 49, SiLU, softmax, trained with the Kullback-
// Leibler divergence (Eq.(kullback_leibler)) against measured f_eq.
//
// Matrix products run on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16):
// bf16 operands, fp32 accumulation, fp32 master weights and Adam state.  One
// GEMM kernel serves the forward pass and both backward products through
// strided operand access; its epilogue fuses the bias and the SiLU.
#include <cmath>
#include <cstring>
#include <vector>

#include "mdlg_internal.h"

namespace mdlg {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 6, kHid = 256, kOut = 49;
constexpr long kW1 = 0, kB1 = 1536, kW2 = 1792, kB2 = 67328, kW3 = 67584, kB3 = 133120, kW4 = 133376, kB4 = 145920;
constexpr long kParams = 145969;
// fixed input scaling: phi / 0.4, kT / 20, (dt_cg/dx) * 100, |u| / 0.2, cos, sin
__constant__ float c_scale[kIn] = {2.5f, 0.05f, 100.0f, 5.0f, 1.0f, 1.0f};

enum { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_BIAS = 2 };

struct GemmArgs {
    int M, N, K;
    const bf16* A;
    long a_sm, a_sk;  // A(m, k) = A[m * a_sm + k * a_sk]
    const bf16* B;
    long b_sk, b_sn;  // B(k, n) = B[k * b_sk + n * b_sn]
    const float* bias;
    float* C;  // C[m * ldc + n]
    long ldc;
    bf16* H;  // SiLU output (EPI_BIAS_SILU)
    long ldh;
    int ones_row;  // row m of A reads as all ones (bias gradient row), -1: none
};

constexpr int BM = 64, BN = 64, BK = 32, LDSK = BK + 8;

// C = A B (+ bias, SiLU).  Block: 256 threads = 4 waves, 64 x 64 outputs;
// each wave owns 32 x 32 = 2 x 2 MFMA tiles of 16 x 16.  Operands are staged
// through LDS with k contiguous: As[m][k], Bt[n][k].  MFMA 16x16x32 lane
// layout: lane l holds A(row l%16, k 8*(l/16) .. +7), B(k 8*(l/16) .. +7,
// col l%16) and D(rows 4*(l/16) .. +3, col l%16).
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) bf16 As[BM][LDSK];
    __shared__ __attribute__((aligned(16))) bf16 Bt[BN][LDSK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = tid >> 2, lk = (tid & 3) * 8;  // staging: row / column and 8 k values per thread
    const bf16 zero = (bf16)0.0f, one = (bf16)1.0f;
    for (int k0 = 0; k0 < g.K; k0 += BK) {
        {
            const int m = m0 + lr;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + lk + e;
                As[lr][lk + e] = (m < g.M && k < g.K) ? (m == g.ones_row ? one : g.A[m * g.a_sm + k * g.a_sk]) : zero;
            }
            const int n = n0 + lr;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + lk + e;
                Bt[lr][lk + e] = (n < g.N && k < g.K) ? g.B[k * g.b_sk + n * g.b_sn] : zero;
            }
        }
        __syncthreads();
        const int kk = (lane >> 4) * 8;
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + i * 16 + (lane & 15)][kk]);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bt[wn + j * 16 + (lane & 15)][kk]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float z = acc[i][j][r];
                if (EPI != EPI_STORE) z += g.bias[n];
                g.C[m * g.ldc + n] = z;
                if (EPI == EPI_BIAS_SILU) g.H[m * g.ldh + n] = (bf16)(z / (1.0f + __expf(-z)));
            }
}

__global__ void k_prep_input(const float* __restrict__ x, int B, bf16* __restrict__ xb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B * kIn) xb[i] = (bf16)(x[i] * c_scale[i % kIn]);
}

// Per sample: q = softmax(z); with a target R: loss_b = sum_i R_i (log R_i - log q_i)
// and the logit gradient G = (q sum_i R_i - R) / B (bf16, for the backward products).
__global__ void k_softmax(const float* __restrict__ z, const float* __restrict__ R, int B, float* __restrict__ q,
                          bf16* __restrict__ G, float* __restrict__ loss_b) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float* zb = z + (long)b * kOut;
    float mx = zb[0];
    for (int i = 1; i < kOut; ++i) mx = fmaxf(mx, zb[i]);
    float s = 0.f;
    for (int i = 0; i < kOut; ++i) s += __expf(zb[i] - mx);
    const float ls = __logf(s);
    float loss = 0.f, rs = 0.f;
    if (R)
        for (int i = 0; i < kOut; ++i) rs += R[(long)b * kOut + i];
    for (int i = 0; i < kOut; ++i) {
        const float logq = zb[i] - mx - ls;
        const float qi = __expf(logq);
        if (q) q[(long)b * kOut + i] = qi;
        if (R) {
            const float ri = R[(long)b * kOut + i];
            if (ri > 0.f) loss += ri * (__logf(ri) - logq);
            G[(long)b * kOut + i] = (bf16)((qi * rs - ri) / (float)B);
        }
    }
    if (R) loss_b[b] = loss;
}

// G = dH * silu'(Z), silu'(z) = s (1 + z (1 - s)), s = 1 / (1 + e^-z)
__global__ void k_silu_bwd(const float* __restrict__ dH, const float* __restrict__ Z, long n, bf16* __restrict__ G) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float z = Z[i];
    const float s = 1.0f / (1.0f + __expf(-z));
    G[i] = (bf16)(dH[i] * s * (1.0f + z * (1.0f - s)));
}

__global__ void k_sum(const float* __restrict__ a, int n, float scale, float* out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += a[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Adam on the fp32 master weights, then the bf16 copies the products read.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2, bf16* __restrict__ wb) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wi;
    wb[i] = (bf16)wi;
}

__global__ void k_to_bf16(const float* __restrict__ w, long n, bf16* __restrict__ wb) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = (bf16)w[i];
}

}  // namespace
}  // namespace mdlg

using namespace mdlg;

struct mdlg_mlp {
    int max_batch = 0;
    long step = 0;
    float* w = nullptr;   // fp32 master parameters
    float* m = nullptr;   // Adam moments
    float* v = nullptr;
    float* grad = nullptr;
    bf16* wb = nullptr;   // bf16 copies
    bf16* xb = nullptr;
    float* Z[3] = {nullptr, nullptr, nullptr};
    bf16* H[3] = {nullptr, nullptr, nullptr};
    float* z4 = nullptr;
    float* q = nullptr;
    bf16* g4 = nullptr;
    float* dh = nullptr;
    bf16* gh = nullptr;
    float* loss_b = nullptr;
    float* loss = nullptr;
    float* x1 = nullptr;  // one-sample staging for the surrogate call
    float* g1 = nullptr;
};

namespace {

hipError_t gemm(int epi, int M, int N, int K, const bf16* A, long a_sm, long a_sk, const bf16* B, long b_sk, long b_sn,
                const float* bias, float* C, long ldc, bf16* H, long ldh, hipStream_t st, int ones_row = -1) {
    GemmArgs g{M, N, K, A, a_sm, a_sk, B, b_sk, b_sn, bias, C, ldc, H, ldh, ones_row};
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
    if (epi == EPI_STORE)
        hipLaunchKernelGGL(k_gemm<EPI_STORE>, grid, dim3(256), 0, st, g);
    else if (epi == EPI_BIAS_SILU)
        hipLaunchKernelGGL(k_gemm<EPI_BIAS_SILU>, grid, dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL(k_gemm<EPI_BIAS>, grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

unsigned nblk(long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// Forward pass on B inputs already in m->xb; leaves z1..z3, h1..h3, z4 and q.
hipError_t forward(mdlg_mlp* m, int B, hipStream_t st) {
    const long in[4] = {kIn, kHid, kHid, kHid};
    const long wo[4] = {kW1, kW2, kW3, kW4};
    const long bo[4] = {kB1, kB2, kB3, kB4};
    hipError_t e = hipSuccess;
    const bf16* a = m->xb;
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
        e = gemm(EPI_BIAS_SILU, B, kHid, (int)in[l], a, in[l], 1, m->wb + wo[l], kHid, 1, m->w + bo[l], m->Z[l], kHid,
                 m->H[l], kHid, st);
        a = m->H[l];
    }
    if (e == hipSuccess)
        e = gemm(EPI_BIAS, B, kOut, kHid, a, kHid, 1, m->wb + wo[3], kOut, 1, m->w + bo[3], m->z4, kOut, nullptr, 0, st);
    return e;
}

// Loss and gradient into m->grad (and m->loss) for targets R.
hipError_t backward(mdlg_mlp* m, const float* R, int B, hipStream_t st) {
    hipLaunchKernelGGL(k_softmax, dim3(nblk(B)), dim3(256), 0, st, (const float*)m->z4, R, B, m->q, m->g4, m->loss_b);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, (const float*)m->loss_b, B, 1.0f / B, m->loss);
    hipError_t e = hipGetLastError();
    // Weight and bias gradients come from one product [prev | 1]^T G: the bias
    // of each layer directly follows its weights in the parameter vector, so
    // the all-ones row fin of the extended operand lands on the bias slot.
    // layer 4: [dW4; db4] = [H3 | 1]^T G4, dH3 = G4 W4^T
    if (e == hipSuccess)
        e = gemm(EPI_STORE, kHid + 1, kOut, B, m->H[2], 1, kHid, m->g4, kOut, 1, nullptr, m->grad + kW4, kOut, nullptr, 0,
                 st, kHid);
    if (e == hipSuccess)
        e = gemm(EPI_STORE, B, kHid, kOut, m->g4, kOut, 1, m->wb + kW4, 1, kOut, nullptr, m->dh, kHid, nullptr, 0, st);
    const long wo[3] = {kW1, kW2, kW3};
    for (int l = 2; l >= 0 && e == hipSuccess; --l) {
        hipLaunchKernelGGL(k_silu_bwd, dim3(nblk((long)B * kHid)), dim3(256), 0, st, (const float*)m->dh,
                           (const float*)m->Z[l], (long)B * kHid, m->gh);
        const bf16* prev = l > 0 ? m->H[l - 1] : m->xb;
        const int fin = l > 0 ? kHid : kIn;
        // [dW; db] = [prev | 1]^T G
        e = gemm(EPI_STORE, fin + 1, kHid, B, prev, 1, fin, m->gh, kHid, 1, nullptr, m->grad + wo[l], kHid, nullptr, 0, st,
                 fin);
        // dH_prev = G W^T (not needed below the first layer)
        if (e == hipSuccess && l > 0)
            e = gemm(EPI_STORE, B, kHid, kHid, m->gh, kHid, 1, m->wb + wo[l], 1, kHid, nullptr, m->dh, kHid, nullptr, 0,
                     st);
    }
    if (e == hipSuccess) e = hipGetLastError();
    return e;
}

template <typename T>
hipError_t dalloc(T** p, size_t n) {
    return hipMalloc((void**)p, sizeof(T) * (n > 0 ? n : 1));
}

mdlg_status check_batch(const mdlg_mlp* m, int B, const char* who) {
    if (!m) return fail(MDLG_EINVAL, std::string(who) + ": NULL handle");
    if (B < 1 || B > m->max_batch)
        return fail(MDLG_EINVAL, std::string(who) + ": batch must be in [1, max_batch]");
    return MDLG_OK;
}

}  // namespace

extern "C" void mdlg_mlp_destroy(mdlg_mlp* m) {
    if (!m) return;
    void* p[] = {m->w, m->m, m->v, m->grad, m->wb, m->xb, m->Z[0], m->Z[1], m->Z[2], m->H[0], m->H[1], m->H[2],
                 m->z4, m->q, m->g4, m->dh, m->gh, m->loss_b, m->loss, m->x1, m->g1};
    for (void* q : p)
        if (q) (void)hipFree(q);
    delete m;
}

extern "C" mdlg_status mdlg_mlp_create(mdlg_mlp** out, const float* params, int32_t max_batch, void* stream) {
    if (!out || !params) return fail(MDLG_EINVAL, "mdlg_mlp_create: NULL argument");
    *out = nullptr;
    if (max_batch < 1 || max_batch > (1 << 20)) return fail(MDLG_EINVAL, "mdlg_mlp_create: max_batch in [1, 2^20]");
    for (long i = 0; i < kParams; ++i)
        if (!std::isfinite(params[i])) return fail(MDLG_EINVAL, "mdlg_mlp_create: non-finite parameter");
    hipStream_t st = (hipStream_t)stream;
    mdlg_mlp* m = new mdlg_mlp();
    m->max_batch = max_batch;
    const size_t B = max_batch;
    hipError_t ae = hipSuccess;
    auto take = [&](hipError_t r) {
        if (ae == hipSuccess) ae = r;
    };
    take(dalloc(&m->w, kParams));
    take(dalloc(&m->m, kParams));
    take(dalloc(&m->v, kParams));
    take(dalloc(&m->grad, kParams));
    take(dalloc(&m->wb, kParams));
    take(dalloc(&m->xb, B * kIn));
    take(dalloc(&m->z4, B * kOut));
    take(dalloc(&m->q, B * kOut));
    take(dalloc(&m->g4, B * kOut));
    take(dalloc(&m->dh, B * kHid));
    take(dalloc(&m->gh, B * kHid));
    take(dalloc(&m->loss_b, B));
    take(dalloc(&m->loss, 1));
    take(dalloc(&m->x1, kIn));
    take(dalloc(&m->g1, kOut));
    for (int l = 0; l < 3; ++l) {
        take(dalloc(&m->Z[l], B * kHid));
        take(dalloc(&m->H[l], B * kHid));
    }
    if (ae != hipSuccess) {
        mdlg_mlp_destroy(m);
        return fail(MDLG_ENOMEM, std::string("mdlg_mlp_create: device allocation failed: ") + hipGetErrorString(ae));
    }
    hipError_t e = hipMemcpyAsync(m->w, params, sizeof(float) * kParams, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, sizeof(float) * kParams, st);
    if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, sizeof(float) * kParams, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_to_bf16, dim3(nblk(kParams)), dim3(256), 0, st, (const float*)m->w, kParams, m->wb);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        mdlg_mlp_destroy(m);
        return fail(MDLG_EHIP, std::string("mdlg_mlp_create: ") + hipGetErrorString(e));
    }
    *out = m;
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_mlp_params(const mdlg_mlp* m, float* host_out, void* stream) {
    if (!m || !host_out) return fail(MDLG_EINVAL, "mdlg_mlp_params: NULL argument");
    MDLG_HIP(hipStreamSynchronize((hipStream_t)stream));
    MDLG_HIP(hipMemcpy(host_out, m->w, sizeof(float) * kParams, hipMemcpyDeviceToHost));
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_mlp_forward(mdlg_mlp* m, const float* x, int32_t B, float* g_out, void* stream) {
    mdlg_status s = check_batch(m, B, "mdlg_mlp_forward");
    if (s != MDLG_OK) return s;
    if (!x || !g_out) return fail(MDLG_EINVAL, "mdlg_mlp_forward: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_prep_input, dim3(nblk((long)B * kIn)), dim3(256), 0, st, x, B, m->xb);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = forward(m, B, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_softmax, dim3(nblk(B)), dim3(256), 0, st, (const float*)m->z4, (const float*)nullptr, B,
                           g_out, (bf16*)nullptr, (float*)nullptr);
        e = hipGetLastError();
    }
    MDLG_HIP(e);
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_mlp_gradient(mdlg_mlp* m, const float* x, const float* target, int32_t B, float* loss,
                                         float* grad, void* stream) {
    mdlg_status s = check_batch(m, B, "mdlg_mlp_gradient");
    if (s != MDLG_OK) return s;
    if (!x || !target) return fail(MDLG_EINVAL, "mdlg_mlp_gradient: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_prep_input, dim3(nblk((long)B * kIn)), dim3(256), 0, st, x, B, m->xb);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = forward(m, B, st);
    if (e == hipSuccess) e = backward(m, target, B, st);
    if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && grad) e = hipMemcpyAsync(grad, m->grad, sizeof(float) * kParams, hipMemcpyDeviceToDevice, st);
    MDLG_HIP(e);
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_mlp_train_step(mdlg_mlp* m, const float* x, const float* target, int32_t B, float lr,
                                           float* loss, void* stream) {
    mdlg_status s = check_batch(m, B, "mdlg_mlp_train_step");
    if (s != MDLG_OK) return s;
    if (!x || !target) return fail(MDLG_EINVAL, "mdlg_mlp_train_step: NULL argument");
    if (!(lr > 0.f) || !std::isfinite(lr)) return fail(MDLG_EINVAL, "mdlg_mlp_train_step: lr must be > 0");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_prep_input, dim3(nblk((long)B * kIn)), dim3(256), 0, st, x, B, m->xb);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = forward(m, B, st);
    if (e == hipSuccess) e = backward(m, target, B, st);
    if (e == hipSuccess) {
        m->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float bc1 = 1.0f - std::pow(b1, (float)m->step), bc2 = 1.0f - std::pow(b2, (float)m->step);
        hipLaunchKernelGGL(k_adam, dim3(nblk(kParams)), dim3(256), 0, st, m->w, m->m, m->v, (const float*)m->grad,
                           kParams, lr, b1, b2, 1e-8f, bc1, bc2, m->wb);
        e = hipGetLastError();
    }
    if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToDevice, st);
    MDLG_HIP(e);
    return MDLG_OK;
}

extern "C" mdlg_status mdlg_feq_surrogate(mdlg_mlp* m, const double* x, double a2, double lambda, double tol,
                                          double* g_out, int32_t* used_fallback, double* err, void* stream) {
    if (!m || !x || !g_out) return fail(MDLG_EINVAL, "mdlg_feq_surrogate: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    float xf[kIn];
    for (int i = 0; i < kIn; ++i) xf[i] = (float)x[i];
    MDLG_HIP(hipMemcpyAsync(m->x1, xf, sizeof(xf), hipMemcpyHostToDevice, st));
    mdlg_status s = mdlg_mlp_forward(m, m->x1, 1, m->g1, stream);
    if (s != MDLG_OK) return s;
    float gf[kOut];
    MDLG_HIP(hipMemcpyAsync(gf, m->g1, sizeof(gf), hipMemcpyDeviceToHost, st));
    MDLG_HIP(hipStreamSynchronize(st));
    // the judge: the Poisson-WSG closed form at the drift (|u| cos, |u| sin)
    const double u[2] = {x[3] * x[4], x[3] * x[5]};
    double gw[MDLG_NQ];
    s = mdlg_feq_wsg(a2, lambda, u, gw);
    if (s != MDLG_OK) return s;
    double e = 0.0;
    for (int i = 0; i < kOut; ++i) e = std::fmax(e, std::fabs((double)gf[i] - gw[i]));
    const bool fallback = !(e <= tol);
    for (int i = 0; i < kOut; ++i) g_out[i] = fallback ? gw[i] : (double)gf[i];
    if (used_fallback) *used_fallback = fallback ? 1 : 0;
    if (err) *err = e;
    return MDLG_OK;
}
