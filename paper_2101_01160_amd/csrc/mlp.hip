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
constexpr int kMaxSplit = 32;
// Fixed input map of x = (phi, kT, dt_cg/dx, |u|, cos, sin): phi / 0.4,
// ln kT / ln 20, (ln(dt_cg/dx) + 6) / 1.5, and the drift as the vector
// 5 |u| (cos, sin) with its length 5 |u|; fp32, every operation rounded once.
__device__ __forceinline__ float encode_in(const float* __restrict__ xr, int k) {
#pragma clang fp contract(off)
    const float inv_ln20 = (float)(1.0 / 2.995732273553991);
    switch (k) {
        case 0: return xr[0] * 2.5f;
        case 1: return logf(fmaxf(xr[1], 1e-30f)) * inv_ln20;
        case 2: return (logf(fmaxf(xr[2], 1e-30f)) + 6.0f) * (float)(1.0 / 1.5);
        case 3: return (xr[3] * xr[4]) * 5.0f;
        case 4: return (xr[3] * xr[5]) * 5.0f;
        default: return xr[3] * 5.0f;
    }
}

// Logistic function and SiLU in fp32, the reciprocal from the hardware
// estimate (about one ulp); every consumer rounds the result to bf16 (8
// significant bits) first.  Training and inference share them.
__device__ __forceinline__ float sigmoid_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_f(float z) { return z * sigmoid_f(z); }

// Epilogues: STORE C; BIAS_SILU C = z = acc + bias and H = silu(z); BIAS C =
// acc + bias; SILU_BWD H = acc * silu'(Z) (the backward pass through an
// activation).
enum { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_BIAS = 2, EPI_SILU_BWD = 4 };
// Operand staging modes: 0 element-wise (any strides), 1 contiguous along k,
// 2 contiguous along the row (A: m, B: n) -- 1 and 2 load 16-byte vectors.
enum { OP_ANY = 0, OP_K = 1, OP_ROW = 2 };

struct GemmArgs {
    int M, N, K;
    const bf16* A;
    long a_sm, a_sk;  // A(m, k) = A[m * a_sm + k * a_sk]
    const bf16* B;
    long b_sk, b_sn;  // B(k, n) = B[k * b_sk + n * b_sn]
    const float* bias;
    float* C;  // C[m * ldc + n] (+ blockIdx.z * split_stride for split-K partials)
    long ldc;
    bf16* H;  // bf16 output (EPI_BIAS_SILU, EPI_SILU_BWD)
    long ldh;
    const float* Z;  // pre-activations read by EPI_SILU_BWD, leading dimension ldh
    int ones_row;  // row m of A reads as all ones (bias gradient row), -1: none
    int kchunk;    // k range of one split
    long split_stride;
};

// Block tile BM x BN, k tile BK (one MFMA step); LDS rows are padded by 8 so
// that the 16-byte fragment reads of consecutive rows spread over the banks.
constexpr int BM = 64, BN = 64, BK = 32, LDSK = BK + 8;

// One thread's share of a 64 x 32 operand tile: 8 values.  For OP_ANY and
// OP_K the thread owns row r = tid / 4, k = 8 (tid % 4) .. +7; for OP_ROW it
// owns k = tid / 8 and rows 8 (tid % 8) .. +7.
template <int MODE>
__device__ __forceinline__ void load_tile(const bf16* __restrict__ P, long s_row, long s_k, int row0, int rows,
                                          int rlim, int ones_row, int k0, int kend, bf16x8& v) {
    const int tid = threadIdx.x;
    const bf16 zero = (bf16)0.0f, one = (bf16)1.0f;
    if (MODE == OP_ROW) {
        const int k = k0 + (tid >> 3), r0 = row0 + (tid & 7) * 8;
        if (k < kend && r0 + 7 < rlim) {
            v = *reinterpret_cast<const bf16x8*>(P + k * s_k + r0);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int r = r0 + e;
                v[e] = (k < kend && r < rows) ? (r == ones_row ? one : P[r * s_row + k * s_k]) : zero;
            }
        }
    } else {
        const int r = row0 + (tid >> 2), kk = k0 + (tid & 3) * 8;
        if (MODE == OP_K && r < rlim && kk + 7 < kend) {
            v = *reinterpret_cast<const bf16x8*>(P + r * s_row + kk);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = kk + e;
                v[e] = (r < rows && k < kend) ? (r == ones_row ? one : P[r * s_row + k * s_k]) : zero;
            }
        }
    }
}

template <int MODE>
__device__ __forceinline__ void store_tile(bf16 (*T)[LDSK], int c0, const bf16x8& v) {
    const int tid = threadIdx.x;
    if (MODE == OP_ROW) {
        const int k = c0 + (tid >> 3), r0 = (tid & 7) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) T[r0 + e][k] = v[e];
    } else {
        *reinterpret_cast<bf16x8*>(&T[tid >> 2][c0 + (tid & 3) * 8]) = v;
    }
}

// C = A B with a fused epilogue.  Block: 256 threads = 4 waves, 64 x 64
// outputs; each wave owns 32 x 32 = 2 x 2 MFMA tiles of 16 x 16.  Operands are
// staged through LDS with k contiguous (As[m][k], Bt[n][k]); the next k tile
// is loaded into registers while the current one is multiplied.  MFMA
// 16x16x32 lane layout: lane l holds A(row l%16, k 8*(l/16) .. +7),
// B(k 8*(l/16) .. +7, col l%16) and D(rows 4*(l/16) .. +3, col l%16).
// blockIdx.z splits k.
template <int EPI, int AM, int BMD>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) bf16 As[BM][LDSK];
    __shared__ __attribute__((aligned(16))) bf16 Bt[BN][LDSK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int kbeg = blockIdx.z * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);
    const int mlim = g.ones_row >= 0 ? g.ones_row : g.M;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 ra, rb;
    load_tile<AM>(g.A, g.a_sm, g.a_sk, m0, g.M, mlim, g.ones_row, kbeg, kend, ra);
    load_tile<BMD>(g.B, g.b_sn, g.b_sk, n0, g.N, g.N, -1, kbeg, kend, rb);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        store_tile<AM>(As, 0, ra);
        store_tile<BMD>(Bt, 0, rb);
        __syncthreads();
        if (k0 + BK < kend) {
            load_tile<AM>(g.A, g.a_sm, g.a_sk, m0, g.M, mlim, g.ones_row, k0 + BK, kend, ra);
            load_tile<BMD>(g.B, g.b_sn, g.b_sk, n0, g.N, g.N, -1, k0 + BK, kend, rb);
        }
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
    float* C = g.C + blockIdx.z * g.split_stride;
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
                if (EPI == EPI_SILU_BWD) {
                    const float zz = g.Z[m * g.ldh + n];
                    const float sg = sigmoid_f(zz);
                    g.H[m * g.ldh + n] = (bf16)(z * sg * (1.0f + zz * (1.0f - sg)));
                    continue;
                }
                if (EPI != EPI_STORE) z += g.bias[n];
                C[m * g.ldc + n] = z;
                if (EPI == EPI_BIAS_SILU) g.H[m * g.ldh + n] = (bf16)silu_f(z);
            }
}

// C[m][n] = sum over splits z (in order) of part[z][m][n]
__global__ void k_splitk_reduce(const float* __restrict__ part, int splits, int M, int N, float* __restrict__ C,
                                long ldc) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long mn = (long)M * N;
    if (i >= mn) return;
    float v[8];
    float s = 0.f;
    for (int z0 = 0; z0 < splits; z0 += 8) {
        const int nz = min(8, splits - z0);
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = e < nz ? part[(long)(z0 + e) * mn + i] : 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) s += v[e];
    }
    C[(i / N) * ldc + i % N] = s;
}

__global__ void k_prep_input(const float* __restrict__ x, int B, bf16* __restrict__ xb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B * kIn) xb[i] = (bf16)encode_in(x + (long)(i / kIn) * kIn, i % kIn);
}

__device__ __forceinline__ float wave_max_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave per sample, lane i < 49 holds logit i: q = softmax(z); with a
// target R the per-sample loss sum_i R_i (log R_i - log q_i) and the logit
// gradient G = (q sum_i R_i - R) / B (bf16, for the backward products).  The
// block's four losses are summed in order into loss_part[block].
__global__ __launch_bounds__(256) void k_softmax(const float* __restrict__ z, const float* __restrict__ R, int B,
                                                 float* __restrict__ q, bf16* __restrict__ G,
                                                 float* __restrict__ loss_part) {
    __shared__ float wl[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.x * 4 + w;
    const bool on = b < B && lane < kOut;
    const long o = (long)b * kOut + lane;
    const float zi = on ? z[o] : -INFINITY;
    const float mx = wave_max_f(zi);
    const float ei = on ? __expf(zi - mx) : 0.f;
    const float ls = __logf(wave_sum_f(ei));
    const float logq = zi - mx - ls;
    const float qi = on ? __expf(logq) : 0.f;
    if (on && q) q[o] = qi;
    if (!R) return;
    const float ri = on ? R[o] : 0.f;
    const float rs = wave_sum_f(ri);
    const float li = wave_sum_f(on && ri > 0.f ? ri * (__logf(ri) - logq) : 0.f);
    if (on) G[o] = (bf16)((qi * rs - ri) / (float)B);
    if (lane == 0) wl[w] = b < B ? li : 0.f;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = (wl[0] + wl[1]) + (wl[2] + wl[3]);
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

// Position of parameter i in the transposed weight copy (W_l [fin][fout]
// stored as [fout][fin] at the same offset), or -1 for a bias.
__device__ __forceinline__ long transposed_pos(long i) {
    long o = 0, fin = 0, fout = 0;
    if (i < kB1) {
        o = kW1, fin = kIn, fout = kHid;
    } else if (i >= kW2 && i < kB2) {
        o = kW2, fin = kHid, fout = kHid;
    } else if (i >= kW3 && i < kB3) {
        o = kW3, fin = kHid, fout = kHid;
    } else if (i >= kW4 && i < kB4) {
        o = kW4, fin = kHid, fout = kOut;
    } else {
        return -1;
    }
    const long r = i - o;
    return o + (r % fout) * fin + r / fout;
}

// Adam on the fp32 master weights, then the bf16 copies the products read:
// wb in the parameter layout (backward products), wt with every weight
// matrix transposed (forward products, whose k then runs contiguously).
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2, bf16* __restrict__ wb, bf16* __restrict__ wt) {
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
    const long t = transposed_pos(i);
    if (t >= 0) wt[t] = (bf16)wi;
}

__global__ void k_to_bf16(const float* __restrict__ w, long n, bf16* __restrict__ wb, bf16* __restrict__ wt) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    wb[i] = (bf16)w[i];
    const long t = transposed_pos(i);
    if (t >= 0) wt[t] = (bf16)w[i];
}

// Whole-network inference for 64 samples per block.  The activations stay
// in LDS from layer to layer; the weights come from the transposed bf16 copy
// (k contiguous per output), from L2, straight into MFMA operand registers.
// Wave w computes output columns 64 w .. 64 w + 63 of a hidden layer (4 x 4
// tiles of 16 x 16, accumulators in registers), then every wave's results
// replace the layer input in LDS; the last layer (49 outputs, padded to 64)
// gives wave w the 16 rows 16 w .. 16 w + 15, whose softmax is reduced across
// the 16 lanes that hold a row.  Same roundings as the layer-wise products:
// scaled inputs, weights and hidden activations in bf16, fp32 accumulation,
// fp32 biases.
constexpr int kFB = 64;            // samples per block
constexpr int kHLD = kHid + 8;     // LDS row stride of the activations (bf16)

__device__ __forceinline__ void hidden_epilogue(const f32x4 (&acc)[4][4], const float* __restrict__ bias,
                                                bf16 (*H)[kHLD], int wv, int lane) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = 64 * wv + 16 * j + (lane & 15);
        const float bj = bias[col];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = acc[i][j][r] + bj;
                H[16 * i + 4 * (lane >> 4) + r][col] = (bf16)silu_f(z);
            }
    }
}

// At most 128 registers per lane: four waves per SIMD, so that one block's
// epilogue overlaps another's products.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_mlp_infer(const float* __restrict__ x, int B, const bf16* __restrict__ wt,
                                                   const float* __restrict__ w, float* __restrict__ g) {
    __shared__ __attribute__((aligned(16))) bf16 H[kFB][kHLD];
    __shared__ __attribute__((aligned(16))) bf16 X[kFB][40];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int row0 = blockIdx.x * kFB;
    for (int i = tid; i < kFB * 32; i += 256) {
        const int r = i >> 5, k = i & 31;
        float v = 0.f;
        if (k < kIn && row0 + r < B) v = encode_in(x + (long)(row0 + r) * kIn, k);
        X[r][k] = (bf16)v;
    }
    __syncthreads();
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    const bf16 zero = (bf16)0.0f;
    f32x4 acc[4][4];
    // layer 1: k = 6, one MFMA step over k padded to 32
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    {
        bf16x8 a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&X[16 * i + lr][lk]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = 64 * wv + 16 * j + lr;
            bf16x8 b;
#pragma unroll
            for (int e = 0; e < 8; ++e) b[e] = lk + e < kIn ? wt[kW1 + col * kIn + lk + e] : zero;
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[i][j], 0, 0, 0);
        }
    }
    // layers 2 and 3: k = 256; the first weight fragments of a layer are loaded
    // before the previous layer's epilogue
    const long wo[2] = {kW2, kW3}, bo[2] = {kB2, kB3};
    bf16x8 b[4], bn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        b[j] = *reinterpret_cast<const bf16x8*>(wt + kW2 + (64 * wv + lr) * kHid + lk + 16 * j * kHid);
    hidden_epilogue(acc, w + kB1, H, wv, lane);
    __syncthreads();
#pragma unroll
    for (int l = 0; l < 2; ++l) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        const bf16* __restrict__ W = wt + wo[l] + (64 * wv + lr) * kHid + lk;
        // the weight fragments of the next k step are in flight during this one's products
#pragma unroll 2
        for (int ks = 0; ks < kHid / 32; ++ks) {
            if (ks + 1 < kHid / 32) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bn[j] = *reinterpret_cast<const bf16x8*>(W + 16 * j * kHid + 32 * (ks + 1));
            }
            bf16x8 a[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&H[16 * i + lr][32 * ks + lk]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            if (ks + 1 < kHid / 32) {
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = bn[j];
            }
        }
        if (l == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(wt + kW3 + (64 * wv + lr) * kHid + lk + 16 * j * kHid);
        }
        __syncthreads();  // every wave has read this layer's input
        hidden_epilogue(acc, w + bo[l], H, wv, lane);
        __syncthreads();
    }
    // layer 4: 49 outputs; wave wv takes rows 16 wv .. 16 wv + 15
    f32x4 o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int ks = 0; ks < kHid / 32; ++ks) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&H[16 * wv + lr][32 * ks + lk]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = 16 * j + lr;
            bf16x8 b;
            if (col < kOut) {
                b = *reinterpret_cast<const bf16x8*>(wt + kW4 + col * kHid + 32 * ks + lk);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) b[e] = zero;
            }
            o[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, o[j], 0, 0, 0);
        }
    }
    // softmax of each row over the 16 lanes (x 4 tiles) that hold it
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = row0 + 16 * wv + 4 * (lane >> 4) + r;
        float z[4], mx = -INFINITY;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = 16 * j + lr;
            z[j] = col < kOut ? o[j][r] + w[kB4 + col] : -INFINITY;
            mx = fmaxf(mx, z[j]);
        }
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) mx = fmaxf(mx, __shfl_xor(mx, d, 64));
        float e[4], sum = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            e[j] = 16 * j + lr < kOut ? __expf(z[j] - mx) : 0.f;
            sum += e[j];
        }
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) sum += __shfl_xor(sum, d, 64);
        if (row < B) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = 16 * j + lr;
                if (col < kOut) g[(long)row * kOut + col] = e[j] / sum;
            }
        }
    }
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
    bf16* wb = nullptr;   // bf16 copies: parameter layout
    bf16* wt = nullptr;   // and weight matrices transposed
    bf16* xb = nullptr;
    float* Z[3] = {nullptr, nullptr, nullptr};
    bf16* H[3] = {nullptr, nullptr, nullptr};
    float* z4 = nullptr;
    bf16* g4 = nullptr;
    bf16* gh[2] = {nullptr, nullptr};  // activation gradients, ping-pong
    float* loss_b = nullptr;
    float* loss = nullptr;
    float* ws = nullptr;  // split-k partials of the weight gradients
    float* x1 = nullptr;  // one-sample staging for the surrogate call
    float* g1 = nullptr;
};

namespace {

template <int EPI, int AM>
void launch_b(int bm, dim3 grid, hipStream_t st, const GemmArgs& g) {
    if (bm == OP_K)
        hipLaunchKernelGGL((k_gemm<EPI, AM, OP_K>), grid, dim3(256), 0, st, g);
    else if (bm == OP_ROW)
        hipLaunchKernelGGL((k_gemm<EPI, AM, OP_ROW>), grid, dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL((k_gemm<EPI, AM, OP_ANY>), grid, dim3(256), 0, st, g);
}

template <int EPI>
void launch_ab(int am, int bm, dim3 grid, hipStream_t st, const GemmArgs& g) {
    if (am == OP_K)
        launch_b<EPI, OP_K>(bm, grid, st, g);
    else if (am == OP_ROW)
        launch_b<EPI, OP_ROW>(bm, grid, st, g);
    else
        launch_b<EPI, OP_ANY>(bm, grid, st, g);
}

// staging mode of an operand with element strides (s_row, s_k)
int op_mode(const bf16* p, long s_row, long s_k) {
    const bool aligned = ((uintptr_t)p & 15) == 0;
    if (aligned && s_k == 1 && s_row % 8 == 0) return OP_K;
    if (aligned && s_row == 1 && s_k % 8 == 0) return OP_ROW;
    return OP_ANY;
}

// C = A B with the epilogue epi.  Long-k products (the weight gradients, k =
// batch) are split over blockIdx.z into partials in `ws` (room for
// max_split x M x N floats) and summed in a fixed order.
hipError_t gemm(int epi, int M, int N, int K, const bf16* A, long a_sm, long a_sk, const bf16* B, long b_sk, long b_sn,
                const float* bias, float* C, long ldc, bf16* H, long ldh, hipStream_t st, int ones_row = -1,
                float* ws = nullptr, int max_split = 1, const float* Z = nullptr) {
    const int tiles = ((N + BN - 1) / BN) * ((M + BM - 1) / BM);
    int split = 1;
    if (epi == EPI_STORE && ws && max_split > 1) {
        // about one block per compute unit, at least eight k tiles per split
        while (split * 2 <= max_split && tiles * split < 256 && K / (split * 2) >= 8 * BK) split *= 2;
    }
    const int kchunk = ((K + split - 1) / split + BK - 1) / BK * BK;
    GemmArgs g{M, N, K, A, a_sm, a_sk, B, b_sk, b_sn, bias, C, ldc, H, ldh, Z, ones_row, kchunk, 0};
    if (split > 1) {
        g.C = ws;
        g.ldc = N;
        g.split_stride = (long)M * N;
    }
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, split);
    const int am = op_mode(A, a_sm, a_sk), bm = op_mode(B, b_sn, b_sk);
    switch (epi) {
        case EPI_STORE: launch_ab<EPI_STORE>(am, bm, grid, st, g); break;
        case EPI_BIAS_SILU: launch_ab<EPI_BIAS_SILU>(am, bm, grid, st, g); break;
        case EPI_BIAS: launch_ab<EPI_BIAS>(am, bm, grid, st, g); break;
        default: launch_ab<EPI_SILU_BWD>(am, bm, grid, st, g); break;
    }
    if (split > 1) {
        hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)(((long)M * N + 255) / 256)), dim3(256), 0, st,
                           (const float*)ws, split, M, N, C, ldc);
    }
    return hipGetLastError();
}

unsigned nblk(long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// Forward pass for training on B inputs already in m->xb: pre-activations
// z1..z3, activations h1..h3 and the logits z4 (inference uses k_mlp_infer).
hipError_t forward(mdlg_mlp* m, int B, hipStream_t st) {
    const long in[4] = {kIn, kHid, kHid, kHid};
    const long wo[4] = {kW1, kW2, kW3, kW4};
    const long bo[4] = {kB1, kB2, kB3, kB4};
    hipError_t e = hipSuccess;
    const bf16* a = m->xb;
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
        e = gemm(EPI_BIAS_SILU, B, kHid, (int)in[l], a, in[l], 1, m->wt + wo[l], 1, in[l],
                 m->w + bo[l], m->Z[l], kHid, m->H[l], kHid, st);
        a = m->H[l];
    }
    if (e == hipSuccess)
        e = gemm(EPI_BIAS, B, kOut, kHid, a, kHid, 1, m->wt + wo[3], 1, kHid, m->w + bo[3], m->z4, kOut, nullptr, 0, st);
    return e;
}

// Loss and gradient into m->grad (and m->loss) for targets R.
hipError_t backward(mdlg_mlp* m, const float* R, int B, hipStream_t st) {
    const int sb = (B + 3) / 4;
    hipLaunchKernelGGL(k_softmax, dim3(sb), dim3(256), 0, st, (const float*)m->z4, R, B, (float*)nullptr, m->g4,
                       m->loss_b);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, (const float*)m->loss_b, sb, 1.0f / B, m->loss);
    hipError_t e = hipGetLastError();
    // Weight and bias gradients come from one product [prev | 1]^T G: the bias
    // of each layer directly follows its weights in the parameter vector, so
    // the all-ones row fin of the extended operand lands on the bias slot.
    // layer 4: [dW4; db4] = [H3 | 1]^T G4, dH3 = G4 W4^T
    if (e == hipSuccess)
        e = gemm(EPI_STORE, kHid + 1, kOut, B, m->H[2], 1, kHid, m->g4, kOut, 1, nullptr, m->grad + kW4, kOut, nullptr, 0,
                 st, kHid, m->ws, kMaxSplit);
    // G3 = (G4 W4^T) * silu'(z3), fused into the product's epilogue
    if (e == hipSuccess)
        e = gemm(EPI_SILU_BWD, B, kHid, kOut, m->g4, kOut, 1, m->wb + kW4, 1, kOut, nullptr, nullptr, 0, m->gh[0], kHid,
                 st, -1, nullptr, 1, m->Z[2]);
    const long wo[3] = {kW1, kW2, kW3};
    int cur = 0;
    for (int l = 2; l >= 0 && e == hipSuccess; --l) {
        const bf16* prev = l > 0 ? m->H[l - 1] : m->xb;
        const int fin = l > 0 ? kHid : kIn;
        // [dW; db] = [prev | 1]^T G
        e = gemm(EPI_STORE, fin + 1, kHid, B, prev, 1, fin, m->gh[cur], kHid, 1, nullptr, m->grad + wo[l], kHid, nullptr,
                 0, st, fin, m->ws, kMaxSplit);
        // G_prev = (G W^T) * silu'(z_prev) (not needed below the first layer)
        if (e == hipSuccess && l > 0)
            e = gemm(EPI_SILU_BWD, B, kHid, kHid, m->gh[cur], kHid, 1, m->wb + wo[l], 1, kHid, nullptr, nullptr, 0,
                     m->gh[1 - cur], kHid, st, -1, nullptr, 1, m->Z[l - 1]);
        cur = 1 - cur;
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
    void* p[] = {m->w, m->m, m->v, m->grad, m->wb, m->wt, m->xb, m->Z[0], m->Z[1], m->Z[2], m->H[0], m->H[1], m->H[2],
                 m->z4, m->g4, m->gh[0], m->gh[1], m->loss_b, m->loss, m->ws, m->x1, m->g1};
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
    take(dalloc(&m->wt, kParams));
    take(dalloc(&m->xb, B * kIn));
    take(dalloc(&m->z4, B * kOut));
    take(dalloc(&m->g4, B * kOut));
    take(dalloc(&m->gh[0], B * kHid));
    take(dalloc(&m->gh[1], B * kHid));
    take(dalloc(&m->loss_b, (B + 3) / 4));
    take(dalloc(&m->loss, 1));
    take(dalloc(&m->ws, (size_t)kMaxSplit * (kHid + 1) * kHid));
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
        hipLaunchKernelGGL(k_to_bf16, dim3(nblk(kParams)), dim3(256), 0, st, (const float*)m->w, kParams, m->wb, m->wt);
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
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((B + kFB - 1) / kFB)), dim3(256), 0, st, x, B,
                       (const bf16*)m->wt, (const float*)m->w, g_out);
    MDLG_HIP(hipGetLastError());
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
                           kParams, lr, b1, b2, 1e-8f, bc1, bc2, m->wb, m->wt);
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
    // the guard: the Poisson-WSG closed form at the drift (|u| cos, |u| sin)
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

extern "C" mdlg_status mdlg_feq_surrogate_table(mdlg_mlp* m, const mdlg_moment_table* table, const double* x,
                                                double tol, double* g_out, int32_t* used_fallback, double* err,
                                                double* a2_out, double* lambda_out, void* stream) {
    if (!m || !table || !x || !g_out) return fail(MDLG_EINVAL, "mdlg_feq_surrogate_table: NULL argument");
    double a2 = 0.0, lambda = 0.0;
    mdlg_status s = mdlg_moment_table_eval(table, x, &a2, &lambda, nullptr);
    if (s != MDLG_OK) return s;
    if (a2_out) *a2_out = a2;
    if (lambda_out) *lambda_out = lambda;
    return mdlg_feq_surrogate(m, x, a2, lambda, tol, g_out, used_fallback, err, stream);
}
