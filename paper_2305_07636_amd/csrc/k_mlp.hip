// The weight-window network on the GPU: an 8-64-64-64-1 perceptron with
// tanh hidden layers, trained in FP32 on matrix cores and run in BF16 on
// matrix cores.
//
// Training: one 64-lane wave per block (about 512 blocks: a block takes one
// or a few groups of 16 samples); each wave streams its groups through
// forward and backward passes built from
// v_mfma_f32_16x16x4_f32 tiles (A 16x4, B 4x16, D 16x16), with weights and
// activations in LDS and the weight-gradient tiles in registers across the
// wave's groups.  Each block writes its gradient as one partial row; a
// second kernel sums the rows in block order (deterministic split-K, no
// float atomics) and applies Adam.
//
// Inference: v_mfma_f32_16x16x32_bf16 with weights and activations rounded
// to bfloat16, FP32 accumulation, FP32 tanh.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "mcdc_internal.hpp"

namespace mcdc {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kIn = 8, kH = 64;
constexpr int P_W1 = 0, P_B1 = 512, P_W2 = 576, P_B2 = 4672, P_W3 = 4736, P_B3 = 8832, P_W4 = 8896,
              P_B4 = 8960, NP = 8961;
constexpr int LD = kH + 1;   // padded LDS row (floats)

struct TrainLds {
    float W1[kIn][LD], W2[kH][LD], W3[kH][LD];
    float b1[kH], b2[kH], b3[kH], w4[kH], b4;
    float X[16][kIn + 1];
    float H1[16][LD], H2[16][LD], H3[16][LD];
    float dA[16][LD], dB[16][LD];
    float t[16], wt[16], dy[16];
};

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Z = A(16 x K, LDS rows) * W(K x 64, LDS rows) + bias, then tanh into Hout.
template <int K>
__device__ __forceinline__ void dense_tanh(const float (*A)[K == kIn ? kIn + 1 : LD], const float (*W)[LD],
                                           const float *bias, float (*Hout)[LD], int l) {
    const int col = l & 15, grp = l >> 4;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < K / 4; ++kc) acc = mfma4(A[col][4 * kc + grp], W[4 * kc + grp][16 * ct + col], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * grp + r, j = 16 * ct + col;
            Hout[i][j] = tanhf(acc[r] + bias[j]);
        }
    }
}

// dW(rows x 64) += Hin^T(rows x 16 samples) * dZ(16 x 64): RT row tiles.
template <int RT, int HW>
__device__ __forceinline__ void grad_w(v4f (&acc)[RT][4], const float (*Hin)[HW], const float (*dZ)[LD], int l,
                                       int nrows) {
    const int col = l & 15, grp = l >> 4;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                const int m = 16 * rt + col;
                const float a = (m < nrows) ? Hin[4 * kc + grp][m] : 0.f;
                acc[rt][ct] = mfma4(a, dZ[4 * kc + grp][16 * ct + col], acc[rt][ct]);
            }
}

// dZprev = (dZ * W^T) (.) (1 - Hprev^2)
__device__ __forceinline__ void back_tanh(const float (*dZ)[LD], const float (*W)[LD], const float (*Hprev)[LD],
                                          float (*out)[LD], int l) {
    const int col = l & 15, grp = l >> 4;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 16; ++kc) acc = mfma4(dZ[col][4 * kc + grp], W[16 * ct + col][4 * kc + grp], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * grp + r, j = 16 * ct + col;
            const float h = Hprev[i][j];
            out[i][j] = acc[r] * (1.f - h * h);
        }
    }
}

// Fused forward + backward over this block's sample groups.  partial row:
// [NP] gradient + [1] loss.
__global__ void __launch_bounds__(64) k_mlp_grad(const float *__restrict__ params, const float *__restrict__ X,
                                                 const float *__restrict__ T, const float *__restrict__ Wt,
                                                 int64_t n, int groups_per_block, float *partial) {
    extern __shared__ char smem[];
    TrainLds &S = *reinterpret_cast<TrainLds *>(smem);
    const int l = threadIdx.x;
    for (int p = l; p < kIn * kH; p += 64) S.W1[p / kH][p % kH] = params[P_W1 + p];
    for (int p = l; p < kH * kH; p += 64) {
        S.W2[p / kH][p % kH] = params[P_W2 + p];
        S.W3[p / kH][p % kH] = params[P_W3 + p];
    }
    S.b1[l] = params[P_B1 + l];
    S.b2[l] = params[P_B2 + l];
    S.b3[l] = params[P_B3 + l];
    S.w4[l] = params[P_W4 + l];
    if (l == 0) S.b4 = params[P_B4];
    __syncthreads();

    v4f g1[1][4], g2[4][4], g3[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        g1[0][a] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) g2[a][b] = g3[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, gw4 = 0.f, gb4 = 0.f, lsum = 0.f;

    const int64_t g0 = (int64_t)blockIdx.x * groups_per_block;
    for (int gi = 0; gi < groups_per_block; ++gi) {
        const int64_t row0 = (g0 + gi) * 16;
        if (row0 >= n) break;
        // stage the 16 samples (padded rows carry weight 0)
        for (int p = l; p < 16 * kIn; p += 64) {
            const int i = p / kIn, k = p % kIn;
            S.X[i][k] = (row0 + i < n) ? X[(row0 + i) * kIn + k] : 0.f;
        }
        if (l < 16) {
            S.t[l] = (row0 + l < n) ? T[row0 + l] : 0.f;
            S.wt[l] = (row0 + l < n) ? Wt[row0 + l] : 0.f;
        }
        __syncthreads();
        dense_tanh<kIn>(S.X, S.W1, S.b1, S.H1, l);
        __syncthreads();
        dense_tanh<kH>(S.H1, S.W2, S.b2, S.H2, l);
        __syncthreads();
        dense_tanh<kH>(S.H2, S.W3, S.b3, S.H3, l);
        __syncthreads();
        // output y_i = H3[i] . w4 + b4: 4 lanes per sample, then combine
        {
            const int i = l & 15, part = l >> 4;
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < 16; ++j) s += S.H3[i][16 * part + j] * S.w4[16 * part + j];
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            if (l < 16) {
                const float r = (s + S.b4) - S.t[l];
                S.dy[l] = 2.f * S.wt[l] * r;
                lsum += S.wt[l] * r * r;
            }
        }
        __syncthreads();
        // output layer gradients and dZ3 (lane = column j)
        {
            float a4 = 0.f, ab3 = 0.f;
            const float w4j = S.w4[l];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const float h = S.H3[i][l];
                const float dyi = S.dy[i];
                a4 += h * dyi;
                const float dz = dyi * w4j * (1.f - h * h);
                S.dA[i][l] = dz;
                ab3 += dz;
            }
            gw4 += a4;
            gb3 += ab3;
            if (l == 0) {
                float sdy = 0.f;
#pragma unroll
                for (int i = 0; i < 16; ++i) sdy += S.dy[i];
                gb4 += sdy;
            }
        }
        __syncthreads();
        grad_w<4, LD>(g3, S.H2, S.dA, l, kH);             // dW3 += H2^T dZ3
        back_tanh(S.dA, S.W3, S.H2, S.dB, l);            // dZ2
        __syncthreads();
        {
            float a = 0.f;
#pragma unroll
            for (int i = 0; i < 16; ++i) a += S.dB[i][l];
            gb2 += a;
        }
        grad_w<4, LD>(g2, S.H1, S.dB, l, kH);             // dW2 += H1^T dZ2
        back_tanh(S.dB, S.W2, S.H1, S.dA, l);            // dZ1
        __syncthreads();
        {
            float a = 0.f;
#pragma unroll
            for (int i = 0; i < 16; ++i) a += S.dA[i][l];
            gb1 += a;
        }
        grad_w<1, kIn + 1>(g1, S.X, S.dA, l, kIn);        // dW1 += X^T dZ1
        __syncthreads();
    }

    float *out = partial + (int64_t)blockIdx.x * (NP + 1);
    const int col = l & 15, grp = l >> 4;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * rt + 4 * grp + r, j = 16 * ct + col;
                out[P_W2 + i * kH + j] = g2[rt][ct][r];
                out[P_W3 + i * kH + j] = g3[rt][ct][r];
            }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * grp + r, j = 16 * ct + col;
            if (i < kIn) out[P_W1 + i * kH + j] = g1[0][ct][r];
        }
    out[P_B1 + l] = gb1;
    out[P_B2 + l] = gb2;
    out[P_B3 + l] = gb3;
    out[P_W4 + l] = gw4;
    // loss: lanes 0..15 hold partial sums
    float ls = lsum;
    for (int o = 32; o > 0; o >>= 1) ls += __shfl_xor(ls, o);
    if (l == 0) {
        out[P_B4] = gb4;
        out[NP] = ls;
    }
}

// Sum the partial rows in block order; optionally apply Adam.
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *__restrict__ partial, int nblk, float *grad_out,
                                                    float *params, float *m, float *v, float lr, float bc1,
                                                    float bc2, float *loss_slot, int adam) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NP) return;
    float g = 0.f;
    for (int b = 0; b < nblk; ++b) g += partial[(int64_t)b * (NP + 1) + p];
    if (p == NP) {
        if (loss_slot) *loss_slot = g;
        return;
    }
    if (grad_out) grad_out[p] = g;
    if (adam) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float mm = b1 * m[p] + (1.f - b1) * g;
        const float vv = b2 * v[p] + (1.f - b2) * g * g;
        m[p] = mm;
        v[p] = vv;
        params[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    }
}

// ---------------------------------------------------------------------------
// BF16 inference
// ---------------------------------------------------------------------------
constexpr int LB = kH + 8;   // bf16 row pitch (144 B) against bank conflicts

struct InferLds {
    __bf16 W1t[kH][LB];      // transposed: [out j][in k], k < 8 used (rest 0)
    __bf16 W2t[kH][LB], W3t[kH][LB];
    float b1[kH], b2[kH], b3[kH], w4[kH], b4;
    __bf16 A[4][16][LB];     // per-wave activations
};

__device__ __forceinline__ v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v8bf load8(const __bf16 *p) {
    v8bf r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = p[e];
    return r;
}

__device__ __forceinline__ void dense_bf16(__bf16 (*A)[LB], const __bf16 (*Wt)[LB], const float *bias, int K,
                                           int l) {
    const int col = l & 15, grp = l >> 4;
    v4f acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        acc[ct] = v4f{0.f, 0.f, 0.f, 0.f};
        for (int kc = 0; kc < K / 32; ++kc)
            acc[ct] = mfma_bf16(load8(&A[col][32 * kc + 8 * grp]), load8(&Wt[16 * ct + col][32 * kc + 8 * grp]),
                                acc[ct]);
    }
    __syncthreads();   // all lanes have read A before it is overwritten
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * grp + r, j = 16 * ct + col;
            A[i][j] = (__bf16)tanhf(acc[ct][r] + bias[j]);
        }
}

__global__ void __launch_bounds__(256) k_mlp_infer(const float *__restrict__ params, const float *__restrict__ X,
                                                   int64_t n, float *Y) {
    extern __shared__ char smem[];
    InferLds &S = *reinterpret_cast<InferLds *>(smem);
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    for (int p = tid; p < kH * LB; p += 256) {
        const int j = p / LB, k = p % LB;
        S.W1t[j][k] = (__bf16)((k < kIn) ? params[P_W1 + k * kH + j] : 0.f);
        S.W2t[j][k] = (__bf16)((k < kH) ? params[P_W2 + k * kH + j] : 0.f);
        S.W3t[j][k] = (__bf16)((k < kH) ? params[P_W3 + k * kH + j] : 0.f);
    }
    if (tid < kH) {
        S.b1[tid] = params[P_B1 + tid];
        S.b2[tid] = params[P_B2 + tid];
        S.b3[tid] = params[P_B3 + tid];
        S.w4[tid] = (float)(__bf16)params[P_W4 + tid];
    }
    if (tid == 0) S.b4 = params[P_B4];
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + w) * 16;
    for (int p = l; p < 16 * LB; p += 64) {
        const int i = p / LB, k = p % LB;
        S.A[w][i][k] = (__bf16)((k < kIn && row0 + i < n) ? X[(row0 + i) * kIn + k] : 0.f);
    }
    __syncthreads();
    dense_bf16(S.A[w], S.W1t, S.b1, 32, l);
    __syncthreads();
    dense_bf16(S.A[w], S.W2t, S.b2, kH, l);
    __syncthreads();
    dense_bf16(S.A[w], S.W3t, S.b3, kH, l);
    __syncthreads();
    const int i = l & 15, part = l >> 4;
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) s += (float)S.A[w][i][16 * part + j] * S.w4[16 * part + j];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (l < 16 && row0 + l < n) Y[row0 + l] = s + S.b4;
}

}  // namespace
}  // namespace mcdc

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace mcdc;

struct mcdc_mlp {
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    float *partial = nullptr;
    size_t partial_rows = 0;
    int64_t step = 0;
    int device = 0;
};

namespace {

int mlp_invalid(const char *m) {
    set_error(std::string("invalid argument: ") + m);
    return MCDC_E_INVALID;
}

// Xavier-uniform initial weights, zero biases, from SplitMix64(seed).
std::vector<float> xavier(uint64_t seed) {
    std::vector<float> p(NP, 0.f);
    uint64_t s = seed;
    auto u01 = [&]() {
        s += 0x9E3779B97F4A7C15ULL;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        return (double)(z >> 11) * 0x1p-53;
    };
    auto fill = [&](int off, int fan_in, int fan_out) {
        const double a = std::sqrt(6.0 / (fan_in + fan_out));
        for (int k = 0; k < fan_in * fan_out; ++k) p[off + k] = (float)((2.0 * u01() - 1.0) * a);
    };
    fill(P_W1, kIn, kH);
    fill(P_W2, kH, kH);
    fill(P_W3, kH, kH);
    fill(P_W4, kH, 1);
    return p;
}

int ensure_partial(mcdc_mlp *m, size_t rows) {
    if (m->partial_rows >= rows) return MCDC_OK;
    if (m->partial) (void)hipFree(m->partial);
    m->partial = nullptr;
    hipError_t e = hipMalloc(&m->partial, rows * (NP + 1) * sizeof(float));
    if (e != hipSuccess) {
        m->partial_rows = 0;
        return hip_fail(e, "hipMalloc(mlp partials)");
    }
    m->partial_rows = rows;
    return MCDC_OK;
}

// Sample groups of 16 per block: as few as keep about this many blocks in
// flight (a block's groups run one after the other, so fewer groups per
// block shorten the step; the partial rows they add stay few enough for the
// ordered reduction).
constexpr int64_t kTargetBlocks = 512;

int grad_pass(mcdc_mlp *m, const float *X, const float *T, const float *W, int64_t n, hipStream_t st,
              int &nblk) {
    const int64_t groups = (n + 15) / 16;
    const int64_t per = (groups + kTargetBlocks - 1) / kTargetBlocks;
    nblk = (int)((groups + per - 1) / per);
    int rc = ensure_partial(m, (size_t)nblk);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(64), sizeof(TrainLds), st, m->params, X, T, W, n, (int)per,
                       m->partial);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "mlp grad launch");
}

}  // namespace

extern "C" int mcdc_mlp_create(const int32_t *widths, int32_t n_layers, uint64_t seed, mcdc_mlp **out) {
    if (!out || !widths) return mlp_invalid("NULL argument");
    *out = nullptr;
    const int32_t want[5] = {8, 64, 64, 64, 1};
    if (n_layers != 4) {
        set_error("only the 8-64-64-64-1 network (4 layers) is supported");
        return MCDC_E_UNSUPPORTED;
    }
    for (int i = 0; i < 5; ++i)
        if (widths[i] != want[i]) {
            set_error("only the 8-64-64-64-1 network (4 layers) is supported");
            return MCDC_E_UNSUPPORTED;
        }
    mcdc_mlp *m = new (std::nothrow) mcdc_mlp();
    if (!m) return MCDC_E_NOMEM;
    hipError_t e = hipGetDevice(&m->device);
    float **bufs[] = {&m->params, &m->m, &m->v, &m->grad, &m->loss};
    for (auto b : bufs)
        if (e == hipSuccess) e = hipMalloc(b, (NP + 1) * sizeof(float));
    if (e != hipSuccess) {
        mcdc_mlp_destroy(m);
        return hip_fail(e, "hipMalloc(mlp)");
    }
    std::vector<float> p = xavier(seed);
    e = hipMemcpy(m->params, p.data(), NP * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->m, 0, (NP + 1) * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->v, 0, (NP + 1) * sizeof(float));
    if (e != hipSuccess) {
        mcdc_mlp_destroy(m);
        return hip_fail(e, "mlp init");
    }
    *out = m;
    return MCDC_OK;
}

extern "C" int mcdc_mlp_destroy(mcdc_mlp *m) {
    if (!m) return MCDC_OK;
    float *bufs[] = {m->params, m->m, m->v, m->grad, m->loss, m->partial};
    for (auto b : bufs)
        if (b) (void)hipFree(b);
    delete m;
    return MCDC_OK;
}

extern "C" int mcdc_mlp_get_params(const mcdc_mlp *m, float *params) {
    if (!m || !params) return mlp_invalid("NULL argument");
    hipError_t e = hipMemcpy(params, m->params, NP * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "copy params");
}

extern "C" int mcdc_mlp_set_params(mcdc_mlp *m, const float *params) {
    if (!m || !params) return mlp_invalid("NULL argument");
    hipError_t e = hipMemcpy(m->params, params, NP * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->m, 0, (NP + 1) * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->v, 0, (NP + 1) * sizeof(float));
    m->step = 0;
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "set params");
}

extern "C" int mcdc_mlp_grad(mcdc_mlp *m, const float *X, const float *T, const float *W, int64_t n, float *loss,
                             float *grads, void *stream) {
    if (!m || !X || !T || !W || n <= 0) return mlp_invalid("NULL argument or n <= 0");
    hipStream_t st = (hipStream_t)stream;
    int nblk = 0;
    int rc = grad_pass(m, X, T, W, n, st, nblk);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NP + 1 + 255) / 256), dim3(256), 0, st, m->partial, nblk, m->grad,
                       m->params, m->m, m->v, 0.f, 1.f, 1.f, m->loss, 0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && grads) e = hipMemcpyAsync(grads, m->grad, NP * sizeof(float), hipMemcpyDeviceToHost, st);
    float l = 0.f;
    if (e == hipSuccess) e = hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "mlp grad");
    if (loss) *loss = l;
    return MCDC_OK;
}

extern "C" int mcdc_mlp_train(mcdc_mlp *m, const float *X, const float *T, const float *W, int64_t n,
                              int32_t steps, float lr, float *loss_out, void *stream) {
    if (!m || !X || !T || !W || n <= 0 || steps < 0) return mlp_invalid("NULL argument, n <= 0 or steps < 0");
    if (!(lr > 0.f)) return mlp_invalid("lr must be > 0");
    hipStream_t st = (hipStream_t)stream;
    float *dloss = nullptr;
    hipError_t e = hipSuccess;
    if (loss_out && steps > 0) e = hipMalloc(&dloss, (size_t)steps * sizeof(float));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(loss history)");
    for (int s = 0; s < steps; ++s) {
        int nblk = 0;
        int rc = grad_pass(m, X, T, W, n, st, nblk);
        if (rc) {
            if (dloss) (void)hipFree(dloss);
            return rc;
        }
        m->step += 1;
        const double bc1 = 1.0 - std::pow(0.9, (double)m->step);
        const double bc2 = 1.0 - std::pow(0.999, (double)m->step);
        hipLaunchKernelGGL(k_mlp_reduce, dim3((NP + 1 + 255) / 256), dim3(256), 0, st, m->partial, nblk, m->grad,
                           m->params, m->m, m->v, lr, (float)bc1, (float)bc2, dloss ? dloss + s : m->loss, 1);
    }
    e = hipGetLastError();
    if (e == hipSuccess && dloss)
        e = hipMemcpyAsync(loss_out, dloss, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (dloss) (void)hipFree(dloss);
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "mlp train");
}

extern "C" int mcdc_mlp_infer(mcdc_mlp *m, const float *X, int64_t n, float *Y, void *stream) {
    if (!m || !X || !Y || n <= 0) return mlp_invalid("NULL argument or n <= 0");
    hipStream_t st = (hipStream_t)stream;
    const int64_t blocks = (n + 63) / 64;
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)blocks), dim3(256), sizeof(InferLds), st, m->params, X, n, Y);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? MCDC_OK : hip_fail(e, "mlp infer");
}
