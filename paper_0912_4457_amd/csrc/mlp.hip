// The ell/k predictor network: MLP 16 -> 64 -> 64 -> 2 with SiLU, trained and
// evaluated on the GPU by hand-written kernels.
//
// Numerics: every matrix product runs on the bf16 MFMA units
// (v_mfma_f32_16x16x16_bf16) with bfloat16 operands (weights and layer inputs
// rounded to nearest-even from float32) and float32 accumulation; bias,
// activation, loss and the Adam update are float32; master weights are float32.
//
// Parameter vector (float32, 5378 entries): W1[16][64], b1[64], W2[64][64],
// b2[64], W3[64][2], b3[2]; a layer computes z = h W + b (row vectors).
#include "nks_internal.h"

namespace nks {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int IN = 16, HID = 64, OUT = 2;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + IN * HID, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID * OUT, NPARAM = OFF_B3 + OUT;
static_assert(NPARAM == 5378, "parameter count");
constexpr int ROWS = 64;     // batch rows per chunk
constexpr int MT = 256;      // threads per workgroup (4 waves)

// float32 -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ inline unsigned short bf16_bits(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_val(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

__device__ inline float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float dsilu(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// One 16x16 output tile: acc += A[m0:m0+16, k0:k0+16] * B[k0:k0+16, n0:n0+16],
// operands read through accessors returning bf16 bits.  Lane layout of the
// 16x16x16 bf16 MFMA: A row (lane % 16), k = 4*(lane/16)..+3; B column
// (lane % 16), same k; result rows 4*(lane/16)..+3 of column (lane % 16).
template <typename FA, typename FB>
__device__ inline f32x4 mfma_tile(f32x4 acc, FA a, FB b, int m0, int n0, int k0) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, kg = (lane >> 4) * 4;
    bf16x4 av, bv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        av[i] = (short)a(m0 + r, k0 + kg + i);
        bv[i] = (short)b(k0 + kg + i, n0 + r);
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
}

struct Lds {
    unsigned short w1[IN * HID];     // bf16 weights
    unsigned short w2[HID * HID];
    unsigned short w3[HID * 16];     // W3 padded to 16 columns
    unsigned short h0[ROWS * IN];    // bf16 layer inputs
    unsigned short h1[ROWS * HID];
    unsigned short h2[ROWS * HID];
    float z1[ROWS * HID];            // float32 pre-activations
    float z2[ROWS * HID];
    unsigned short e3[ROWS * 16];    // bf16 output error, padded to 16 columns
    unsigned short e2[ROWS * HID];   // bf16 backpropagated errors
    unsigned short e1[ROWS * HID];
    float y[ROWS * OUT];
};

__device__ void load_weights(Lds& L, const float* __restrict__ P) {
    for (int i = threadIdx.x; i < IN * HID; i += MT) L.w1[i] = bf16_bits(P[OFF_W1 + i]);
    for (int i = threadIdx.x; i < HID * HID; i += MT) L.w2[i] = bf16_bits(P[OFF_W2 + i]);
    for (int i = threadIdx.x; i < HID * 16; i += MT) {
        const int r = i / 16, c = i % 16;
        L.w3[i] = c < OUT ? bf16_bits(P[OFF_W3 + r * OUT + c]) : 0;
    }
}

// forward pass of the rows [row0, row0 + nrows) of X into the chunk buffers
__device__ void forward_chunk(Lds& L, const float* __restrict__ P, const float* __restrict__ X, int row0,
                              int nrows) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < ROWS * IN; i += MT) {
        const int r = i / IN;
        L.h0[i] = r < nrows ? bf16_bits(X[(size_t)(row0 + r) * IN + (i % IN)]) : 0;
    }
    __syncthreads();
    // layer 1: 64 x 64 outputs = 16 tiles, 4 per wave, K = 16
    for (int t = wave; t < 16; t += 4) {
        const int m0 = (t / 4) * 16, n0 = (t % 4) * 16;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma_tile(acc, [&](int m, int k) { return L.h0[m * IN + k]; },
                        [&](int k, int n) { return L.w1[k * HID + n]; }, m0, n0, 0);
        const int n = n0 + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + (lane >> 4) * 4 + i;
            const float z = acc[i] + P[OFF_B1 + n];
            L.z1[m * HID + n] = z;
            L.h1[m * HID + n] = bf16_bits(silu(z));
        }
    }
    __syncthreads();
    // layer 2: K = 64
    for (int t = wave; t < 16; t += 4) {
        const int m0 = (t / 4) * 16, n0 = (t % 4) * 16;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < HID; k0 += 16)
            acc = mfma_tile(acc, [&](int m, int k) { return L.h1[m * HID + k]; },
                            [&](int k, int n) { return L.w2[k * HID + n]; }, m0, n0, k0);
        const int n = n0 + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + (lane >> 4) * 4 + i;
            const float z = acc[i] + P[OFF_B2 + n];
            L.z2[m * HID + n] = z;
            L.h2[m * HID + n] = bf16_bits(silu(z));
        }
    }
    __syncthreads();
    // layer 3: 64 x 16 (2 used) = 4 tiles, one per wave
    {
        const int m0 = wave * 16;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < HID; k0 += 16)
            acc = mfma_tile(acc, [&](int m, int k) { return L.h2[m * HID + k]; },
                            [&](int k, int n) { return L.w3[k * 16 + n]; }, m0, 0, k0);
        const int n = lane & 15;
        if (n < OUT) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + (lane >> 4) * 4 + i;
                L.y[m * OUT + n] = acc[i] + P[OFF_B3 + n];
            }
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(MT) void mlp_forward_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                        int B, float* __restrict__ Y) {
    __shared__ Lds L;
    load_weights(L, P);
    const int row0 = blockIdx.x * ROWS;
    const int nrows = min(ROWS, B - row0);
    forward_chunk(L, P, X, row0, nrows);
    for (int i = threadIdx.x; i < nrows * OUT; i += MT) Y[(size_t)row0 * OUT + i] = L.y[i];
}

// Full-batch gradient of 0.5 * mean ||y - t||^2 (one workgroup; the batch is
// processed in chunks of 64 rows, gradients accumulate in fixed order).
__global__ __launch_bounds__(MT) void mlp_backward_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                         const float* __restrict__ T, int B, float* __restrict__ G,
                                                         float* __restrict__ loss) {
    __shared__ Lds L;
    __shared__ float gb[HID + HID + OUT];   // bias gradients
    __shared__ float lsum[MT];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    load_weights(L, P);
    for (int i = threadIdx.x; i < HID + HID + OUT; i += MT) gb[i] = 0.f;
    float lacc = 0.f;
    // per-wave accumulators of the weight gradients (MFMA tiles)
    f32x4 gw2[4], gw1, gw3;
    for (int t = 0; t < 4; ++t) gw2[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    gw1 = f32x4{0.f, 0.f, 0.f, 0.f};
    gw3 = f32x4{0.f, 0.f, 0.f, 0.f};
    const float invB = 1.0f / (float)B;
    for (int row0 = 0; row0 < B; row0 += ROWS) {
        const int nrows = min(ROWS, B - row0);
        __syncthreads();
        forward_chunk(L, P, X, row0, nrows);
        // output error e3 = (y - t) / B (float32 kept in L.y, bf16 copy padded to 16 columns)
        for (int i = threadIdx.x; i < ROWS * 16; i += MT) {
            const int r = i / 16, c = i % 16;
            float e = 0.f;
            if (r < nrows && c < OUT) {
                const float d = L.y[r * OUT + c] - T[(size_t)(row0 + r) * OUT + c];
                lacc += 0.5f * d * d;
                e = d * invB;
                L.y[r * OUT + c] = e;
            }
            L.e3[i] = bf16_bits(e);
        }
        __syncthreads();
        if (threadIdx.x < OUT) {
            float s = 0.f;
            for (int m = 0; m < nrows; ++m) s += L.y[m * OUT + threadIdx.x];
            gb[HID + HID + threadIdx.x] += s;
        }
        // dW3 (64 x 16 padded) += h2^T e3 : wave w owns rows 16w..16w+15 of dW3, K = chunk rows
        for (int k0 = 0; k0 < ROWS; k0 += 16)
            gw3 = mfma_tile(gw3, [&](int m, int k) { return L.h2[k * HID + m]; },
                            [&](int k, int n) { return L.e3[k * 16 + n]; }, wave * 16, 0, k0);
        // dh2 = e3 W3^T (64 x 64), K = 16 (2 used); e2 = dh2 * silu'(z2)
        for (int t = wave; t < 16; t += 4) {
            const int m0 = (t / 4) * 16, n0 = (t % 4) * 16;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma_tile(acc, [&](int m, int k) { return L.e3[m * 16 + k]; },
                            [&](int k, int n) { return L.w3[n * 16 + k]; }, m0, n0, 0);
            const int n = n0 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + (lane >> 4) * 4 + i;
                const float e = m < nrows ? acc[i] * dsilu(L.z2[m * HID + n]) : 0.f;
                L.z2[m * HID + n] = e;   // keep float32 e2 in place of z2
                L.e2[m * HID + n] = bf16_bits(e);
            }
        }
        __syncthreads();
        for (int n = threadIdx.x; n < HID; n += MT) {
            float s = 0.f;
            for (int m = 0; m < nrows; ++m) s += L.z2[m * HID + n];
            gb[HID + n] += s;
        }
        // dW2 (64 x 64) += h1^T e2 : wave w owns tiles w, w+4, w+8, w+12
        for (int t = 0; t < 4; ++t) {
            const int tt = wave + 4 * t;
            const int m0 = (tt / 4) * 16, n0 = (tt % 4) * 16;
            for (int k0 = 0; k0 < ROWS; k0 += 16)
                gw2[t] = mfma_tile(gw2[t], [&](int m, int k) { return L.h1[k * HID + m]; },
                                   [&](int k, int n) { return L.e2[k * HID + n]; }, m0, n0, k0);
        }
        // dh1 = e2 W2^T ; e1 = dh1 * silu'(z1)
        for (int t = wave; t < 16; t += 4) {
            const int m0 = (t / 4) * 16, n0 = (t % 4) * 16;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < HID; k0 += 16)
                acc = mfma_tile(acc, [&](int m, int k) { return L.e2[m * HID + k]; },
                                [&](int k, int n) { return L.w2[n * HID + k]; }, m0, n0, k0);
            const int n = n0 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + (lane >> 4) * 4 + i;
                const float e = m < nrows ? acc[i] * dsilu(L.z1[m * HID + n]) : 0.f;
                L.z1[m * HID + n] = e;
                L.e1[m * HID + n] = bf16_bits(e);
            }
        }
        __syncthreads();
        for (int n = threadIdx.x; n < HID; n += MT) {
            float s = 0.f;
            for (int m = 0; m < nrows; ++m) s += L.z1[m * HID + n];
            gb[n] += s;
        }
        // dW1 (16 x 64) += h0^T e1 : wave w owns columns 16w..16w+15
        for (int k0 = 0; k0 < ROWS; k0 += 16)
            gw1 = mfma_tile(gw1, [&](int m, int k) { return L.h0[k * IN + m]; },
                            [&](int k, int n) { return L.e1[k * HID + n]; }, 0, wave * 16, k0);
    }
    __syncthreads();
    // write the gradient
    {
        const int n = lane & 15;
        for (int t = 0; t < 4; ++t) {
            const int tt = wave + 4 * t;
            const int m0 = (tt / 4) * 16, n0 = (tt % 4) * 16;
#pragma unroll
            for (int i = 0; i < 4; ++i) G[OFF_W2 + (m0 + (lane >> 4) * 4 + i) * HID + n0 + n] = gw2[t][i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) G[OFF_W1 + ((lane >> 4) * 4 + i) * HID + wave * 16 + n] = gw1[i];
        if (n < OUT) {
#pragma unroll
            for (int i = 0; i < 4; ++i) G[OFF_W3 + (wave * 16 + (lane >> 4) * 4 + i) * OUT + n] = gw3[i];
        }
    }
    for (int i = threadIdx.x; i < HID; i += MT) {
        G[OFF_B1 + i] = gb[i];
        G[OFF_B2 + i] = gb[HID + i];
    }
    if (threadIdx.x < OUT) G[OFF_B3 + threadIdx.x] = gb[HID + HID + threadIdx.x];
    lsum[threadIdx.x] = lacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < MT; ++i) s += lsum[i];
        *loss = s * invB;
    }
}

__global__ void mlp_adam_kernel(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                                float* __restrict__ Vv, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    const float g = G[i];
    const float m = 0.9f * M[i] + 0.1f * g;
    const float v = 0.999f * Vv[i] + 0.001f * g * g;
    M[i] = m;
    Vv[i] = v;
    P[i] = P[i] - lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
}

}  // namespace

int mlp_nparams() { return NPARAM; }

void launch_mlp_forward(const float* P, const float* X, int B, float* Y, hipStream_t s) {
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + ROWS - 1) / ROWS), dim3(MT), 0, s, P, X, B, Y);
}

void launch_mlp_backward(const float* P, const float* X, const float* T, int B, float* G, float* loss,
                         hipStream_t s) {
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(1), dim3(MT), 0, s, P, X, T, B, G, loss);
}

void launch_mlp_adam(float* P, const float* G, float* M, float* V, int t, float lr, hipStream_t s) {
    const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s, P, G, M, V, lr, c1, c2);
}

}  // namespace nks
