// mlp.hip -- the density surrogate on gfx950: forward, backward, gradient
// reduction and Adam for a 3-128-128-128-1 GELU perceptron (see
// include/pcpd_mlp.h for the arithmetic contract).
//
// Work split: one workgroup of 256 lanes (4 wavefronts) per tile of 64 rows.
// The two 128x128 layers and the weight gradients are matrix products on
// v_mfma_f32_16x16x32_bf16 (bfloat16 operands, float32 accumulation); the
// 3-input first layer, the 128-input output unit, GELU, biases and the loss
// are float32 vector work. Activations live in LDS as bfloat16 (row-major
// for the products that read them along a row, transposed for the weight
// gradients that read them along a column); pre-activations z are kept in
// HBM between the forward and backward passes. Weight gradients are written
// per workgroup and summed in a fixed order, so results do not depend on
// scheduling.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "../../include/pcpd_mlp.h"
#include "philox.h"

namespace pcpd {
namespace {

constexpr int H = 128;
constexpr int ROWS = 64;          // rows per workgroup
constexpr int THREADS = 256;
constexpr int LDH = H + 8;        // LDS pitch (bf16) of row-major [ROWS][H] tiles
constexpr int LDR = ROWS + 8;     // LDS pitch (bf16) of transposed [H][ROWS] tiles

constexpr int oW1 = 0, ob1 = oW1 + H * 3, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H,
              ob3 = oW3 + H * H, ow4 = ob3 + H, ob4 = ow4 + H, NP = ob4 + 1;
static_assert(NP == PCPD_MLP_PARAMS, "parameter layout");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t bfbits;

// float32 -> bfloat16 bits, round to nearest, ties to even (NaN stays NaN)
__device__ __forceinline__ bfbits f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0u;
    return static_cast<bfbits>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(bfbits b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }
__device__ __forceinline__ float rbf(float f) { return bf2f(f2bf(f)); }

// tanh form of GELU and its derivative
__device__ __forceinline__ float gelu(float z) {
    const float c = 0.7978845608028654f, a = 0.044715f;
    return 0.5f * z * (1.0f + tanhf(c * (z + a * z * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z) {
    const float c = 0.7978845608028654f, a = 0.044715f;
    const float t = tanhf(c * (z + a * z * z * z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * c * (1.0f + 3.0f * a * z * z);
}

// eight consecutive bfloat16 values (16-byte aligned) as an MFMA operand
__device__ __forceinline__ bf16x8 load8(const bfbits *p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(p));
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// One hidden layer of the forward pass on the tile: Z = Hin W^T + b with
// Hin [ROWS][H] bf16 in LDS and W [H][H] bf16 in HBM (output-major, so the
// operand B[k][n] = W[n][k] is contiguous in k). Wavefront w computes rows
// 16w..16w+15, all 128 outputs. MFMA operand layout (16x16x32): lane l holds
// A[l%16][8(l/16)..+7], B[8(l/16)..+7][l%16]; result lane l holds
// D[4(l/16)+j][l%16], j = 0..3.
__device__ __forceinline__ void hidden_layer(const bfbits *hin, const bfbits *__restrict__ W,
                                             const float *__restrict__ bias, float *__restrict__ zout,
                                             bfbits *hout, uint32_t r0, uint32_t N) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    f32x4 acc[8];
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int k0 = 32 * kk + 8 * (lane >> 4);
        const bf16x8 a = load8(hin + (16 * wave + (lane & 15)) * LDH + k0);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
            acc[nt] = mfma(a, load8(W + (16 * nt + (lane & 15)) * H + k0), acc[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = 16 * wave + 4 * (lane >> 4) + j, u = 16 * nt + (lane & 15);
            const float z = acc[nt][j] + bias[u];
            if (zout && r0 + r < N) zout[static_cast<size_t>(r0 + r) * H + u] = z;
            hout[r * LDH + u] = f2bf(gelu(z));
        }
    }
}

// Forward pass of one 64-row tile; with a target, also the tile's masked
// squared error and mask count (part[2*wg], part[2*wg+1]). The pre-activations
// z1..z3 are kept for the backward pass only when z1 is not null.
__global__ void __launch_bounds__(THREADS)
mlp_forward(const float *__restrict__ x, uint32_t N, const float *__restrict__ theta,
            const bfbits *__restrict__ W2b, const bfbits *__restrict__ W3b,
            float *__restrict__ z1, float *__restrict__ z2, float *__restrict__ z3,
            float *__restrict__ y, const float *__restrict__ target,
            const float *__restrict__ mask, float *__restrict__ loss_part) {
    __shared__ __attribute__((aligned(16))) bfbits hA[ROWS * LDH];
    __shared__ __attribute__((aligned(16))) bfbits hB[ROWS * LDH];
    __shared__ float red[2][THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t r0 = blockIdx.x * ROWS;

    for (int idx = tid; idx < ROWS * H; idx += THREADS) {  // layer 1: 3 inputs
        const int r = idx / H, u = idx % H;
        const uint32_t gr = r0 + r;
        float z = 0.f;
        if (gr < N) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                acc = fmaf(rbf(x[static_cast<size_t>(gr) * 3 + k]), rbf(theta[oW1 + u * 3 + k]), acc);
            z = acc + theta[ob1 + u];
            if (z1) z1[static_cast<size_t>(gr) * H + u] = z;
        }
        hA[r * LDH + u] = f2bf(gelu(z));
    }
    __syncthreads();
    hidden_layer(hA, W2b, theta + ob2, z2, hB, r0, N);
    __syncthreads();
    hidden_layer(hB, W3b, theta + ob3, z3, hA, r0, N);
    __syncthreads();

    // output unit: four lanes per row, 32 inputs each
    const int r = 16 * wave + (lane >> 2), q = lane & 3;
    float acc = 0.f;
    for (int j = 0; j < 32; ++j) {
        const int u = 32 * q + j;
        acc = fmaf(bf2f(hA[r * LDH + u]), rbf(theta[ow4 + u]), acc);
    }
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    const float yv = acc + theta[ob4];
    const uint32_t gr = r0 + r;
    float se = 0.f, cnt = 0.f;
    if (q == 0 && gr < N) {
        y[gr] = yv;
        if (target) {
            const float m = (mask == nullptr || mask[gr] != 0.f) ? 1.f : 0.f;
            const float d = yv - target[gr];
            se = m * d * d;
            cnt = m;
        }
    }
    if (target) {
        for (int sh = 32; sh >= 1; sh >>= 1) {
            se += __shfl_xor(se, sh);
            cnt += __shfl_xor(cnt, sh);
        }
        if (lane == 0) {
            red[0][wave] = se;
            red[1][wave] = cnt;
        }
        __syncthreads();
        if (tid == 0) {
            float a = 0.f, b = 0.f;
            for (int w = 0; w < THREADS / 64; ++w) {
                a += red[0][w];
                b += red[1][w];
            }
            loss_part[2 * blockIdx.x] = a;
            loss_part[2 * blockIdx.x + 1] = b;
        }
    }
}

// Masked loss and row count from the per-tile partials (one workgroup, fixed order).
__global__ void __launch_bounds__(THREADS)
mlp_loss_finalize(const float *__restrict__ loss_part, uint32_t nwg, float *__restrict__ scal) {
    __shared__ double a[THREADS], b[THREADS];
    double sa = 0.0, sb = 0.0;
    for (uint32_t i = threadIdx.x; i < nwg; i += THREADS) {
        sa += loss_part[2 * i];
        sb += loss_part[2 * i + 1];
    }
    a[threadIdx.x] = sa;
    b[threadIdx.x] = sb;
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int i = 0; i < THREADS; ++i) {
            ta += a[i];
            tb += b[i];
        }
        scal[0] = tb > 0.0 ? static_cast<float>(ta / tb) : 0.f;  // loss
        scal[1] = static_cast<float>(tb);                          // M
    }
}

// dW [H][H] (+)= dzT^T-product: C[i][j] = sum_r dz[r][i] h[r][j] over the
// tile, from the transposed tiles dzT [H][ROWS] and hT [H][ROWS] in LDS.
// Wavefront w computes i in 32w..32w+31 (two row blocks), all j.
__device__ __forceinline__ void weight_grad(const bfbits *dzT, const bfbits *hT,
                                            float *__restrict__ out, bool accumulate) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int mt = 2 * wave + half;
        f32x4 acc[8];
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < ROWS / 32; ++kk) {
            const int k0 = 32 * kk + 8 * (lane >> 4);
            const bf16x8 a = load8(dzT + (16 * mt + (lane & 15)) * LDR + k0);
#pragma unroll
            for (int nt = 0; nt < 8; ++nt)
                acc[nt] = mfma(a, load8(hT + (16 * nt + (lane & 15)) * LDR + k0), acc[nt]);
        }
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float *o = out + (16 * mt + 4 * (lane >> 4) + j) * H + 16 * nt + (lane & 15);
                *o = accumulate ? *o + acc[nt][j] : acc[nt][j];
            }
    }
}

// dh [ROWS][H] = dz W: A = dz row-major bf16 [ROWS][H] in LDS, B[k][n] = W[k][n]
// read from the transposed weight copy WT[n][k] in HBM. Result kept in registers:
// lane holds dh[16w + 4(l/16) + j][16nt + l%16].
__device__ __forceinline__ void input_grad(const bfbits *dz, const bfbits *__restrict__ WT,
                                           f32x4 (&acc)[8]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int k0 = 32 * kk + 8 * (lane >> 4);
        const bf16x8 a = load8(dz + (16 * wave + (lane & 15)) * LDH + k0);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
            acc[nt] = mfma(a, load8(WT + (16 * nt + (lane & 15)) * H + k0), acc[nt]);
    }
}

// Backward pass of the 64-row tiles blockIdx.x, blockIdx.x + gridDim.x, ...
// in that order: their gradients summed into part[wg * NP .. + NP) (then
// summed over workgroups by mlp_reduce). The grid is capped, so the partials
// take at most kBwdGrid * NP floats whatever the number of rows. Every
// partial element is read and written by one fixed thread, in program order.
__global__ void __launch_bounds__(THREADS)
mlp_backward(const float *__restrict__ x, const float *__restrict__ target,
             const float *__restrict__ mask, uint32_t N, const float *__restrict__ theta,
             const bfbits *__restrict__ W2bT, const bfbits *__restrict__ W3bT,
             const float *__restrict__ z1, const float *__restrict__ z2,
             const float *__restrict__ z3, const float *__restrict__ y,
             const float *__restrict__ scal, float *__restrict__ part) {
    __shared__ __attribute__((aligned(16))) bfbits dz[ROWS * LDH];   // bf(dz) row-major
    __shared__ __attribute__((aligned(16))) bfbits dzT[H * LDR];     // bf(dz) transposed
    __shared__ __attribute__((aligned(16))) bfbits hT[H * LDR];      // bf(h) transposed
    __shared__ float zf[ROWS * H];                                   // dz float32
    __shared__ float dy[ROWS];
    __shared__ float colsum[2][H];
    const int tid = threadIdx.x;
    float *out = part + static_cast<size_t>(blockIdx.x) * NP;
    const float M = scal[1];
    const uint32_t ntiles = (N + ROWS - 1) / ROWS;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint32_t r0 = tile * ROWS;
    const bool acc_on = tile != blockIdx.x;  // add to the partial of earlier tiles
    auto put = [&](uint32_t i, float v) { out[i] = acc_on ? out[i] + v : v; };
    __syncthreads();  // the previous tile is done with the shared buffers

    if (tid < ROWS) {
        const uint32_t gr = r0 + tid;
        float v = 0.f;
        if (gr < N && M > 0.f) {
            const float m = (mask == nullptr || mask[gr] != 0.f) ? 1.f : 0.f;
            v = m * 2.f * (y[gr] - target[gr]) / M;
        }
        dy[tid] = v;
    }
    __syncthreads();

    // output unit and layer 3 pre-activation gradient; h2 transposed
    {
        const int j = tid & (H - 1), rh = tid >> 7;  // two lanes per unit, 32 rows each
        const float w4 = rbf(theta[ow4 + j]);
        float sw4 = 0.f, sb3 = 0.f;
        for (int rr = 0; rr < ROWS / 2; ++rr) {
            const int r = rh * (ROWS / 2) + rr;
            const uint32_t gr = r0 + r;
            float d = 0.f, h2 = 0.f;
            if (gr < N) {
                const float zz3 = z3[static_cast<size_t>(gr) * H + j];
                sw4 = fmaf(dy[r], rbf(gelu(zz3)), sw4);
                d = dy[r] * w4 * gelu_grad(zz3);
                h2 = gelu(z2[static_cast<size_t>(gr) * H + j]);
            }
            sb3 += d;
            const bfbits db = f2bf(d);
            dz[r * LDH + j] = db;
            dzT[j * LDR + r] = db;
            hT[j * LDR + r] = f2bf(h2);
        }
        if (rh == 1) {
            colsum[0][j] = sw4;
            colsum[1][j] = sb3;
        }
        __syncthreads();
        if (rh == 0) {
            put(ow4 + j, sw4 + colsum[0][j]);
            put(ob3 + j, sb3 + colsum[1][j]);
        }
        if (tid == 0) {
            float s = 0.f;
            for (int r = 0; r < ROWS; ++r) s += dy[r];
            put(ob4, s);
        }
    }
    __syncthreads();
    weight_grad(dzT, hT, out + oW3, acc_on);

    // layer 2: dh2 = bf(dz3) W3, dz2 = dh2 gelu'(z2)
    {
        f32x4 acc[8];
        input_grad(dz, W3bT, acc);
        __syncthreads();  // every wavefront is done reading dz / dzT / hT
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 16 * wave + 4 * (lane >> 4) + j, u = 16 * nt + (lane & 15);
                const uint32_t gr = r0 + r;
                float d = 0.f;
                if (gr < N) d = acc[nt][j] * gelu_grad(z2[static_cast<size_t>(gr) * H + u]);
                zf[r * H + u] = d;
                const bfbits db = f2bf(d);
                dz[r * LDH + u] = db;
                dzT[u * LDR + r] = db;
            }
        for (int idx = tid; idx < ROWS * H; idx += THREADS) {  // h1 transposed
            const int r = idx / H, u = idx % H;
            const uint32_t gr = r0 + r;
            hT[u * LDR + r] = f2bf(gr < N ? gelu(z1[static_cast<size_t>(gr) * H + u]) : 0.f);
        }
    }
    __syncthreads();
    if (tid < H) {
        float s = 0.f;
        for (int r = 0; r < ROWS; ++r) s += zf[r * H + tid];
        put(ob2 + tid, s);
    }
    weight_grad(dzT, hT, out + oW2, acc_on);

    // layer 1: dh1 = bf(dz2) W2, dz1 = dh1 gelu'(z1), 3-input weights on vector lanes
    {
        f32x4 acc[8];
        input_grad(dz, W2bT, acc);
        __syncthreads();
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 16 * wave + 4 * (lane >> 4) + j, u = 16 * nt + (lane & 15);
                const uint32_t gr = r0 + r;
                float d = 0.f;
                if (gr < N) d = acc[nt][j] * gelu_grad(z1[static_cast<size_t>(gr) * H + u]);
                zf[r * H + u] = d;
            }
    }
    __syncthreads();
    for (int idx = tid; idx < H * 4; idx += THREADS) {  // dW1[i][k] (k < 3) and db1[i] (k = 3)
        const int i = idx >> 2, k = idx & 3;
        float s = 0.f;
        for (int r = 0; r < ROWS; ++r) {
            const uint32_t gr = r0 + r;
            const float xv = (k < 3) ? (gr < N ? rbf(x[static_cast<size_t>(gr) * 3 + k]) : 0.f) : 1.f;
            s = fmaf(zf[r * H + i], xv, s);
        }
        if (k < 3)
            put(oW1 + i * 3 + k, s);
        else
            put(ob1 + i, s);
    }
    }
}

// grad[p] = sum over tiles of part[tile][p], tiles in order.
__global__ void mlp_reduce(const float *__restrict__ part, uint32_t nwg, float *__restrict__ grad) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= static_cast<uint32_t>(NP)) return;
    float s = 0.f;
    for (uint32_t w = 0; w < nwg; ++w) s += part[static_cast<size_t>(w) * NP + p];
    grad[p] = s;
}

// Adam with bias corrections c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t).
__global__ void mlp_adam(float *__restrict__ theta, const float *__restrict__ grad,
                         float *__restrict__ m, float *__restrict__ v, float lr, float c1,
                         float c2) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= static_cast<uint32_t>(NP)) return;
    const float g = grad[p];
    const float mm = 0.9f * m[p] + 0.1f * g;
    const float vv = 0.999f * v[p] + 0.001f * g * g;
    m[p] = mm;
    v[p] = vv;
    theta[p] -= lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
}

// bfloat16 copies of the hidden-layer weights, output-major and transposed.
__global__ void mlp_prep(const float *__restrict__ theta, bfbits *__restrict__ W2b,
                         bfbits *__restrict__ W2bT, bfbits *__restrict__ W3b,
                         bfbits *__restrict__ W3bT) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= static_cast<uint32_t>(H * H)) return;
    const uint32_t o = i / H, k = i % H;
    const bfbits a = f2bf(theta[oW2 + i]), b = f2bf(theta[oW3 + i]);
    W2b[i] = a;
    W2bT[k * H + o] = a;
    W3b[i] = b;
    W3bT[k * H + o] = b;
}

// Initial parameters: uniform in (-1/sqrt(fan_in), 1/sqrt(fan_in)) from
// Philox-4x32-10, key (seed, 0x4D4C5031), counter (p, 0, 0, 0).
__global__ void mlp_init_params(float *__restrict__ theta, uint32_t seed) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= static_cast<uint32_t>(NP)) return;
    const U4 r = philox10(U4{p, 0u, 0u, 0u}, seed, 0x4D4C5031u);
    const float u = (static_cast<float>(r.x >> 8) + 0.5f) * (1.0f / 16777216.0f);
    const float fan_in = (p < static_cast<uint32_t>(ob1 + H)) ? 3.f : static_cast<float>(H);
    theta[p] = (2.f * u - 1.f) / sqrtf(fan_in);
}

}  // namespace
}  // namespace pcpd

using pcpd::bfbits;

struct pcpd_mlp {
    hipStream_t stream = nullptr;
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    bfbits *wb = nullptr;  // W2b, W2bT, W3b, W3bT
    float *scal = nullptr;  // loss, M
    float *z = nullptr;     // z1, z2, z3 for cap_rows rows
    float *ytmp = nullptr;  // cap_rows
    float *loss_part = nullptr;  // 2 * cap_wg
    float *part = nullptr;  // bwd_grid(cap_rows) * NP
    uint32_t cap_rows = 0, cap_wg = 0;
    float *h_scal = nullptr;  // pinned
    int64_t step = 0;
    bool broken = false;
};

namespace {

int mfail(pcpd_mlp *net, hipError_t e) {
    if (e == hipSuccess) return PCPD_OK;
    if (net) net->broken = true;
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? PCPD_ENOMEM : PCPD_EDEVICE;
}

bfbits *W2b(pcpd_mlp *n) { return n->wb; }
bfbits *W2bT(pcpd_mlp *n) { return n->wb + pcpd::H * pcpd::H; }
bfbits *W3b(pcpd_mlp *n) { return n->wb + 2 * pcpd::H * pcpd::H; }
bfbits *W3bT(pcpd_mlp *n) { return n->wb + 3 * pcpd::H * pcpd::H; }

hipError_t prep(pcpd_mlp *n) {
    hipLaunchKernelGGL(pcpd::mlp_prep, dim3((pcpd::H * pcpd::H + 255) / 256), dim3(256), 0,
                       n->stream, n->theta, W2b(n), W2bT(n), W3b(n), W3bT(n));
    return hipGetLastError();
}

// Workgroups of the backward pass at most: each sums the gradients of its
// tiles into one partial (NP floats), so the partials take at most
// kBwdGrid * NP * 4 bytes (69 MB) for any number of rows; 512 workgroups
// cover the 256 CUs twice.
constexpr uint32_t kBwdGrid = 512;

uint32_t bwd_grid(uint32_t N) {
    const uint32_t nwg = (N + pcpd::ROWS - 1) / pcpd::ROWS;
    return nwg < kBwdGrid ? nwg : kBwdGrid;
}

// Scratch for N rows, grown on demand (the stream is synchronised first):
// the loss partials (2 floats per 64-row tile) always; for a gradient
// (train = true, N <= PCPD_MLP_MAX_TRAIN_ROWS) also the pre-activations of
// every row (3 * 128 floats), the outputs and the backward partials.
hipError_t reserve(pcpd_mlp *n, uint32_t N, bool train) {
    const uint32_t nwg = (N + pcpd::ROWS - 1) / pcpd::ROWS;
    const size_t rows = static_cast<size_t>(nwg) * pcpd::ROWS;
    hipError_t e = hipSuccess;
    if (nwg > n->cap_wg) {
        if ((e = hipStreamSynchronize(n->stream)) != hipSuccess) return e;
        (void)hipFree(n->loss_part);
        n->loss_part = nullptr;
        n->cap_wg = 0;
        if ((e = hipMalloc(&n->loss_part, 2 * static_cast<size_t>(nwg) * sizeof(float))) != hipSuccess)
            return e;
        n->cap_wg = nwg;
    }
    if (train && rows > n->cap_rows) {
        if ((e = hipStreamSynchronize(n->stream)) != hipSuccess) return e;
        (void)hipFree(n->z);
        (void)hipFree(n->ytmp);
        (void)hipFree(n->part);
        n->z = n->ytmp = n->part = nullptr;
        n->cap_rows = 0;
        if ((e = hipMalloc(&n->z, 3 * rows * pcpd::H * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc(&n->ytmp, rows * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc(&n->part, static_cast<size_t>(bwd_grid(N)) * pcpd::NP * sizeof(float))) !=
            hipSuccess)
            return e;
        n->cap_rows = static_cast<uint32_t>(rows);
    }
    return hipSuccess;
}

// keep_z: store the pre-activations for a backward pass (scratch reserved
// with train = true).
hipError_t forward(pcpd_mlp *n, const float *x, uint32_t N, float *y, const float *target,
                   const float *mask, bool keep_z) {
    const uint32_t nwg = (N + pcpd::ROWS - 1) / pcpd::ROWS;
    const size_t rows = static_cast<size_t>(n->cap_rows);
    float *z1 = keep_z ? n->z : nullptr;
    float *z2 = keep_z ? n->z + rows * pcpd::H : nullptr;
    float *z3 = keep_z ? n->z + 2 * rows * pcpd::H : nullptr;
    hipLaunchKernelGGL(pcpd::mlp_forward, dim3(nwg), dim3(pcpd::THREADS), 0, n->stream, x, N,
                       n->theta, W2b(n), W3b(n), z1, z2, z3, y, target, mask, n->loss_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !target) return e;
    hipLaunchKernelGGL(pcpd::mlp_loss_finalize, dim3(1), dim3(pcpd::THREADS), 0, n->stream,
                       n->loss_part, nwg, n->scal);
    return hipGetLastError();
}

hipError_t backward(pcpd_mlp *n, const float *x, const float *target, const float *mask,
                    uint32_t N) {
    const uint32_t nwg = bwd_grid(N);
    const size_t rows = static_cast<size_t>(n->cap_rows);
    hipLaunchKernelGGL(pcpd::mlp_backward, dim3(nwg), dim3(pcpd::THREADS), 0, n->stream, x,
                       target, mask, N, n->theta, W2bT(n), W3bT(n), n->z, n->z + rows * pcpd::H,
                       n->z + 2 * rows * pcpd::H, n->ytmp, n->scal, n->part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pcpd::mlp_reduce, dim3((pcpd::NP + 255) / 256), dim3(256), 0, n->stream,
                       n->part, nwg, n->grad);
    return hipGetLastError();
}

bool rows_ok(uint32_t N) { return N >= 1 && N <= PCPD_MLP_MAX_ROWS; }
bool train_rows_ok(uint32_t N) { return N >= 1 && N <= PCPD_MLP_MAX_TRAIN_ROWS; }

}  // namespace

extern "C" {

int pcpd_mlp_init(pcpd_mlp **out, uint32_t seed, const pcpd_device *dev) {
    if (!out) return PCPD_EINVAL;
    pcpd_mlp *n = new (std::nothrow) pcpd_mlp();
    if (!n) return PCPD_ENOMEM;
    n->stream = dev ? static_cast<hipStream_t>(dev->hip_stream) : nullptr;
    const size_t P = pcpd::NP * sizeof(float);
    hipError_t e;
    if ((e = hipMalloc(&n->theta, P)) != hipSuccess || (e = hipMalloc(&n->m, P)) != hipSuccess ||
        (e = hipMalloc(&n->v, P)) != hipSuccess || (e = hipMalloc(&n->grad, P)) != hipSuccess ||
        (e = hipMalloc(&n->wb, 4 * pcpd::H * pcpd::H * sizeof(bfbits))) != hipSuccess ||
        (e = hipMalloc(&n->scal, 2 * sizeof(float))) != hipSuccess ||
        (e = hipHostMalloc(&n->h_scal, 2 * sizeof(float), hipHostMallocDefault)) != hipSuccess ||
        (e = hipMemsetAsync(n->m, 0, P, n->stream)) != hipSuccess ||
        (e = hipMemsetAsync(n->v, 0, P, n->stream)) != hipSuccess) {
        pcpd_mlp_free(n);
        return mfail(nullptr, e);
    }
    hipLaunchKernelGGL(pcpd::mlp_init_params, dim3((pcpd::NP + 255) / 256), dim3(256), 0,
                       n->stream, n->theta, seed);
    if ((e = hipGetLastError()) != hipSuccess || (e = prep(n)) != hipSuccess ||
        (e = hipStreamSynchronize(n->stream)) != hipSuccess) {
        pcpd_mlp_free(n);
        return mfail(nullptr, e);
    }
    *out = n;
    return PCPD_OK;
}

int pcpd_mlp_get_params(pcpd_mlp *n, float *host_params) {
    if (!n || !host_params) return PCPD_EINVAL;
    if (n->broken) return PCPD_ESTATE;
    hipError_t e = hipMemcpyAsync(host_params, n->theta, pcpd::NP * sizeof(float),
                                  hipMemcpyDeviceToHost, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    return mfail(n, e);
}

int pcpd_mlp_set_params(pcpd_mlp *n, const float *host_params) {
    if (!n || !host_params) return PCPD_EINVAL;
    if (n->broken) return PCPD_ESTATE;
    const size_t P = pcpd::NP * sizeof(float);
    hipError_t e = hipMemcpyAsync(n->theta, host_params, P, hipMemcpyHostToDevice, n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n->m, 0, P, n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n->v, 0, P, n->stream);
    if (e == hipSuccess) e = prep(n);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    n->step = 0;
    return mfail(n, e);
}

int pcpd_mlp_predict(pcpd_mlp *n, const float *x_dev, uint32_t N, float *y_dev) {
    if (!n || !x_dev || !y_dev || !rows_ok(N)) return PCPD_EINVAL;
    if (n->broken) return PCPD_ESTATE;
    hipError_t e = reserve(n, N, false);
    if (e == hipSuccess) e = forward(n, x_dev, N, y_dev, nullptr, nullptr, false);
    return mfail(n, e);
}

int pcpd_mlp_loss(pcpd_mlp *n, const float *x_dev, const float *target_dev,
                  const float *mask_dev, uint32_t N, float *y_dev, float *loss_out) {
    if (!n || !x_dev || !target_dev || !y_dev || !loss_out || !rows_ok(N)) return PCPD_EINVAL;
    if (n->broken) return PCPD_ESTATE;
    hipError_t e = reserve(n, N, false);
    if (e == hipSuccess) e = forward(n, x_dev, N, y_dev, target_dev, mask_dev, false);
    if (e == hipSuccess)
        e = hipMemcpyAsync(n->h_scal, n->scal, 2 * sizeof(float), hipMemcpyDeviceToHost, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) return mfail(n, e);
    *loss_out = n->h_scal[0];
    return PCPD_OK;
}

int pcpd_mlp_grads(pcpd_mlp *n, const float *x_dev, const float *target_dev,
                   const float *mask_dev, uint32_t N, float *host_grads, float *loss_out) {
    if (!n || !x_dev || !target_dev || !host_grads || !train_rows_ok(N)) return PCPD_EINVAL;
    if (n->broken) return PCPD_ESTATE;
    hipError_t e = reserve(n, N, true);
    if (e == hipSuccess) e = forward(n, x_dev, N, n->ytmp, target_dev, mask_dev, true);
    if (e == hipSuccess) e = backward(n, x_dev, target_dev, mask_dev, N);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_grads, n->grad, pcpd::NP * sizeof(float), hipMemcpyDeviceToHost,
                           n->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(n->h_scal, n->scal, 2 * sizeof(float), hipMemcpyDeviceToHost, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) return mfail(n, e);
    if (loss_out) *loss_out = n->h_scal[0];
    return PCPD_OK;
}

int pcpd_mlp_train_step(pcpd_mlp *n, const float *x_dev, const float *target_dev,
                        const float *mask_dev, uint32_t N, float lr, float *loss_out) {
    if (!n || !x_dev || !target_dev || !train_rows_ok(N) || !(lr >= 0.f)) return PCPD_EINVAL;
    if (n->broken) return PCPD_ESTATE;
    hipError_t e = reserve(n, N, true);
    if (e == hipSuccess) e = forward(n, x_dev, N, n->ytmp, target_dev, mask_dev, true);
    if (e == hipSuccess) e = backward(n, x_dev, target_dev, mask_dev, N);
    if (e == hipSuccess && loss_out)
        e = hipMemcpyAsync(n->h_scal, n->scal, 2 * sizeof(float), hipMemcpyDeviceToHost, n->stream);
    if (e != hipSuccess) return mfail(n, e);
    n->step += 1;
    const double c1 = 1.0 / (1.0 - std::pow(0.9, static_cast<double>(n->step)));
    const double c2 = 1.0 / (1.0 - std::pow(0.999, static_cast<double>(n->step)));
    hipLaunchKernelGGL(pcpd::mlp_adam, dim3((pcpd::NP + 255) / 256), dim3(256), 0, n->stream,
                       n->theta, n->grad, n->m, n->v, lr, static_cast<float>(c1),
                       static_cast<float>(c2));
    e = hipGetLastError();
    if (e == hipSuccess) e = prep(n);
    if (e == hipSuccess && loss_out) {
        e = hipStreamSynchronize(n->stream);
        if (e == hipSuccess) *loss_out = n->h_scal[0];
    }
    return mfail(n, e);
}

int pcpd_mlp_free(pcpd_mlp *n) {
    if (!n) return PCPD_EINVAL;
    (void)hipStreamSynchronize(n->stream);
    (void)hipFree(n->theta);
    (void)hipFree(n->m);
    (void)hipFree(n->v);
    (void)hipFree(n->grad);
    (void)hipFree(n->wb);
    (void)hipFree(n->scal);
    (void)hipFree(n->z);
    (void)hipFree(n->ytmp);
    (void)hipFree(n->loss_part);
    (void)hipFree(n->part);
    if (n->h_scal) (void)hipHostFree(n->h_scal);
    delete n;
    return PCPD_OK;
}

}  // extern "C"
