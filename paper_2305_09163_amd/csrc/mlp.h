// Learned smoothness indicator (a project extension beside the WENO5
// reconstruction of Sec. 3.2): a 15 -> 32 -> 32 -> 1 perceptron with GELU
// (tanh form) on both hidden layers and a logistic output, evaluated by
// whole wavefronts on bf16 matrix cores (FP32 accumulation).
//
// Inputs of one (cell, direction): for alpha1, rho = a1r1 + a2r2 and p, the 5
// stencil values minus the centre value, divided by
// max(max_j |v_j - v_centre|, sqrt(eps)); a 16th input is always 0.
//
// Number formats: the operands of every matrix product (inputs, W1, W2, the
// hidden activations H1 and, in training, dZ2 and dZ1) are rounded to bf16
// (nearest, ties to even); biases, W3, the output layer, GELU and all other
// element-wise work are FP32.  Parameters arrive as FP32 in the flat order
// W1 [15][32] (input-major), b1 [32], W2 [32][32] (input-major), b2 [32],
// W3 [32], b3.
//
// Wavefront layout.  A tile is 16 samples; lane l has s = l % 16 (sample of
// the tile) and g = l / 16 (k group).  All products are formed transposed
// (hidden units x samples), so the output of one layer is already the input
// operand of the next:
//   Z1^T = W1^T X^T      16x16x16 MFMA per 16 hidden units: lane l supplies
//                        X[s][4g .. 4g+3] and receives Z1[s][16b + 4g + t];
//   Z2^T = W2^T H1^T     16x16x32 MFMA: the k slots of lane group g are taken
//                        as hidden units u(g, t) = 4g + t (t < 4) and
//                        16 + 4g + t - 4 (t >= 4), exactly the units the lane
//                        holds after layer 1, and W2^T is loaded with the same
//                        permutation;
//   z = W3 . H2 + b3     per-lane partial sums over its 8 units, then a sum
//                        over the 4 lane groups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfc {
namespace mlp {

constexpr int NIN = 15, NH = 32, NPARAM = 1601;
constexpr int OW1 = 0, OB1 = 480, OW2 = 512, OB2 = 1536, OW3 = 1568, OB3 = 1600;

typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// float -> bf16 bits, nearest with ties to even (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// double -> bf16 bits, rounded once from the double: round the significand
// to 8 bits in the double's own encoding, after which the conversion to
// float and the truncation to 16 bits are exact.
__device__ __forceinline__ uint16_t bf16_bits(double x)
{
    uint64_t u = (uint64_t)__double_as_longlong(x);
    u += ((1ull << 44) - 1) + ((u >> 45) & 1ull);
    u &= ~((1ull << 45) - 1);
    return (uint16_t)(__float_as_uint((float)__longlong_as_double((long long)u)) >> 16);
}

__device__ __forceinline__ __bf16 as_bf16(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

// u(g, t): the hidden unit in k slot t of lane group g (see the header)
__device__ __forceinline__ int unit(int g, int t) { return t < 4 ? 4 * g + t : 12 + 4 * g + t; }

constexpr float kC = 0.7978845608028654f;  // sqrt(2 / pi)
constexpr float kA = 0.044715f;

__device__ __forceinline__ float tanh_f(float u)
{
    // 1 - 2 / (1 + e^(2u)); saturates to +-1 for large |u| (rcp(inf) = 0)
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * u));
}

__device__ __forceinline__ float gelu(float x)
{
    const float t = tanh_f(kC * x * (1.0f + kA * x * x));
    return 0.5f * x * (1.0f + t);
}

__device__ __forceinline__ float gelu_grad(float x)
{
    const float t = tanh_f(kC * x * (1.0f + kA * x * x));
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * kC * (1.0f + 3.0f * kA * x * x);
}

// Parameters staged in LDS in lane order: every lane reads its own operands
// with one 8- or 16-byte access.
struct Params {
    s4 a1[2][64];     // W1^T rows 16b + s, k = 4g + t   (layer 1, A operand)
    bf8 a2[2][64];    // W2^T rows 16b + s, k slot t -> unit u(g, t)   (layer 2)
    float b1[NH], b2[NH], w3[NH];
    float b3, pad[3];
};

// Backward-only operand: W2 rows 16b + s (input units), k slot t -> output
// unit u(g, t), for dH1^T = W2 dZ2^T.
struct ParamsT {
    bf8 a2t[2][64];
};

// Fill P from the flat FP32 parameters; call with all threads of the block,
// then synchronise.
__device__ inline void stage_params(Params &P, ParamsT *PT, const float *__restrict__ w, int tid, int nthreads)
{
    for (int e = tid; e < 2 * 64; e += nthreads) {
        const int b = e / 64, l = e % 64, g = l / 16, s = l % 16;
        s4 a;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int f = 4 * g + t;
            a[t] = (short)(f < NIN ? bf16_bits(w[OW1 + f * NH + 16 * b + s]) : 0);
        }
        P.a1[b][l] = a;
        bf8 a2, a2t;
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const int u = unit(g, t);
            a2[t] = as_bf16(bf16_bits(w[OW2 + u * NH + 16 * b + s]));
            a2t[t] = as_bf16(bf16_bits(w[OW2 + (16 * b + s) * NH + u]));
        }
        P.a2[b][l] = a2;
        if (PT) PT->a2t[b][l] = a2t;
    }
    for (int e = tid; e < NH; e += nthreads) {
        P.b1[e] = w[OB1 + e];
        P.b2[e] = w[OB2 + e];
        P.w3[e] = w[OW3 + e];
    }
    if (tid == 0) P.b3 = w[OB3];
}

// Forward state of one tile, as held by one lane (its sample s, its 8 units).
struct Fwd {
    float z1[8], z2[8], h2[8];  // pre-activations and layer-2 activations, slot order
    bf8 h1;                     // layer-1 activations (bf16), slot order
    uint16_t h1_bits[8];        // the same activations as bit patterns
    float z;                    // output logit of sample s (all 4 lane groups)
};

// One tile through the network.  xb: features 4g .. 4g+3 of sample s.
__device__ __forceinline__ void forward_tile(const Params &P, s4 xb, int lane, Fwd &F)
{
    const int g = lane >> 4;
#pragma unroll
    for (int b = 0; b < 2; b++) {
        f4 c = *(const f4 *)&P.b1[16 * b + 4 * g];
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(P.a1[b][lane], xb, c, 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; t++) {
            F.z1[4 * b + t] = c[t];
            F.h1_bits[4 * b + t] = bf16_bits(gelu(c[t]));
            F.h1[4 * b + t] = as_bf16(F.h1_bits[4 * b + t]);
        }
    }
    float z = 0.0f;
#pragma unroll
    for (int b = 0; b < 2; b++) {
        f4 c = *(const f4 *)&P.b2[16 * b + 4 * g];
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(P.a2[b][lane], F.h1, c, 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; t++) {
            F.z2[4 * b + t] = c[t];
            F.h2[4 * b + t] = gelu(c[t]);
            z += P.w3[16 * b + 4 * g + t] * F.h2[4 * b + t];
        }
    }
    z += __shfl_xor(z, 16, 64);
    z += __shfl_xor(z, 32, 64);
    F.z = z + P.b3;
}

// Inference-only forward: the logit of sample s of the tile.
__device__ __forceinline__ float logit_tile(const Params &P, s4 xb, int lane)
{
    const int g = lane >> 4;
    bf8 h1;
#pragma unroll
    for (int b = 0; b < 2; b++) {
        f4 c = *(const f4 *)&P.b1[16 * b + 4 * g];
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(P.a1[b][lane], xb, c, 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; t++) h1[4 * b + t] = as_bf16(bf16_bits(gelu(c[t])));
    }
    float z = 0.0f;
#pragma unroll
    for (int b = 0; b < 2; b++) {
        f4 c = *(const f4 *)&P.b2[16 * b + 4 * g];
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(P.a2[b][lane], h1, c, 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; t++) z += P.w3[16 * b + 4 * g + t] * gelu(c[t]);
    }
    z += __shfl_xor(z, 16, 64);
    z += __shfl_xor(z, 32, 64);
    return z + P.b3;
}

// Features of one (cell, direction) from the three 5-cell stencils, as bf16
// bits (16 values, the last 0).  sqrt_eps is sqrt(weno eps).
template <class T>
__device__ __forceinline__ void features(const T *a, const T *r, const T *p, T sqrt_eps, uint16_t *out)
{
    const T *v3[3] = {a, r, p};
#pragma unroll
    for (int m = 0; m < 3; m++) {
        const T *v = v3[m];
        T d[5], mx = T(0);
#pragma unroll
        for (int j = 0; j < 5; j++) {
            d[j] = v[j] - v[2];
            mx = d[j] < T(0) ? (-d[j] > mx ? -d[j] : mx) : (d[j] > mx ? d[j] : mx);
        }
        const T scale = mx > sqrt_eps ? mx : sqrt_eps;
#pragma unroll
        for (int j = 0; j < 5; j++) out[5 * m + j] = bf16_bits(d[j] / scale);
    }
    out[15] = 0;
}

// Wavefront-cooperative decision: every lane supplies the features of its
// own sample (64 samples, 4 tiles) and gets back whether its sample's logit
// exceeds `logit_tau`.  `scratch` is this wavefront's 64 x 16 bf16 LDS area.
// All 64 lanes must execute this call.
__device__ __forceinline__ bool smooth_wave(const Params &P, uint16_t *scratch, const uint16_t *feat, float logit_tau,
                                            int lane)
{
    uint4 *row = (uint4 *)(scratch + lane * 16);
    const uint32_t *f32 = (const uint32_t *)feat;
    row[0] = make_uint4(f32[0], f32[1], f32[2], f32[3]);
    row[1] = make_uint4(f32[4], f32[5], f32[6], f32[7]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int g = lane >> 4, s = lane & 15;
    bool smooth = false;
#pragma unroll
    for (int tile = 0; tile < 4; tile++) {
        const s4 xb = *(const s4 *)(scratch + (16 * tile + s) * 16 + 4 * g);
        const float z = logit_tile(P, xb, lane);
        if (g == tile) smooth = z > logit_tau;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return smooth;
}

// smooth_wave for a stencil read from memory with a stride: alpha1, the two
// partial densities (summed to rho) and p at positions 0, stride, .., 4 stride.
template <class T>
__device__ __forceinline__ bool smooth_stencil(const Params &P, uint16_t *scratch, const T *a, const T *r1,
                                               const T *r2, const T *p, int stride, T sqrt_eps, float logit_tau,
                                               int lane)
{
    T av[5], rv[5], pv[5];
#pragma unroll
    for (int j = 0; j < 5; j++) {
        av[j] = a[j * stride];
        rv[j] = r1[j * stride] + r2[j * stride];
        pv[j] = p[j * stride];
    }
    uint16_t f[16];
    features<T>(av, rv, pv, sqrt_eps, f);
    return smooth_wave(P, scratch, f, logit_tau, lane);
}

}  // namespace mlp
}  // namespace mfc
