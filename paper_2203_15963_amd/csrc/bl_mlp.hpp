// bl_mlp.hpp -- the step-proposal network on gfx950 matrix cores.
//
// An MLP 11 -> 64 -> 64 -> 64 -> 1 with SiLU hidden activations maps the state
// at the start of a step (x^mu, k_mu, spin, log|h| and log eps of the last
// accepted step) to log|h| of the step to try.  Weights are BF16 on the matrix
// cores with FP32 accumulation; FP32 master weights are trained with Adam.
//
// Layout on the matrix cores (v_mfma_f32_16x16x32_bf16): rays are the N
// dimension.  A layer computes Z^T = W X^T with W (out x in) as the A operand
// and the activations X^T (in x rays) as B.  In that orientation lane (g, j)
// (g = lane / 16, j = lane % 16) of an output tile (mt, nt) holds units
// 16 mt + 4 g + e (e = 0..3) of ray 16 nt + j, and the next layer's B operand
// for K chunk kk can be assembled from the lane's own registers by letting
// the lane's eight K elements be units 32 kk + 4 g + e and 32 kk + 16 + 4 g + e:
// the matching A operands (weights) are stored in that K order.  The input
// layer reads its B operand from a per-wave LDS staging row per ray.
//
// Model vector (FP32, the layout of bl_mlp_* buffers): W1[64][11], b1[64],
// W2[64][64], b2[64], W3[64][64], b3[64], w4[64], b4, then the input mean[11]
// and standard deviation[11] used to normalise the features.
#pragma once

#include "bl_common.hpp"

namespace bl {

constexpr int kMlpIn = 11, kMlpH = 64;
constexpr int kW1 = 0, kB1 = kW1 + kMlpH * kMlpIn, kW2 = kB1 + kMlpH, kB2 = kW2 + kMlpH * kMlpH, kW3 = kB2 + kMlpH,
              kB3 = kW3 + kMlpH * kMlpH, kW4 = kB3 + kMlpH, kB4 = kW4 + kMlpH, kMlpNParam = kB4 + 1;
constexpr int kMu = kMlpNParam, kSig = kMu + kMlpIn, kMlpNModel = kSig + kMlpIn;
constexpr int kLogRec = 12;   // floats per step-log record: 11 features + target

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Packed model: A-operand fragments (8 BF16 per lane) in the order the lanes
// read them, then an FP32 tail.  Units of u32x4.
constexpr int kPkL1 = 0;                   // forward layer 1: [mt 4][lane 64]
constexpr int kPkL2 = kPkL1 + 4 * 64;      // forward layer 2: [mt 4][kk 2][lane 64]
constexpr int kPkL3 = kPkL2 + 8 * 64;      // forward layer 3
constexpr int kPkFwd = kPkL3 + 8 * 64;     // end of the forward fragments
constexpr int kPkB2 = kPkFwd;              // backward (W^T) layer 2: [mt 4][kk 2][lane 64]
constexpr int kPkB3 = kPkB2 + 8 * 64;      // backward layer 3
constexpr int kPkAll = kPkB3 + 8 * 64;
// FP32 tail (floats): b1, b2, b3, w4, b4, feature mean, 1 / feature std
constexpr int kTB1 = 0, kTB2 = 64, kTB3 = 128, kTW4 = 192, kTB4 = 256, kTMu = 257, kTISig = 268, kTailN = 288;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// two floats to BF16 (round to nearest even; one v_cvt_pk_bf16_f32), lo in
// the low half
__device__ __forceinline__ unsigned int pack2(float lo, float hi) {
    return __builtin_bit_cast(unsigned int, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

__device__ __forceinline__ f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// SiLU and its derivative with the hardware exp and a fast reciprocal (a few
// ulp, far below the BF16 resolution of the values they feed)
__device__ __forceinline__ float silu(float z) { return __fdividef(z, 1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    float s = __fdividef(1.0f, 1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// K index of element e of lane group g in chunk kk for a hidden-layer input.
__host__ __device__ __forceinline__ int hid_k(int kk, int g, int e) {
    return 32 * kk + (e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4));
}

// Wave-scope ordering of LDS traffic between the lanes of one wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc[mt][nt] = sum_kk A[mt][kk] B[nt][kk] for a 64-output layer.
template <int KK>
__device__ __forceinline__ void mm_layer(const u32x4 *frag, const u32x4 (&bq)[4][KK], f32x4 (&acc)[4][4], int lane) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            const u32x4 a = frag[(mt * KK + kk) * 64 + lane];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mma(a, bq[nt][kk], acc[mt][nt]);
        }
    }
}

// B operands of the next layer from this layer's outputs (own registers).
__device__ __forceinline__ void to_bfrag(const f32x4 (&h)[4][4], u32x4 (&bq)[4][2]) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const f32x4 &lo = h[2 * kk][nt], &hi = h[2 * kk + 1][nt];
            bq[nt][kk] = u32x4{pack2(lo[0], lo[1]), pack2(lo[2], lo[3]), pack2(hi[0], hi[1]), pack2(hi[2], hi[3])};
        }
}

// Normalised input features of one lane into its staging row (32 BF16).
__device__ __forceinline__ void stage_input(const float *tail, const float x[kMlpIn], u32x4 *stage, int lane) {
    float xn[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) xn[i] = i < kMlpIn ? (x[i] - tail[kTMu + i]) * tail[kTISig + i] : 0.0f;
    stage[lane * 4 + 0] = u32x4{pack2(xn[0], xn[1]), pack2(xn[2], xn[3]), pack2(xn[4], xn[5]), pack2(xn[6], xn[7])};
    stage[lane * 4 + 1] = u32x4{pack2(xn[8], xn[9]), pack2(xn[10], xn[11]), pack2(xn[12], xn[13]),
                                pack2(xn[14], xn[15])};
    stage[lane * 4 + 2] = u32x4{0u, 0u, 0u, 0u};
    stage[lane * 4 + 3] = u32x4{0u, 0u, 0u, 0u};
}

// Layer-1 B operands: lane (g, j) takes features 8g..8g+7 of ray 16 nt + j.
__device__ __forceinline__ void input_bfrag(const u32x4 *stage, u32x4 (&bq)[4][1], int lane) {
    const int g = lane >> 4, j = lane & 15;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) bq[nt][0] = stage[(16 * nt + j) * 4 + g];
}

__device__ __forceinline__ void bias_act(f32x4 (&acc)[4][4], const float *b, int lane) {
    const int g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float bb = b[16 * mt + 4 * g + e];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt][e] = silu(acc[mt][nt][e] + bb);
        }
}

// Output unit: y(ray 16 nt + j) summed over the four lane groups; lane l
// receives the output of ray l.
__device__ __forceinline__ float out_layer(const f32x4 (&h)[4][4], const float *tail, int lane) {
    const int g = lane >> 4;
    float p[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        float s = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int e = 0; e < 4; ++e) s += tail[kTW4 + 16 * mt + 4 * g + e] * h[mt][nt][e];
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        p[nt] = s;
    }
    const float y = g == 0 ? p[0] : g == 1 ? p[1] : g == 2 ? p[2] : p[3];
    return y + tail[kTB4];
}

// Forward pass of the wave: every lane of the wave must call it together
// (full EXEC).  x: this lane's raw features; returns this lane's output.
__device__ __forceinline__ float mlp_forward(const u32x4 *pk, const float *tail, const float x[kMlpIn],
                                             u32x4 *stage) {
    const int lane = threadIdx.x & 63;
    wave_lds_sync();   // earlier reads of the staging rows are complete
    stage_input(tail, x, stage, lane);
    wave_lds_sync();
    u32x4 b1[4][1];
    input_bfrag(stage, b1, lane);
    f32x4 h[4][4];
    mm_layer<1>(pk + kPkL1, b1, h, lane);
    bias_act(h, tail + kTB1, lane);
    u32x4 bq[4][2];
    to_bfrag(h, bq);
    mm_layer<2>(pk + kPkL2, bq, h, lane);
    bias_act(h, tail + kTB2, lane);
    to_bfrag(h, bq);
    mm_layer<2>(pk + kPkL3, bq, h, lane);
    bias_act(h, tail + kTB3, lane);
    return out_layer(h, tail, lane);
}

// Features of the state at the start of a step: x^mu, k_mu (k_t held
// fixed), spin, log|h| and log eps (eps floored at 1e-10) of the last
// accepted step.
__device__ __forceinline__ void step_features(const double y[7], double kt, double a, double h_last, double eps_last,
                                              float x[kMlpIn]) {
    x[0] = (float)y[0];
    x[1] = (float)y[1];
    x[2] = (float)y[2];
    x[3] = (float)y[3];
    x[4] = (float)kt;
    x[5] = (float)y[4];
    x[6] = (float)y[5];
    x[7] = (float)y[6];
    x[8] = (float)a;
    x[9] = __logf(fabsf((float)h_last));
    x[10] = __logf(fmaxf((float)eps_last, 1e-10f));
}

}  // namespace bl
