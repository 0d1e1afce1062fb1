// The indicator network's arithmetic shared by the fused reconstruction kernel and the
// stand-alone inference kernels: parameter layout, bf16 matrix-core evaluation of 32 rows by one
// wave, and the features computed from a cell's reconstruction right-hand sides.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gks {

constexpr int MLP_IN = 44, MLP_K = 48, MLP_H = 64;
constexpr int MLP_NP = MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;  // 7105
constexpr int OFF_B1 = MLP_IN * MLP_H, OFF_W2 = OFF_B1 + MLP_H, OFF_B2 = OFF_W2 + MLP_H * MLP_H,
              OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_H;


typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline short to_bf16(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (short)(u >> 16);
}

constexpr int IND_WAVES = 4;

// LDS row strides (in bf16 elements) of the feature and hidden-activation tiles: multiples of 8
// (16-byte aligned operand reads), not of 64 (bank spread)
constexpr int FB = MLP_K + 8, HB = MLP_H + 8;

// eight bf16 operands (stored as their bit patterns) for the matrix core
__device__ inline bf16x8 bf16_operand(const short *p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const s16x8 *>(p));
}

// The network on 32 rows held in LDS as bf16: featb[32][FB] (features, zero padded to 48),
// hidb[32][HB] (first hidden layer), one wave per block of 32 hidden units.  The matrix products use
// v_mfma_f32_32x32x16_bf16: lane l supplies row l%32 of A and column l%32 of B for
// k = 8 (l/32) + 0..7; accumulator register r of lane l holds row 8 (r/4) + 4 (l/32) + r%4, column
// l%32.  The weights come pre-arranged in that operand order (k_weights_bf16), eight bf16 per lane
// and step.  The caller synchronises between the two halves.
__device__ inline void mlp_layer1(const short (*featb)[FB], short (*hidb)[HB], int lane, int nbk,
                                  const short *__restrict__ W1r, const float *__restrict__ P)
{
    // hidden units 32 nbk .. 32 nbk + 31
    const int row = lane & 31, half = lane >> 5;
    f32x16 acc = f32x16{0};
#pragma unroll
    for (int s = 0; s < MLP_K / 16; s++) {
        const bf16x8 a = bf16_operand(&featb[row][16 * s + 8 * half]);
        const bf16x8 b = bf16_operand(W1r + ((nbk * (MLP_K / 16) + s) * 64 + lane) * 8);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    const float bias = P[OFF_B1 + 32 * nbk + row];
#pragma unroll
    for (int r = 0; r < 16; r++)
        hidb[8 * (r / 4) + 4 * half + (r % 4)][32 * nbk + row] = to_bf16(fmaxf(acc[r] + bias, 0.f));
}

// the output unit's partial sum over the second hidden layer's units 32 nbk .. 32 nbk + 31:
// z_i = sum_j relu(acc_ij + b2_j) w3_j; on return lanes 0 and 32 hold rows 8 (r/4) + 4 (l/32) + r%4
// in z[r].  The logit is b3 plus the two partial sums, added as z(0) + z(1) + b3.
__device__ inline void mlp_layer2(const short (*hidb)[HB], int lane, int nbk, const short *__restrict__ W2r,
                                  const float *__restrict__ P, float z[16])
{
    const int row = lane & 31, half = lane >> 5;
    f32x16 acc = f32x16{0};
#pragma unroll
    for (int s = 0; s < MLP_H / 16; s++) {
        const bf16x8 a = bf16_operand(&hidb[row][16 * s + 8 * half]);
        const bf16x8 b = bf16_operand(W2r + ((nbk * (MLP_H / 16) + s) * 64 + lane) * 8);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    // column j lives in lane j of each half: reduce over the half's 32 lanes
    const float b2 = P[OFF_B2 + 32 * nbk + row], w3 = P[OFF_W3 + 32 * nbk + row];
#pragma unroll
    for (int r = 0; r < 16; r++) z[r] = fmaxf(acc[r] + b2, 0.f) * w3;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < 16; r++) z[r] += __shfl_xor(z[r], off);
}

// the whole network for 32 rows on one wave; on return lanes 0 and 32 hold the logits of rows
// 8 (r/4) + 4 (l/32) + r%4 in z[r].  The caller synchronises between the hidden layers.
__device__ inline void mlp_layer2_out(const short (*hidb)[HB], int lane, const short *__restrict__ W2r,
                                      const float *__restrict__ P, float z[16])
{
    float z1[16];
    mlp_layer2(hidb, lane, 0, W2r, P, z);
    mlp_layer2(hidb, lane, 1, W2r, P, z1);
    const float b3 = P[OFF_B3];
#pragma unroll
    for (int r = 0; r < 16; r++) z[r] = z[r] + z1[r] + b3;
}

// The weight matrices in the operand order of mlp_layer1 / mlp_layer2, bf16 (round to nearest
// even): element ((nbk * steps + s) * 64 + l) * 8 + i holds W[k][col] with k = 16 s + 8 (l / 32) + i,
// col = 32 nbk + l % 32; W1 rows 44..47 (input padding) are zero.  W1r [3072], W2r [4096].
__global__ void k_weights_bf16(const float *__restrict__ P, short *__restrict__ W1r, short *__restrict__ W2r)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int ii = i & 7, l = (i >> 3) & 63, blk = i >> 9;
    const int k0 = 8 * (l >> 5) + ii, col = (l & 31);
    if (i < MLP_K * MLP_H) {
        const int nbk = blk / (MLP_K / 16), s = blk % (MLP_K / 16), k = 16 * s + k0;
        W1r[i] = k < MLP_IN ? to_bf16(P[k * MLP_H + 32 * nbk + col]) : (short)0;
    }
    if (i < MLP_H * MLP_H) {
        const int nbk = blk / (MLP_H / 16), s = blk % (MLP_H / 16), k = 16 * s + k0;
        W2r[i] = to_bf16(P[OFF_W2 + k * MLP_H + 32 * nbk + col]);
    }
}

// Features of one thickness field from its reconstruction right-hand side rhs (9 differences,
// then hs times the gradients of the cell and its face neighbours, in the bulk precision):
// x[l] = rhs[l] / s with s = max_l |rhs[l]| + 1e-12 |Q0| (l < 17), x[17] = log10(s / h) / 4 with
// h the layer thickness
template <typename R>
__device__ inline void thick_features(const R *rhs, double Q0, double h, float *x)
{
    double s = 0;
#pragma unroll
    for (int l = 0; l < 9; l++) s = fmax(s, fabs((double)rhs[l]));
    s += 1e-12 * fabs(Q0);
    const double is = 1.0 / s;
#pragma unroll
    for (int l = 0; l < 17; l++) x[l] = (float)((double)rhs[l] * is);
    x[17] = (float)(log10(s / h) * 0.25);
}

// largest stencil difference of one variable
template <typename R>
__device__ inline double max_diff(const R *rhs)
{
    double s = 0;
#pragma unroll
    for (int l = 0; l < 9; l++) s = fmax(s, fabs((double)rhs[l]));
    return s;
}

// size of a layer's momentum variation sm against h sqrt(G h)
__device__ inline float mom_feature(double sm, double h, double G)
{
    const double cm = h * sqrt(G * h);
    return (float)(log10((sm + 1e-12 * cm) / cm) * 0.25);
}

}  // namespace gks
