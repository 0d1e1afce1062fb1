// Learned smoothness indicator: a small MLP (44 -> 64 -> 64 -> 1, ReLU) predicts from a cell's
// compact stencil whether the nonlinear weights of the reconstruction may be skipped (the linear
// P^3 reconstruction is then used, which the nonlinear one reproduces on smooth data).
//
//   features  per cell, for the interface level eta1 = h1 + B and then h2: the 9 stencil differences
//             (Q_l - Q_0)/s and the 8 scaled gradients hs grad Q_l / s of the cell and its face
//             neighbours, s = max_l |Q_l - Q_0| + 1e-12 |Q_0|; the size of the variation,
//             log10(s / h)/4, and of the layer's momentum variation against h sqrt(G h); then the
//             face neighbours' area ratios and the cell's edge lengths over hs (static, from the mesh)
//   inference BF16 MFMA (v_mfma_f32_32x32x8_bf16), FP32 accumulation, one wave per 32 cells; the
//             44 inputs are padded with zeros to 48 (six K-steps of 8)
//   training  FP32: per-sample forward and backward deltas, deterministic weight-gradient sums
//             (one thread per parameter, fixed order over the batch), Adam
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gks_kernels.h"

namespace gks {

constexpr int MLP_IN = 44, MLP_K = 48, MLP_H = 64;
constexpr int MLP_NP = MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;  // 7105
constexpr int OFF_B1 = MLP_IN * MLP_H, OFF_W2 = OFF_B1 + MLP_H, OFF_B2 = OFF_W2 + MLP_H * MLP_H,
              OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_H;

// Features of field f of cell c (f = 0: eta1 with the lower layer's momenta, f = 1: h2 with the
// upper layer's): x[0..16] the stencil differences and scaled gradients, x[17] the size of the
// variation, x[18] the size of the momentum variation.
template <typename R>
__device__ inline void field_features(const MeshDev &m, double G, const double *__restrict__ Wh,
                                      const R *__restrict__ Wm, const R *__restrict__ gW, int f, int64_t c,
                                      const int32_t *nb, float *x)
{
    const int64_t T = m.T, TG = m.T + m.NG;
    const double *Q = Wh + (f == 0 ? TG : 0);
    const int v = f == 0 ? 3 : 0;
    const double Q0 = Q[c];
    const double h = f == 0 ? Q0 - m.Bbar[c] : Q0;
    double d[9], s = 0;
#pragma unroll
    for (int l = 0; l < 9; l++) {
        d[l] = Q[nb[l]] - Q0;
        s = fmax(s, fabs(d[l]));
    }
    s += 1e-12 * fabs(Q0);
    const double is = 1.0 / s, hs = (double)tab<R>(m.hs)[c];
#pragma unroll
    for (int l = 0; l < 9; l++) x[l] = (float)(d[l] * is);
    x[9] = (float)(hs * (double)gW[(2 * v) * TG + c] * is);
    x[10] = (float)(hs * (double)gW[(2 * v + 1) * TG + c] * is);
#pragma unroll
    for (int l = 0; l < 3; l++) {
        x[11 + 2 * l] = (float)(hs * (double)gW[(2 * v) * TG + nb[l]] * is);
        x[12 + 2 * l] = (float)(hs * (double)gW[(2 * v + 1) * TG + nb[l]] * is);
    }
    x[17] = (float)(log10(s / h) * 0.25);
    // momentum slots: upper layer 0, 1; lower layer 2, 3
    const R *mu = Wm + (f == 0 ? 2 : 0) * TG, *mv = mu + TG;
    const double mu0 = (double)mu[c], mv0 = (double)mv[c];
    double sm = 0;
#pragma unroll
    for (int l = 0; l < 9; l++) sm = fmax(sm, fmax(fabs((double)mu[nb[l]] - mu0), fabs((double)mv[nb[l]] - mv0)));
    const double cm = h * sqrt(G * h);
    x[18] = (float)(log10((sm + 1e-12 * cm) / cm) * 0.25);
}

// all 44 features of cell c (training export)
template <typename R>
__global__ void k_features(MeshDev m, double G, const double *__restrict__ Wh, const R *__restrict__ Wm,
                           const R *__restrict__ gW, float *__restrict__ X)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m.T) return;
    const int64_t T = m.T;
    int32_t nb[9];
#pragma unroll
    for (int s = 0; s < 9; s++) nb[s] = m.sten[s * T + c];
    float *x = X + c * MLP_IN;
#pragma unroll
    for (int f = 0; f < 2; f++) {
        float y[19];
        field_features<R>(m, G, Wh, Wm, gW, f, c, nb, y);
#pragma unroll
        for (int k = 0; k < 17; k++) x[17 * f + k] = y[k];
        x[34 + f] = y[17];
        x[36 + f] = y[18];
    }
#pragma unroll
    for (int k = 0; k < 6; k++) x[38 + k] = m.igeo[k * T + c];
}

// ---------------------------------------------------------------------------------------------
// inference: 4 waves per block, one wave per 32 cells

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline short to_bf16(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (short)(u >> 16);
}

constexpr int IND_WAVES = 4;

// One wave evaluates the MLP on 32 feature rows held in LDS (feat[32][49], hid[32][65] are the
// wave's own slices).  The matrix products use v_mfma_f32_32x32x8_bf16: lane l supplies row l%32
// of A and column l%32 of B for k = 4 (l/32) + 0..3; accumulator register r of lane l holds row
// 8 (r/4) + 4 (l/32) + r%4, column l%32.  The caller synchronises between the two halves.
__device__ inline void mlp_layer1(const float (*feat)[MLP_K + 1], float (*hid)[MLP_H + 1], int lane,
                                  const short *__restrict__ W1b, const float *__restrict__ P)
{
    const int row = lane & 31, half = lane >> 5;
#pragma unroll
    for (int nbk = 0; nbk < 2; nbk++) {
        f32x16 acc = f32x16{0};
#pragma unroll
        for (int s = 0; s < MLP_K / 8; s++) {
            bf16x4 a, b;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int k = 8 * s + 4 * half + i;
                a[i] = to_bf16(feat[row][k]);
                b[i] = W1b[k * MLP_H + 32 * nbk + row];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
        }
        const float bias = P[OFF_B1 + 32 * nbk + row];
#pragma unroll
        for (int r = 0; r < 16; r++) hid[8 * (r / 4) + 4 * half + (r % 4)][32 * nbk + row] = fmaxf(acc[r] + bias, 0.f);
    }
}

// second hidden layer and the output unit; on return lanes 0 and 32 hold the logits of rows
// 8 (r/4) + 4 (l/32) + r%4 in z[r]
__device__ inline void mlp_layer2_out(const float (*hid)[MLP_H + 1], int lane, const short *__restrict__ W2b,
                                      const float *__restrict__ P, float z[16])
{
    const int row = lane & 31, half = lane >> 5;
    f32x16 acc[2];
#pragma unroll
    for (int nbk = 0; nbk < 2; nbk++) {
        acc[nbk] = f32x16{0};
#pragma unroll
        for (int s = 0; s < MLP_H / 8; s++) {
            bf16x4 a, b;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int k = 8 * s + 4 * half + i;
                a[i] = to_bf16(hid[row][k]);
                b[i] = W2b[k * MLP_H + 32 * nbk + row];
            }
            acc[nbk] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc[nbk], 0, 0, 0);
        }
    }
    // z_i = b3 + sum_j relu(acc_ij + b2_j) w3_j: column j lives in lane j (and j + 32 of the
    // second block), so reduce over the 32 lanes of each half
    const float b2a = P[OFF_B2 + row], b2b = P[OFF_B2 + 32 + row];
    const float w3a = P[OFF_W3 + row], w3b = P[OFF_W3 + 32 + row];
#pragma unroll
    for (int r = 0; r < 16; r++) z[r] = fmaxf(acc[0][r] + b2a, 0.f) * w3a + fmaxf(acc[1][r] + b2b, 0.f) * w3b;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < 16; r++) z[r] += __shfl_xor(z[r], off);
    const float b3 = P[OFF_B3];
#pragma unroll
    for (int r = 0; r < 16; r++) z[r] += b3;
}

// W1b: bf16 [48][64] (zero rows 44..47), W2b: bf16 [64][64]; P: FP32 parameters (biases and the
// output layer).
// Writes mask[c] = (logit > thr) and, when logit is not null, the logit.
template <typename R>
__global__ void __launch_bounds__(64 * IND_WAVES) k_indicator(MeshDev m, double G, const double *__restrict__ Wh,
                                                               const R *__restrict__ Wm, const R *__restrict__ gW,
                                                               const short *__restrict__ W1b,
                                                               const short *__restrict__ W2b,
                                                               const float *__restrict__ P, float thr,
                                                               uint8_t *__restrict__ mask, float *__restrict__ logit)
{
    __shared__ float feat[IND_WAVES][32][MLP_K + 1];
    __shared__ float hid[IND_WAVES][32][MLP_H + 1];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 31, half = lane >> 5;
    const int64_t T = m.T, TG = m.T + m.NG;
    const int64_t base = ((int64_t)blockIdx.x * IND_WAVES + wv) * 32;
    const int64_t c = base + row;
    // features: lanes 0..31 the interface level (and the geometry), lanes 32..63 h2 (and the
    // zero padding of the inputs)
    {
        float x[19];
        if (c < T) {
            int32_t nb[9];
#pragma unroll
            for (int s = 0; s < 9; s++) nb[s] = m.sten[s * T + c];
            field_features<R>(m, G, Wh, Wm, gW, half, c, nb, x);
        } else {
#pragma unroll
            for (int k = 0; k < 19; k++) x[k] = 0.f;
        }
#pragma unroll
        for (int k = 0; k < 17; k++) feat[wv][row][17 * half + k] = x[k];
        feat[wv][row][34 + half] = x[17];
        feat[wv][row][36 + half] = x[18];
        if (!half) {
#pragma unroll
            for (int k = 0; k < 6; k++) feat[wv][row][38 + k] = c < T ? m.igeo[k * T + c] : 0.f;
        } else {
#pragma unroll
            for (int k = MLP_IN; k < MLP_K; k++) feat[wv][row][k] = 0.f;
        }
    }
    __syncthreads();
    mlp_layer1(feat[wv], hid[wv], lane, W1b, P);
    __syncthreads();
    float z[16];
    mlp_layer2_out(hid[wv], lane, W2b, P, z);
    if (row == 0) {
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int64_t ci = base + 8 * (r / 4) + 4 * half + (r % 4);
            if (ci < T) {
                mask[ci] = z[r] > thr ? 1 : 0;
                if (logit) logit[ci] = z[r];
            }
        }
    }
}

// the same network on stored feature rows X[n][40] (threshold selection on training samples)
__global__ void __launch_bounds__(64 * IND_WAVES) k_mlp_infer(const float *__restrict__ X, int64_t n,
                                                               const short *__restrict__ W1b,
                                                               const short *__restrict__ W2b,
                                                               const float *__restrict__ P, float *__restrict__ logit)
{
    __shared__ float feat[IND_WAVES][32][MLP_K + 1];
    __shared__ float hid[IND_WAVES][32][MLP_H + 1];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 31, half = lane >> 5;
    const int64_t base = ((int64_t)blockIdx.x * IND_WAVES + wv) * 32;
    for (int k = half; k < MLP_K; k += 2)
        feat[wv][row][k] = (base + row < n && k < MLP_IN) ? X[(base + row) * MLP_IN + k] : 0.f;
    __syncthreads();
    mlp_layer1(feat[wv], hid[wv], lane, W1b, P);
    __syncthreads();
    float z[16];
    mlp_layer2_out(hid[wv], lane, W2b, P, z);
    if (row == 0) {
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int64_t i = base + 8 * (r / 4) + 4 * half + (r % 4);
            if (i < n) logit[i] = z[r];
        }
    }
}

// round the two weight matrices of P to bf16 (round to nearest even); W1b [48][64] carries zero
// rows for the input padding
__global__ void k_weights_bf16(const float *__restrict__ P, short *__restrict__ W1b, short *__restrict__ W2b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_K * MLP_H) W1b[i] = i < MLP_IN * MLP_H ? to_bf16(P[i]) : (short)0;
    if (i < MLP_H * MLP_H) W2b[i] = to_bf16(P[OFF_W2 + i]);
}

// ---------------------------------------------------------------------------------------------
// labels: 1 where the nonlinear and the linear reconstructions agree at every Gauss point within
// tol times the variable's scale (layer thickness, or h sqrt(G h) for momenta)

template <typename R>
__global__ void k_label(MeshDev m, double G, double tol, const double *__restrict__ Wh,
                        const GpHead<R> *__restrict__ rec_nl, const GpHead<R> *__restrict__ rec_li, uint8_t *__restrict__ y)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m.T) return;
    const int64_t TG = m.T + m.NG;
    const double h2 = Wh[c], h1 = Wh[TG + c] - m.Bbar[c];
    const double sh[2] = {h2, h1}, sm[2] = {h2 * sqrt(G * h2), h1 * sqrt(G * h1)};
    bool ok = true;
    for (int slot = 0; slot < 6; slot++) {
        const GpHead<R> &a = rec_nl[6 * c + slot], &b = rec_li[6 * c + slot];
        for (int q = 0; q < 2; q++) ok = ok && fabs(a.h[q] - b.h[q]) <= tol * sh[q];
        for (int q = 0; q < 4; q++) ok = ok && fabs((double)a.q[q] - (double)b.q[q]) <= tol * sm[q / 2];
    }
    y[c] = ok ? 1 : 0;
}

__global__ void k_u8_to_f32(const uint8_t *__restrict__ a, int64_t n, float *__restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// ---------------------------------------------------------------------------------------------
// training (FP32)

constexpr int TRAIN_BLOCK = 128;

// per sample s of the batch (rows idx[s] of X, Y): forward pass, logistic loss L[s] and the
// back-propagated pre-activation gradients of the mean loss, dz (output), D2, D1 (hidden layers);
// keeps H1, H2 for the weight gradients.  Per-sample arrays are [B][64].
__global__ void __launch_bounds__(TRAIN_BLOCK) k_mlp_forward_delta(const float *__restrict__ P,
                                                                    const float *__restrict__ X,
                                                                    const float *__restrict__ Y,
                                                                    const int32_t *__restrict__ idx, int B,
                                                                    float *__restrict__ H1, float *__restrict__ H2,
                                                                    float *__restrict__ D1, float *__restrict__ D2,
                                                                    float *__restrict__ DZ, float *__restrict__ L)
{
    __shared__ float Ps[MLP_NP];
    for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) Ps[i] = P[i];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const int64_t r = idx[s];
    const float *x = X + r * MLP_IN;
    float h1[MLP_H];
    {
        float xin[MLP_IN];
#pragma unroll
        for (int i = 0; i < MLP_IN; i++) xin[i] = x[i];
#pragma unroll
        for (int j = 0; j < MLP_H; j++) {
            float a = Ps[OFF_B1 + j];
#pragma unroll
            for (int i = 0; i < MLP_IN; i++) a = fmaf(xin[i], Ps[i * MLP_H + j], a);
            h1[j] = fmaxf(a, 0.f);
        }
    }
    float *h2o = H2 + (int64_t)s * MLP_H;
    float z = Ps[OFF_B3];
    for (int j = 0; j < MLP_H; j++) {
        float a = Ps[OFF_B2 + j];
#pragma unroll
        for (int i = 0; i < MLP_H; i++) a = fmaf(h1[i], Ps[OFF_W2 + i * MLP_H + j], a);
        const float h2 = fmaxf(a, 0.f);
        h2o[j] = h2;
        z = fmaf(h2, Ps[OFF_W3 + j], z);
    }
    const float y = Y[r];
    // softplus(z) - y z, evaluated without overflow
    L[s] = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - y * z;
    const float dz = (1.f / (1.f + expf(-z)) - y) / (float)B;
    DZ[s] = dz;
    float acc[MLP_H];
#pragma unroll
    for (int i = 0; i < MLP_H; i++) acc[i] = 0.f;
    float *d2o = D2 + (int64_t)s * MLP_H;
    for (int j = 0; j < MLP_H; j++) {
        const float d2 = h2o[j] > 0.f ? dz * Ps[OFF_W3 + j] : 0.f;
        d2o[j] = d2;
#pragma unroll
        for (int i = 0; i < MLP_H; i++) acc[i] = fmaf(Ps[OFF_W2 + i * MLP_H + j], d2, acc[i]);
    }
    float *d1o = D1 + (int64_t)s * MLP_H, *h1o = H1 + (int64_t)s * MLP_H;
#pragma unroll
    for (int i = 0; i < MLP_H; i++) {
        d1o[i] = h1[i] > 0.f ? acc[i] : 0.f;
        h1o[i] = h1[i];
    }
}

// one thread per parameter: sum over the batch in sample order (deterministic, no atomics)
__global__ void k_mlp_weight_grad(const float *__restrict__ X, const int32_t *__restrict__ idx, int B,
                                  const float *__restrict__ H1, const float *__restrict__ H2,
                                  const float *__restrict__ D1, const float *__restrict__ D2,
                                  const float *__restrict__ DZ, float *__restrict__ grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NP) return;
    float acc = 0.f;
    if (p < OFF_B1) {
        const int i = p / MLP_H, j = p % MLP_H;
        for (int s = 0; s < B; s++) acc = fmaf(X[(int64_t)idx[s] * MLP_IN + i], D1[(int64_t)s * MLP_H + j], acc);
    } else if (p < OFF_W2) {
        const int j = p - OFF_B1;
        for (int s = 0; s < B; s++) acc += D1[(int64_t)s * MLP_H + j];
    } else if (p < OFF_B2) {
        const int i = (p - OFF_W2) / MLP_H, j = (p - OFF_W2) % MLP_H;
        for (int s = 0; s < B; s++) acc = fmaf(H1[(int64_t)s * MLP_H + i], D2[(int64_t)s * MLP_H + j], acc);
    } else if (p < OFF_W3) {
        const int j = p - OFF_B2;
        for (int s = 0; s < B; s++) acc += D2[(int64_t)s * MLP_H + j];
    } else if (p < OFF_B3) {
        const int j = p - OFF_W3;
        for (int s = 0; s < B; s++) acc = fmaf(DZ[s], H2[(int64_t)s * MLP_H + j], acc);
    } else {
        for (int s = 0; s < B; s++) acc += DZ[s];
    }
    grad[p] = acc;
}

__global__ void k_adam(float *__restrict__ P, const float *__restrict__ g, float *__restrict__ mo,
                       float *__restrict__ ve, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NP) return;
    const float m = b1 * mo[p] + (1.f - b1) * g[p];
    const float v = b2 * ve[p] + (1.f - b2) * g[p] * g[p];
    mo[p] = m;
    ve[p] = v;
    P[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// mean of the per-sample losses (one block, fixed-order tree)
__global__ void k_mean(const float *__restrict__ L, int B, float *__restrict__ out)
{
    __shared__ float sh[256];
    float a = 0.f;
    for (int i = threadIdx.x; i < B; i += 256) a += L[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] / (float)B;
}

}  // namespace gks
