// Learned smoothness indicator: a small MLP (44 -> 64 -> 64 -> 1, ReLU) predicts from a cell's
// compact stencil whether the nonlinear weights of the reconstruction may be skipped (the linear
// P^3 reconstruction is then used, which the nonlinear one reproduces on smooth data).
//
//   features  per cell, for the interface level eta1 = h1 + B and then h2: the 9 stencil differences
//             (Q_l - Q_0)/s and the 8 scaled gradients hs grad Q_l / s of the cell and its face
//             neighbours, s = max_l |Q_l - Q_0| + 1e-12 |Q_0|; the size of the variation,
//             log10(s / h)/4, and of the layer's momentum variation against h sqrt(G h); then the
//             face neighbours' area ratios and the cell's edge lengths over hs (static, from the mesh)
//   inference BF16 MFMA (v_mfma_f32_32x32x16_bf16), FP32 accumulation, 32 cells per wave; the
//             44 inputs are padded with zeros to 48 (six K-steps of 8)
//   training  FP32: per-sample forward and backward deltas, deterministic weight-gradient sums
//             (one thread per parameter, fixed order over the batch), Adam
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gks_kernels.h"
#include "gks_mlp.h"

namespace gks {

// Features of field f of cell c (f = 0: eta1 with the lower layer's momenta, f = 1: h2 with the
// upper layer's): x[0..16] the stencil differences and scaled gradients, x[17] the size of the
// variation, x[18] the size of the momentum variation.  Computed from the reconstruction's own
// right-hand sides, with the arithmetic of the reconstruction kernel's fused indicator.
template <typename R>
__device__ inline void field_features(const MeshDev &m, double G, const double *__restrict__ Wh,
                                      const R *__restrict__ Wm, const R *__restrict__ gW, int f, int64_t c, float *x)
{
    const int vt = f == 0 ? 3 : 0, vu = f == 0 ? 4 : 1;
    ReconRhs<R> q, qu, qv;
    recon_rhs<R>(m, Wh, Wm, gW, vt, true, c, q);
    recon_rhs<R>(m, Wh, Wm, gW, vu, false, c, qu);
    recon_rhs<R>(m, Wh, Wm, gW, vu + 1, false, c, qv);
    const double h = f == 0 ? q.Q0h - m.Bbar[c] : q.Q0h;
    thick_features<R>(q.rhs, q.Q0h, h, x);
    x[18] = mom_feature(fmax(max_diff<R>(qu.rhs), max_diff<R>(qv.rhs)), h, G);
}

// all 44 features of cell c (training export)
template <typename R>
__global__ void k_features(MeshDev m, double G, const double *__restrict__ Wh, const R *__restrict__ Wm,
                           const R *__restrict__ gW, float *__restrict__ X)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m.T) return;
    float *x = X + c * MLP_IN;
#pragma unroll
    for (int f = 0; f < 2; f++) {
        float y[19];
        field_features<R>(m, G, Wh, Wm, gW, f, c, y);
#pragma unroll
        for (int k = 0; k < 17; k++) x[17 * f + k] = y[k];
        x[34 + f] = y[17];
        x[36 + f] = y[18];
    }
#pragma unroll
    for (int k = 0; k < 6; k++) x[38 + k] = m.igeo[k * m.T + c];
}

// ---------------------------------------------------------------------------------------------
// inference: 4 waves per block, one wave per 32 cells (the network itself is in gks_mlp.h)

// W1b, W2b: the weight matrices in operand order (k_weights_bf16); P: FP32 parameters (biases and
// the output layer).
// Writes mask[c] = (logit > thr) and, when logit is not null, the logit.
template <typename R>
__global__ void __launch_bounds__(64 * IND_WAVES) k_indicator(MeshDev m, double G, const double *__restrict__ Wh,
                                                               const R *__restrict__ Wm, const R *__restrict__ gW,
                                                               const short *__restrict__ W1b,
                                                               const short *__restrict__ W2b,
                                                               const float *__restrict__ P, float thr,
                                                               uint8_t *__restrict__ mask, float *__restrict__ logit)
{
    __shared__ __align__(16) short feat[IND_WAVES][32][FB];
    __shared__ __align__(16) short hid[IND_WAVES][32][HB];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 31, half = lane >> 5;
    const int64_t T = m.T;
    const int64_t base = ((int64_t)blockIdx.x * IND_WAVES + wv) * 32;
    const int64_t c = base + row;
    // features: lanes 0..31 the interface level (and the geometry), lanes 32..63 h2 (and the
    // zero padding of the inputs)
    {
        float x[19];
        if (c < T) {
            field_features<R>(m, G, Wh, Wm, gW, half, c, x);
        } else {
#pragma unroll
            for (int k = 0; k < 19; k++) x[k] = 0.f;
        }
#pragma unroll
        for (int k = 0; k < 17; k++) feat[wv][row][17 * half + k] = to_bf16(x[k]);
        feat[wv][row][34 + half] = to_bf16(x[17]);
        feat[wv][row][36 + half] = to_bf16(x[18]);
        if (!half) {
#pragma unroll
            for (int k = 0; k < 6; k++) feat[wv][row][38 + k] = to_bf16(c < T ? m.igeo[k * T + c] : 0.f);
        } else {
#pragma unroll
            for (int k = MLP_IN; k < MLP_K; k++) feat[wv][row][k] = 0;
        }
    }
    __syncthreads();
    mlp_layer1(feat[wv], hid[wv], lane, 0, W1b, P);
    mlp_layer1(feat[wv], hid[wv], lane, 1, W1b, P);
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
    __shared__ __align__(16) short feat[IND_WAVES][32][FB];
    __shared__ __align__(16) short hid[IND_WAVES][32][HB];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 31, half = lane >> 5;
    const int64_t base = ((int64_t)blockIdx.x * IND_WAVES + wv) * 32;
    for (int k = half; k < MLP_K; k += 2)
        feat[wv][row][k] = to_bf16((base + row < n && k < MLP_IN) ? X[(base + row) * MLP_IN + k] : 0.f);
    __syncthreads();
    mlp_layer1(feat[wv], hid[wv], lane, 0, W1b, P);
    mlp_layer1(feat[wv], hid[wv], lane, 1, W1b, P);
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
