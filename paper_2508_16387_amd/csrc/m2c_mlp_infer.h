// m2c_mlp_infer.h -- matrix-core inference of the learned star-pressure
// guess inside other kernels (the FIVER kernel of the grid step and the
// kernel-level guess kernels).  Layouts and the network are those of
// m2c_mlp.h; the 16x16x16 BF16 MFMA lane layout is described in k_mlp.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "m2c_mlp.h"

namespace m2c {

typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ short to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Inference for the guess kernels.  A wave keeps the weights in registers
// (the A operands of layers 1 and 2, and its lanes' biases and output
// weights in the D layout) and evaluates 64 samples per pass: each lane
// computes the features of one sample once, and the four 16-sample MFMA
// tiles take their B operands from the owning lanes by shuffles.
struct MlpRegs {
    bf16x4 a1[4], a2[4][4];
    float b1[4][4], b2[4][4], w3[4][4], b3;
};

__device__ __forceinline__ void mlp_load_regs(const float* __restrict__ P, const uint16_t* __restrict__ wbf,
                                              MlpRegs& w)
{
    const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * g + e, h = 16 * t + 4 * g + e;
            w.a1[t][e] = k < MLP_IN ? (short)wbf[MLP_OFF_W1 + (16 * t + r) * MLP_IN + k] : (short)0;
            w.b1[t][e] = P[MLP_OFF_B1 + h];
            w.b2[t][e] = P[MLP_OFF_B2 + h];
            w.w3[t][e] = P[MLP_OFF_W3 + h];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) w.a2[t][c][e] = (short)wbf[512 + (16 * t + r) * MLP_H + 16 * c + 4 * g + e];
    }
    w.b3 = P[MLP_OFF_B3];
}

// tanh through the hardware exponential and reciprocal: 1 - 2/(e^{2x} + 1)
// (about 1e-7 absolute error, far below the BF16 rounding of the operands;
// saturates correctly for large |x|).
__device__ __forceinline__ float tanh_fast(float x)
{
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * x) + 1.0f);
}

// y of the 16 samples whose layer-1 B operand is xb (sample l%16 in every
// lane of that sample).
__device__ __forceinline__ float mlp_infer16(const MlpRegs& w, bf16x4 xb)
{
    bf16x4 hb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x4 z = mfma(w.a1[t], xb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int e = 0; e < 4; ++e) hb[t][e] = to_bf16(tanh_fast(z[e] + w.b1[t][e]));
    }
    float part = 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) z = mfma(w.a2[u][c], hb[c], z);
#pragma unroll
        for (int e = 0; e < 4; ++e) part += w.w3[u][e] * tanh_fast(z[e] + w.b2[u][e]);
    }
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    return part + w.b3;
}

// A problem whose two states differ by less than 1e-3 in pressure (relative
// to the smaller p + p_c) and in normal velocity (relative to the smaller
// sound speed): the acoustic guess is then exact to about 1e-6, far closer
// than the network's, and is taken directly (the guess is left non-finite,
// which the solver reads as "no candidate").
__device__ __forceinline__ bool acoustic_suffices(double rL, double uL, double pL, double gL, double pcL, double rR,
                                                  double uR, double pR, double gR, double pcR)
{
    // du^2 <= 1e-6 min(c_L^2, c_R^2), with c_K^2 = g_K a_K / r_K, written
    // without divisions
    const double aL = pL + pcL, aR = pR + pcR, du = uL - uR, du2 = du * du;
    return fabs(pL - pR) <= 1e-3 * fmin(aL, aR) && du2 * rL <= 1e-6 * (gL * aL) && du2 * rR <= 1e-6 * (gR * aR);
}

// Guesses of the wave's 64 samples (one per lane): features x, p_lo, P and
// `skip` (no network: invalid lane or acoustic_suffices).  Tiles whose 16
// samples all skip are not evaluated.
__device__ __forceinline__ double guess64(const MlpRegs& w, const float x[8], double plo, double P, bool skip)
{
    const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
    const uint64_t need = __ballot(!skip);
    float y = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (((need >> (16 * t)) & 0xffffull) == 0ull) continue;     // wave-uniform
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = __shfl(x[k], 16 * t + r);
        bf16x4 xb;
#pragma unroll
        for (int e = 0; e < 4; ++e) xb[e] = g == 0 ? to_bf16(v[e]) : (g == 1 ? to_bf16(v[4 + e]) : (short)0);
        const float yt = mlp_infer16(w, xb);
        const float mine = __shfl(yt, r);
        if (g == t) y = mine;
    }
    return skip ? __builtin_nan("") : plo + P * exp((double)y);
}

// The same evaluation with the operands read from the weights in memory as
// they are needed (cache hits after the first wave), for kernels that would
// lose occupancy by holding the whole network in registers (the FIVER
// kernel of the grid step, where most wavefronts never need it).
__device__ __forceinline__ float mlp_infer16_mem(const float* __restrict__ P, const uint16_t* __restrict__ wbf,
                                                 bf16x4 xb)
{
    const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
    bf16x4 hb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        bf16x4 a1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * g + e;
            a1[e] = k < MLP_IN ? (short)wbf[MLP_OFF_W1 + (16 * t + r) * MLP_IN + k] : (short)0;
        }
        const f32x4 z = mfma(a1, xb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int e = 0; e < 4; ++e) hb[t][e] = to_bf16(tanh_fast(z[e] + P[MLP_OFF_B1 + 16 * t + 4 * g + e]));
    }
    float part = 0.f;
#pragma unroll 1
    for (int u = 0; u < 4; ++u) {
        f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            bf16x4 a2;
#pragma unroll
            for (int e = 0; e < 4; ++e) a2[e] = (short)wbf[512 + (16 * u + r) * MLP_H + 16 * c + 4 * g + e];
            z = mfma(a2, hb[c], z);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int h = 16 * u + 4 * g + e;
            part += P[MLP_OFF_W3 + h] * tanh_fast(z[e] + P[MLP_OFF_B2 + h]);
        }
    }
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    return part + P[MLP_OFF_B3];
}

// guess64 with the operands read from memory (see mlp_infer16_mem).
__device__ __forceinline__ double guess64_mem(const MlpDev& m, const float x[8], double plo, double P, bool skip)
{
    const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
    const uint64_t need = __ballot(!skip);
    float y = 0.f;
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
        if (((need >> (16 * t)) & 0xffffull) == 0ull) continue;     // wave-uniform
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = __shfl(x[k], 16 * t + r);
        bf16x4 xb;
#pragma unroll
        for (int e = 0; e < 4; ++e) xb[e] = g == 0 ? to_bf16(v[e]) : (g == 1 ? to_bf16(v[4 + e]) : (short)0);
        const float yt = mlp_infer16_mem(m.master, m.wbf, xb);
        const float mine = __shfl(yt, r);
        if (g == t) y = mine;
    }
    return skip ? __builtin_nan("") : plo + P * exp((double)y);
}

}  // namespace m2c
