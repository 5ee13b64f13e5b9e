// k_mlp.hip -- BF16 matrix-core inference and training of the learned
// star-pressure guess, and the guess kernel of the FIVER work queue.
//
// One wavefront evaluates 16 samples at a time with the 16x16x16 BF16 MFMA
// (FP32 accumulation), in the transposed orientation Z^T = W X^T so that the
// output tile of one layer is already the B operand of the next:
//   MFMA lane layout (checked on gfx950): A[i][k] in lane i + 16(k/4),
//   element k%4; B[k][j] in lane j + 16(k/4), element k%4; D[i][j] in lane
//   j + 16(i/4), element i%4.
// Layer 1: Z1^T (64x16) = W1 (64x8, K padded to 16) X^T   -> 4 MFMA
// Layer 2: Z2^T (64x16) = W2 (64x64) H1^T                 -> 16 MFMA
// Layer 3: y (16) = w3 . H2^T + b3                         -> lane sums + shuffles
// Backward (training): dW2 = dZ2^T H1 and dW1 = dZ1^T X accumulate over the
// wave's chunks in MFMA accumulators (the transposes go through LDS),
// dH1^T = W2^T dZ2^T reuses dZ2^T in place as the B operand.
#include "m2c_device.h"
#include "m2c_internal.h"
#include "m2c_kernels.h"
#include "m2c_mlp.h"
#include "m2c_mlp_infer.h"

namespace m2c {

// Sum over the 16 lanes of this lane's group (lanes with equal lane/16).
__device__ __forceinline__ float group16_sum(float v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// Forward pass of 16 samples held by one wave.  xb: this lane's B operand of
// layer 1 (features 4g..4g+3 of sample l%16, zero for g >= 2).  Produces the
// hidden activations in D layout (h1[c][e] = H1^T[16c+4g+e][l%16], same for
// h2) and y of sample l%16 in every lane of that sample.
struct Fwd {
    float h1[4][4], h2[4][4];
    float y;
};

__device__ __forceinline__ void mlp_fwd16(const float* __restrict__ P, const uint16_t* __restrict__ wbf, bf16x4 xb,
                                          Fwd& f)
{
    const int l = threadIdx.x & 63, g = l >> 4, r = l & 15;
    // layer 1
    bf16x4 hb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        bf16x4 a;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * g + e;
            a[e] = k < MLP_IN ? (short)wbf[MLP_OFF_W1 + (16 * t + r) * MLP_IN + k] : (short)0;
        }
        f32x4 z = mfma(a, xb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float h = tanhf(z[e] + P[MLP_OFF_B1 + 16 * t + 4 * g + e]);
            f.h1[t][e] = h;
            hb[t][e] = to_bf16(h);
        }
    }
    // layer 2
    float part = 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            bf16x4 a;
#pragma unroll
            for (int e = 0; e < 4; ++e) a[e] = (short)wbf[512 + (16 * u + r) * MLP_H + 16 * c + 4 * g + e];
            z = mfma(a, hb[c], z);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int h = 16 * u + 4 * g + e;
            const float v = tanhf(z[e] + P[MLP_OFF_B2 + h]);
            f.h2[u][e] = v;
            part += P[MLP_OFF_W3 + h] * v;
        }
    }
    // layer 3: sum the four lane groups of each sample
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    f.y = part + P[MLP_OFF_B3];
}

// This lane's layer-1 B operand from the 8 features of its sample.
__device__ __forceinline__ bf16x4 xb_of(const float x[8])
{
    const int g = (threadIdx.x & 63) >> 4;
    bf16x4 b;
#pragma unroll
    for (int e = 0; e < 4; ++e) b[e] = g < 2 ? to_bf16(x[4 * g + e]) : (short)0;
    return b;
}

// ---------------------------------------------------------------------------
// Features of n Riemann problems (SoA in [6][n], eos [4][n]) -> X [8][n],
// and, when p* is given, the targets ln((p* - p_lo)/P).
__global__ __launch_bounds__(256) void k_mlp_features(long long n, const double* __restrict__ in,
                                                      const double* __restrict__ eos, const double* __restrict__ ps,
                                                      float* __restrict__ X, float* __restrict__ tg)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        float x[8];
        double plo, P;
        mlp_features(in[i], in[n + i], in[2 * n + i], eos[i], eos[n + i], in[3 * n + i], in[4 * n + i],
                     in[5 * n + i], eos[2 * n + i], eos[3 * n + i], x, plo, P);
#pragma unroll
        for (int k = 0; k < 8; ++k) X[k * n + i] = x[k];
        if (ps && tg) tg[i] = (float)log((ps[i] - plo) / P);
    }
}

hipError_t launch_mlp_features(long long n, const double* in, const double* eos, const double* ps, float* X,
                               float* tg, hipStream_t s)
{
    long long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)nb), dim3(256), 0, s, n, in, eos, ps, X, tg);
    return hipGetLastError();
}

// Inference on n feature vectors X [8][n] -> y [n].  One wave per 16-sample
// chunk (grid-stride); samples past n are computed on zeros and dropped.
__global__ __launch_bounds__(256) void k_mlp_forward(long long n, const float* __restrict__ X,
                                                     const float* __restrict__ P, const uint16_t* __restrict__ wbf,
                                                     float* __restrict__ y)
{
    const int l = threadIdx.x & 63, r = l & 15;
    const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
    const long long nw = ((long long)gridDim.x * blockDim.x) >> 6;
    for (long long c = wave; c * 16 < n; c += nw) {
        const long long i = c * 16 + r;
        float x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = i < n ? X[k * n + i] : 0.f;
        Fwd f;
        mlp_fwd16(P, wbf, xb_of(x), f);
        if (l < 16 && i < n) y[i] = f.y;
    }
}

hipError_t launch_mlp_forward(long long n, const float* X, const MlpDev& m, float* y, hipStream_t s)
{
    long long nb = (n + 63) / 64;               // 4 waves x 16 samples per block
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)nb), dim3(256), 0, s, n, X, m.master, m.wbf, y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gradient of the mean squared error over samples [i0, i0 + cnt) of a
// minibatch of size B, accumulated (atomically) into grad[MLP_NPARAM]; the
// sum of squared errors goes to *sse.  One wave per CHUNKS x 16 samples.
constexpr int GRAD_CHUNKS = 4;

__global__ __launch_bounds__(64) void k_mlp_grad(long long i0, long long cnt, long long ntot, float invB,
                                                 const float* __restrict__ X, const float* __restrict__ T,
                                                 const float* __restrict__ P, const uint16_t* __restrict__ wbf,
                                                 float* __restrict__ grad, float* __restrict__ sse)
{
    __shared__ short sA[64 * 16];      // dZ2^T or dZ1^T as [hidden][sample]
    __shared__ short sB[64 * 16];      // H1^T as [hidden][sample]
    __shared__ short sX[16 * 16];      // X as [sample][feature] (features 8..15 zero)
    const int l = threadIdx.x, g = l >> 4, r = l & 15;
    f32x4 dW2[4][4], dW1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        dW1[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int v = 0; v < 4; ++v) dW2[u][v] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float gw3[4][4] = {}, gb2[4][4] = {}, gb1[4][4] = {};
    float gb3 = 0.f, err2 = 0.f;
    const long long base = i0 + (long long)blockIdx.x * GRAD_CHUNKS * 16;
    for (int ch = 0; ch < GRAD_CHUNKS; ++ch) {
        const long long j0 = base + ch * 16;
        if (j0 >= i0 + cnt) break;
        const long long i = j0 + r;
        const bool live = i < i0 + cnt;
        float x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = live ? X[k * ntot + i] : 0.f;
        Fwd f;
        mlp_fwd16(P, wbf, xb_of(x), f);
        const float dy = live ? 2.f * (f.y - T[i]) * invB : 0.f;
        if (l < 16 && live) err2 += (f.y - T[i]) * (f.y - T[i]);
        if (l < 16) gb3 += dy;
        // dZ2^T (D layout) and the per-hidden-unit sums
        float dz2[4][4];
        bf16x4 dz2b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int h = 16 * u + 4 * g + e;
                const float h2 = f.h2[u][e];
                gw3[u][e] += dy * h2;
                const float d = P[MLP_OFF_W3 + h] * dy * (1.f - h2 * h2);
                dz2[u][e] = d;
                gb2[u][e] += d;
                dz2b[u][e] = to_bf16(d);
            }
        // transposes through LDS: sA[h][j] = dZ2^T, sB[h][j] = H1^T, sX[j][k] = X
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int h = 16 * u + 4 * g + e;
                sA[h * 16 + r] = dz2b[u][e];
                sB[h * 16 + r] = to_bf16(f.h1[u][e]);
            }
        if (g < 4) {
#pragma unroll
            for (int e = 0; e < 4; ++e) sX[r * 16 + 4 * g + e] = (4 * g + e) < 8 ? to_bf16(x[4 * g + e]) : (short)0;
        }
        __syncthreads();
        // dW2[a][b] += sum_j dZ2^T[a][j] H1^T[b][j]: A[i][k=j] = sA[16u+i][j],
        // B[k=j][n] = sB[16v+n][j]
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            bf16x4 a;
#pragma unroll
            for (int e = 0; e < 4; ++e) a[e] = sA[(16 * u + r) * 16 + 4 * g + e];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                bf16x4 b;
#pragma unroll
                for (int e = 0; e < 4; ++e) b[e] = sB[(16 * v + r) * 16 + 4 * g + e];
                dW2[u][v] = mfma(a, b, dW2[u][v]);
            }
        }
        // dH1^T = W2^T dZ2^T: A[i][k] = W2[16c+k][16v+i], B = dZ2^T tile c
        float dz1[4][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                bf16x4 a;
#pragma unroll
                for (int e = 0; e < 4; ++e) a[e] = (short)wbf[512 + (16 * c + 4 * g + e) * MLP_H + 16 * v + r];
                z = mfma(a, dz2b[c], z);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float h1 = f.h1[v][e];
                const float d = z[e] * (1.f - h1 * h1);
                dz1[v][e] = d;
                gb1[v][e] += d;
            }
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) sA[(16 * v + 4 * g + e) * 16 + r] = to_bf16(dz1[v][e]);
        __syncthreads();
        // dW1[a][k] += sum_j dZ1^T[a][j] X[j][k]: A[i][k=j] = sA[16u+i][j],
        // B[k=j][n] = sX[j][n]
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            bf16x4 a, b;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                a[e] = sA[(16 * u + r) * 16 + 4 * g + e];
                b[e] = sX[(4 * g + e) * 16 + r];
            }
            dW1[u] = mfma(a, b, dW1[u]);
        }
    }
    // reduce and accumulate into the global gradient
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int h = 16 * u + 4 * g + e;
            const float s3 = group16_sum(gw3[u][e]), s2 = group16_sum(gb2[u][e]), s1 = group16_sum(gb1[u][e]);
            if (r == 0) {
                atomicAdd(&grad[MLP_OFF_W3 + h], s3);
                atomicAdd(&grad[MLP_OFF_B2 + h], s2);
                atomicAdd(&grad[MLP_OFF_B1 + h], s1);
            }
        }
    gb3 = group16_sum(gb3);
    err2 = group16_sum(err2);
    if (l == 0) {
        atomicAdd(&grad[MLP_OFF_B3], gb3);
        atomicAdd(sse, err2);
    }
    // D layout: dW2 tile (u,v) element e of lane l = dW2[16u + 4g + e][16v + r]
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                atomicAdd(&grad[MLP_OFF_W2 + (16 * u + 4 * g + e) * MLP_H + 16 * v + r], dW2[u][v][e]);
        if (r < MLP_IN) {
#pragma unroll
            for (int e = 0; e < 4; ++e) atomicAdd(&grad[MLP_OFF_W1 + (16 * u + 4 * g + e) * MLP_IN + r], dW1[u][e]);
        }
    }
}

__global__ void k_fill_f32(float* p, long long n, float v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_mlp_grad(long long i0, long long cnt, long long ntot, float invB, const float* X, const float* T,
                           const MlpDev& m, float* grad, float* sse, hipStream_t s)
{
    const long long per = GRAD_CHUNKS * 16;
    const long long nb = (cnt + per - 1) / per;
    if (nb < 1) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)nb), dim3(64), 0, s, i0, cnt, ntot, invB, X, T, m.master, m.wbf,
                       grad, sse);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, long long n, float v, hipStream_t s)
{
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Adam (Kingma and Ba) on the FP32 master parameters, then refresh the BF16
// copies and clear the gradient for the next minibatch.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ P, uint16_t* __restrict__ wbf,
                                              float* __restrict__ m, float* __restrict__ v, float* __restrict__ grad,
                                              float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MLP_NPARAM; i += gridDim.x * blockDim.x) {
        const float gi = grad[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float p = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        P[i] = p;
        grad[i] = 0.f;
        if (i < MLP_OFF_B1) wbf[i] = (uint16_t)to_bf16(p);
        else if (i >= MLP_OFF_W2 && i < MLP_OFF_B2) wbf[512 + (i - MLP_OFF_W2)] = (uint16_t)to_bf16(p);
    }
}

hipError_t launch_adam(const MlpDev& md, float* m, float* v, float* grad, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(19), dim3(256), 0, s, md.master, md.wbf, m, v, grad, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// BF16 copies of the weight matrices from the master parameters.
__global__ void k_mlp_sync_bf16(const float* __restrict__ P, uint16_t* __restrict__ wbf)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MLP_NBF; i += gridDim.x * blockDim.x) {
        const float p = i < 512 ? P[MLP_OFF_W1 + i] : P[MLP_OFF_W2 + i - 512];
        wbf[i] = (uint16_t)to_bf16(p);
    }
}

hipError_t launch_mlp_sync(const MlpDev& m, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_sync_bf16, dim3(18), dim3(256), 0, s, m.master, m.wbf);
    return hipGetLastError();
}

// Learned guesses of independent problems (in [6][n], eos [4][n]) for the
// kernel-level solver.
__global__ __launch_bounds__(256) void k_points_guess(long long n, const double* __restrict__ in,
                                                      const double* __restrict__ eos, const MlpDev m,
                                                      double* __restrict__ guess)
{
    const int l = threadIdx.x & 63;
    const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
    const long long nw = ((long long)gridDim.x * blockDim.x) >> 6;
    if (wave * 64 >= n) return;                                   // wave-uniform
    MlpRegs w;
    mlp_load_regs(m.master, m.wbf, w);
    for (long long c = wave; c * 64 < n; c += nw) {
        const long long i = c * 64 + l;
        float x[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        double plo = 0.0, P = 1.0;
        bool skip = true;
        if (i < n) {
            const double rL = in[i], uL = in[n + i], pL = in[2 * n + i], rR = in[3 * n + i], uR = in[4 * n + i],
                         pR = in[5 * n + i];
            const double gL = eos[i], pcL = eos[n + i], gR = eos[2 * n + i], pcR = eos[3 * n + i];
            skip = acoustic_suffices(rL, uL, pL, gL, pcL, rR, uR, pR, gR, pcR);
            if (!skip) mlp_features(rL, uL, pL, gL, pcL, rR, uR, pR, gR, pcR, x, plo, P);
        }
        const double gs = guess64(w, x, plo, P, skip);
        if (i < n) guess[i] = gs;
    }
}

hipError_t launch_points_guess(long long n, const double* in, const double* eos, const MlpDev& m, double* guess,
                               hipStream_t s)
{
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_points_guess, dim3((unsigned)nb), dim3(256), 0, s, n, in, eos, m, guess);
    return hipGetLastError();
}

}  // namespace m2c
