// m2c_mlp.h -- learned star-pressure guess: parameter layout and the
// feature map shared by the inference, training and FIVER-guess kernels.
//
// Network 8 -> 64 -> 64 -> 1 with tanh hidden layers.  Parameter vector
// (4801 FP32 values, the master copy): W1 (64x8, row-major), b1 (64),
// W2 (64x64, row-major), b2 (64), w3 (64), b3 (1).  The two weight matrices
// also live as BF16 copies, the operands of the matrix-core products.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace m2c {

constexpr int MLP_IN = 8, MLP_H = 64;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 512, MLP_OFF_W2 = 576, MLP_OFF_B2 = 4672, MLP_OFF_W3 = 4736,
              MLP_OFF_B3 = 4800, MLP_NPARAM = 4801;
constexpr int MLP_NBF = 512 + 4096;            // BF16 copies: W1 then W2

struct MlpDev {
    float* master;                             // [MLP_NPARAM]
    uint16_t* wbf;                             // [MLP_NBF]
};

// Dimensionless features of a two-material Riemann problem and the scale of
// the target: the network predicts y = ln((p* - p_lo)/P), with
// p_lo = -min(pc_L, pc_R) and P = sqrt((p_L - p_lo)(p_R - p_lo)), so the
// guess p_lo + P exp(y) is admissible for any y.
__device__ __forceinline__ void mlp_features(double rL, double uL, double pL, double gL, double pcL, double rR,
                                             double uR, double pR, double gR, double pcR, float x[8],
                                             double& plo, double& P)
{
    plo = -fmin(pcL, pcR);
    const double aL = pL - plo, aR = pR - plo;
    P = sqrt(aL * aR);
    const double rb = sqrt(rL * rR);
    const double U = sqrt(P / rb);
    const double ub = 0.5 * (uL + uR);
    x[0] = (float)log(rL / rb);
    x[1] = (float)log(rR / rb);
    x[2] = (float)((uL - ub) / U);
    x[3] = (float)((uR - ub) / U);
    x[4] = (float)log(aL / P);
    x[5] = (float)log(aR / P);
    x[6] = (float)log(gL / gR);
    x[7] = (float)((pcL - pcR) / (pcL + pcR + P));
}

}  // namespace m2c
