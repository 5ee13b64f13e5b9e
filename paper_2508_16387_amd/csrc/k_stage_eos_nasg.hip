// k_stage_eos_nasg.hip -- general-EOS stage kernels of the default scheme on
// the 16x15 tile for the family sets that hold the Noble-Abel stiffened gas:
// {NASG}, {NASG, Mie-Grueneisen}, {NASG, JWL} (each kernel carries only the
// code of its families; k_stage_eos_other.hip has the other sets, so that
// the two files compile in parallel).
#include "m2c_stage.h"

namespace m2c {

hipError_t launch_stage_eos_nasg(int stage, int fs, const StageArgs& a, hipStream_t s)
{
    constexpr int N = 1 << M2C_EOS_NASG, M = 1 << M2C_EOS_MG, J = 1 << M2C_EOS_JWL;
    switch (fs) {
        case N: return launch_tile<16, 15, double, false, true, N>(stage, a, s);
        case N | M: return launch_tile<16, 15, double, false, true, N | M>(stage, a, s);
        case N | J: return launch_tile<16, 15, double, false, true, N | J>(stage, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace m2c
