// k_stage_eos_other.hip -- general-EOS stage kernels of the default scheme on
// the 16x15 tile for the family sets without the Noble-Abel stiffened gas:
// {Mie-Grueneisen}, {JWL}, {Mie-Grueneisen, JWL} (each kernel carries only
// the code of its families).
#include "m2c_stage.h"

namespace m2c {

hipError_t launch_stage_eos_other(int stage, int fs, const StageArgs& a, hipStream_t s)
{
    constexpr int M = 1 << M2C_EOS_MG, J = 1 << M2C_EOS_JWL;
    switch (fs) {
        case M: return launch_tile<16, 15, double, false, true, M>(stage, a, s);
        case J: return launch_tile<16, 15, double, false, true, J>(stage, a, s);
        case M | J: return launch_tile<16, 15, double, false, true, M | J>(stage, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace m2c
