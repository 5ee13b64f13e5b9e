// k_stage_eos.hip -- the stage kernels with a general equation of state per
// material (NASG, Mie-Grueneisen, JWL; section "Equations of state"): every
// conversion, sound speed and single-material flux takes the material's EOS,
// and the limiter, flux and level-set band come from the configuration at
// run time.  FP64 only, and two tile shapes (16x16, and 64x2 for grids one
// cell high); kept apart from the stiffened-gas kernels, whose register
// allocation the EOS code would otherwise enlarge.
#include "m2c_stage.h"

namespace m2c {

bool stage_tile_supported_eos(int tx, int ty) { return (tx == 16 && ty == 16) || (tx == 64 && ty == 2); }

hipError_t launch_stage_eos(int stage, int tx, int ty, const StageArgs& a, hipStream_t s)
{
    const bool opts = a.g.limiter != LIM_MC || a.g.flux != FLUX_HLLC || a.g.ls_band > 0.0;
    // default scheme on the 16x16 tile without a Mie-Grueneisen material:
    // kernels without its code
    const bool nomg = a.g.ek[0].fam != M2C_EOS_MG && a.g.ek[1].fam != M2C_EOS_MG;
    if (tx == 16 && ty == 16 && !opts && nomg) return launch_tile<16, 16, double, false, true, true>(stage, a, s);
    if (tx == 16 && ty == 16)
        return opts ? launch_tile<16, 16, double, true, true>(stage, a, s)
                    : launch_tile<16, 16, double, false, true>(stage, a, s);
    if (tx == 64 && ty == 2)
        return opts ? launch_tile<64, 2, double, true, true>(stage, a, s)
                    : launch_tile<64, 2, double, false, true>(stage, a, s);
    return hipErrorInvalidValue;
}

}  // namespace m2c
