// k_stage_eos.hip -- the stage kernels with a general equation of state per
// material (NASG, Mie-Grueneisen, JWL; section "Equations of state"): every
// conversion, sound speed and single-material flux takes the material's EOS.
// FP64 only, and two tile shapes (16x15, and 64x2 for grids one cell high);
// kept apart from the stiffened-gas kernels, whose register allocation the
// EOS code would otherwise enlarge.
//
// The default scheme (MC, HLLC, whole grid) on the 16x15 tile runs kernels
// compiled for the set of the two materials' families (k_stage_eos_nasg.hip
// for the sets that hold NASG, k_stage_eos_other.hip for the rest), each
// carrying only the code of those families; the run-time options (limiter,
// flux, level-set band) and the 64x2 tile take the kernels of this file,
// which dispatch on the families at run time.
#include "m2c_stage.h"

namespace m2c {

bool stage_tile_supported_eos(int tx, int ty) { return (tx == 16 && ty == 15) || (tx == 64 && ty == 2); }

hipError_t launch_stage_eos(int stage, int tx, int ty, const StageArgs& a, hipStream_t s)
{
    const bool opts = a.g.limiter != LIM_MC || a.g.flux != FLUX_HLLC || a.g.ls_band > 0.0;
    if (tx == 16 && ty == 15 && !opts) {
        const int f0 = a.g.ek[0].fam, f1 = a.g.ek[1].fam;
        if (f0 < 0 || f0 > 2 || f1 < 0 || f1 > 2) return hipErrorInvalidValue;
        const int fs = eos::fam_set(f0) | eos::fam_set(f1);
        return (fs & eos::fam_set(M2C_EOS_NASG)) ? launch_stage_eos_nasg(stage, fs, a, s)
                                                 : launch_stage_eos_other(stage, fs, a, s);
    }
    if (tx == 16 && ty == 15) return launch_tile<16, 15, double, true, true>(stage, a, s);
    if (tx == 64 && ty == 2)
        return opts ? launch_tile<64, 2, double, true, true>(stage, a, s)
                    : launch_tile<64, 2, double, false, true>(stage, a, s);
    return hipErrorInvalidValue;
}

}  // namespace m2c
