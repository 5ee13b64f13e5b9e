// k_stage_opts.hip -- the stage kernels with the limiter, numerical flux and
// level-set band taken from the configuration at run time (MC, Van Albada or
// modified Van Albada slopes; HLLC or local Lax-Friedrichs fluxes; whole-grid
// or narrow-band level set).  Kept apart from the
// default kernels, whose register allocation the run-time choice would
// otherwise enlarge.
#include "m2c_stage.h"

namespace m2c {

hipError_t launch_stage_opts(int stage, bool mixed, int tx, int ty, const StageArgs& a, hipStream_t s)
{
#define M2C_TILE(TX_, TY_)                                                              \
    if (tx == TX_ && ty == TY_)                                                         \
        return mixed ? launch_tile<TX_, TY_, float, true>(stage, a, s)                 \
                     : launch_tile<TX_, TY_, double, true>(stage, a, s);
    M2C_TILES(M2C_TILE)
#undef M2C_TILE
    return hipErrorInvalidValue;
}

}  // namespace m2c
