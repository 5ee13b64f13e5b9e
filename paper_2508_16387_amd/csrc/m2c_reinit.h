// m2c_reinit.h -- level-set reinitialization launch interface (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace m2c {

struct ReinitGrid {
    int nx, ny, nz;
    int per[3];                    // axis is periodic
    int act[3];                    // axis has more than one cell
    double h[3], rh[3];            // width, 1/width
    double hmin;                   // smallest width over the active axes
    int rz;                        // planes per block
    int bx, by, bz;                // blocks per axis (64 x 4 x rz cells each)
};

// false for invalid sizes, widths or boundary codes (periodic must pair up)
bool reinit_grid(int nx, int ny, int nz, const double h[3], const int32_t bc[6], ReinitGrid& g);
long long reinit_blocks(const ReinitGrid& g);
// workspace: S [N] and the second iterate [N] (FP64), the list of moving
// blocks with its count in front [1 + blocks of one plane each] (int32)
inline long long reinit_workspace_bytes(const ReinitGrid& g)
{
    const long long N = (long long)g.nx * g.ny * g.nz;
    return 16 * N + 4 * (1 + (long long)g.bx * g.by * g.nz);
}
// iters pseudo-time steps on phi (device, in place) with the given
// workspace; synchronises the stream once (the count of moving blocks)
hipError_t reinit_run(const ReinitGrid& g, double* phi, double* S, double* tmp, int32_t* list, int iters,
                      double band, hipStream_t s);

}  // namespace m2c
