// k_stage.hip -- the stage kernels with the default limiter and flux (MC,
// HLLC) and the persistent batched stage kernel; the kernel body is in
// m2c_stage.h.
#include "m2c_stage.h"

namespace m2c {

// Persistent batched stage: the grid is sized to the resident capacity and
// walks a list of (run, tile) items of many independent grids; each XCD
// takes a contiguous share of the list.  The state parity of each run lives
// in its device scalars, so one captured graph serves every step.
template <int STAGE, int TX, int TY, typename TF>
__global__ M2C_STAGE_BOUNDS(TX, TY, TF) void k_stage_batch(const RunDesc* __restrict__ runs,
                                                           const int2* __restrict__ items, int nitems)
{
    const int G = gridDim.x;
    int lb, per, lo, hi;
    if (G >= 8) {
        const int xcd = blockIdx.x % 8;
        lb = blockIdx.x / 8;
        per = (G + 7 - xcd) / 8;                           // blocks on this XCD
        lo = (int)((long long)nitems * xcd / 8);
        hi = (int)((long long)nitems * (xcd + 1) / 8);
    } else {
        lb = blockIdx.x;
        per = G;
        lo = 0;
        hi = nitems;
    }
    for (int t = lo + lb; t < hi; t += per) {
        const int2 it = items[t];
        const RunDesc& R = runs[it.x];
        const int cur = R.sc->cur;
        StageArgs a;
        a.g = R.g;
        a.Win = STAGE == 1 ? R.W[cur] : R.W1;
        a.W0 = R.W[cur];
        a.Wout = STAGE == 1 ? R.W1 : R.W[cur ^ 1];
        a.chi = R.chi[cur];
        a.chi_next = R.chi[cur ^ 1];
        a.flips = R.flips;
        a.fslot = R.fslot;
        a.fluxF = R.fluxF;
        a.qcap = R.qcap;
        a.sc = R.sc;
        a.tiles_x = R.tiles_x;
        a.tiles_y = R.tiles_y;
        a.tiles_z = R.tiles_z;
        a.kz = R.kz;
        a.c0 = 0.5;
        a.c1 = 0.5;
        stage_tile<STAGE, TX, TY, TF, false, false>(a, it.y);
    }
}

// ---- launchers ----------------------------------------------------------------
template <int TX, int TY, typename TF>
static hipError_t launch_tile_batch(int stage, const RunDesc* runs, const int2* items, int nitems, hipStream_t s)
{
    int dev = 0, ncu = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = stage == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stage_batch<1, TX, TY, TF>,
                                                                     stage_threads(TX, TY), 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stage_batch<2, TX, TY, TF>,
                                                                     stage_threads(TX, TY), 0);
    if (e != hipSuccess) return e;
    long long nblk = (long long)ncu * (per > 0 ? per : 1);
    if (nblk > nitems) nblk = nitems > 0 ? nitems : 1;
    if (stage == 1)
        hipLaunchKernelGGL((k_stage_batch<1, TX, TY, TF>), dim3((unsigned)nblk), dim3(stage_threads(TX, TY)), 0, s,
                           runs, items, nitems);
    else
        hipLaunchKernelGGL((k_stage_batch<2, TX, TY, TF>), dim3((unsigned)nblk), dim3(stage_threads(TX, TY)), 0, s,
                           runs, items, nitems);
    return hipGetLastError();
}

bool stage_tile_supported(int tx, int ty)
{
    return (tx == 16 && ty == 15) || (tx == 32 && ty == 7) || (tx == 16 && ty == 16) || (tx == 32 && ty == 8) ||
           (tx == 64 && ty == 2);
}

hipError_t launch_stage(int stage, bool mixed, int tx, int ty, const StageArgs& a, hipStream_t s)
{
    if (a.g.eosg) return mixed ? hipErrorInvalidValue : launch_stage_eos(stage, tx, ty, a, s);
    if (a.g.limiter != LIM_MC || a.g.flux != FLUX_HLLC || a.g.ls_band > 0.0)
        return launch_stage_opts(stage, mixed, tx, ty, a, s);
#define M2C_TILE(TX_, TY_)                                                              \
    if (tx == TX_ && ty == TY_)                                                         \
        return mixed ? launch_tile<TX_, TY_, float, false>(stage, a, s)                \
                     : launch_tile<TX_, TY_, double, false>(stage, a, s);
    M2C_TILES(M2C_TILE)
#undef M2C_TILE
    return hipErrorInvalidValue;
}

hipError_t launch_stage_batch(int stage, bool mixed, int tx, int ty, const RunDesc* runs, const int2* items,
                              int nitems, hipStream_t s)
{
#define M2C_TILE(TX_, TY_)                                                                          \
    if (tx == TX_ && ty == TY_)                                                                     \
        return mixed ? launch_tile_batch<TX_, TY_, float>(stage, runs, items, nitems, s)           \
                     : launch_tile_batch<TX_, TY_, double>(stage, runs, items, nitems, s);
    M2C_TILES(M2C_TILE)
#undef M2C_TILE
    return hipErrorInvalidValue;
}

}  // namespace m2c
