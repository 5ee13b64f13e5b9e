// k_reinit.hip -- level-set reinitialization (section "Level set method",
// eq. reinit): pseudo-time steps of
//     d phi / d tau + S(phi_0) (|grad phi| - 1) = 0,
//     S(phi_0) = phi_0 / sqrt(phi_0^2 + eps^2),
// with the upwind (Godunov) |grad phi| of one-sided differences a = D^- phi,
// b = D^+ phi per active axis:
//     S > 0: sum_d max(max(a_d, 0)^2, min(b_d, 0)^2)
//     S < 0: sum_d max(min(a_d, 0)^2, max(b_d, 0)^2)
// and forward-Euler steps dtau = 0.5 min_d h_d (Jacobi: every cell reads the
// previous iterate).  First-layer cells (a face neighbour on the other side
// of the zero level set, phi >= 0 counting as the non-negative side) keep
// phi_0, which is the paper's fixed-first-layer treatment; with a narrow
// band only cells with |phi_0| < band move.  Both are expressed as S = 0.
//
// Boundary images: one layer, periodic axes wrap, transmissive and wall
// boundaries repeat the boundary cell (the zero-gradient and mirror images
// of phi coincide for one layer).
//
// Work decomposition (MI355X): a 256-thread block owns a 64 x 4 tile of an
// xy-plane and a few consecutive planes; x is the contiguous axis and every
// wavefront holds one 512-byte row per plane.  A cell's x neighbours come
// from the adjacent lanes (shuffles), its y neighbours from the other rows
// of the block through LDS, its z neighbours from a three-plane register
// window; only the tile's edge lanes and rows load halo values.  The speed kernel
// appends the blocks that hold any cell with S != 0 to a list, and the step
// kernel runs on that list only.  The iterate is kept in two buffers that
// both start as phi_0; a frozen cell never changes, so it is never written
// -- a narrow band costs only the blocks it touches.  Per iteration and
// moving cell the algorithmic traffic is phi and S read, phi written: 24
// bytes.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "m2c.h"
#include "m2c_reinit.h"

namespace m2c {
namespace {

constexpr int RX = 64, RY = 4;
// planes per block: 4 over the whole grid; 1 in a narrow band, where few
// blocks move and the serial plane loop of each would be exposed latency
// (measured at 128^3: whole grid 15.5 us per step with 4 planes against
// 17.3 with 8; band of six cells 5.3 us with 1 against 7.5 with 4)
constexpr int RZ_FULL = 4, RZ_BAND = 1;

__device__ __forceinline__ int image(int i, int n, int periodic)
{
    return i < 0 ? (periodic ? i + n : 0) : (i >= n ? (periodic ? i - n : n - 1) : i);
}

struct Tile {
    int i, j, k0, k1;
};

__device__ __forceinline__ Tile tile_of(const ReinitGrid& g, int b)
{
    const int bx = b % g.bx, r = b / g.bx;
    const int by = r % g.by, bz = r / g.by;
    Tile t;
    t.i = bx * RX + (int)(threadIdx.x % RX);
    t.j = by * RY + (int)(threadIdx.x / RX);
    t.k0 = bz * g.rz;
    t.k1 = min(t.k0 + g.rz, g.nz);
    return t;
}

__global__ __launch_bounds__(256) void k_reinit_speed(const ReinitGrid g, const double* __restrict__ phi0,
                                                      double eps2, double band, double* __restrict__ S,
                                                      int32_t* __restrict__ list)
{
    const Tile t = tile_of(g, blockIdx.x);
    const bool in = t.i < g.nx && t.j < g.ny;
    int any = 0;
    if (in) {
        for (int k = t.k0; k < t.k1; ++k) {
            const long long c = (long long)t.i + (long long)g.nx * (t.j + (long long)g.ny * k);
            const double p = phi0[c];
            const bool pos = p >= 0.0;
            bool fl = false;
            if (g.nx > 1) {
                fl |= (phi0[c - t.i + image(t.i - 1, g.nx, g.per[0])] >= 0.0) != pos;
                fl |= (phi0[c - t.i + image(t.i + 1, g.nx, g.per[0])] >= 0.0) != pos;
            }
            if (g.ny > 1) {
                const long long r0 = c - (long long)g.nx * t.j;
                fl |= (phi0[r0 + (long long)g.nx * image(t.j - 1, g.ny, g.per[1])] >= 0.0) != pos;
                fl |= (phi0[r0 + (long long)g.nx * image(t.j + 1, g.ny, g.per[1])] >= 0.0) != pos;
            }
            if (g.nz > 1) {
                const long long pl = (long long)g.nx * g.ny, r0 = c - pl * k;
                fl |= (phi0[r0 + pl * image(k - 1, g.nz, g.per[2])] >= 0.0) != pos;
                fl |= (phi0[r0 + pl * image(k + 1, g.nz, g.per[2])] >= 0.0) != pos;
            }
            double s = p / sqrt(p * p + eps2);
            if (fl || (band > 0.0 && fabs(p) >= band)) s = 0.0;
            S[c] = s;
            any |= s != 0.0;
        }
    }
    any = __syncthreads_or(any);
    // list[0] counts the blocks with moving cells, list[1..] holds them
    if (threadIdx.x == 0 && any) list[1 + atomicAdd(&list[0], 1)] = blockIdx.x;
}

// LIST: the block runs tile list[1 + blockIdx.x] (narrow band); otherwise
// the tile of the 3D block index (whole grid, no integer division)
template <bool LIST>
__global__ __launch_bounds__(256) void k_reinit_step(const ReinitGrid g, const double* __restrict__ phi,
                                                     double* __restrict__ out, const double* __restrict__ S,
                                                     const int32_t* __restrict__ list, double dtau)
{
    // one wavefront per x-row of the tile: x neighbours by lane shuffles, y
    // neighbours through a double-buffered LDS copy of the block's four rows,
    // z neighbours in a register window; only the tile's edges load halos.
    // Offsets are 32-bit (grids up to 2^31 cells); the one-sided
    // differences multiply by 1/h.
    __shared__ double sRow[2][RY][RX];
    Tile t;
    if (LIST) {
        t = tile_of(g, list[1 + blockIdx.x]);
    } else {
        t.i = (int)blockIdx.x * RX + (int)(threadIdx.x % RX);
        t.j = (int)blockIdx.y * RY + (int)(threadIdx.x / RX);
        t.k0 = (int)blockIdx.z * g.rz;
        t.k1 = min(t.k0 + g.rz, g.nz);
    }
    const int lane = (int)(threadIdx.x % RX), w = (int)(threadIdx.x / RX);
    const bool live = t.i < g.nx && t.j < g.ny;
    const int ic = min(t.i, g.nx - 1), jc = min(t.j, g.ny - 1);      // clamped: loads stay in range
    const uint32_t pl = (uint32_t)g.nx * (uint32_t)g.ny;
    const uint32_t row0 = (uint32_t)g.nx * (uint32_t)jc, col = row0 + (uint32_t)ic;
    const bool xlo = lane == 0 || ic == 0, xhi = lane == RX - 1 || ic == g.nx - 1;
    const bool ylo = w == 0 || jc == 0, yhi = w == RY - 1 || jc == g.ny - 1;
    const uint32_t xm = row0 + image(ic - 1, g.nx, g.per[0]), xp = row0 + image(ic + 1, g.nx, g.per[0]);
    const uint32_t ym = (uint32_t)g.nx * image(jc - 1, g.ny, g.per[1]) + ic;
    const uint32_t yp = (uint32_t)g.nx * image(jc + 1, g.ny, g.per[1]) + ic;
    double pzm = phi[col + pl * image(t.k0 - 1, g.nz, g.per[2])];
    double p = phi[col + pl * t.k0];
    int buf = 0;
    for (int k = t.k0; k < t.k1; ++k, buf ^= 1) {
        const uint32_t o = pl * (uint32_t)k;
        const double pzp = phi[col + pl * image(k + 1, g.nz, g.per[2])];
        const double s = S[col + o];
        sRow[buf][w][lane] = p;
        const double su = __shfl_up(p, 1), sd = __shfl_down(p, 1);
        __syncthreads();
        const double xa = xlo ? phi[xm + o] : su, xb = xhi ? phi[xp + o] : sd;
        const double ya = ylo ? phi[ym + o] : sRow[buf][w - 1][lane];
        const double yb = yhi ? phi[yp + o] : sRow[buf][w + 1][lane];
        if (live && s != 0.0) {                       // frozen: both buffers hold phi_0
            const bool up = s > 0.0;
            auto term = [&](double lo, double hi, double rh) {
                const double a = (p - lo) * rh, b = (hi - p) * rh;
                const double u = up ? fmax(a, 0.0) : fmin(a, 0.0), v = up ? fmin(b, 0.0) : fmax(b, 0.0);
                return fmax(u * u, v * v);
            };
            double g2 = 0.0;
            if (g.act[0]) g2 += term(xa, xb, g.rh[0]);
            if (g.act[1]) g2 += term(ya, yb, g.rh[1]);
            if (g.act[2]) g2 += term(pzm, pzp, g.rh[2]);
            out[col + o] = p - dtau * s * (sqrt(g2) - 1.0);
        }
        pzm = p;
        p = pzp;
    }
}

}  // namespace

long long reinit_blocks(const ReinitGrid& g)
{
    return (long long)g.bx * g.by * g.bz;
}

bool reinit_grid(int nx, int ny, int nz, const double h[3], const int32_t bc[6], ReinitGrid& g)
{
    if (nx < 1 || ny < 1 || nz < 1) return false;
    if ((long long)nx * ny * nz > (1LL << 31)) return false;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    const int n[3] = {nx, ny, nz};
    double hmin = INFINITY;
    for (int d = 0; d < 3; ++d) {
        if (!(h[d] > 0.0) || !isfinite(h[d])) return false;
        for (int s = 0; s < 2; ++s)
            if (bc[2 * d + s] < M2C_BC_TRANSMISSIVE || bc[2 * d + s] > M2C_BC_PERIODIC) return false;
        if ((bc[2 * d] == M2C_BC_PERIODIC) != (bc[2 * d + 1] == M2C_BC_PERIODIC)) return false;
        g.per[d] = bc[2 * d] == M2C_BC_PERIODIC;
        g.act[d] = n[d] > 1;
        g.h[d] = h[d];
        g.rh[d] = 1.0 / h[d];
        if (g.act[d]) hmin = fmin(hmin, h[d]);
    }
    g.hmin = isfinite(hmin) ? hmin : fmin(h[0], fmin(h[1], h[2]));
    g.bx = (nx + RX - 1) / RX;
    g.by = (ny + RY - 1) / RY;
    g.rz = RZ_FULL;
    g.bz = (nz + g.rz - 1) / g.rz;
    return true;
}

hipError_t reinit_run(const ReinitGrid& g0, double* phi, double* S, double* tmp, int32_t* list, int iters,
                      double band, hipStream_t s)
{
    ReinitGrid g = g0;
    g.rz = band > 0.0 ? RZ_BAND : RZ_FULL;
    g.bz = (g.nz + g.rz - 1) / g.rz;
    const long long N = (long long)g.nx * g.ny * g.nz;
    const long long nb = reinit_blocks(g);
    if (iters <= 0) return hipSuccess;
    const double eps = g.hmin;                        // smallest cell width
    hipError_t e = hipMemsetAsync(list, 0, sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reinit_speed, dim3((unsigned)nb), dim3(256), 0, s, g, phi, eps * eps, band, S, list);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(tmp, phi, N * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    // the number of moving blocks sizes every step launch
    int32_t nact = 0;
    e = hipMemcpyAsync(&nact, list, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (nact < 0 || nact > nb) return hipErrorUnknown;
    const double dtau = 0.5 * g.hmin;
    // whole grid: a 3D launch over every tile (nearly all move); band: the list
    const bool use_list = band > 0.0 || g.by > 65535 || g.bz > 65535;
    for (int it = 0; it < iters && nact > 0; ++it) {
        const double* src = (it & 1) ? tmp : phi;
        double* dst = (it & 1) ? phi : tmp;
        if (use_list)
            hipLaunchKernelGGL(k_reinit_step<true>, dim3((unsigned)nact), dim3(256), 0, s, g, src, dst, S, list,
                               dtau);
        else
            hipLaunchKernelGGL(k_reinit_step<false>, dim3((unsigned)g.bx, (unsigned)g.by, (unsigned)g.bz),
                               dim3(256), 0, s, g, src, dst, S, list, dtau);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if ((iters & 1) && nact > 0) e = hipMemcpyAsync(phi, tmp, N * sizeof(double), hipMemcpyDeviceToDevice, s);
    return e;
}

}  // namespace m2c

using namespace m2c;

extern "C" int m2c_reinit_workspace(int32_t nx, int32_t ny, int32_t nz, int64_t* bytes)
{
    const double h[3] = {1.0, 1.0, 1.0};
    const int32_t bc[6] = {0, 0, 0, 0, 0, 0};
    ReinitGrid g;
    if (!bytes || !reinit_grid(nx, ny, nz, h, bc, g)) return M2C_ERR_ARG;
    *bytes = reinit_workspace_bytes(g);
    return M2C_OK;
}

extern "C" int m2c_reinit_field(int32_t nx, int32_t ny, int32_t nz, const double h[3], const int32_t bc[6],
                                double* phi, void* work, int32_t iters, double band, void* hip_stream)
{
    ReinitGrid g;
    if (!h || !bc || !reinit_grid(nx, ny, nz, h, bc, g)) return M2C_ERR_ARG;
    if (iters < 0 || !(band >= 0.0) || !isfinite(band)) return M2C_ERR_ARG;
    if (iters == 0) return M2C_OK;
    if (!phi || !work) return M2C_ERR_ARG;
    const long long N = (long long)nx * ny * nz;
    double* S = (double*)work;
    double* tmp = S + N;
    int32_t* active = (int32_t*)(tmp + N);
    return reinit_run(g, phi, S, tmp, active, iters, band, (hipStream_t)hip_stream) == hipSuccess ? M2C_OK
                                                                                                  : M2C_ERR_DEVICE;
}
