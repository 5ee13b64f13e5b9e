// k_riemann_eos.hip -- kernels and C entry points of the general-EOS exact
// two-material Riemann solver and of the EOS evaluation; the per-problem
// numerics are in m2c_eos.h.
//
// Work decomposition: one thread per problem, grid-stride, FP64 throughout;
// the material table travels in the kernel arguments (materials may differ
// between the lanes of a wavefront).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "m2c.h"
#include "m2c_eos.h"

namespace m2c {
namespace {

using namespace m2c::eos;

__global__ __launch_bounds__(256) void k_riemann_eos(long long n, const double* __restrict__ in,
                                                     const int32_t* __restrict__ mat, const EosTable tab,
                                                     double rtol, int maxit, double hmax,
                                                     double* __restrict__ out, int32_t* __restrict__ iters,
                                                     int32_t* __restrict__ nbad)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double q[6], res[4];
        for (int k = 0; k < 6; ++k) q[k] = in[k * n + i];
        const int its = solve_one(tab, mat[i], mat[n + i], q, rtol, maxit, hmax, res);
        if (its == 0) atomicAdd(nbad, 1);
        for (int k = 0; k < 4; ++k) out[k * n + i] = res[k];
        if (iters) iters[i] = its;
    }
}

__global__ __launch_bounds__(256) void k_eos_eval(long long n, const double* __restrict__ rho,
                                                  const double* __restrict__ e, const int32_t* __restrict__ mat,
                                                  const EosTable tab, double* __restrict__ p,
                                                  double* __restrict__ c)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int k = mat[i];
        double pp = __builtin_nan(""), cc = __builtin_nan("");
        if (k >= 0 && k < tab.n && rho[i] > 0.0) {
            const EosK& m = tab.m[k];
            const double v = 1.0 / rho[i];
            pp = eos_p(m, v, e[i]);
            const double c2 = eos_c2(m, v, pp);
            cc = c2 > 0.0 ? sqrt(c2) : __builtin_nan("");
            if (!(c2 > 0.0)) pp = __builtin_nan("");
        }
        p[i] = pp;
        c[i] = cc;
    }
}

unsigned grid_for(long long n)
{
    long long b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace
}  // namespace m2c

using namespace m2c;

extern "C" int m2c_riemann_solve_eos(int64_t n, const double* in, const int32_t* mat, int32_t nmat,
                                     const m2c_eos* eos, double rtol, int32_t maxit, double ds, double* out,
                                     int32_t* iters, void* hip_stream)
{
    if (n < 0 || (n > 0 && (!in || !mat || !out))) return M2C_ERR_ARG;
    if (!(rtol > 0.0) || maxit < 1) return M2C_ERR_ARG;
    if (ds == 0.0) ds = 0.01;
    if (!(ds >= 1e-3 && ds <= 0.5)) return M2C_ERR_ARG;
    EosTable tab;
    if (!prepare(nmat, eos, tab)) return M2C_ERR_ARG;
    if (n == 0) return M2C_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    int32_t* dbad = nullptr;
    if (hipMalloc((void**)&dbad, sizeof(int32_t)) != hipSuccess) return M2C_ERR_NOMEM;
    int32_t hb = 0;
    int rc = M2C_OK;
    if (hipMemsetAsync(dbad, 0, sizeof(int32_t), s) != hipSuccess) rc = M2C_ERR_DEVICE;
    if (rc == M2C_OK) {
        hipLaunchKernelGGL(k_riemann_eos, dim3(grid_for(n)), dim3(256), 0, s, (long long)n, in, mat, tab, rtol,
                           (int)maxit, ds, out, iters, dbad);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&hb, dbad, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = M2C_ERR_DEVICE;
    }
    (void)hipFree(dbad);
    if (rc == M2C_OK && hb > 0) rc = M2C_ERR_RIEMANN;
    return rc;
}

extern "C" int m2c_eos_eval(int64_t n, const double* rho, const double* e, const int32_t* mat, int32_t nmat,
                            const m2c_eos* eos, double* p, double* c, void* hip_stream)
{
    if (n < 0 || (n > 0 && (!rho || !e || !mat || !p || !c))) return M2C_ERR_ARG;
    EosTable tab;
    if (!prepare(nmat, eos, tab)) return M2C_ERR_ARG;
    if (n == 0) return M2C_OK;
    hipLaunchKernelGGL(k_eos_eval, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, (long long)n, rho, e,
                       mat, tab, p, c);
    return hipGetLastError() == hipSuccess ? M2C_OK : M2C_ERR_DEVICE;
}
