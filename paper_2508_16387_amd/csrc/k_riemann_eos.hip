// k_riemann_eos.hip -- kernels and C entry points of the general-EOS exact
// two-material Riemann solver and of the EOS evaluation; the per-problem
// numerics are in m2c_eos.h.
//
// Work decomposition: one thread per problem, grid-stride, FP64 throughout;
// the material table travels in the kernel arguments.  The work of one
// problem depends strongly on its two materials (closed forms for NASG and
// JWL, RK4 walks for Mie-Grueneisen), and a wavefront runs as long as its
// slowest lane, so a set that mixes material pairs is first grouped by pair
// (a counting sort over the at most 64 pair keys) and solved through that
// permutation: the lanes of a wavefront then share their materials.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "m2c.h"
#include "m2c_eos.h"

namespace m2c {
namespace {

using namespace m2c::eos;

// pair key of problem i: ml * nmat + mr, or nmat^2 for an index outside the table
__device__ __forceinline__ int pair_key(const int32_t* mat, long long n, long long i, int nmat)
{
    const int ml = mat[i], mr = mat[n + i];
    return (ml >= 0 && ml < nmat && mr >= 0 && mr < nmat) ? ml * nmat + mr : nmat * nmat;
}

constexpr int NKEY = M2C_EOS_MAX * M2C_EOS_MAX + 1;

// counts[key] += problems of that key (block histogram in LDS first)
__global__ __launch_bounds__(256) void k_pair_count(long long n, const int32_t* __restrict__ mat, int nmat,
                                                    int32_t* __restrict__ counts)
{
    __shared__ int32_t h[NKEY];
    for (int k = threadIdx.x; k < NKEY; k += blockDim.x) h[k] = 0;
    __syncthreads();
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&h[pair_key(mat, n, i, nmat)], 1);
    __syncthreads();
    for (int k = threadIdx.x; k < NKEY; k += blockDim.x)
        if (h[k]) atomicAdd(&counts[k], h[k]);
}

// cursor = exclusive prefix sum of counts (one thread; NKEY entries)
__global__ void k_pair_scan(const int32_t* __restrict__ counts, int32_t* __restrict__ cursor)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int32_t acc = 0;
        for (int k = 0; k < NKEY; ++k) {
            cursor[k] = acc;
            acc += counts[k];
        }
    }
}

// perm[slot] = i, slots of one key contiguous: each block reserves its
// share of every key with one atomic and ranks its problems in LDS
__global__ __launch_bounds__(256) void k_pair_place(long long n, const int32_t* __restrict__ mat, int nmat,
                                                    int32_t* __restrict__ cursor, int32_t* __restrict__ perm)
{
    __shared__ int32_t h[NKEY], base[NKEY];
    for (int k = threadIdx.x; k < NKEY; k += blockDim.x) h[k] = 0;
    __syncthreads();
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int key = 0, rank = 0;
    if (i < n) {
        key = pair_key(mat, n, i, nmat);
        rank = atomicAdd(&h[key], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NKEY; k += blockDim.x)
        if (h[k]) base[k] = atomicAdd(&cursor[k], h[k]);
    __syncthreads();
    if (i < n) perm[base[key] + rank] = (int32_t)i;
}

// perm (nullable): thread t solves problem perm[t]
__global__ __launch_bounds__(256) void k_riemann_eos(long long n, const double* __restrict__ in,
                                                     const int32_t* __restrict__ mat, const EosTable tab,
                                                     double rtol, int maxit, double hmax,
                                                     double* __restrict__ out, int32_t* __restrict__ iters,
                                                     int32_t* __restrict__ nbad, const int32_t* __restrict__ perm)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const long long i = perm ? (long long)perm[t] : t;
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
    // grouping by material pair pays once the set is large and mixes pairs
    const bool group = nmat > 1 && n >= 4096 && n < (1LL << 31);
    // workspace (int32): failure count, key counts, key cursors, permutation
    const long long words = 1 + 2 * NKEY + (group ? n : 0);
    int32_t* dbad = nullptr;
    if (hipMalloc((void**)&dbad, words * sizeof(int32_t)) != hipSuccess) return M2C_ERR_NOMEM;
    int32_t* counts = dbad + 1;
    int32_t* cursor = counts + NKEY;
    int32_t* perm = group ? cursor + NKEY : nullptr;
    int32_t hb = 0;
    int rc = M2C_OK;
    if (hipMemsetAsync(dbad, 0, (1 + NKEY) * sizeof(int32_t), s) != hipSuccess) rc = M2C_ERR_DEVICE;
    if (rc == M2C_OK && group) {
        const unsigned nb = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_pair_count, dim3(nb), dim3(256), 0, s, (long long)n, mat, (int)nmat, counts);
        hipLaunchKernelGGL(k_pair_scan, dim3(1), dim3(64), 0, s, counts, cursor);
        hipLaunchKernelGGL(k_pair_place, dim3(nb), dim3(256), 0, s, (long long)n, mat, (int)nmat, cursor, perm);
        if (hipGetLastError() != hipSuccess) rc = M2C_ERR_DEVICE;
    }
    if (rc == M2C_OK) {
        hipLaunchKernelGGL(k_riemann_eos, dim3(grid_for(n)), dim3(256), 0, s, (long long)n, in, mat, tab, rtol,
                           (int)maxit, ds, out, iters, dbad, (const int32_t*)perm);
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
