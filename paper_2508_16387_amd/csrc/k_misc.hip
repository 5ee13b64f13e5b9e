// k_misc.hip -- per-step bookkeeping, state conversion and the point
// kernels behind the kernel-level entry points.
#include "m2c_device.h"
#include "m2c_internal.h"
#include "m2c_kernels.h"

namespace m2c {

static unsigned grid_for(long long n, int threads, long long cap = 65536)
{
    long long b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// ---------------------------------------------------------------------------
// Batched begin / end of a step: one thread per run; dt from the CFL rule
// (section "Time integration"; the reading is dt = CFL / max_i sum over the
// axes with more than one cell of (|V_d| + c)/h_d) or imposed, accumulators
// cleared; a completed step advances the counters and flips the run's state
// parity.
__global__ void k_begin_batch(const RunDesc* __restrict__ runs, int n, double dt_imposed)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const RunDesc& R = runs[r];
    DevScalars* sc = R.sc;
    if (sc->err != 0) return;
    double dt;
    if (dt_imposed > 0.0) dt = dt_imposed;
    else if (R.g.dt_fixed > 0.0) dt = R.g.dt_fixed;
    else dt = R.g.cfl / __longlong_as_double((long long)sc->lam_bits);
    sc->dt = dt;
    sc->lam_bits = 0ull;
    sc->nflip = 0;
}

__global__ void k_end_batch(const RunDesc* __restrict__ runs, int n, int stages)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    DevScalars* sc = runs[r].sc;
    if (sc->err != 0) return;
    sc->steps_done += 1;
    sc->t += sc->dt;
    sc->dt_last = sc->dt;
    sc->solves += (long long)sc->qlen * stages;
    sc->flips += sc->nflip;
    sc->cur ^= 1;
}

hipError_t launch_begin_batch(const RunDesc* runs, int nruns, double dt_imposed, hipStream_t s)
{
    hipLaunchKernelGGL(k_begin_batch, dim3((nruns + 63) / 64), dim3(64), 0, s, runs, nruns, dt_imposed);
    return hipGetLastError();
}

hipError_t launch_end_batch(const RunDesc* runs, int nruns, int stages, hipStream_t s)
{
    hipLaunchKernelGGL(k_end_batch, dim3((nruns + 63) / 64), dim3(64), 0, s, runs, nruns, stages);
    return hipGetLastError();
}

// max_i lambda_i of a state (the CFL maximum of the first step after a
// state is set); non-negative doubles order like their bit patterns.
template <bool EG>
__global__ __launch_bounds__(256) void k_lambda(const Grid G, const double* __restrict__ W,
                                                const uint8_t* __restrict__ chi, DevScalars* sc)
{
    __shared__ double sRed[4];
    __shared__ eos::EosK sEos[EG ? 2 : 1];
    if constexpr (EG) geos_stage(G, sEos);
    const long long N = G.N;
    double lam = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const int x = chi[c];
        double u, v, w;
        const double r = W[c];
        double cs;
        if constexpr (EG) {
            const double p = geos_prim(sEos[x], r, W[N + c], W[2 * N + c], W[3 * N + c], W[4 * N + c], u, v, w);
            cs = sqrt(geos_c2(sEos[x], r, p));
        } else {
            const double p = eos_prim(r, W[N + c], W[2 * N + c], W[3 * N + c], W[4 * N + c], pick(G.gamma, x) - 1.0,
                                      pick(G.gpc, x), u, v, w);
            cs = sqrt(pick(G.gamma, x) * (p + pick(G.pc, x)) / r);
        }
        double l = 0.0;
        if (G.act[0]) l += (fabs(u) + cs) * G.rh[0];
        if (G.act[1]) l += (fabs(v) + cs) * G.rh[1];
        if (G.act[2]) l += (fabs(w) + cs) * G.rh[2];
        lam = fmax(lam, l);
    }
    for (int o = 32; o > 0; o >>= 1) lam = fmax(lam, __shfl_xor(lam, o));
    if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = lam;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) m = fmax(m, sRed[k]);
        atomic_max_nonneg(&sc->lam_bits, m);
    }
}

__global__ void k_zero_lam(DevScalars* sc) { sc->lam_bits = 0ull; }

hipError_t launch_lambda(const Grid& g, const double* W, const uint8_t* chi, DevScalars* sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_lam, dim3(1), dim3(1), 0, s, sc);
    if (g.eosg)
        hipLaunchKernelGGL(k_lambda<true>, dim3(grid_for(g.N, 256, 4096)), dim3(256), 0, s, g, W, chi, sc);
    else
        hipLaunchKernelGGL(k_lambda<false>, dim3(grid_for(g.N, 256, 4096)), dim3(256), 0, s, g, W, chi, sc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Primitive [rho,u,v,w,p,phi][N] -> conservative state and material ids,
// with the admissibility check (rho > 0, p + p_c > 0, all finite; with a
// general EOS p above the material's floor and c^2 > 0).  The first failing
// cell (smallest index) is reported through err_cell.
template <bool EG>
__global__ __launch_bounds__(256) void k_prim_to_cons(const Grid G, const double* __restrict__ P,
                                                      double* __restrict__ W, uint8_t* __restrict__ chi,
                                                      DevScalars* sc)
{
    __shared__ eos::EosK sEos[EG ? 2 : 1];
    if constexpr (EG) geos_stage(G, sEos);
    const long long N = G.N;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const double r = P[c], u = P[N + c], v = P[2 * N + c], w = P[3 * N + c], p = P[4 * N + c];
        const double phi = P[5 * N + c];
        const int x = phi < 0.0 ? 1 : 0;
        const bool adm = EG ? geos_ok(sEos[x], r, p) : r > 0.0 && p + pick(G.pc, x) > 0.0;
        const bool ok = isfinite(r) && isfinite(u) && isfinite(v) && isfinite(w) && isfinite(p) &&
                        isfinite(phi) && adm;
        if (!ok) report_error(&sc->err, &sc->err_cell, ST_NONPHYSICAL, c);
        W[c] = r;
        W[N + c] = r * u;
        W[2 * N + c] = r * v;
        W[3 * N + c] = r * w;
        if constexpr (EG) W[4 * N + c] = geos_energy(sEos[x], r, u, v, w, p);
        else W[4 * N + c] = eos_energy<double>(r, u, v, w, p, pick(G.gpc, x), pick(G.inv_gm1, x));
        W[5 * N + c] = phi;
        chi[c] = (uint8_t)x;
    }
}

hipError_t launch_prim_to_cons(const Grid& g, const double* prim6, double* W, uint8_t* chi, DevScalars* sc,
                               hipStream_t s)
{
    if (g.eosg)
        hipLaunchKernelGGL(k_prim_to_cons<true>, dim3(grid_for(g.N, 256)), dim3(256), 0, s, g, prim6, W, chi, sc);
    else
        hipLaunchKernelGGL(k_prim_to_cons<false>, dim3(grid_for(g.N, 256)), dim3(256), 0, s, g, prim6, W, chi, sc);
    return hipGetLastError();
}

template <bool EG>
__global__ __launch_bounds__(256) void k_cons_to_prim(const Grid G, const double* __restrict__ W,
                                                      const uint8_t* __restrict__ chi, double* __restrict__ P)
{
    __shared__ eos::EosK sEos[EG ? 2 : 1];
    if constexpr (EG) geos_stage(G, sEos);
    const long long N = G.N;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const int x = chi[c];
        double u, v, w, p;
        if constexpr (EG) p = geos_prim(sEos[x], W[c], W[N + c], W[2 * N + c], W[3 * N + c], W[4 * N + c], u, v, w);
        else p = eos_prim(W[c], W[N + c], W[2 * N + c], W[3 * N + c], W[4 * N + c], pick(G.gamma, x) - 1.0,
                          pick(G.gpc, x), u, v, w);
        P[c] = W[c];
        P[N + c] = u;
        P[2 * N + c] = v;
        P[3 * N + c] = w;
        P[4 * N + c] = p;
        P[5 * N + c] = W[5 * N + c];
    }
}

hipError_t launch_cons_to_prim(const Grid& g, const double* W, const uint8_t* chi, double* prim6, hipStream_t s)
{
    if (g.eosg)
        hipLaunchKernelGGL(k_cons_to_prim<true>, dim3(grid_for(g.N, 256)), dim3(256), 0, s, g, W, chi, prim6);
    else
        hipLaunchKernelGGL(k_cons_to_prim<false>, dim3(grid_for(g.N, 256)), dim3(256), 0, s, g, W, chi, prim6);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_chi_from_phi(const Grid G, const double* __restrict__ W,
                                                      uint8_t* __restrict__ chi)
{
    const long long N = G.N;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x)
        chi[c] = W[5 * N + c] < 0.0 ? 1 : 0;
}

hipError_t launch_chi_from_phi(const Grid& g, const double* W, uint8_t* chi, hipStream_t s)
{
    hipLaunchKernelGGL(k_chi_from_phi, dim3(grid_for(g.N, 256)), dim3(256), 0, s, g, W, chi);
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, long long n, int32_t v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, long long n, int32_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// HLLC at independent faces (face frame, SoA [5][n]); TF = float gives the
// flux of the mixed-precision form on the same inputs.
template <typename TF>
__global__ __launch_bounds__(256) void k_hllc_points(long long n, const double* __restrict__ qL,
                                                     const double* __restrict__ qR, double g, double pc,
                                                     double* __restrict__ F)
{
    const TF gpc = TF(g * pc), igm1 = TF(1.0 / (g - 1.0));
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        TF f[5];
        hllc<TF>(TF(qL[i]), TF(qL[n + i]), TF(qL[2 * n + i]), TF(qL[3 * n + i]), TF(qL[4 * n + i]), TF(qR[i]),
                 TF(qR[n + i]), TF(qR[2 * n + i]), TF(qR[3 * n + i]), TF(qR[4 * n + i]), TF(g), TF(pc), gpc,
                 igm1, f);
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v * n + i] = (double)f[v];
    }
}

hipError_t launch_hllc_points(long long n, const double* qL, const double* qR, double gamma, double pc,
                              bool mixed, double* F, hipStream_t s)
{
    if (mixed)
        hipLaunchKernelGGL(k_hllc_points<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, qL, qR, gamma, pc, F);
    else
        hipLaunchKernelGGL(k_hllc_points<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, qL, qR, gamma, pc, F);
    return hipGetLastError();
}

// Independent two-material Riemann problems, in = [6][n], eos = [4][n],
// out = [4][n] (p*, u*, rho*_L, rho*_R); optional candidate guesses.
__global__ __launch_bounds__(64) void k_riemann_points(long long n, const double* __restrict__ in,
                                                       const double* __restrict__ eos,
                                                       const double* __restrict__ guess, double rtol, int maxit,
                                                       double* __restrict__ out, int32_t* __restrict__ iters,
                                                       int32_t* nvac, unsigned long long* nfb)
{
    unsigned long long fb = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double o[4];
        bool used = false;
        const int it = riemann_solve(in[i], in[n + i], in[2 * n + i], eos[i], eos[n + i], in[3 * n + i],
                                     in[4 * n + i], in[5 * n + i], eos[2 * n + i], eos[3 * n + i], rtol, maxit,
                                     guess != nullptr, guess ? guess[i] : 0.0, o, &used);
        if (it == 0) atomicAdd(nvac, 1);
        fb += guess != nullptr && !used && it != 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) out[v * n + i] = o[v];
        if (iters) iters[i] = it;
    }
    for (int o = 32; o > 0; o >>= 1) fb += __shfl_xor(fb, o);
    if (nfb && (threadIdx.x & 63) == 0 && fb) atomicAdd(nfb, fb);
}

hipError_t launch_riemann_points(long long n, const double* in, const double* eos, const double* guess, double rtol,
                                 int maxit, double* out, int32_t* iters, int32_t* nvac, unsigned long long* nfb,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_riemann_points, dim3(grid_for(n, 64)), dim3(64), 0, s, n, in, eos, guess, rtol, maxit, out,
                       iters, nvac, nfb);
    return hipGetLastError();
}

}  // namespace m2c
