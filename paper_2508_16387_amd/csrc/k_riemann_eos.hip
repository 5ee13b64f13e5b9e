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
// permutation: the lanes of a wavefront then share their materials.  The
// keys are laid out by unordered family pair (NASG, Mie-Grueneisen, JWL),
// costliest group first, and a problem whose right side has the lower
// family is solved mirrored.  A set of one family pair (in either order) is
// solved by a kernel compiled for exactly those two families, which carries
// neither the code nor the registers of the others; a set of several family
// pairs takes one launch of the kernel that dispatches on the families at
// run time, so that the groups run side by side (launches per group, one
// after another on the stream, would each wait for the slowest wavefront of
// the one before).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "m2c.h"
#include "m2c_eos.h"
#include "m2c_mlp_eos.h"
#include "m2c_mlp_infer.h"

const m2c::MlpDev* m2c_mlp_dev(const m2c_mlp* m);   // m2c_learned.hip

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

// Family-pair group of every key: 3 min(famL, famR) + max(famL, famR) for
// the keys of the table (a problem whose right family is the lower one is
// solved mirrored), NFP - 1 for the key of indices outside it.
constexpr int NFP = 10;
struct KeyGroups {
    int32_t g[NKEY];
};

// Order of the groups in the permutation: the costliest first (both sides
// Mie-Grueneisen, whose rarefactions walk the isentrope by RK4, then one
// side, then JWL, then NASG), so that a launch over a mixed set starts its
// slowest wavefronts first instead of ending on them.  The groups 3 MG +
// NASG, 3 JWL + NASG and 3 JWL + MG stay empty.
constexpr int kGroupOrder[NFP] = {3 * M2C_EOS_MG + M2C_EOS_MG,    3 * M2C_EOS_NASG + M2C_EOS_MG,
                                  3 * M2C_EOS_MG + M2C_EOS_JWL,   3 * M2C_EOS_JWL + M2C_EOS_JWL,
                                  3 * M2C_EOS_NASG + M2C_EOS_JWL, 3 * M2C_EOS_NASG + M2C_EOS_NASG,
                                  3 * M2C_EOS_MG + M2C_EOS_NASG,  3 * M2C_EOS_JWL + M2C_EOS_NASG,
                                  3 * M2C_EOS_JWL + M2C_EOS_MG,   NFP - 1};

// cursor = exclusive prefix sum of counts with the keys taken group by group
// in kGroupOrder, so that each family pair's problems occupy one range of
// slots: range[2 f] .. range[2 f + 1] (one thread; NKEY x NFP steps)
__global__ void k_pair_scan(const int32_t* __restrict__ counts, int32_t* __restrict__ cursor, const KeyGroups kg,
                            int32_t* __restrict__ range)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int32_t acc = 0;
        for (int o = 0; o < NFP; ++o) {
            const int f = kGroupOrder[o];
            range[2 * f] = acc;
            for (int k = 0; k < NKEY; ++k)
                if (kg.g[k] == f) {
                    cursor[k] = acc;
                    acc += counts[k];
                }
            range[2 * f + 1] = acc;
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

// Waves per SIMD the compiler fits a family pair's kernel to: two where
// neither side is Mie-Grueneisen (a few registers spilled at most), one with
// its branch-point walks and for the run-time dispatch (no spills there).
template <int FA, int FB>
constexpr int kWavesPerSimd = (FA >= 0 && FB >= 0 && FA != M2C_EOS_MG && FB != M2C_EOS_MG) ? 2 : 1;

// Slots range[0] .. range[1] of the permutation perm (whole set without
// them: thread t solves problem t).  FA <= FB: every problem of the range
// has one material of family FA and one of family FB, in either order,
// inside the table (the grouping guarantees it).  FA = FB = -1: any
// materials, indices checked, families dispatched at run time.  A problem
// whose right side has the lower family is solved mirrored (x -> -x: the
// sides swap and the velocities change sign), which leaves p* and negates
// u*, so a problem and its image take the same arithmetic.
template <int FA, int FB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd<FA, FB>))) void k_riemann_eos(
    long long n, const double* __restrict__ in, const int32_t* __restrict__ mat, const EosTable tab, double rtol,
    int maxit, double hmax, double* __restrict__ out, int32_t* __restrict__ iters, int32_t* __restrict__ nbad,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ range)
{
    static_assert(FA <= FB, "family pair in canonical order");
    const long long lo = range ? (long long)range[0] : 0, hi = range ? (long long)range[1] : n;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = lo + (long long)blockIdx.x * blockDim.x + threadIdx.x; t < hi; t += stride) {
        const long long i = perm ? (long long)perm[t] : t;
        double q[6], res[4];
        for (int k = 0; k < 6; ++k) q[k] = in[k * n + i];
        const int ml = mat[i], mr = mat[n + i];
        int its;
        const bool valid = FA >= 0 || (ml >= 0 && ml < tab.n && mr >= 0 && mr < tab.n);
        if (valid) {
            const bool flip = FA >= 0 ? (FA != FB && tab.m[ml].fam != FA) : tab.m[ml].fam > tab.m[mr].fam;
            const double qm[6] = {flip ? q[3] : q[0], flip ? -q[4] : q[1], flip ? q[5] : q[2],
                                  flip ? q[0] : q[3], flip ? -q[1] : q[4], flip ? q[2] : q[5]};
            its = solve_pair<fam_set(FA), fam_set(FB)>(tab.m[flip ? mr : ml], tab.m[flip ? ml : mr], qm, rtol, maxit,
                                                       hmax, res);
            if (flip) {
                const double r = res[2];
                res[1] = -res[1];
                res[2] = res[3];
                res[3] = r;
            }
        } else {
            its = 0;
            for (int k = 0; k < 4; ++k) res[k] = __builtin_nan("");
        }
        if (its == 0) atomicAdd(nbad, 1);
        for (int k = 0; k < 4; ++k) out[k * n + i] = res[k];
        if (iters) iters[i] = its;
    }
}

// The same with the learned start (the grouping as for k_riemann_eos).  The
// network is evaluated on the matrix cores by whole wavefronts, so the
// range is walked in wavefronts; a wavefront evaluates it only for its
// 16-lane groups that hold a problem away from equilibrium whose families
// take it (learned_pair).  nfb counts the problems that started from the
// acoustic guess.
template <int FA, int FB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd<FA, FB>))) void k_riemann_eos_learned(
    long long n, const double* __restrict__ in, const int32_t* __restrict__ mat, const EosTable tab, double rtol,
    int maxit, double hmax, double* __restrict__ out, int32_t* __restrict__ iters, int32_t* __restrict__ nbad,
    unsigned long long* __restrict__ nfb, const int32_t* __restrict__ perm, const int32_t* __restrict__ range,
    const MlpDev net)
{
    static_assert(FA <= FB, "family pair in canonical order");
    const long long lo = range ? (long long)range[0] : 0, hi = range ? (long long)range[1] : n;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    unsigned long long fb = 0;
    for (long long t0 = lo + (long long)blockIdx.x * blockDim.x + (threadIdx.x & ~63); t0 < hi; t0 += stride) {
        const long long t = t0 + lane;
        const bool live = t < hi;
        long long i = 0;
        int ml = 0, mr = 0;
        bool flip = false, ok = false;
        Pair P;
        if (live) {
            i = perm ? (long long)perm[t] : t;
            ml = mat[i];
            mr = mat[n + i];
            const bool valid = FA >= 0 || (ml >= 0 && ml < tab.n && mr >= 0 && mr < tab.n);
            if (valid) {
                double q[6];
                for (int k = 0; k < 6; ++k) q[k] = in[k * n + i];
                flip = FA >= 0 ? (FA != FB && tab.m[ml].fam != FA) : tab.m[ml].fam > tab.m[mr].fam;
                const double qm[6] = {flip ? q[3] : q[0], flip ? -q[4] : q[1], flip ? q[5] : q[2],
                                      flip ? q[0] : q[3], flip ? -q[1] : q[4], flip ? q[2] : q[5]};
                ok = pair_init<fam_set(FA), fam_set(FB)>(tab.m[flip ? mr : ml], tab.m[flip ? ml : mr], qm, P);
            }
        }
        float x[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        double plo = 0.0, Pn = 1.0;
        bool skip = !ok || eos_near_equilibrium(P);
        if (!skip) {
            const int fa = tab.m[flip ? mr : ml].fam, fb = tab.m[flip ? ml : mr].fam;
            skip = !learned_pair(fa, fb) || !eos_features(P, fa, fb, x, plo, Pn);
        }
        const double g = guess64_mem(net, x, plo, Pn, skip);              // whole wavefront
        if (!live) continue;
        double res[4] = {__builtin_nan(""), __builtin_nan(""), __builtin_nan(""), __builtin_nan("")};
        int its = 0;
        bool used = false;
        if (ok)
            its = pair_solve<fam_set(FA), fam_set(FB)>(tab.m[flip ? mr : ml], tab.m[flip ? ml : mr], P, rtol, maxit,
                                                       hmax, g, res, &used);
        if (flip) {
            const double r = res[2];
            res[1] = -res[1];
            res[2] = res[3];
            res[3] = r;
        }
        fb += its != 0 && !used;
        if (its == 0) atomicAdd(nbad, 1);
        for (int k = 0; k < 4; ++k) out[k * n + i] = res[k];
        if (iters) iters[i] = its;
    }
    for (int o = 32; o > 0; o >>= 1) fb += __shfl_xor(fb, o);
    if (lane == 0 && fb) atomicAdd(nfb, fb);
}

// Features X [8][n] and targets t [n] (pstar given) of the learned start,
// in the orientation the solver takes (lower family on the left); zeros and
// NaN targets for an inadmissible problem or an index outside the table.
__global__ __launch_bounds__(256) void k_eos_features(long long n, const double* __restrict__ in,
                                                      const int32_t* __restrict__ mat, const EosTable tab,
                                                      const double* __restrict__ pstar, float* __restrict__ X,
                                                      float* __restrict__ tg)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float x[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        double plo = 0.0, Pn = 1.0;
        bool ok = false;
        const int ml = mat[i], mr = mat[n + i];
        if (ml >= 0 && ml < tab.n && mr >= 0 && mr < tab.n) {
            double q[6];
            for (int k = 0; k < 6; ++k) q[k] = in[k * n + i];
            const bool flip = tab.m[ml].fam > tab.m[mr].fam;
            const double qm[6] = {flip ? q[3] : q[0], flip ? -q[4] : q[1], flip ? q[5] : q[2],
                                  flip ? q[0] : q[3], flip ? -q[1] : q[4], flip ? q[2] : q[5]};
            Pair P;
            const EosK& a = tab.m[flip ? mr : ml];
            const EosK& b = tab.m[flip ? ml : mr];
            ok = pair_init(a, b, qm, P) && eos_features(P, a.fam, b.fam, x, plo, Pn);
        }
        for (int k = 0; k < 8; ++k) X[k * n + i] = ok ? x[k] : 0.f;
        if (tg) {
            const double ps = pstar ? pstar[i] : __builtin_nan("");
            tg[i] = ok && ps > plo ? (float)log((ps - plo) / Pn) : __builtin_nanf("");
        }
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

struct SolveArgs {
    long long n;
    const double* in;
    const int32_t* mat;
    EosTable tab;
    double rtol;
    int maxit;
    double hmax;
    double* out;
    int32_t* iters;
    int32_t* nbad;
    const int32_t* perm;
    const MlpDev* net;                 // learned start (nullable)
    unsigned long long* nfb;           // acoustic starts (with net)
};

// (the learned kernel only for a family pair that takes the learned start,
// or for the run-time dispatch)
// Returns whether the learned kernel was launched.
template <int FA, int FB>
bool launch_solve(const SolveArgs& a, unsigned grid, const int32_t* range, hipStream_t s)
{
    if constexpr (FA < 0 || learned_pair(FA, FB)) {
        if (a.net) {
            hipLaunchKernelGGL((k_riemann_eos_learned<FA, FB>), dim3(grid), dim3(256), 0, s, a.n, a.in, a.mat, a.tab,
                               a.rtol, a.maxit, a.hmax, a.out, a.iters, a.nbad, a.nfb, a.perm, range, *a.net);
            return true;
        }
    }
    hipLaunchKernelGGL((k_riemann_eos<FA, FB>), dim3(grid), dim3(256), 0, s, a.n, a.in, a.mat, a.tab, a.rtol,
                       a.maxit, a.hmax, a.out, a.iters, a.nbad, a.perm, range);
    return false;
}

using SolveLaunch = bool (*)(const SolveArgs&, unsigned, const int32_t*, hipStream_t);
// by family-pair group 3 FA + FB, FA <= FB (families M2C_EOS_NASG, _MG, _JWL
// = 0, 1, 2; the other groups stay empty)
constexpr SolveLaunch kSolvePair[9] = {launch_solve<0, 0>, launch_solve<0, 1>, launch_solve<0, 2>,
                                       nullptr,            launch_solve<1, 1>, launch_solve<1, 2>,
                                       nullptr,            nullptr,            launch_solve<2, 2>};
static_assert(M2C_EOS_NASG == 0 && M2C_EOS_MG == 1 && M2C_EOS_JWL == 2, "family-pair table order");

}  // namespace
}  // namespace m2c

using namespace m2c;

namespace {

int solve_eos(const MlpDev* net, int64_t n, const double* in, const int32_t* mat, int32_t nmat, const m2c_eos* eos,
              double rtol, int32_t maxit, double ds, double* out, int32_t* iters, int64_t* n_fallback,
              void* hip_stream)
{
    if (n < 0 || (n > 0 && (!in || !mat || !out))) return M2C_ERR_ARG;
    if (!(rtol > 0.0) || maxit < 1) return M2C_ERR_ARG;
    if (ds == 0.0) ds = 0.01;
    if (!(ds >= 1e-3 && ds <= 0.5)) return M2C_ERR_ARG;
    EosTable tab;
    if (!prepare(nmat, eos, tab)) return M2C_ERR_ARG;
    if (n == 0) return M2C_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    // grouped by material pair, and within that by family pair (32-bit slots)
    const bool group = n < (1LL << 31);
    // workspace (int32): failure count, key counts, key cursors, family-pair
    // ranges, acoustic-start count (64-bit), permutation
    const long long words = 1 + 2 * NKEY + 2 * NFP + 3 + (group ? n : 0);
    int32_t* dbad = nullptr;
    if (hipMalloc((void**)&dbad, words * sizeof(int32_t)) != hipSuccess) return M2C_ERR_NOMEM;
    int32_t* counts = dbad + 1;
    int32_t* cursor = counts + NKEY;
    int32_t* range = cursor + NKEY;
    unsigned long long* nfb = (unsigned long long*)(range + 2 * NFP + 1);   // 8-byte aligned
    int32_t* perm = group ? range + 2 * NFP + 3 : nullptr;
    int32_t hb = 0;
    int rc = M2C_OK;
    unsigned long long hfb = 0;
    bool learned = false;              // a learned kernel counted the acoustic starts
    const SolveArgs sa{(long long)n, in, mat, tab, rtol, (int)maxit, ds, out, iters, dbad, perm, net, nfb};
    if (hipMemsetAsync(dbad, 0, (1 + NKEY) * sizeof(int32_t), s) != hipSuccess ||
        hipMemsetAsync(nfb, 0, sizeof(unsigned long long), s) != hipSuccess)
        rc = M2C_ERR_DEVICE;
    if (rc == M2C_OK && group) {
        KeyGroups kg;
        for (int k = 0; k < NKEY; ++k) {
            kg.g[k] = NFP - 1;
            if (k >= nmat * nmat) continue;
            const int fl = tab.m[k / (int)nmat].fam, fr = tab.m[k % (int)nmat].fam;
            kg.g[k] = fl < fr ? 3 * fl + fr : 3 * fr + fl;
        }
        const unsigned nb = (unsigned)((n + 255) / 256);
        int32_t hr[2 * NFP] = {};
        hipLaunchKernelGGL(k_pair_count, dim3(nb), dim3(256), 0, s, (long long)n, mat, (int)nmat, counts);
        hipLaunchKernelGGL(k_pair_scan, dim3(1), dim3(64), 0, s, counts, cursor, kg, range);
        hipLaunchKernelGGL(k_pair_place, dim3(nb), dim3(256), 0, s, (long long)n, mat, (int)nmat, cursor, perm);
        // the group sizes decide the launch (one read-back; the call
        // synchronises at its end anyway)
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(hr, range, sizeof(hr), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = M2C_ERR_DEVICE;
        int only = -1, nonempty = 0;
        for (int f = 0; f < NFP; ++f)
            if (hr[2 * f + 1] > hr[2 * f]) {
                only = f;
                ++nonempty;
            }
        if (rc == M2C_OK && nonempty == 1 && only < NFP - 1 && kSolvePair[only]) {
            learned = kSolvePair[only](sa, grid_for(hr[2 * only + 1] - hr[2 * only]), range + 2 * only, s);
        } else if (rc == M2C_OK) {
            // several family pairs in one launch: the learned start only
            // where it pays for the whole launch, i.e. no Mie-Grueneisen
            // group (its walks set the time of a mixed launch) and some
            // group that takes it
            bool mg = false, takes = false;
            for (int f = 0; f < NFP - 1; ++f)
                if (hr[2 * f + 1] > hr[2 * f]) {
                    mg = mg || f / 3 == M2C_EOS_MG || f % 3 == M2C_EOS_MG;
                    takes = takes || learned_pair(f / 3, f % 3);
                }
            SolveArgs sm = sa;
            if (mg || !takes) sm.net = nullptr;
            learned = launch_solve<-1, -1>(sm, grid_for(n), nullptr, s);
        }
        if (rc == M2C_OK && hipGetLastError() != hipSuccess) rc = M2C_ERR_DEVICE;
    } else if (rc == M2C_OK) {
        learned = launch_solve<-1, -1>(sa, grid_for(n), nullptr, s);
        if (hipGetLastError() != hipSuccess) rc = M2C_ERR_DEVICE;
    }
    if (rc == M2C_OK &&
        (hipMemcpyAsync(&hb, dbad, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipMemcpyAsync(&hfb, nfb, sizeof(hfb), hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
        rc = M2C_ERR_DEVICE;
    (void)hipFree(dbad);
    // without a learned launch every solved problem started from the
    // acoustic guess
    if (n_fallback) *n_fallback = learned ? (int64_t)hfb : (int64_t)n - hb;
    if (rc == M2C_OK && hb > 0) rc = M2C_ERR_RIEMANN;
    return rc;
}

}  // namespace

extern "C" int m2c_riemann_solve_eos(int64_t n, const double* in, const int32_t* mat, int32_t nmat,
                                     const m2c_eos* eos, double rtol, int32_t maxit, double ds, double* out,
                                     int32_t* iters, void* hip_stream)
{
    return solve_eos(nullptr, n, in, mat, nmat, eos, rtol, maxit, ds, out, iters, nullptr, hip_stream);
}

extern "C" int m2c_riemann_solve_eos_learned(const m2c_mlp* m, int64_t n, const double* in, const int32_t* mat,
                                             int32_t nmat, const m2c_eos* eos, double rtol, int32_t maxit,
                                             double ds, double* out, int32_t* iters, int64_t* n_fallback,
                                             void* hip_stream)
{
    if (n_fallback) *n_fallback = 0;
    return solve_eos(m2c_mlp_dev(m), n, in, mat, nmat, eos, rtol, maxit, ds, out, iters, n_fallback, hip_stream);
}

extern "C" int m2c_mlp_features_eos(int64_t n, const double* in, const int32_t* mat, int32_t nmat,
                                    const m2c_eos* eos, const double* pstar, float* X8, float* target,
                                    void* hip_stream)
{
    if (n < 0 || (n > 0 && (!in || !mat || !X8))) return M2C_ERR_ARG;
    EosTable tab;
    if (!prepare(nmat, eos, tab)) return M2C_ERR_ARG;
    if (n == 0) return M2C_OK;
    hipLaunchKernelGGL(k_eos_features, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream, (long long)n, in,
                       mat, tab, pstar, X8, target);
    return hipGetLastError() == hipSuccess ? M2C_OK : M2C_ERR_DEVICE;
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
