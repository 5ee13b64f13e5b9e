// k_interface.hip -- interface-face work queue, FIVER fluxes and the phase
// update.
//
// FIVER (section "Spatial discretization of governing equations", eq.
// 1DRiemannProblem): at a face whose two cells hold different materials the
// flux is not one HLLC flux but two one-sided fluxes built on the exact
// solution of the two-material Riemann problem along the face normal.  Those
// faces are a thin sheet (well under 1% of all faces), so they are gathered
// into a dense queue once per step (material ids are frozen during a step)
// and solved by one thread each, away from the bulk stage kernel whose
// wavefronts would otherwise diverge on the Newton iteration.
//
// Queue order is ascending face id f = 3c + d (face between cell c and its
// +d neighbour); the compaction is a deterministic three-pass scan
// (per-block count, one-block exclusive scan, scatter with wavefront prefix
// sums), so the queue is bit-identical from run to run.  The face -> slot
// map is written only at the faces of the new queue and read only at faces
// whose cells differ in material under the same frozen ids, so entries left
// from earlier queues are never read and need no clearing.
#include "m2c_device.h"
#include "m2c_internal.h"
#include "m2c_kernels.h"
#include "m2c_mlp_eos.h"
#include "m2c_mlp_infer.h"

namespace m2c {

// Interface-face bits of cell c: bit d set when the face towards the +d
// neighbour separates two materials.  A face on a non-periodic domain
// boundary is never an interface (the boundary image carries the boundary
// cell's material); a periodic axis wraps.  Cell indices fit in 32 bits
// (grids are limited to 2^29 cells).
// A lane walks its cells c, c + 64, c + 128, ... with their coordinates
// (i, j, k) advanced incrementally (no division per cell).
struct CellWalk {
    uint32_t c, i, j, k;
};

__device__ __forceinline__ void walk_start(const Grid& G, uint32_t c, CellWalk& w)
{
    const uint32_t nx = G.nx, sxy = nx * (uint32_t)G.ny;
    w.c = c;
    w.k = c / sxy;
    const uint32_t r = c - w.k * sxy;
    w.j = r / nx;
    w.i = r - w.j * nx;
}

__device__ __forceinline__ void walk_advance(const Grid& G, CellWalk& w, uint32_t step = 64u)
{
    const uint32_t nx = G.nx, ny = G.ny;
    w.c += step;
    w.i += step;
    while (w.i >= nx) {
        w.i -= nx;
        if (++w.j == ny) {
            w.j = 0;
            ++w.k;
        }
    }
}

__device__ __forceinline__ unsigned cell_face_bits(const Grid& G, const uint8_t* __restrict__ chi, const CellWalk& w)
{
    const uint32_t nx = G.nx, ny = G.ny, nz = G.nz, sxy = nx * ny;
    const uint32_t c = w.c, i = w.i, j = w.j, k = w.k;
    const uint8_t x = chi[c];
    unsigned bits = 0;
    if (G.act[0] && (i + 1 < nx || G.bc[1] == BC_PERIODIC)) {
        const uint32_t n = i + 1 < nx ? c + 1 : c - (nx - 1);
        if (chi[n] != x) bits |= 1u;
    }
    if (G.act[1] && (j + 1 < ny || G.bc[3] == BC_PERIODIC)) {
        const uint32_t n = j + 1 < ny ? c + nx : c - (ny - 1) * nx;
        if (chi[n] != x) bits |= 2u;
    }
    if (G.act[2] && (k + 1 < nz || G.bc[5] == BC_PERIODIC)) {
        const uint32_t n = k + 1 < nz ? c + sxy : c - (nz - 1) * sxy;
        if (chi[n] != x) bits |= 4u;
    }
    return bits;
}

// Cells of a compaction block: wave w owns the 64 * COMPACT_CELLS_PER_THREAD
// consecutive cells from blk * COMPACT_CELLS_PER_BLOCK + w * 64 *
// COMPACT_CELLS_PER_THREAD (how its lanes share them: lane_bits_* below), so
// the queue order over waves and blocks is ascending cell order.
__device__ __forceinline__ uint32_t compact_wave_base(int blk)
{
    return (uint32_t)blk * COMPACT_CELLS_PER_BLOCK + (threadIdx.x >> 6) * (64 * COMPACT_CELLS_PER_THREAD);
}

__device__ __forceinline__ int block_sum(int v, int* sRed)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sRed[w] = v;
    __syncthreads();
    int t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sRed[k];
    return t;
}

// Face bits of the lane's cells.  Byte path (any grid): in round e the lane
// takes cell wbase + 64 e + l, packed at bits 3e..3e+2.  Word path (nx a
// multiple of 4, ids 4-byte aligned): in round e the lane takes the four
// cells wbase + 256 e + 4 l + b (b = 0..3) with one aligned 32-bit load of
// their ids and one per neighbouring row, plane and (for b = 3) the next
// word, packed at bits 3(4e + b)...; a quarter of the memory instructions.
__device__ __forceinline__ bool compact_words(const Grid& G, const uint8_t* chi)
{
    return G.nx % 4 == 0 && ((uintptr_t)chi & 3u) == 0;
}

__device__ __forceinline__ uint64_t lane_bits_bytes(const Grid& G, const uint8_t* __restrict__ chi, uint32_t wbase,
                                                    int& cnt)
{
    const uint32_t N = (uint32_t)G.N;
    uint64_t packed = 0;
    cnt = 0;
    CellWalk cw;
    walk_start(G, wbase + (threadIdx.x & 63), cw);
#pragma unroll
    for (int e = 0; e < COMPACT_CELLS_PER_THREAD; ++e) {
        const unsigned bits = cw.c < N ? cell_face_bits(G, chi, cw) : 0u;
        walk_advance(G, cw);
        packed |= (uint64_t)bits << (3 * e);
        cnt += __popc(bits);
    }
    return packed;
}

__device__ __forceinline__ uint32_t ld_word(const uint8_t* __restrict__ chi, uint32_t c)
{
    return *reinterpret_cast<const uint32_t*>(chi + c);
}

__device__ __forceinline__ uint64_t lane_bits_words(const Grid& G, const uint8_t* __restrict__ chi, uint32_t wbase,
                                                    int& cnt)
{
    const uint32_t N = (uint32_t)G.N, nx = G.nx, ny = G.ny, nz = G.nz, sxy = nx * ny;
    const bool py = G.bc[3] == BC_PERIODIC, pz = G.bc[5] == BC_PERIODIC, px = G.bc[1] == BC_PERIODIC;
    uint64_t packed = 0;
    cnt = 0;
    CellWalk cw;
    walk_start(G, wbase + 4u * (threadIdx.x & 63), cw);
#pragma unroll
    for (int e = 0; e < COMPACT_CELLS_PER_THREAD / 4; ++e) {
        if (cw.c < N) {
            const uint32_t c = cw.c;
            const uint32_t d0 = ld_word(chi, c);
            // neighbour words (all 4-byte aligned since nx % 4 == 0)
            const bool hx = cw.i + 4 < nx || px;
            const bool hy = G.act[1] && (cw.j + 1 < ny || py);
            const bool hz = G.act[2] && (cw.k + 1 < nz || pz);
            const uint32_t dx = hx ? ld_word(chi, cw.i + 4 < nx ? c + 4 : c + 4 - nx) : 0u;
            const uint32_t dy = hy ? ld_word(chi, cw.j + 1 < ny ? c + nx : c - (ny - 1) * nx) : 0u;
            const uint32_t dz = hz ? ld_word(chi, cw.k + 1 < nz ? c + sxy : c - (nz - 1) * sxy) : 0u;
            const uint32_t nxw = (d0 >> 8) | (dx << 24);     // +x neighbour of each byte
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t x = (d0 >> (8 * b)) & 0xffu;
                unsigned bits = 0;
                if ((b < 3 || hx) && ((nxw >> (8 * b)) & 0xffu) != x) bits |= 1u;
                if (hy && ((dy >> (8 * b)) & 0xffu) != x) bits |= 2u;
                if (hz && ((dz >> (8 * b)) & 0xffu) != x) bits |= 4u;
                packed |= (uint64_t)bits << (3 * (4 * e + b));
                cnt += __popc(bits);
            }
        }
        walk_advance(G, cw, 256u);
    }
    return packed;
}

__device__ __forceinline__ void count_body(const IfaceArgs& a, int blk)
{
    __shared__ int sRed[COMPACT_THREADS / 64];
    const uint32_t wbase = compact_wave_base(blk);
    int cnt = 0;
    if (compact_words(a.g, a.chi)) (void)lane_bits_words(a.g, a.chi, wbase, cnt);
    else (void)lane_bits_bytes(a.g, a.chi, wbase, cnt);
    const int t = block_sum(cnt, sRed);
    if (threadIdx.x == 0) a.blockcnt[blk] = t;
}

// A step whose predecessor flipped no cell has the material ids the queue
// was built from (the last stage writes every id, and a flip is exactly a
// changed id), so the single-grid compaction keeps the queue and the face
// slots.  The decision is read here before the scan kernel clears the flip
// count, and the scan records it for the scatter.
__device__ __forceinline__ bool queue_kept(const DevScalars* sc) { return sc->qvalid && sc->nflip == 0; }

__global__ __launch_bounds__(COMPACT_THREADS) void k_count(const IfaceArgs a)
{
    if (queue_kept(a.sc)) return;
    count_body(a, blockIdx.x);
}

// One block: exclusive scan of the block counts (in place), total -> qlen.
// Each thread sums a contiguous segment of the counts, the block scans the
// segment sums, and each thread rewrites its segment from its offset.
__device__ __forceinline__ void scan_body(const IfaceArgs& a)
{
    __shared__ long long sW[16];
    const int nb = a.nblk;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int per = (nb + (int)blockDim.x - 1) / (int)blockDim.x;
    const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
    long long sum = 0;
    for (int b = b0; b < b1; ++b) sum += a.blockcnt[b];
    long long incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) sW[w] = incl;
    __syncthreads();
    long long run = incl - sum, total = 0;
    for (int k = 0; k < nw; ++k) {
        if (k < w) run += sW[k];
        total += sW[k];
    }
    for (int b = b0; b < b1; ++b) {
        const int v = a.blockcnt[b];
        a.blockcnt[b] = (int)run;
        run += v;
    }
    if (threadIdx.x == 0) {
        if (total > a.qcap) {
            atomicCAS(&a.sc->err, 0, ST_OVERFLOW);
            a.sc->qlen = 0;
        } else {
            a.sc->qlen = (int)total;
        }
    }
}

// End of a step (single grid): counters and simulated time, only when no
// kernel of the step reported an error.
__device__ __forceinline__ void end_step_body(DevScalars* sc, int stages)
{
    if (sc->err != 0) return;
    sc->steps_done += 1;
    sc->t += sc->dt;
    sc->dt_last = sc->dt;
    sc->solves += (long long)sc->qlen * stages;
    sc->flips += sc->nflip;
}

// Start of a step (single grid): dt from the CFL rule (section "Time
// integration"; the rule itself is not printed, the reading is dt = CFL /
// max_i sum over the axes with more than one cell of (|V_d| + c)/h_d) or
// imposed; clear the accumulators that the step fills for the next step.
__device__ __forceinline__ void begin_step_body(DevScalars* sc, double cfl, double dt_fixed, double dt_imposed)
{
    if (sc->err != 0) return;
    double dt;
    if (dt_imposed > 0.0) dt = dt_imposed;
    else if (dt_fixed > 0.0) dt = dt_fixed;
    else dt = cfl / __longlong_as_double((long long)sc->lam_bits);
    sc->dt = dt;
    sc->lam_bits = 0ull;
    sc->nflip = 0;
}

// The scan kernel of a step also closes the previous step of the same
// m2c_step call (end_prev) and opens this one (begin): both must precede
// every kernel that reads dt, and follow the phase update of the previous
// step, which is where the single-block scan sits in the stream.
__global__ __launch_bounds__(1024) void k_scan(const IfaceArgs a, int end_prev, int begin, double cfl,
                                               double dt_fixed, double dt_imposed)
{
    __shared__ int sKeep;
    if (threadIdx.x == 0) {
        const int keep = queue_kept(a.sc) ? 1 : 0;
        sKeep = keep;
        a.sc->qreuse = keep;
        if (end_prev) end_step_body(a.sc, a.g.rk_stages);
        if (begin) begin_step_body(a.sc, cfl, dt_fixed, dt_imposed);
    }
    __syncthreads();
    if (sKeep) return;
    scan_body(a);
    // the scatter that follows completes the queue unless a kernel failed
    if (threadIdx.x == 0) a.sc->qvalid = a.sc->err == 0 ? 1 : 0;
}

__global__ void k_end_step(DevScalars* sc, int stages) { end_step_body(sc, stages); }

hipError_t launch_end_step(DevScalars* sc, int stages, hipStream_t s)
{
    hipLaunchKernelGGL(k_end_step, dim3(1), dim3(1), 0, s, sc, stages);
    return hipGetLastError();
}

__device__ __forceinline__ void scatter_body(const IfaceArgs& a, int blk)
{
    __shared__ int sW[COMPACT_THREADS / 64];
    if (a.sc->err != 0) return;
    const uint32_t wbase = compact_wave_base(blk);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool words = compact_words(a.g, a.chi);
    int cnt = 0;
    const uint64_t packed = words ? lane_bits_words(a.g, a.chi, wbase, cnt) : lane_bits_bytes(a.g, a.chi, wbase, cnt);
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane == 0) sW[w] = cnt;
    __syncthreads();
    if (cnt == 0) return;                     // wave-uniform
    int off = a.blockcnt[blk];
    for (int k = 0; k < w; ++k) off += sW[k];
    if (words) {
        // the lane's 16 cells are 4 runs of 4 consecutive cells; faces in
        // ascending id order within a round: by lane, cell, axis
        for (int e = 0; e < COMPACT_CELLS_PER_THREAD / 4; ++e) {
            const unsigned bits12 = (unsigned)(packed >> (12 * e)) & 0xfffu;
            const int n = __popc(bits12);
            int incl = n;
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            const int tot = __shfl(incl, 63);
            if (tot == 0) continue;                               // wave-uniform
            int o = off + incl - n;
            const int f0 = (int)(3u * (wbase + 256u * e + 4u * lane));
            for (int q = 0; q < 12; ++q)
                if (bits12 & (1u << q)) {
                    a.queue[o] = f0 + q;                          // 3 (c0 + b) + d = f0 + 3b + d
                    a.fslot[f0 + q] = o;
                    ++o;
                }
            off += tot;
        }
        return;
    }
    // byte path: faces in ascending id order: by cell, then by axis
    const uint64_t below = (1ull << lane) - 1ull;
    for (int e = 0; e < COMPACT_CELLS_PER_THREAD; ++e) {
        const unsigned bits = (unsigned)(packed >> (3 * e)) & 7u;
        const uint64_t b0 = __ballot(bits & 1u), b1 = __ballot(bits & 2u), b2 = __ballot(bits & 4u);
        if ((b0 | b1 | b2) == 0ull) continue;
        int o = off + __popcll(b0 & below) + __popcll(b1 & below) + __popcll(b2 & below);
        const int f0 = (int)(3u * (wbase + lane + 64u * e));
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (bits & (1u << d)) {
                a.queue[o] = f0 + d;
                a.fslot[f0 + d] = o;
                ++o;
            }
        off += __popcll(b0) + __popcll(b1) + __popcll(b2);
    }
}

__global__ __launch_bounds__(COMPACT_THREADS) void k_scatter(const IfaceArgs a)
{
    if (a.sc->qreuse) return;
    scatter_body(a, blockIdx.x);
}


// ---------------------------------------------------------------------------
// FIVER: one thread per queued face.  The Riemann data are the two cells'
// own (first-order) primitive states in the face frame (rho, u_n, p); the
// star states W*_L = (rho*_L, u*, tangential V_L, p*) and W*_R likewise feed
//   F_lower = HLLC(W_L, W*_L; EOS of the lower cell)
//   F_upper = HLLC(W*_R, W_R; EOS of the upper cell)
// with the arguments ordered along the face normal.
// FS: the set of the materials' families (EG; eos::fam_set)
template <bool EG, int FS = eos::FAM_ALL>
__device__ __forceinline__ void cell_prim(const Grid& G, const eos::EosK* sEos, const double* __restrict__ W,
                                          uint32_t c, int x, double q[5])
{
    const uint32_t N = (uint32_t)G.N;
    double u, v, w;
    if constexpr (EG)
        q[4] = geos_prim<FS>(sEos[x], ldf(W, c), ldf(W + N, c), ldf(W + 2 * N, c), ldf(W + 3 * N, c),
                             ldf(W + 4 * N, c), u, v, w);
    else
        q[4] = eos_prim(ldf(W, c), ldf(W + N, c), ldf(W + 2 * N, c), ldf(W + 3 * N, c), ldf(W + 4 * N, c),
                        pick(G.gamma, x) - 1.0, pick(G.gpc, x), u, v, w);
    q[0] = ldf(W, c);
    q[1] = u;
    q[2] = v;
    q[3] = w;
}

// EG: general EOS per material (the Riemann solve of section "Equations of
// state" with Hugoniot and isentrope wave curves, fluxes with each side's
// EOS).  LG: learned star-pressure guess (stiffened gases): each face first
// takes the near-equilibrium test, and only a wavefront holding a face that
// fails it loads the network and evaluates it (on the matrix cores, 64 faces
// per pass); every other face starts Newton from the acoustic guess at no
// extra cost.  The queue is then walked in whole wavefronts, since the
// network needs every lane of one; its operands are read from memory as
// they are needed, so that the kernel keeps the acoustic kernel's registers.
// F0, F1 (EG): families of materials 0 and 1 fixed at compile time, so that
// a kernel carries the wave curves and EOS forms of those two families only
// (-1: dispatched at run time).
template <bool EG, bool LG = false, int F0 = -1, int F1 = -1>
__device__ __forceinline__ void fiver_body(const IfaceArgs& a, int record, int blk, int nblk,
                                           const MlpDev* m = nullptr)
{
    static_assert(!(EG && LG) || (F0 >= 0 && F1 >= 0), "the general-EOS learned start needs the families");
    __shared__ unsigned long long sCnt[3][4];
    __shared__ int sErr;
    __shared__ eos::EosK sEos[EG ? 2 : 1];
    DevScalars* sc = a.sc;
    // skip when an earlier kernel failed; read once so that the whole block
    // takes the same branch (this kernel's own reports may raise the flag)
    if (threadIdx.x == 0) sErr = sc->err;
    if (EG && threadIdx.x == 0) {
        const double* src = reinterpret_cast<const double*>(a.g.ek);
        double* dst = reinterpret_cast<double*>(sEos);
#pragma unroll
        for (int t = 0; t < (int)(2 * sizeof(eos::EosK) / sizeof(double)); ++t) dst[t] = src[t];
    }
    __syncthreads();
    if (sErr != 0) return;
    const Grid& G = a.g;
    constexpr int FS = eos::fam_set(F0) | eos::fam_set(F1);
    const int n = sc->qlen;
    long long iters = 0, fallbacks = 0, mlp_fb = 0;
    const int stride = nblk * blockDim.x;
    // LG: wave-uniform trip count (q may pass n in the last pass)
    const int qend = LG ? (n + 63) / 64 * 64 : n;
    for (int q = blk * blockDim.x + threadIdx.x; q < qend; q += stride) {
        const bool live = !LG || q < n;
        uint32_t c = 0, cn = 0;
        int d = 0;
        if (live) face_cells(G.nx, G.ny, G.nz, (uint32_t)a.queue[q], c, cn, d);
        const int xa = live ? a.chi[c] : 0, xb = live ? a.chi[cn] : 0;
        double qa[5], qb[5];
        cell_prim<EG, FS>(G, sEos, a.Win, c, xa, qa);
        cell_prim<EG, FS>(G, sEos, a.Win, cn, xb, qb);
        const int t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
        const double ua = qa[1 + d], ub = qb[1 + d];
        const double gA = pick(G.gamma, xa), pcA = pick(G.pc, xa), gB = pick(G.gamma, xb), pcB = pick(G.pc, xb);
        double out[4];
        bool used = false;
        bool hg = false;
        double gs = 0.0;
        if constexpr (LG && !EG) {
            const bool skip = !live || acoustic_suffices(qa[0], ua, qa[4], gA, pcA, qb[0], ub, qb[4], gB, pcB);
            if (__ballot(!skip) != 0ull) {                       // wave-uniform
                float x[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                double plo = 0.0, P = 1.0;
                if (!skip) mlp_features(qa[0], ua, qa[4], gA, pcA, qb[0], ub, qb[4], gB, pcB, x, plo, P);
                gs = guess64_mem(*m, x, plo, P, skip);
                hg = !skip;
            }
            if (!live) continue;
        }
        int it;
        if constexpr (EG) {
            // material 0 always on the left: where the lower cell holds
            // material 1 the mirrored problem is solved (p* unchanged, u*
            // negated, the star densities swapped), so that every lane of a
            // wavefront runs the same families' code on each side
            const bool flip = xa != 0;
            const double in[6] = {flip ? qb[0] : qa[0], flip ? -ub : ua, flip ? qb[4] : qa[4],
                                  flip ? qa[0] : qb[0], flip ? -ua : ub, flip ? qa[4] : qb[4]};
            double o[4];
            constexpr int S0 = eos::fam_set(F0), S1 = eos::fam_set(F1);
            if constexpr (LG) {
                // learned start (the families take it, see learned_pair):
                // the network evaluated by whole wavefronts for the faces
                // away from equilibrium, then the judged outer iteration
                eos::Pair P;
                const bool ok = live && eos::pair_init<S0, S1>(sEos[0], sEos[1], in, P);
                float x[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                double plo = 0.0, Pn = 1.0;
                const bool skip = !ok || eos_near_equilibrium(P) || !eos_features(P, F0, F1, x, plo, Pn);
                double g = __builtin_nan("");
                if (__ballot(!skip) != 0ull) g = guess64_mem(*m, x, plo, Pn, skip);      // wave-uniform
                if (!live) continue;
                it = 0;
                for (int k = 0; k < 4; ++k) o[k] = __builtin_nan("");
                if (ok) it = eos::pair_solve<S0, S1>(sEos[0], sEos[1], P, G.rtol, G.maxit, G.rds, g, o, &used);
            } else {
                it = eos::solve_pair<S0, S1>(sEos[0], sEos[1], in, G.rtol, G.maxit, G.rds, o);
            }
            out[0] = o[0];
            out[1] = flip ? -o[1] : o[1];
            out[2] = flip ? o[3] : o[2];
            out[3] = flip ? o[2] : o[3];
        } else {
            it = riemann_solve(qa[0], ua, qa[4], gA, pcA, qb[0], ub, qb[4], gB, pcB, G.rtol, G.maxit, hg, gs, out,
                               &used);
        }
        // faces that started from the acoustic guess (near equilibrium, or
        // the judge preferred it)
        mlp_fb += LG && !used && it != 0;
        if (it == 0) {
            report_error(&sc->err, &sc->err_cell, ST_RIEMANN, c);
            continue;
        }
        iters += it < 0 ? -it : it;
        fallbacks += it < 0;
        const double ps = out[0], us = out[1];
        double Fl[5], Fu[5];
        if constexpr (EG) {
            geos_flux<FS>(sEos[xa], G.flux, qa[0], ua, qa[t1], qa[t2], qa[4], out[2], us, qa[t1], qa[t2], ps, Fl);
            geos_flux<FS>(sEos[xb], G.flux, out[3], us, qb[t1], qb[t2], ps, qb[0], ub, qb[t1], qb[t2], qb[4], Fu);
        } else {
            num_flux<double>(G.flux, qa[0], ua, qa[t1], qa[t2], qa[4], out[2], us, qa[t1], qa[t2], ps, gA, pcA,
                             pick(G.gpc, xa), pick(G.inv_gm1, xa), Fl);
            num_flux<double>(G.flux, out[3], us, qb[t1], qb[t2], ps, qb[0], ub, qb[t1], qb[t2], qb[4], gB, pcB,
                             pick(G.gpc, xb), pick(G.inv_gm1, xb), Fu);
        }
        // face frame (mass, normal, t1, t2, energy) -> global components;
        // the ten fluxes of a face are contiguous (one address per face for
        // the stage kernel that reads them)
        double* const fq = a.fluxF + 10 * (long long)q;
        double fo[10];
        fo[0] = Fl[0];
        fo[1 + d] = Fl[1];
        fo[t1] = Fl[2];
        fo[t2] = Fl[3];
        fo[4] = Fl[4];
        fo[5] = Fu[0];
        fo[6 + d] = Fu[1];
        fo[5 + t1] = Fu[2];
        fo[5 + t2] = Fu[3];
        fo[9] = Fu[4];
#pragma unroll
        for (int v = 0; v < 10; ++v) fq[v] = fo[v];
        if (record) {
            const long long Q = a.qcap;
            a.star[0 * Q + q] = ps;
            a.star[1 * Q + q] = us;
            a.star[2 * Q + q] = out[2];
            a.star[3 * Q + q] = out[3];
            a.star[4 * Q + q] = qa[t1];
            a.star[5 * Q + q] = qa[t2];
            a.star[6 * Q + q] = qb[t1];
            a.star[7 * Q + q] = qb[t2];
        }
    }
    // counters: one atomic per block and counter (same-address atomics from
    // every wavefront serialise into a measurable tail)
    for (int o = 32; o > 0; o >>= 1) {
        iters += __shfl_xor(iters, o);
        fallbacks += __shfl_xor(fallbacks, o);
        mlp_fb += __shfl_xor(mlp_fb, o);
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sCnt[0][w] = iters;
        sCnt[1][w] = fallbacks;
        sCnt[2][w] = mlp_fb;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long t = 0;
        for (int k = 0; k < nw; ++k) t += sCnt[threadIdx.x][k];
        unsigned long long* dst = threadIdx.x == 0 ? (unsigned long long*)&sc->newton_iters
                                 : (threadIdx.x == 1 ? (unsigned long long*)&sc->fallbacks
                                                     : (unsigned long long*)&sc->mlp_fallbacks);
        if (t) atomicAdd(dst, t);
    }
}

__global__ __launch_bounds__(256) void k_fiver(const IfaceArgs a, int record)
{
    fiver_body<false>(a, record, blockIdx.x, gridDim.x);
}

template <int F0, int F1>
__global__ __launch_bounds__(256) void k_fiver_eos(const IfaceArgs a, int record)
{
    fiver_body<true, false, F0, F1>(a, record, blockIdx.x, gridDim.x);
}

// with the learned start, for the family pairs that take it (learned_pair)
template <int F0, int F1>
__global__ __launch_bounds__(256) void k_fiver_eos_learned(const IfaceArgs a, int record, const MlpDev m)
{
    fiver_body<true, true, F0, F1>(a, record, blockIdx.x, gridDim.x, &m);
}

template <int F0, int F1>
void launch_fiver_eos(const IfaceArgs& a, unsigned nb, int record, const MlpDev* mlp, hipStream_t s)
{
    if constexpr (learned_pair(F0, F1)) {
        if (mlp) {
            hipLaunchKernelGGL((k_fiver_eos_learned<F0, F1>), dim3(nb), dim3(256), 0, s, a, record, *mlp);
            return;
        }
    }
    hipLaunchKernelGGL((k_fiver_eos<F0, F1>), dim3(nb), dim3(256), 0, s, a, record);
}
using FiverEosLaunch = void (*)(const IfaceArgs&, unsigned, int, const MlpDev*, hipStream_t);
// by 3 family(material 0) + family(material 1), families NASG, MG, JWL = 0, 1, 2
constexpr FiverEosLaunch kFiverEos[9] = {launch_fiver_eos<0, 0>, launch_fiver_eos<0, 1>, launch_fiver_eos<0, 2>,
                                         launch_fiver_eos<1, 0>, launch_fiver_eos<1, 1>, launch_fiver_eos<1, 2>,
                                         launch_fiver_eos<2, 0>, launch_fiver_eos<2, 1>, launch_fiver_eos<2, 2>};
static_assert(M2C_EOS_NASG == 0 && M2C_EOS_MG == 1 && M2C_EOS_JWL == 2, "family-pair table order");

__global__ __launch_bounds__(256) void k_fiver_learned(const IfaceArgs a, int record, const MlpDev m)
{
    fiver_body<false, true>(a, record, blockIdx.x, gridDim.x, &m);
}

hipError_t launch_fiver(const IfaceArgs& a, bool record, const MlpDev* mlp, hipStream_t s)
{
    long long nb = (a.qcap + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    if (a.g.eosg) {
        const int f0 = a.g.ek[0].fam, f1 = a.g.ek[1].fam;
        if (f0 < 0 || f0 > 2 || f1 < 0 || f1 > 2) return hipErrorInvalidValue;
        kFiverEos[3 * f0 + f1](a, (unsigned)nb, record ? 1 : 0, mlp, s);
    } else if (mlp)
        hipLaunchKernelGGL(k_fiver_learned, dim3((unsigned)nb), dim3(256), 0, s, a, record ? 1 : 0, *mlp);
    else
        hipLaunchKernelGGL(k_fiver, dim3((unsigned)nb), dim3(256), 0, s, a, record ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phase update (step 6 of the time-step outline, section "Code structure"):
// material ids follow the sign of the new level set; a cell that changed
// from material A to B takes the mean, over its faces in the order
// -x,+x,-y,+y,-z,+z whose neighbour held B during the step, of the B-side
// star state of the last stage's Riemann problem there (rho*_B, the B
// cell's velocity with its normal component replaced by u*, p*), encoded
// with B's equation of state.  Without such a face it keeps its primitive
// state (an "orphan").  The new state also enters the next step's CFL
// maximum.
template <bool EG>
__device__ __forceinline__ void phase_body(const PhaseArgs& a, int blk, int nblk)
{
    DevScalars* sc = a.sc;
    const Grid& G = a.g;
    __shared__ eos::EosK sEos[EG ? 2 : 1];
    if constexpr (EG) geos_stage(G, sEos);
    if (sc->err != 0) return;
    const int n = sc->nflip;
    const long long N = G.N, sxy = (long long)G.nx * G.ny, Q = a.qcap;
    const long long cstr[3] = {1, G.nx, sxy};
    const int nd[3] = {G.nx, G.ny, G.nz};
    double lam = 0.0;
    long long orphans = 0;
    for (int e = blk * blockDim.x + threadIdx.x; e < n; e += nblk * blockDim.x) {
        const long long c = a.flips[e];
        const int A = a.chi_old[c], B = a.chi_new[c];
        const int k = (int)(c / sxy);
        const long long r = c - (long long)k * sxy;
        const int j = (int)(r / G.nx);
        const int i = (int)(r - (long long)j * G.nx);
        const int ijk[3] = {i, j, k};
        double sum[5] = {0, 0, 0, 0, 0};
        int cnt = 0;
        for (int d = 0; d < 3; ++d) {
            if (!G.act[d]) continue;
            for (int side = 0; side < 2; ++side) {
                int nb = ijk[d] + (side ? 1 : -1);
                if (nb < 0 || nb >= nd[d]) {
                    if (G.bc[2 * d + side] != BC_PERIODIC) continue;
                    nb = (nb + nd[d]) % nd[d];
                }
                const long long ck = c + (long long)(nb - ijk[d]) * cstr[d];
                if (a.chi_old[ck] != B) continue;
                const long long lower = side ? c : ck;
                const int sl = a.fslot[3 * lower + d];
                if (sl < 0) continue;
                const int t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
                double qv[5];
                qv[0] = a.star[(side ? 3 : 2) * Q + sl];
                qv[1 + d] = a.star[1 * Q + sl];
                qv[t1] = a.star[(side ? 6 : 4) * Q + sl];
                qv[t2] = a.star[(side ? 7 : 5) * Q + sl];
                qv[4] = a.star[0 * Q + sl];
#pragma unroll
                for (int v = 0; v < 5; ++v) sum[v] += qv[v];
                ++cnt;
            }
        }
        double q[5];
        if (cnt) {
#pragma unroll
            for (int v = 0; v < 5; ++v) q[v] = sum[v] / cnt;
        } else {
            double u, vv, w;
            if constexpr (EG)
                q[4] = geos_prim(sEos[A], a.W[c], a.W[N + c], a.W[2 * N + c], a.W[3 * N + c], a.W[4 * N + c], u, vv, w);
            else
                q[4] = eos_prim(a.W[c], a.W[N + c], a.W[2 * N + c], a.W[3 * N + c], a.W[4 * N + c],
                                pick(G.gamma, A) - 1.0, pick(G.gpc, A), u, vv, w);
            q[0] = a.W[c];
            q[1] = u;
            q[2] = vv;
            q[3] = w;
            ++orphans;
        }
        bool ok = EG ? geos_ok(sEos[B], q[0], q[4]) : q[0] > 0.0 && q[4] + pick(G.pc, B) > 0.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) ok = ok && isfinite(q[v]);
        if (!ok) report_error(&sc->err, &sc->err_cell, ST_NONPHYSICAL, c);
        a.W[c] = q[0];
        a.W[N + c] = q[0] * q[1];
        a.W[2 * N + c] = q[0] * q[2];
        a.W[3 * N + c] = q[0] * q[3];
        if constexpr (EG) a.W[4 * N + c] = geos_energy(sEos[B], q[0], q[1], q[2], q[3], q[4]);
        else a.W[4 * N + c] = eos_energy<double>(q[0], q[1], q[2], q[3], q[4], pick(G.gpc, B), pick(G.inv_gm1, B));
        if (ok) {
            const double cs = EG ? sqrt(geos_c2(sEos[B], q[0], q[4])) : sqrt(pick(G.gamma, B) * (q[4] + pick(G.pc, B)) / q[0]);
            double l = 0.0;
            for (int d = 0; d < 3; ++d)
                if (G.act[d]) l += (fabs(q[1 + d]) + cs) * G.rh[d];
            lam = fmax(lam, l);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lam = fmax(lam, __shfl_xor(lam, o));
        orphans += __shfl_xor(orphans, o);
    }
    if ((threadIdx.x & 63) == 0) {
        if (lam > 0.0) atomic_max_nonneg(&sc->lam_bits, lam);
        if (orphans) atomicAdd((unsigned long long*)&sc->orphans, (unsigned long long)orphans);
    }
}

__global__ __launch_bounds__(256) void k_phase(const PhaseArgs a) { phase_body<false>(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(256) void k_phase_eos(const PhaseArgs a) { phase_body<true>(a, blockIdx.x, gridDim.x); }

hipError_t launch_phase(const PhaseArgs& a, hipStream_t s)
{
    long long nb = (a.g.N + 255) / 256;
    if (nb > 256) nb = 256;
    if (a.g.eosg)
        hipLaunchKernelGGL(k_phase_eos, dim3((unsigned)nb), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_phase, dim3((unsigned)nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

// The phase update of the previous step run by the count kernel of the next
// one: the phase update writes the state at flipped cells, the CFL maximum
// and error reports; the count reads only material ids, and the scan that
// forms dt from that maximum and closes the previous step comes after.
__global__ __launch_bounds__(COMPACT_THREADS) void k_count_phase(const IfaceArgs a, const PhaseArgs pa)
{
    phase_body<false>(pa, blockIdx.x, gridDim.x);
    if (!queue_kept(a.sc)) count_body(a, blockIdx.x);
}

__global__ __launch_bounds__(COMPACT_THREADS) void k_count_phase_eos(const IfaceArgs a, const PhaseArgs pa)
{
    phase_body<true>(pa, blockIdx.x, gridDim.x);
    if (!queue_kept(a.sc)) count_body(a, blockIdx.x);
}

hipError_t launch_compact(const IfaceArgs& a, const PhaseArgs* prev_phase, bool end_prev, bool begin,
                          double dt_imposed, hipStream_t s)
{
    if (prev_phase && a.g.eosg)
        hipLaunchKernelGGL(k_count_phase_eos, dim3(a.nblk), dim3(COMPACT_THREADS), 0, s, a, *prev_phase);
    else if (prev_phase)
        hipLaunchKernelGGL(k_count_phase, dim3(a.nblk), dim3(COMPACT_THREADS), 0, s, a, *prev_phase);
    else
        hipLaunchKernelGGL(k_count, dim3(a.nblk), dim3(COMPACT_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, a, end_prev ? 1 : 0, begin ? 1 : 0, a.g.cfl,
                       a.g.dt_fixed, dt_imposed);
    hipLaunchKernelGGL(k_scatter, dim3(a.nblk), dim3(COMPACT_THREADS), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched forms: the same bodies over many independent runs.  Each run's
// arguments are rebuilt on the device from its descriptor and its
// device-side state parity (sc->cur), so a captured graph is valid for
// every step.
__device__ __forceinline__ IfaceArgs iface_of_run(const RunDesc& R, int stage)
{
    IfaceArgs a;
    const int cur = R.sc->cur;
    a.g = R.g;
    a.Win = stage == 2 ? R.W1 : R.W[cur];
    a.chi = R.chi[cur];
    a.queue = R.queue;
    a.fslot = R.fslot;
    a.fluxF = R.fluxF;
    a.star = R.star;
    a.blockcnt = R.blockcnt;
    a.qcap = R.qcap;
    a.nblk = R.nblk_compact;
    a.sc = R.sc;
    return a;
}

__global__ __launch_bounds__(COMPACT_THREADS) void k_count_batch(const RunDesc* __restrict__ runs,
                                                                 const int2* __restrict__ cmap)
{
    const int2 m = cmap[blockIdx.x];
    count_body(iface_of_run(runs[m.x], 1), m.y);
}

__global__ __launch_bounds__(1024) void k_scan_batch(const RunDesc* __restrict__ runs)
{
    scan_body(iface_of_run(runs[blockIdx.x], 1));
}

__global__ __launch_bounds__(COMPACT_THREADS) void k_scatter_batch(const RunDesc* __restrict__ runs,
                                                                   const int2* __restrict__ cmap)
{
    const int2 m = cmap[blockIdx.x];
    scatter_body(iface_of_run(runs[m.x], 1), m.y);
}

hipError_t launch_compact_batch(const RunDesc* runs, int nruns, const int2* cmap, int ncblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_batch, dim3(ncblocks), dim3(COMPACT_THREADS), 0, s, runs, cmap);
    hipLaunchKernelGGL(k_scan_batch, dim3(nruns), dim3(1024), 0, s, runs);
    hipLaunchKernelGGL(k_scatter_batch, dim3(ncblocks), dim3(COMPACT_THREADS), 0, s, runs, cmap);
    return hipGetLastError();
}

constexpr int FIVER_BLOCKS_PER_RUN = 32;
constexpr int PHASE_BLOCKS_PER_RUN = 8;

__global__ __launch_bounds__(64) void k_fiver_batch(const RunDesc* __restrict__ runs, int stage)
{
    const int r = blockIdx.x / FIVER_BLOCKS_PER_RUN, b = blockIdx.x % FIVER_BLOCKS_PER_RUN;
    fiver_body<false>(iface_of_run(runs[r], stage), stage == 2, b, FIVER_BLOCKS_PER_RUN);
}

hipError_t launch_fiver_batch(const RunDesc* runs, int nruns, int stage, hipStream_t s)
{
    hipLaunchKernelGGL(k_fiver_batch, dim3(nruns * FIVER_BLOCKS_PER_RUN), dim3(64), 0, s, runs, stage);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_phase_batch(const RunDesc* __restrict__ runs)
{
    const int r = blockIdx.x / PHASE_BLOCKS_PER_RUN, b = blockIdx.x % PHASE_BLOCKS_PER_RUN;
    const RunDesc& R = runs[r];
    const int cur = R.sc->cur;
    PhaseArgs a;
    a.g = R.g;
    a.W = R.W[cur ^ 1];
    a.chi_old = R.chi[cur];
    a.chi_new = R.chi[cur ^ 1];
    a.flips = R.flips;
    a.fslot = R.fslot;
    a.star = R.star;
    a.qcap = R.qcap;
    a.sc = R.sc;
    phase_body<false>(a, b, PHASE_BLOCKS_PER_RUN);
}

hipError_t launch_phase_batch(const RunDesc* runs, int nruns, hipStream_t s)
{
    hipLaunchKernelGGL(k_phase_batch, dim3(nruns * PHASE_BLOCKS_PER_RUN), dim3(256), 0, s, runs);
    return hipGetLastError();
}

}  // namespace m2c
