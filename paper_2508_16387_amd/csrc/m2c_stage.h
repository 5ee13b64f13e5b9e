// m2c_stage.h -- fused bulk kernel of one Runge-Kutta stage (internal).
//
// One launch evaluates, for every cell, the finite-volume residual of eq.
// NS_discretized (inviscid, no source) and of the level-set equation, and
// applies one stage of a TVD Runge-Kutta scheme (section "Time
// integration"), W_out = c0 W^n + c1 (W_in + dt R(W_in)):
//   TVD-RK2: W(1) = W^n + dt R(W^n); W^{n+1} = 1/2 W^n + 1/2 (W(1) + dt R(W(1)))
//   TVD-RK3: the same first stage; W(2) = 3/4 W^n + 1/4 (W(1) + dt R(W(1)));
//            W^{n+1} = 1/3 W^n + 2/3 (W(2) + dt R(W(2)))
//   forward Euler: W^{n+1} = W^n + dt R(W^n)
// with R_i = -sum_d (F_{i,d+} - F_{i,d-}) / h_d and L_i = -sum_d V_d D_d phi.
//
// Layout on the device: SoA FP64 fields [rho, rho u, rho v, rho w, rho E, phi],
// x fastest, no ghost cells (boundary images are produced on load).
//
// Work decomposition (MI355X): a block owns a TX x TY tile of an xy-plane
// and marches along z over kz planes (2.5D).  Per plane the tile's
// primitives plus a 2-cell halo ring are staged in LDS; the x- and y-faces
// of the tile are evaluated once each as one flat work list over the
// block's threads, laid out so that each wavefront holds faces of one axis
// (no divergence between x and y faces, and LDS strides and component
// order fixed at compile time per axis), and parked in LDS; the z-face above each column is
// computed by the column's own thread from a 3-plane register window and
// carried to the next plane.  Each face flux is therefore evaluated once.
// Faces whose two cells hold different materials are not evaluated here:
// their two one-sided FIVER fluxes come from the interface kernel through
// the face -> queue slot map.  Blocks are renumbered so that each XCD
// receives a contiguous run of neighbouring tiles (halo reuse in its L2).
//
// Register budget: the column window keeps primitives of three planes,
// the z-slope and lower z-flux of the current plane, phi of five planes and
// the raw state of the prefetched plane; the stage-input conservative state
// of the cell being updated is not carried: the FP64 stiffened-gas kernels
// rebuild it from the cell's primitives, the other forms re-read it.
//
// Precision: TF is the type of reconstruction, HLLC and of the primitives
// and single-material fluxes staged in LDS and registers (double, or float
// for the mixed form).  EOS inversion, the level set, the FIVER fluxes of
// interface faces (read straight from their FP64 buffer), the residual
// accumulation and the update are FP64 in both forms.
#pragma once
#include <type_traits>

#include "m2c_device.h"
#include "m2c_internal.h"
#include "m2c_kernels.h"

#ifndef M2C_STAGE_WAVES
// Minimum waves per SIMD imposed on the register allocation.  Measured on
// the 128^3 shock-bubble stage: an imposed 2 or 3 waves (spills) is slower
// than the unconstrained allocation, which lands at 2 waves per SIMD.
#define M2C_STAGE_WAVES 1
#endif
#ifndef M2C_STAGE_WAVES_MIXED
// Mixed form: three waves per SIMD fit without private-memory spills
// (142-144 VGPRs); four needed ~60 B of scratch per lane and measured slower
// on the 384^3 cloud (3.62 against 3.31 ms per stage launch).
#define M2C_STAGE_WAVES_MIXED 3
#endif

namespace m2c {

// Fields of the per-block material table (FP64): gamma, p_c, gamma p_c,
// gamma - 1 and 1/(gamma - 1) of each material.
enum { MAT_GAMMA = 0, MAT_PC, MAT_GPC, MAT_GM1, MAT_IGM1, MAT_FIELDS };

// Threads of a stage block: the tile's cells rounded up to whole wavefronts.
constexpr int stage_threads(int tx, int ty) { return (tx * ty + 63) / 64 * 64; }

// One tile (TX x TY columns, a.kz planes) of one stage.  Called once per
// block by the single-grid kernel and once per work item by the persistent
// batched kernel; the whole block takes part.  SG: the single-grid kernel
// (material table in LDS for FP64, halo prefetched one plane ahead).  OPTS: limiter, flux and level-set band as
// configured (Van Albada, local Lax-Friedrichs, narrow band); otherwise MC,
// HLLC and the whole grid, fixed at compile time so that the default kernels
// carry neither the code nor the registers of the other options.  EG: a
// general EOS per material; FS: the set of the two materials' families (bit
// mask, eos::fam_set), so that the kernel carries only their code
// (eos::FAM_ALL: dispatched on the materials' tags at run time).
template <int STAGE, int TX, int TY, typename TF, bool SG, bool OPTS, bool EG = false, int FS = eos::FAM_ALL>
__device__ __forceinline__ void stage_tile(const StageArgs& a, const int tile)
{
    // Stage kinds: 1 first stage of RK2 / RK3 (W_out = W_in + dt R); 2 last
    // stage of RK2 / RK3 (blend with W^n, then the next step's CFL maximum,
    // new material ids and flipped cells); 3 middle stage of RK3 (blend
    // only); 4 forward Euler (first and last).
    static_assert(STAGE >= 1 && STAGE <= 4, "stage kind");
    constexpr bool BLEND = STAGE == 2 || STAGE == 3;
    constexpr bool LAST = STAGE == 2 || STAGE == 4;
    // CT cells per tile; the block is CT rounded up to whole wavefronts (a
    // 16x15 tile has 511 in-plane faces: exactly two rounds of the 256
    // threads, where a 16x16 tile needs a third, one-wave round)
    constexpr int CT = TX * TY, NT = stage_threads(TX, TY), LX = TX + 4, LY = TY + 4, PL = LX * LY;
    constexpr int NXF = (TX + 1) * TY, NYF = TX * (TY + 1), NF = NXF + NYF;
    // plane tiles are double-buffered (even / odd planes), so the next
    // plane can be staged while slow waves still read the current one
    __shared__ TF sQ2[2][5 * PL];          // primitives rho,u,v,w,p of the plane + halo
    __shared__ double sPhi2[2][PL];        // level set of the plane + halo (always FP64)
    __shared__ uint8_t sX2[2][PL];         // material ids
    __shared__ TF sF[5 * NF];              // in-plane single-material face fluxes
    __shared__ int sS[NF];                 // queue slot of an interface face, else -1
    __shared__ double sRed[NT / 64];
    __shared__ int sErr;
    // LMAT: material parameters indexed by material id, so that a per-lane
    // id costs one LDS read per parameter instead of a select between two
    // scalar register pairs.  Measured faster for the single-grid FP64
    // kernel; the mixed form and the batched kernel (whose register budget
    // it would exceed) keep the selects.
    constexpr bool LMAT = SG && !EG && sizeof(TF) == sizeof(double);
    __shared__ double sMat[2][MAT_FIELDS];
    // EG: general EOS of the two materials (FP64 form only)
    static_assert(!EG || sizeof(TF) == sizeof(double), "general EOS runs in FP64");
    __shared__ eos::EosK sEos[EG ? 2 : 1];

    // Skip the tile when an earlier kernel of the step failed; the flag is
    // read once per block so that the whole block takes the same branch
    // (other blocks may raise it meanwhile).
    DevScalars* sc = a.sc;
    const Grid& G = a.g;
    __syncthreads();
    if (threadIdx.x == 0) sErr = sc->err;
    if (EG && threadIdx.x == 0) {
        const double* src = reinterpret_cast<const double*>(a.g.ek);
        double* dst = reinterpret_cast<double*>(sEos);
#pragma unroll
        for (int t = 0; t < (int)(2 * sizeof(eos::EosK) / sizeof(double)); ++t) dst[t] = src[t];
    }
    if (LMAT && threadIdx.x < 2) {
        const int m = threadIdx.x;
        sMat[m][MAT_GAMMA] = G.gamma[m];
        sMat[m][MAT_PC] = G.pc[m];
        sMat[m][MAT_GPC] = G.gpc[m];
        sMat[m][MAT_GM1] = G.gamma[m] - 1.0;
        sMat[m][MAT_IGM1] = G.inv_gm1[m];
    }
    __syncthreads();
    if (sErr != 0) return;
    // parameter f of material x
    auto mat = [&](int x, int f) -> double {
        if constexpr (LMAT) return sMat[x][f];
        switch (f) {
            case MAT_GAMMA: return pick(G.gamma, x);
            case MAT_PC: return pick(G.pc, x);
            case MAT_GPC: return pick(G.gpc, x);
            case MAT_GM1: return pick(G.gamma, x) - 1.0;
            default: return pick(G.inv_gm1, x);
        }
    };

    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const long long N = G.N;
    const bool xact = G.act[0], yact = G.act[1], zact = G.act[2];
    const double* __restrict__ Win = a.Win;
    const uint8_t* __restrict__ chi = a.chi;

    const int bx = tile % a.tiles_x;
    const int rest = tile / a.tiles_x;
    const int by = rest % a.tiles_y;
    const int bz = rest / a.tiles_y;
    const int i0 = bx * TX, j0 = by * TY;
    const int kz0 = bz * a.kz, kz1 = min(nz, kz0 + a.kz);

    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const bool cellt = tid < CT;                       // thread owns a tile column
    const int gi = i0 + tx, gj = j0 + ty;
    const bool inside = cellt && gi < nx && gj < ny;
    bool mirx = false, miry = false;
    const int si = bc_index(gi, nx, G.bc[0], G.bc[1], mirx);
    const int sj = bc_index(gj, ny, G.bc[2], G.bc[3], miry);
    if (!xact) mirx = false;
    if (!yact) miry = false;
    const uint32_t sxy = (uint32_t)nx * ny;
    const uint32_t col = si + (uint32_t)nx * sj;
    const TF halpha = TF(0.5) * (TF)G.alpha;
    const int lim = OPTS ? G.limiter : (int)LIM_MC, limk = G.limk;
    const int flux = OPTS ? G.flux : (int)FLUX_HLLC;

    // Raw state of this thread's column at plane k (any k in [-2, nz+1]).
    auto load_raw = [&](int k, double w[6], uint8_t& x, bool& mz) {
        const int sk = bc_index(k, nz, G.bc[4], G.bc[5], mz);
        const uint32_t c = col + sxy * sk;
#pragma unroll
        for (int v = 0; v < 6; ++v) w[v] = ldf(Win + v * N, c);
        x = chi[c];
    };
    // Primitives of a raw state, velocities mirrored at wall images.
    auto to_prim = [&](const double w[6], uint8_t x, bool mz, TF q[5]) {
        double u, vv, ww, p;
        if constexpr (EG) p = geos_prim<FS>(sEos[x], w[0], w[1], w[2], w[3], w[4], u, vv, ww);
        else p = eos_prim(w[0], w[1], w[2], w[3], w[4], mat(x, MAT_GM1), mat(x, MAT_GPC), u, vv, ww);
        q[0] = TF(w[0]);
        q[1] = TF(mirx ? -u : u);
        q[2] = TF(miry ? -vv : vv);
        q[3] = TF((mz && zact) ? -ww : ww);
        q[4] = TF(p);
    };
    // half the z-slope of a cell from its column neighbours (zero next to
    // another material along z).
    auto zslope = [&](const TF qm[5], const TF q0[5], const TF qp[5], uint8_t xm, uint8_t x0, uint8_t xp,
                      TF s[5]) {
        const bool flat = (xm != x0) || (xp != x0);
#pragma unroll
        for (int v = 0; v < 5; ++v) s[v] = lim_half_slope_flat<TF>(lim, limk, q0[v] - qm[v], qp[v] - q0[v], halpha, flat);
    };
    // z-face between planes k (lower) and k+1.  A single-material face gets
    // its HLLC flux in F and slot -1; an interface face returns the queue
    // slot of its two FP64 one-sided FIVER fluxes.
    auto zface = [&](int k, const TF ql[5], const TF sl[5], uint8_t xl, const TF qu[5], const TF su[5],
                     uint8_t xu, TF F[5]) -> int {
        if (xl == xu) {
            TF Fr[5];
            // face frame: normal w, tangential u, v
            if constexpr (EG) {
                geos_flux<FS>(sEos[xl], flux, ql[0] + sl[0], ql[3] + sl[3], ql[1] + sl[1], ql[2] + sl[2],
                          ql[4] + sl[4], qu[0] - su[0], qu[3] - su[3], qu[1] - su[1], qu[2] - su[2], qu[4] - su[4],
                          Fr);
            } else {
                const TF g = TF(mat(xl, MAT_GAMMA)), pc = TF(mat(xl, MAT_PC)), gpc = TF(mat(xl, MAT_GPC)),
                         igm1 = TF(mat(xl, MAT_IGM1));
                num_flux<TF>(flux, ql[0] + sl[0], ql[3] + sl[3], ql[1] + sl[1], ql[2] + sl[2], ql[4] + sl[4],
                             qu[0] - su[0], qu[3] - su[3], qu[1] - su[1], qu[2] - su[2], qu[4] - su[4], g, pc, gpc,
                             igm1, Fr);
            }
            F[0] = Fr[0];
            F[3] = Fr[1];
            F[1] = Fr[2];
            F[2] = Fr[3];
            F[4] = Fr[4];
            return -1;
        }
        bool m;
        const int lk = bc_index(k, nz, G.bc[4], G.bc[5], m);
        const uint32_t fid = 3 * (col + sxy * lk) + 2;
        const int q = a.fslot[fid];
        if (q < 0) report_error(&sc->err, &sc->err_cell, ST_NONPHYSICAL, fid / 3);
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] = TF(0);
        return q < 0 ? 0 : q;
    };

    // ---- prologue: column window and the z-face below plane kz0 ----------
    TF Q0[5], Q1[5], Q2[5];           // primitives at k, k+1, k+2
    double PH[5];                     // phi at k-2 .. k+2
    uint8_t X0, X1, X2;               // ids at k .. k+2
    TF S0[5];                         // half z-slope of plane k
    TF Fzlo[5];                       // single-material flux through the lower z-face of plane k
    int qzlo = -1;                    // or the queue slot of that face's FIVER fluxes
    {
        double w[6];
        TF qm1[5];
        uint8_t xm1;
        bool mz;
        if (zact) {
            TF qm2[5];
            uint8_t xm2;
            load_raw(kz0 - 2, w, xm2, mz);
            PH[0] = w[5];
            to_prim(w, xm2, mz, qm2);
            load_raw(kz0 - 1, w, xm1, mz);
            PH[1] = w[5];
            to_prim(w, xm1, mz, qm1);
            load_raw(kz0, w, X0, mz);
            PH[2] = w[5];
            to_prim(w, X0, mz, Q0);
            load_raw(kz0 + 1, w, X1, mz);
            PH[3] = w[5];
            to_prim(w, X1, mz, Q1);
            load_raw(kz0 + 2, w, X2, mz);
            PH[4] = w[5];
            to_prim(w, X2, mz, Q2);
            zslope(qm1, Q0, Q1, xm1, X0, X1, S0);
            TF Sm[5];
            zslope(qm2, qm1, Q0, xm2, xm1, X0, Sm);
            if (inside) qzlo = zface(kz0 - 1, qm1, Sm, xm1, Q0, S0, X0, Fzlo);
        } else {
            load_raw(kz0, w, X0, mz);
            to_prim(w, X0, mz, Q0);
            PH[2] = w[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                S0[v] = TF(0);
                Fzlo[v] = TF(0);
                Q1[v] = Q2[v] = Q0[v];
            }
            PH[0] = PH[1] = PH[3] = PH[4] = PH[2];
            X1 = X2 = X0;
        }
    }

    const double dt = sc->dt;
    double lam = 0.0;                 // last stage: max wave-speed sum of own cells

    // Halo ring of a plane (x-halo: 4 columns x TY rows; y-halo: 4 rows x TX
    // columns), HPT cells per thread at most; its raw state is loaded one
    // plane ahead (in the single-grid default kernels right after the
    // previous plane's halo is staged, so that the face work hides its
    // latency; otherwise after the face work) and turned into primitives
    // when the plane is staged.
    constexpr int HPT = (4 * TX + 4 * TY + NT - 1) / NT;
    const int nxh = xact ? 4 * TY : 0, nyh = yact ? 4 * TX : 0;
    auto halo_pos = [&](int h, int& li, int& lj) {
        if (h < nxh) {
            const int r = h / 4, s = h % 4;
            lj = r + 2;
            li = s < 2 ? s : TX + s;
        } else {
            const int hh = h - nxh;
            const int r = hh / TX, s = hh % TX;
            li = s + 2;
            lj = r < 2 ? r : TY + r;
        }
    };
    // The halo of the next plane is prefetched into registers (FP64, and
    // the single-grid mixed form on tiles with one halo cell per thread);
    // the batched mixed form keeps its register budget for three waves per
    // SIMD and loads the halo when it stages the plane.
    constexpr bool PF = sizeof(TF) == sizeof(double) || (SG && HPT == 1);
    // plane-independent part of the halo elements of this thread: LDS
    // offset (-1: none), source column in the xy-plane, wall-image flags
    int hofs[HPT];
    uint32_t hcol[HPT];
    unsigned hmir = 0;
#pragma unroll
    for (int q = 0; q < HPT; ++q) {
        const int h = tid + q * NT;
        hofs[q] = -1;
        hcol[q] = 0;
        if (h < nxh + nyh) {
            int li, lj;
            halo_pos(h, li, lj);
            bool mx, my;
            const int hi_ = bc_index(i0 + li - 2, nx, G.bc[0], G.bc[1], mx);
            const int hj_ = bc_index(j0 + lj - 2, ny, G.bc[2], G.bc[3], my);
            hofs[q] = lj * LX + li;
            hcol[q] = hi_ + (uint32_t)nx * hj_;
            hmir |= ((mx && xact) ? 1u : 0u) << (2 * q);
            hmir |= ((my && yact) ? 2u : 0u) << (2 * q);
        }
    }
    double hw[HPT][6] = {};
    uint8_t hx[HPT] = {};
    auto halo_load = [&](int k) {
#pragma unroll
        for (int q = 0; q < HPT; ++q) {
            if (hofs[q] >= 0) {
                const uint32_t c = hcol[q] + sxy * k;
#pragma unroll
                for (int v = 0; v < 6; ++v) hw[q][v] = ldf(Win + v * N, c);
                hx[q] = chi[c];
            }
        }
    };
    // Consume the prefetched raw halo (the empty asm): a use after this
    // point never waits on the vector-memory counter, which counts stores as
    // well as loads in issue order, so placing this before a plane's stores
    // keeps the staging of the next plane from waiting for them.
    auto halo_consume = [&]() {
#pragma unroll
        for (int q = 0; q < HPT; ++q) {
            uint32_t x = hx[q];
            asm volatile("" : "+v"(hw[q][0]), "+v"(hw[q][1]), "+v"(hw[q][2]), "+v"(hw[q][3]), "+v"(hw[q][4]),
                         "+v"(hw[q][5]), "+v"(x));
            hx[q] = (uint8_t)x;
        }
    };
    // Tiles with one halo cell per thread: the halo of the next plane is
    // loaded right after this plane's halo is staged and consumed after the
    // face work, before this plane's stores; the 64x2 tile (three per
    // thread), whose register budget this would exceed, loads it after the
    // face work.
    constexpr bool EARLY_HALO = PF && HPT == 1;
    // wave priorities by phase of the plane (see the face work below)
    constexpr bool PRIO = sizeof(TF) == sizeof(double) && !OPTS;
    // stage-input state of the cell fetched at the top of the plane (forms
    // that do not rebuild it from the primitives)
    constexpr bool WIE = HPT == 1 && (EG || sizeof(TF) != sizeof(double));
    double wie[5] = {};
    // blended stages: the step-start state of the cell, fetched likewise
    constexpr bool W0E = BLEND && ((HPT == 1 && (SG || sizeof(TF) == sizeof(double))) ||
                                   (sizeof(TF) == sizeof(double) && !EG && !OPTS));
    double w0[6] = {};
    if (PF) halo_load(kz0);
    if (EARLY_HALO) halo_consume();

    // In-plane face list: slot t < NXF is the x-face left of tile column
    // t % (TX+1) in row t / (TX+1); slot t in [YB, YB + NYF) is the y-face
    // below row (t - YB) / TX.  YB is NXF rounded up to whole wavefronts, so
    // that each wavefront holds faces of one axis and runs that axis's code
    // path, whose LDS strides and component order are compile-time
    // constants.  Per round: LDS offset of the lower cell << 1 | face inside
    // the grid.
    constexpr int YB = (NXF + 63) / 64 * 64, NFL = YB + NYF;
    constexpr int FR = (NFL + NT - 1) / NT;
    static_assert(FR <= 3, "at most three rounds of in-plane faces");
    int fdesc[FR];
#pragma unroll
    for (int rr = 0; rr < FR; ++rr) {
        const int t = tid + rr * NT;
        fdesc[rr] = 0;
        const bool isx = t < NXF, isy = t >= YB && t < NFL;
        if (isx || isy) {
            const int tt = isx ? t : t - YB;
            const int W_ = isx ? TX + 1 : TX;
            const int fa = tt % W_, fb = tt / W_;
            const int oA = isx ? (fb + 2) * LX + (fa + 1) : (fb + 1) * LX + (fa + 2);
            const int gx = i0 + fa, gy = j0 + fb;
            const bool valid = isx ? (xact && gx <= nx && gy < ny) : (yact && gx < nx && gy <= ny);
            fdesc[rr] = (oA << 1) | (valid ? 1 : 0);
        }
    }

    for (int k = kz0; k < kz1; ++k) {
        const int buf = (k - kz0) & 1;
        TF* const sQ = sQ2[buf];
        double* const sPhi = sPhi2[buf];
        uint8_t* const sX = sX2[buf];
        // lead load of plane k+3 (turned into primitives before this
        // plane's stores, see below)
        double Wn[6];
        uint8_t Xn;
        bool mzn;
        if (zact) {
            load_raw(k + 3, Wn, Xn, mzn);
        } else {
#pragma unroll
            for (int v = 0; v < 6; ++v) Wn[v] = 1.0;
            Xn = 0;
            mzn = false;
        }
        // stage 2: the step-start state of the cell, fetched early
        if (W0E && inside) {
            const uint32_t c0 = col + sxy * k;
#pragma unroll
            for (int v = 0; v < 6; ++v) w0[v] = ldf(a.W0 + v * N, c0);
        }
        // forms that re-read the stage-input state of the cell (mixed,
        // general EOS): the single-grid default kernels fetch it here, so
        // that the face work covers the load
        if (WIE && inside) {
            const uint32_t c0 = col + sxy * k;
#pragma unroll
            for (int v = 0; v < 5; ++v) wie[v] = ldf(Win + v * N, c0);
        }

        // (1) own plane-k values into the LDS tile
        if (cellt) {
            const int o = (ty + 2) * LX + tx + 2;
#pragma unroll
            for (int v = 0; v < 5; ++v) sQ[v * PL + o] = Q0[v];
            sPhi[o] = PH[2];
            sX[o] = X0;
        }
        // (2) halo ring of plane k from the prefetched raw state
        if (!PF) halo_load(k);
#pragma unroll
        for (int q = 0; q < HPT; ++q) {
            if (hofs[q] >= 0) {
                const bool mx = (hmir >> (2 * q)) & 1u, my = (hmir >> (2 * q)) & 2u;
                const uint8_t x = hx[q];
                double u, vv, ww, p;
                if constexpr (EG) p = geos_prim<FS>(sEos[x], hw[q][0], hw[q][1], hw[q][2], hw[q][3], hw[q][4], u, vv, ww);
                else p = eos_prim(hw[q][0], hw[q][1], hw[q][2], hw[q][3], hw[q][4], mat(x, MAT_GM1), mat(x, MAT_GPC),
                                  u, vv, ww);
                const int o = hofs[q];
                sQ[o] = TF(hw[q][0]);
                sQ[PL + o] = TF(mx ? -u : u);
                sQ[2 * PL + o] = TF(my ? -vv : vv);
                sQ[3 * PL + o] = TF(ww);
                sQ[4 * PL + o] = TF(p);
                sPhi[o] = hw[q][5];
                sX[o] = x;
            }
        }
        // halo of the next plane: its registers are free once this plane's
        // halo is staged, and the face work below covers the load latency
        if (EARLY_HALO && k + 1 < kz1) halo_load(k + 1);
        __syncthreads();
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);

        // (3) x- and y-faces of the tile as one work list (the list
        // decomposition is the same for every plane, see fdesc).  One face:
        // axis ISX, list slot t, LDS offset oA of its lower cell; its fluxes
        // go to face index f of sF / sS (x-faces first, then y-faces).
        auto face = [&](auto axis_tag, const int t, const int oA) {
            constexpr bool ISX = decltype(axis_tag)::value;
            constexpr int step = ISX ? 1 : LX;
            constexpr int nrm = ISX ? 1 : 2, ta = ISX ? 2 : 3, tb = ISX ? 3 : 1;
            const int tt = ISX ? t : t - YB;
            const int f = ISX ? t : NXF + tt;
            const int oB = oA + step;
            const uint8_t xa = sX[oA], xb = sX[oB];
            if (xa == xb) {
                const bool flatA = sX[oA - step] != xa || sX[oB] != xa;
                const bool flatB = sX[oA] != xb || sX[oB + step] != xb;
                TF qa[5], qb[5];
                constexpr int comp[5] = {0, nrm, ta, tb, 4};
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    const TF* s = sQ + comp[v] * PL;
                    const TF m1 = s[oA - step], a0 = s[oA], b0 = s[oB], p1 = s[oB + step];
                    qa[v] = a0 + lim_half_slope_flat<TF>(lim, limk, a0 - m1, b0 - a0, halpha, flatA);
                    qb[v] = b0 - lim_half_slope_flat<TF>(lim, limk, b0 - a0, p1 - b0, halpha, flatB);
                }
                TF Fr[5];
                if constexpr (EG)
                    geos_flux<FS>(sEos[xa], flux, qa[0], qa[1], qa[2], qa[3], qa[4], qb[0], qb[1], qb[2], qb[3], qb[4], Fr);
                else
                    num_flux<TF>(flux, qa[0], qa[1], qa[2], qa[3], qa[4], qb[0], qb[1], qb[2], qb[3], qb[4],
                                 TF(mat(xa, MAT_GAMMA)), TF(mat(xa, MAT_PC)), TF(mat(xa, MAT_GPC)), TF(mat(xa, MAT_IGM1)),
                                 Fr);
                sF[f] = Fr[0];
                sF[nrm * NF + f] = Fr[1];
                sF[ta * NF + f] = Fr[2];
                sF[tb * NF + f] = Fr[3];
                sF[4 * NF + f] = Fr[4];
                sS[f] = -1;
            } else {
                bool m;
                constexpr int W_ = ISX ? TX + 1 : TX;
                const int gx = i0 + tt % W_, gy = j0 + tt / W_;   // x: face left of cell gx; y: below gy
                uint32_t lower;
                if constexpr (ISX) {
                    const int lx = bc_index(gx - 1, nx, G.bc[0], G.bc[1], m);
                    lower = lx + (uint32_t)nx * gy;
                } else {
                    const int ly = bc_index(gy - 1, ny, G.bc[2], G.bc[3], m);
                    lower = gx + (uint32_t)nx * ly;
                }
                const uint32_t fid = 3 * (lower + sxy * k) + (ISX ? 0 : 1);
                const int q = a.fslot[fid];
                if (q < 0) report_error(&sc->err, &sc->err_cell, ST_NONPHYSICAL, fid / 3);
                sS[f] = q < 0 ? 0 : q;
            }
        };
        if constexpr (YB == NT && FR == 2 && sizeof(TF) == sizeof(double) && !EG) {
            // the first round holds every x-face and the second every y-face
            if (fdesc[0] & 1) face(std::integral_constant<bool, true>(), tid, fdesc[0] >> 1);
            if (fdesc[FR - 1] & 1) face(std::integral_constant<bool, false>(), tid + NT, fdesc[FR - 1] >> 1);
        } else {
#pragma unroll 1
            for (int rr = 0; rr < FR; ++rr) {
                const int t = tid + rr * NT;
                const int fd = rr == 0 ? fdesc[0] : (rr == 1 ? fdesc[1 % FR] : fdesc[2 % FR]);
                // the wavefront's first slot decides its axis (uniform across it)
                const int wt = __builtin_amdgcn_readfirstlane((tid & ~63) + rr * NT);
                if (!(fd & 1)) continue;
                if (wt < YB) face(std::integral_constant<bool, true>(), t, fd >> 1);
                else face(std::integral_constant<bool, false>(), t, fd >> 1);
            }
        }

        // Wave priority (FP64 default-scheme kernels): the end of the face
        // work (the z-face) at 2, the update and the staging of the next
        // plane at 3, the in-plane face rounds at 0.  A block whose waves are
        // finishing a plane is preferred over the other block on the CU,
        // which is in the middle of its face rounds, so the barriers release
        // sooner and the two blocks take turns (384^3 stage launch 2.64 ->
        // 2.46 ms).  The mixed form (three blocks per CU) and the option
        // kernels measured no gain or a loss at 128^3 and keep one priority.
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
        // (4) z-face above plane k for this column
        TF S1[5], Fzhi[5];
        int qzhi = -1;
        if (zact) {
            zslope(Q0, Q1, Q2, X0, X1, X2, S1);
            if (inside) qzhi = zface(k, Q0, S0, X0, Q1, S1, X1, Fzhi);
        }
        __syncthreads();
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
        if (PF && !EARLY_HALO && k + 1 < kz1) halo_load(k + 1);
        // the lead-loaded plane is consumed here, before this plane's stores,
        // on every path: the vector-memory counter counts stores as well as
        // loads, in issue order, so a use of the lead load after the stores
        // (or a path on which the compiler cannot see it consumed) would wait
        // for the stores to complete.  Without a z-axis the values are unused.
        TF Qn[5];
        to_prim(Wn, Xn, mzn, Qn);
        double phn = Wn[5];
        uint32_t xnv = Xn;
        asm volatile("" : "+v"(phn), "+v"(xnv));
        if (EARLY_HALO && k + 1 < kz1) halo_consume();
        if (WIE) asm volatile("" : "+v"(wie[0]), "+v"(wie[1]), "+v"(wie[2]), "+v"(wie[3]), "+v"(wie[4]));
        if (W0E)
            asm volatile("" : "+v"(w0[0]), "+v"(w0[1]), "+v"(w0[2]), "+v"(w0[3]), "+v"(w0[4]), "+v"(w0[5]));

        // (5) residual and stage update of cell (gi, gj, k)
        if (inside) {
            const uint32_t c = col + sxy * k;
            double acc[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) acc[v] = 0.0;
            // flux difference across one axis: single-material fluxes from LDS
            // (or registers for z), interface faces from the FP64 FIVER buffer
            // (lower face: the flux seen by its upper cell, i.e. this one;
            // upper face: the flux seen by its lower cell; the ten fluxes of
            // an interface face are contiguous: lower cell's 5, upper cell's 5)
            // (the interface fluxes are fetched under one branch per face, not
            // one per variable: most wavefronts hold no interface face)
            auto axis = [&](int qlo, int qhi, const TF* flo, const TF* fhi, int stride, double rh) {
                double lo[5], hi[5];
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    lo[v] = (double)flo[v * stride];
                    hi[v] = (double)fhi[v * stride];
                }
                // (the empty asm takes the wait for these loads inside the
                // branch, so wavefronts without an interface face do not wait
                // on the vector-memory counter here)
                if (qlo >= 0) {
                    const double* f = a.fluxF + 10 * (long long)qlo + 5;
#pragma unroll
                    for (int v = 0; v < 5; ++v) lo[v] = f[v];
                    asm volatile("" : "+v"(lo[0]), "+v"(lo[1]), "+v"(lo[2]), "+v"(lo[3]), "+v"(lo[4]));
                }
                if (qhi >= 0) {
                    const double* f = a.fluxF + 10 * (long long)qhi;
#pragma unroll
                    for (int v = 0; v < 5; ++v) hi[v] = f[v];
                    asm volatile("" : "+v"(hi[0]), "+v"(hi[1]), "+v"(hi[2]), "+v"(hi[3]), "+v"(hi[4]));
                }
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[v] += (hi[v] - lo[v]) * rh;
            };
            if (xact) {
                const int fl = ty * (TX + 1) + tx, fr = fl + 1;
                axis(sS[fl], sS[fr], sF + fl, sF + fr, NF, G.rh[0]);
            }
            if (yact) {
                const int fl = NXF + ty * TX + tx, fr = fl + TX;
                axis(sS[fl], sS[fr], sF + fl, sF + fr, NF, G.rh[1]);
            }
            if (zact) axis(qzlo, qzhi, Fzlo, Fzhi, 1, G.rh[2]);
            // level set: third-order upwind-biased differences, upwinded by V_d of the cell
            // (both one-sided differences are formed and one is selected, so
            // the five level-set values are read up front rather than inside
            // a divergent branch per axis)
            auto ls_term = [&](double V, double f0, double f1, double f2, double f3, double f4, double rh6) {
                double Dm = (2.0 * f3 + 3.0 * f2 - 6.0 * f1 + f0) * rh6;
                double Dp = (-f4 + 6.0 * f3 - 3.0 * f2 - 2.0 * f1) * rh6;
                // keep both in the straight-line code (the compiler would
                // otherwise sink each, with its LDS reads, into a branch)
                asm volatile("" : "+v"(Dm), "+v"(Dp));
                const double D = V > 0.0 ? Dm : (V < 0.0 ? Dp : 0.0);
                return V * D;
            };
            // stage-input state of the cell (FP64).  The FP64 stiffened-gas
            // kernels rebuild it from the cell's primitives in the column
            // window (a few roundings from the stored values: the update of
            // the conservative state stays conservative to round-off), which
            // saves re-reading 40 B per cell that the cache no longer holds
            // three planes after the lead load; the other forms re-read it.
            double wi[5];
            if constexpr (sizeof(TF) == sizeof(double) && !EG) {
                const double r = Q0[0];
                wi[0] = r;
                wi[1] = r * Q0[1];
                wi[2] = r * Q0[2];
                wi[3] = r * Q0[3];
                wi[4] = eos_energy<double>(r, Q0[1], Q0[2], Q0[3], Q0[4], mat(X0, MAT_GPC), mat(X0, MAT_IGM1));
            } else if constexpr (WIE) {
#pragma unroll
                for (int v = 0; v < 5; ++v) wi[v] = wie[v];
            } else {
#pragma unroll
                for (int v = 0; v < 5; ++v) wi[v] = ldf(Win + v * N, c);
            }
            // cell velocity for the level-set upwinding, in FP64
            double Vc[3];
            if constexpr (sizeof(TF) == sizeof(double)) {
                Vc[0] = Q0[1];
                Vc[1] = Q0[2];
                Vc[2] = Q0[3];
            } else {
                const double ri = 1.0 / wi[0];
                Vc[0] = wi[1] * ri;
                Vc[1] = wi[2] * ri;
                Vc[2] = wi[3] * ri;
            }
            double Ls = 0.0;
            const double* sp = sPhi + (ty + 2) * LX + tx + 2;
            if (xact) Ls += ls_term(Vc[0], sp[-2], sp[-1], sp[0], sp[1], sp[2], G.rh6[0]);
            if (yact) Ls += ls_term(Vc[1], sp[-2 * LX], sp[-LX], sp[0], sp[LX], sp[2 * LX], G.rh6[1]);
            if (zact) Ls += ls_term(Vc[2], PH[0], PH[1], PH[2], PH[3], PH[4], G.rh6[2]);
            // narrow band: phi is held where the stage-input |phi| reaches the bandwidth
            if (OPTS && G.ls_band > 0.0 && fabs(PH[2]) >= G.ls_band) Ls = 0.0;

            double wn[6];
            if (!BLEND) {
#pragma unroll
                for (int v = 0; v < 5; ++v) wn[v] = wi[v] + dt * (-acc[v]);
                wn[5] = PH[2] + dt * (-Ls);
            } else {
                const double c0 = a.c0, c1 = a.c1;
#pragma unroll
                for (int v = 0; v < 5; ++v)
                    wn[v] = c0 * (W0E ? w0[v] : ldf(a.W0 + v * N, c)) + c1 * (wi[v] + dt * (-acc[v]));
                wn[5] = c0 * (W0E ? w0[5] : ldf(a.W0 + 5 * N, c)) + c1 * (PH[2] + dt * (-Ls));
            }
            double u, vv, ww, p, c2 = 0.0;
            bool adm;
            if constexpr (EG) {
                p = geos_prim<FS>(sEos[X0], wn[0], wn[1], wn[2], wn[3], wn[4], u, vv, ww);
                c2 = geos_c2<FS>(sEos[X0], wn[0], p);
                adm = wn[0] > 0.0 && p > sEos[X0].k[eos::KFLOOR] && c2 > 0.0;
            } else {
                p = eos_prim(wn[0], wn[1], wn[2], wn[3], wn[4], mat(X0, MAT_GM1), mat(X0, MAT_GPC), u, vv, ww);
                adm = wn[0] > 0.0 && p + mat(X0, MAT_PC) > 0.0;
            }
            const bool ok = adm && isfinite(p) && isfinite(u) && isfinite(vv) && isfinite(ww) && isfinite(wn[5]);
            if (!ok) report_error(&sc->err, &sc->err_cell, ST_NONPHYSICAL, c);
#pragma unroll
            for (int v = 0; v < 6; ++v) stf(a.Wout + v * N, c, wn[v]);
            if (LAST) {
                const uint8_t xn = wn[5] < 0.0 ? 1 : 0;
                a.chi_next[c] = xn;
                if (xn != X0) {
                    const int slot = atomicAdd(&sc->nflip, 1);
                    a.flips[slot] = (int)c;
                } else if (ok) {
                    double cs;
                    if constexpr (EG) cs = sqrt(c2);
                    else cs = sqrt_nr(mat(X0, MAT_GAMMA) * (p + mat(X0, MAT_PC)) * rcp_nr(wn[0]));
                    double l = 0.0;
                    if (xact) l += (fabs(u) + cs) * G.rh[0];
                    if (yact) l += (fabs(vv) + cs) * G.rh[1];
                    if (zact) l += (fabs(ww) + cs) * G.rh[2];
                    lam = fmax(lam, l);
                }
            }
        }

        // (6) advance the column window
        if (zact) {
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                Q0[v] = Q1[v];
                Q1[v] = Q2[v];
                Q2[v] = Qn[v];
                S0[v] = S1[v];
                Fzlo[v] = Fzhi[v];
            }
            qzlo = qzhi;
            PH[0] = PH[1];
            PH[1] = PH[2];
            PH[2] = PH[3];
            PH[3] = PH[4];
            PH[4] = phn;
            X0 = X1;
            X1 = X2;
            X2 = (uint8_t)xnv;
        }
        // no barrier here: the next plane is staged in the other buffer, and
        // its first barrier orders this plane's reads before any reuse
    }

    if (LAST) {
        // block max of the wave-speed sums -> one atomic per block
        for (int o = 32; o > 0; o >>= 1) lam = fmax(lam, __shfl_xor(lam, o));
        if ((tid & 63) == 0) sRed[tid >> 6] = lam;
        __syncthreads();
        if (tid == 0) {
            double m = 0.0;
            for (int w = 0; w < NT / 64; ++w) m = fmax(m, sRed[w]);
            atomic_max_nonneg(&sc->lam_bits, m);
        }
    }
}

// XCD-aware block numbering: dispatch is round-robin over the 8 XCDs, so
// block b runs on XCD b % 8; map each XCD's blocks onto one contiguous run
// of neighbouring tiles (halo reuse in that XCD's L2).
__device__ __forceinline__ int xcd_tile(int b, int nblk)
{
    const int bq = nblk / 8, br = nblk % 8;
    const int xcd = b % 8, idx = b / 8;
    return (xcd < br ? xcd * (bq + 1) : br * (bq + 1) + (xcd - br) * bq) + idx;
}

#define M2C_STAGE_BOUNDS(TX, TY, TF) \
    __launch_bounds__(stage_threads(TX, TY), sizeof(TF) == 4 ? M2C_STAGE_WAVES_MIXED : M2C_STAGE_WAVES)

template <int STAGE, int TX, int TY, typename TF, bool OPTS, bool EG = false, int FS = eos::FAM_ALL>
__global__ M2C_STAGE_BOUNDS(TX, TY, TF) void k_stage(const StageArgs a)
{
    stage_tile<STAGE, TX, TY, TF, true, OPTS, EG, FS>(a, xcd_tile(blockIdx.x, gridDim.x));
}

// Launch of the single-grid kernel of one stage kind over the whole grid.
template <int TX, int TY, typename TF, bool OPTS, bool EG = false, int FS = eos::FAM_ALL>
static hipError_t launch_tile(int stage, const StageArgs& a, hipStream_t s)
{
    const int nblk = a.tiles_x * a.tiles_y * a.tiles_z;
    const dim3 g(nblk), b(stage_threads(TX, TY));
    switch (stage) {
        case 1: hipLaunchKernelGGL((k_stage<1, TX, TY, TF, OPTS, EG, FS>), g, b, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_stage<2, TX, TY, TF, OPTS, EG, FS>), g, b, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_stage<3, TX, TY, TF, OPTS, EG, FS>), g, b, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_stage<4, TX, TY, TF, OPTS, EG, FS>), g, b, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Tile shapes with compiled stage kernels, applied to a per-tile macro F.
#define M2C_TILES(F)                                                                    \
    F(16, 15)                                                                           \
    F(32, 7)                                                                            \
    F(16, 16)                                                                           \
    F(32, 8)                                                                            \
    F(64, 2)

}  // namespace m2c
