// k_stage.hip -- fused bulk kernel of one Runge-Kutta stage.
//
// One launch evaluates, for every cell, the finite-volume residual of eq.
// NS_discretized (inviscid, no source) and of the level-set equation, and
// applies the TVD-RK2 stage update (section "Time integration"):
//   stage 1: W(1) = W^n + dt R(W^n)
//   stage 2: W^{n+1} = 1/2 W^n + 1/2 (W(1) + dt R(W(1)))
// with R_i = -sum_d (F_{i,d+} - F_{i,d-}) / h_d and L_i = -sum_d V_d D_d phi.
//
// Layout on the device: SoA FP64 fields [rho, rho u, rho v, rho w, rho E, phi],
// x fastest, no ghost cells (boundary images are produced on load).
//
// Work decomposition (MI355X): a block owns a TX x TY tile of an xy-plane
// and marches along z over KZ planes (2.5D).  Per plane the tile's
// primitives plus a 2-cell halo ring are staged in LDS; the x- and y-faces
// of the tile are evaluated once each as a flat work list over the block's
// threads and parked in LDS; the z-face above each column is computed by
// the column's own thread from a 3-plane register window and carried to
// the next plane.  Each face flux is therefore evaluated once.  Faces whose
// two cells hold different materials are not evaluated here: their two
// one-sided FIVER fluxes come from the interface kernel through the face ->
// queue slot map.  Blocks are renumbered so that each XCD receives a
// contiguous run of neighbouring tiles (halo reuse in its L2).
#include "m2c_device.h"
#include "m2c_internal.h"
#include "m2c_kernels.h"

namespace m2c {

// Flux through a face with normal axis D from the two reconstructed face
// states given in global component order (rho, u, v, w, p); result in global
// order (mass, x-, y-, z-momentum, energy).
template <int D, typename T>
__device__ __forceinline__ void face_flux(const T qa[5], const T qb[5], T g, T pc, T gpc, T igm1, T F[5])
{
    constexpr int N = 1 + D, T1 = 1 + (D + 1) % 3, T2 = 1 + (D + 2) % 3;
    T Fr[5];
    hllc<T>(qa[0], qa[N], qa[T1], qa[T2], qa[4], qb[0], qb[N], qb[T1], qb[T2], qb[4], g, pc, gpc, igm1, Fr);
    F[0] = Fr[0];
    F[N] = Fr[1];
    F[T1] = Fr[2];
    F[T2] = Fr[3];
    F[4] = Fr[4];
}

template <int STAGE, int TX, int TY, typename TF>
__global__ __launch_bounds__(TX * TY) void k_stage(const StageArgs a)
{
    constexpr int NT = TX * TY, LX = TX + 4, LY = TY + 4;
    constexpr int NXF = (TX + 1) * TY, NYF = TX * (TY + 1);
    __shared__ double sQ[6][LY][LX];
    __shared__ uint8_t sX[LY][LX];
    __shared__ double sFx[5][TY][TX + 1];
    __shared__ double sFy[5][TY + 1][TX];
    __shared__ int sSx[TY][TX + 1];
    __shared__ int sSy[TY + 1][TX];
    __shared__ double sRed[NT / 64];
    __shared__ int sErr;

    // Skip the launch when an earlier kernel of the step failed; the flag is
    // read once per block so that the whole block takes the same branch
    // (other blocks of this launch may raise it meanwhile).
    DevScalars* sc = a.sc;
    if (threadIdx.x == 0) sErr = sc->err;
    __syncthreads();
    if (sErr != 0) return;
    const Grid& G = a.g;
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const long long N = G.N;
    const bool xact = G.act[0], yact = G.act[1], zact = G.act[2];
    const double* __restrict__ Win = a.Win;
    const uint8_t* __restrict__ chi = a.chi;

    // ---- XCD-aware tile numbering (dispatch is round-robin over 8 XCDs) --
    const int nblk = gridDim.x;
    const int bq = nblk / 8, br = nblk % 8;
    const int xcd = blockIdx.x % 8, idx = blockIdx.x / 8;
    const int tile = (xcd < br ? xcd * (bq + 1) : br * (bq + 1) + (xcd - br) * bq) + idx;
    const int bx = tile % a.tiles_x;
    const int rest = tile / a.tiles_x;
    const int by = rest % a.tiles_y;
    const int bz = rest / a.tiles_y;
    const int i0 = bx * TX, j0 = by * TY;
    const int kz0 = bz * a.kz, kz1 = min(nz, kz0 + a.kz);

    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int gi = i0 + tx, gj = j0 + ty;
    const bool inside = gi < nx && gj < ny;
    bool mirx = false, miry = false;
    const int si = bc_index(gi, nx, G.bc[0], G.bc[1], mirx);
    const int sj = bc_index(gj, ny, G.bc[2], G.bc[3], miry);
    if (!xact) mirx = false;
    if (!yact) miry = false;
    const long long sxy = (long long)nx * ny;
    const long long col = si + (long long)nx * sj;

    const TF alpha = (TF)G.alpha;

    // Load one cell of this thread's column at plane k (any k in [-2, nz+1]).
    auto load_col = [&](int k, double q[5], double w[6], uint8_t& x) {
        bool mz = false;
        const int sk = bc_index(k, nz, G.bc[4], G.bc[5], mz);
        const long long c = col + sxy * sk;
#pragma unroll
        for (int v = 0; v < 6; ++v) w[v] = Win[v * N + c];
        x = chi[c];
        double u, vv, ww;
        const double p = eos_prim(w[0], w[1], w[2], w[3], w[4], G.gamma[x] - 1.0, G.gpc[x], u, vv, ww);
        q[0] = w[0];
        q[1] = mirx ? -u : u;
        q[2] = miry ? -vv : vv;
        q[3] = (mz && zact) ? -ww : ww;
        q[4] = p;
    };

    // z-slope of a cell from its column neighbours (zero next to another
    // material along z).
    auto zslope = [&](const double qm[5], const double q0[5], const double qp[5],
                      uint8_t xm, uint8_t x0, uint8_t xp, TF s[5]) {
        const bool flat = (xm != x0) || (xp != x0);
#pragma unroll
        for (int v = 0; v < 5; ++v)
            s[v] = flat ? TF(0) : mc_slope<TF>(TF(q0[v] - qm[v]), TF(qp[v] - q0[v]), alpha);
    };

    // z-face between planes k (lower) and k+1 of this column: flux seen by the
    // lower cell (Fl) and by the upper cell (Fu).
    auto zface = [&](int k, const double ql[5], const TF sl[5], uint8_t xl,
                     const double qu[5], const TF su[5], uint8_t xu, double Fl[5], double Fu[5]) {
        if (xl == xu) {
            TF fa[5], fb[5], F[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                fa[v] = TF(ql[v]) + TF(0.5) * sl[v];
                fb[v] = TF(qu[v]) - TF(0.5) * su[v];
            }
            face_flux<2, TF>(fa, fb, TF(G.gamma[xl]), TF(G.pc[xl]), TF(G.gpc[xl]), TF(G.inv_gm1[xl]), F);
#pragma unroll
            for (int v = 0; v < 5; ++v) Fl[v] = Fu[v] = (double)F[v];
        } else {
            bool m;
            const int lk = bc_index(k, nz, G.bc[4], G.bc[5], m);
            const long long fid = 3 * (col + sxy * lk) + 2;
            const int q = a.fslot[fid];
            if (q < 0) {
                report_error(&sc->err, &sc->err_cell, ST_NONPHYSICAL, fid / 3);
#pragma unroll
                for (int v = 0; v < 5; ++v) Fl[v] = Fu[v] = 0.0;
                return;
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                Fl[v] = a.fluxF[v * a.qcap + q];
                Fu[v] = a.fluxF[(5 + v) * a.qcap + q];
            }
        }
    };

    // ---- prologue: column window and the z-face below plane kz0 ----------
    double Q0[5], Q1[5], Q2[5];       // primitives at k, k+1, k+2
    double W0c[6], W1c[6], W2c[6];    // stage-input state at k, k+1, k+2
    double PH[5];                     // phi at k-2 .. k+2
    uint8_t Xm, X0, X1, X2;           // ids at k-1 .. k+2
    TF S0[5];                         // z-slope of plane k
    double Fzlo[5];                   // flux seen by plane k through its lower z-face
    {
        double qm2[5], qm1[5], w[6];
        uint8_t xm2;
        load_col(kz0 - 2, qm2, w, xm2);
        PH[0] = w[5];
        load_col(kz0 - 1, qm1, w, Xm);
        PH[1] = w[5];
        load_col(kz0, Q0, W0c, X0);
        PH[2] = W0c[5];
        load_col(kz0 + 1, Q1, W1c, X1);
        PH[3] = W1c[5];
        load_col(kz0 + 2, Q2, W2c, X2);
        PH[4] = W2c[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) Fzlo[v] = 0.0;
        if (zact) {
            zslope(qm1, Q0, Q1, Xm, X0, X1, S0);
            if (inside) {
                // slope of plane kz0-1 needs plane kz0-2
                TF Sm[5];
                zslope(qm2, qm1, Q0, xm2, Xm, X0, Sm);
                double Fl[5];
                zface(kz0 - 1, qm1, Sm, Xm, Q0, S0, X0, Fl, Fzlo);
            }
        } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) S0[v] = TF(0);
        }
    }

    const double dt = sc->dt;
    double lam = 0.0;                 // stage 2: max wave-speed sum of own cells

    for (int k = kz0; k < kz1; ++k) {
        // lead load of plane k+3 (consumed at the end of the iteration)
        double Qn[5], Wn[6];
        uint8_t Xn;
        if (zact) load_col(k + 3, Qn, Wn, Xn);

        // (1) own plane-k values into the LDS tile
#pragma unroll
        for (int v = 0; v < 5; ++v) sQ[v][ty + 2][tx + 2] = Q0[v];
        sQ[5][ty + 2][tx + 2] = PH[2];
        sX[ty + 2][tx + 2] = X0;

        // (2) halo ring of plane k (x-halo: 4 columns x TY rows; y-halo: 4 rows x TX columns)
        {
            const int nxh = xact ? 4 * TY : 0, nyh = yact ? 4 * TX : 0;
            bool mz;
            const int sk = bc_index(k, nz, G.bc[4], G.bc[5], mz);
            for (int h = tid; h < nxh + nyh; h += NT) {
                int li, lj;
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
                bool mx = false, my = false;
                const int hi_ = bc_index(i0 + li - 2, nx, G.bc[0], G.bc[1], mx);
                const int hj_ = bc_index(j0 + lj - 2, ny, G.bc[2], G.bc[3], my);
                const long long c = hi_ + (long long)nx * hj_ + sxy * sk;
                const uint8_t x = chi[c];
                double u, vv, ww;
                const double r0 = Win[c];
                const double p = eos_prim(r0, Win[N + c], Win[2 * N + c], Win[3 * N + c], Win[4 * N + c],
                                          G.gamma[x] - 1.0, G.gpc[x], u, vv, ww);
                sQ[0][lj][li] = r0;
                sQ[1][lj][li] = (mx && xact) ? -u : u;
                sQ[2][lj][li] = (my && yact) ? -vv : vv;
                sQ[3][lj][li] = ww;
                sQ[4][lj][li] = p;
                sQ[5][lj][li] = Win[5 * N + c];
                sX[lj][li] = x;
            }
        }
        __syncthreads();

        // (3) x- and y-faces of the tile as one work list
        {
            const int nxf = xact ? NXF : 0, nyf = yact ? NYF : 0;
            for (int t = tid; t < nxf + nyf; t += NT) {
                if (t < nxf) {
                    const int fi = t % (TX + 1), lj = t / (TX + 1);
                    const int gx = i0 + fi, gy = j0 + lj;
                    if (gx > nx || gy >= ny) continue;
                    const int r = lj + 2, ca = fi + 1, cb = fi + 2;
                    const uint8_t xa = sX[r][ca], xb = sX[r][cb];
                    if (xa == xb) {
                        const bool fa = sX[r][ca - 1] != xa, fb = sX[r][cb + 1] != xb;
                        TF qa[5], qb[5], F[5];
#pragma unroll
                        for (int v = 0; v < 5; ++v) {
                            const double m1 = sQ[v][r][ca - 1], a0 = sQ[v][r][ca];
                            const double b0 = sQ[v][r][cb], p1 = sQ[v][r][cb + 1];
                            const TF sa = fa ? TF(0) : mc_slope<TF>(TF(a0 - m1), TF(b0 - a0), alpha);
                            const TF sb = fb ? TF(0) : mc_slope<TF>(TF(b0 - a0), TF(p1 - b0), alpha);
                            qa[v] = TF(a0) + TF(0.5) * sa;
                            qb[v] = TF(b0) - TF(0.5) * sb;
                        }
                        face_flux<0, TF>(qa, qb, TF(G.gamma[xa]), TF(G.pc[xa]), TF(G.gpc[xa]), TF(G.inv_gm1[xa]), F);
#pragma unroll
                        for (int v = 0; v < 5; ++v) sFx[v][lj][fi] = (double)F[v];
                        sSx[lj][fi] = -1;
                    } else {
                        bool m;
                        const int lx = bc_index(gx - 1, nx, G.bc[0], G.bc[1], m);
                        const long long fid = 3 * (lx + (long long)nx * gy + sxy * k);
                        const int q = a.fslot[fid];
                        if (q < 0) report_error(&sc->err, &sc->err_cell, ST_NONPHYSICAL, fid / 3);
                        const int qq = q < 0 ? 0 : q;
#pragma unroll
                        for (int v = 0; v < 5; ++v) sFx[v][lj][fi] = a.fluxF[v * a.qcap + qq];
                        sSx[lj][fi] = qq;
                    }
                } else {
                    const int tt = t - nxf;
                    const int li = tt % TX, fj = tt / TX;
                    const int gx = i0 + li, gy = j0 + fj;
                    if (gx >= nx || gy > ny) continue;
                    const int c = li + 2, ra = fj + 1, rb = fj + 2;
                    const uint8_t xa = sX[ra][c], xb = sX[rb][c];
                    if (xa == xb) {
                        const bool fa = sX[ra - 1][c] != xa, fb = sX[rb + 1][c] != xb;
                        TF qa[5], qb[5], F[5];
#pragma unroll
                        for (int v = 0; v < 5; ++v) {
                            const double m1 = sQ[v][ra - 1][c], a0 = sQ[v][ra][c];
                            const double b0 = sQ[v][rb][c], p1 = sQ[v][rb + 1][c];
                            const TF sa = fa ? TF(0) : mc_slope<TF>(TF(a0 - m1), TF(b0 - a0), alpha);
                            const TF sb = fb ? TF(0) : mc_slope<TF>(TF(b0 - a0), TF(p1 - b0), alpha);
                            qa[v] = TF(a0) + TF(0.5) * sa;
                            qb[v] = TF(b0) - TF(0.5) * sb;
                        }
                        face_flux<1, TF>(qa, qb, TF(G.gamma[xa]), TF(G.pc[xa]), TF(G.gpc[xa]), TF(G.inv_gm1[xa]), F);
#pragma unroll
                        for (int v = 0; v < 5; ++v) sFy[v][fj][li] = (double)F[v];
                        sSy[fj][li] = -1;
                    } else {
                        bool m;
                        const int ly = bc_index(gy - 1, ny, G.bc[2], G.bc[3], m);
                        const long long fid = 3 * (gx + (long long)nx * ly + sxy * k) + 1;
                        const int q = a.fslot[fid];
                        if (q < 0) report_error(&sc->err, &sc->err_cell, ST_NONPHYSICAL, fid / 3);
                        const int qq = q < 0 ? 0 : q;
#pragma unroll
                        for (int v = 0; v < 5; ++v) sFy[v][fj][li] = a.fluxF[v * a.qcap + qq];
                        sSy[fj][li] = qq;
                    }
                }
            }
        }

        // (4) z-face above plane k for this column
        TF S1[5];
        double Fzhi[5], Fzup[5];
        if (zact) {
            zslope(Q0, Q1, Q2, X0, X1, X2, S1);
            if (inside) zface(k, Q0, S0, X0, Q1, S1, X1, Fzhi, Fzup);
        }
        __syncthreads();

        // (5) residual and stage update of cell (gi, gj, k)
        if (inside) {
            const long long c = col + sxy * k;
            double acc[5];
            if (xact) {
                const int ql = sSx[ty][tx];
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    const double lo = ql >= 0 ? a.fluxF[(5 + v) * a.qcap + ql] : sFx[v][ty][tx];
                    acc[v] = (sFx[v][ty][tx + 1] - lo) * G.rh[0];
                }
            } else {
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[v] = 0.0;
            }
            if (yact) {
                const int ql = sSy[ty][tx];
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    const double lo = ql >= 0 ? a.fluxF[(5 + v) * a.qcap + ql] : sFy[v][ty][tx];
                    acc[v] += (sFy[v][ty + 1][tx] - lo) * G.rh[1];
                }
            }
            if (zact) {
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[v] += (Fzhi[v] - Fzlo[v]) * G.rh[2];
            }
            // level set: third-order upwind-biased differences, upwinded by V_d of the cell
            double Ls = 0.0;
            auto ls_term = [&](double V, double f0, double f1, double f2, double f3, double f4, double rh6) {
                const double D = V > 0.0 ? (2.0 * f3 + 3.0 * f2 - 6.0 * f1 + f0) * rh6
                               : (V < 0.0 ? (-f4 + 6.0 * f3 - 3.0 * f2 - 2.0 * f1) * rh6 : 0.0);
                return V * D;
            };
            if (xact)
                Ls += ls_term(Q0[1], sQ[5][ty + 2][tx], sQ[5][ty + 2][tx + 1], sQ[5][ty + 2][tx + 2],
                              sQ[5][ty + 2][tx + 3], sQ[5][ty + 2][tx + 4], G.rh6[0]);
            if (yact)
                Ls += ls_term(Q0[2], sQ[5][ty][tx + 2], sQ[5][ty + 1][tx + 2], sQ[5][ty + 2][tx + 2],
                              sQ[5][ty + 3][tx + 2], sQ[5][ty + 4][tx + 2], G.rh6[1]);
            if (zact) Ls += ls_term(Q0[3], PH[0], PH[1], PH[2], PH[3], PH[4], G.rh6[2]);

            double wn[6];
            if (STAGE == 1) {
#pragma unroll
                for (int v = 0; v < 5; ++v) wn[v] = W0c[v] + dt * (-acc[v]);
                wn[5] = W0c[5] + dt * (-Ls);
            } else {
#pragma unroll
                for (int v = 0; v < 5; ++v) wn[v] = 0.5 * a.W0[v * N + c] + 0.5 * (W0c[v] + dt * (-acc[v]));
                wn[5] = 0.5 * a.W0[5 * N + c] + 0.5 * (W0c[5] + dt * (-Ls));
            }
            double u, vv, ww;
            const double p = eos_prim(wn[0], wn[1], wn[2], wn[3], wn[4], G.gamma[X0] - 1.0, G.gpc[X0], u, vv, ww);
            const bool ok = wn[0] > 0.0 && p + G.pc[X0] > 0.0 && isfinite(p) && isfinite(u) && isfinite(vv) &&
                            isfinite(ww) && isfinite(wn[5]);
            if (!ok) report_error(&sc->err, &sc->err_cell, ST_NONPHYSICAL, c);
#pragma unroll
            for (int v = 0; v < 6; ++v) a.Wout[v * N + c] = wn[v];
            if (STAGE == 2) {
                const uint8_t xn = wn[5] < 0.0 ? 1 : 0;
                a.chi_next[c] = xn;
                if (xn != X0) {
                    const int slot = atomicAdd(&sc->nflip, 1);
                    a.flips[slot] = (int)c;
                } else if (ok) {
                    const double cs = sqrt(G.gamma[X0] * (p + G.pc[X0]) / wn[0]);
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
                Fzlo[v] = Fzup[v];
            }
#pragma unroll
            for (int v = 0; v < 6; ++v) {
                W0c[v] = W1c[v];
                W1c[v] = W2c[v];
                W2c[v] = Wn[v];
            }
            PH[0] = PH[1];
            PH[1] = PH[2];
            PH[2] = PH[3];
            PH[3] = PH[4];
            PH[4] = Wn[5];
            Xm = X0;
            X0 = X1;
            X1 = X2;
            X2 = Xn;
        }
        __syncthreads();
    }

    if (STAGE == 2) {
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

// ---- launcher ---------------------------------------------------------------
template <int TX, int TY, typename TF>
static hipError_t launch_tile(int stage, const StageArgs& a, hipStream_t s)
{
    const int nblk = a.tiles_x * a.tiles_y * a.tiles_z;
    if (stage == 1)
        hipLaunchKernelGGL((k_stage<1, TX, TY, TF>), dim3(nblk), dim3(TX * TY), 0, s, a);
    else
        hipLaunchKernelGGL((k_stage<2, TX, TY, TF>), dim3(nblk), dim3(TX * TY), 0, s, a);
    return hipGetLastError();
}

bool stage_tile_supported(int tx, int ty)
{
    return (tx == 32 && ty == 8) || (tx == 64 && ty == 4) || (tx == 16 && ty == 16) ||
           (tx == 32 && ty == 4) || (tx == 64 && ty == 2);
}

hipError_t launch_stage(int stage, bool mixed, int tx, int ty, const StageArgs& a, hipStream_t s)
{
#define M2C_TILE(TX_, TY_)                                                              \
    if (tx == TX_ && ty == TY_)                                                         \
        return mixed ? launch_tile<TX_, TY_, float>(stage, a, s) : launch_tile<TX_, TY_, double>(stage, a, s);
    M2C_TILE(32, 8)
    M2C_TILE(64, 4)
    M2C_TILE(16, 16)
    M2C_TILE(32, 4)
    M2C_TILE(64, 2)
#undef M2C_TILE
    return hipErrorInvalidValue;
}

}  // namespace m2c
