// Fused two-phase SMAME step (2D) for gfx950: flow update with the
// surface-tension force, and the Cahn-Hilliard equation (Eq. 2.14) advanced
// by Heun's second-order Runge-Kutta method, all in one launch.
//
// Per step and node (Sec. 2, two-phase paragraphs):
//   mu     = 4 a phi (phi^2 - 1) - kappa L_iso phi
//   flow   = single-phase update (Eqs. 2.10-2.11) + force -dt phi G_iso mu
//   R(f,m) = M L_iso m - (u G_iso,x f + v G_iso,y f)        (u = u^n)
//   phi*   = phi + dt R(phi, mu)
//   phi^{n+1} = (phi + phi* + dt R(phi*, mu*)) / 2,   mu* = mu(phi*)
// with the D2Q9-weighted isotropic stencils
//   G_iso,x f = [4 (f_E - f_W) + (f_NE + f_SE - f_NW - f_SW)] / (12 dx)
//   L_iso f   = [4 (f_E + f_W + f_N + f_S) + (f_NE + f_NW + f_SE + f_SW) - 20 f] / (6 dx^2).
// AXI = true is the axisymmetric form (x axial, y radial, axis on the -y
// face, row j at r = (j + 1/2) dx): L_iso gains (1/r) G_iso,r in mu and in
// the Cahn-Hilliard diffusion, continuity and momentum take the
// cylindrical flux forms of the single-phase axisymmetric step
// (kern_axisym.h); the advection and the surface-tension force are
// unchanged.
// Dependency radii: phi needs a 4-node halo (mu on tile+3, phi* on tile+2,
// mu* on tile+1), the flow fields a 2-node halo.  Ghost positions of every
// intermediate take the value at their mirror node for walls and symmetry
// planes, so they are computed there; phi and phi* ghosts across a wall
// then take the wetting rule of Sec. 2 (identity for a 90 degree angle).
// LDS: phi^n and mu^n are last read in the phi* phase (which also takes
// each output node's phi^n and surface-tension force into registers), so
// mu* and drho' are written over them afterwards; 18.7 KB per 32 x 16 tile
// lets eight workgroups share a CU.
#include "acm_internal.h"
#include "kern_axisym.h"
#include "tile2d.h"

namespace acm {

template <typename T>
__device__ __forceinline__ T momc2(T r, T u, T rho0) { return fmaT(r, u, rho0 * u); }

template <int TX, int TY>
struct Shape2P {
    static constexpr int PX = TX + 8, PY = TY + 8, PXY = PX * PY;   // phi, halo 4
    static constexpr int MX = TX + 6, MY = TY + 6, MXY = MX * MY;   // mu, halo 3
    static constexpr int RX = TX + 4, RY = TY + 4, RXY = RX * RY;   // flow fields / phi*, halo 2
    static constexpr int DX = TX + 2, DY = TY + 2, DXY = DX * DY;   // mu*, drho', halo 1
    static_assert(DXY <= PXY && DXY <= MXY, "mu* and drho' fit in the phi and mu regions");
};

// isotropic Laplacian numerator: 4 (E+W+N+S) + (NE+NW+SE+SW) - 20 C
template <typename T, int W>
__device__ __forceinline__ T liso_num(const T* f, int e)
{
    const T ax = (f[e + 1] + f[e - 1]) + (f[e + W] + f[e - W]);
    const T dg = (f[e + 1 + W] + f[e - 1 + W]) + (f[e + 1 - W] + f[e - 1 - W]);
    return fmaT(T(4), ax, dg) - T(20) * f[e];
}
template <typename T, int W>
__device__ __forceinline__ T gisox_num(const T* f, int e)
{
    return fmaT(T(4), f[e + 1] - f[e - 1], (f[e + 1 + W] + f[e + 1 - W]) - (f[e - 1 + W] + f[e - 1 - W]));
}
template <typename T, int W>
__device__ __forceinline__ T gisoy_num(const T* f, int e)
{
    return fmaT(T(4), f[e + W] - f[e - W], (f[e + 1 + W] + f[e - 1 + W]) - (f[e + 1 - W] + f[e - 1 - W]));
}

// chemical potential from a phi array of row width W at index e
template <typename T, int W>
__device__ __forceinline__ T chem(const Coef<T>& c, const T* f, int e)
{
    const T p = f[e];
    return fmaT(c.a4 * p, fmaT(p, p, T(-1)), -c.kap6 * liso_num<T, W>(f, e));
}

// chemical potential with the cylindrical Laplacian when AXI (irc =
// 1 / (row + 1/2)): -kappa (1/r) G_iso,r phi = -(kappa / 6 dx^2) irc gy / 2
template <typename T, int W, bool AXI>
__device__ __forceinline__ T chem_a(const Coef<T>& c, const T* f, int e, T irc)
{
    const T m = chem<T, W>(c, f, e);
    if constexpr (AXI) return fmaT(T(-0.5) * c.kap6 * irc, gisoy_num<T, W>(f, e), m);
    else return m;
}

// numerator of the (cylindrical when AXI) isotropic Laplacian in units of
// 1 / (6 dx^2): L_iso + (1/r) G_iso,r = [liso_num + irc gy_num / 2] / (6 dx^2)
template <typename T, int W, bool AXI>
__device__ __forceinline__ T lap_a(const T* f, int e, T irc)
{
    if constexpr (AXI) return fmaT(T(0.5) * irc, gisoy_num<T, W>(f, e), liso_num<T, W>(f, e));
    else return liso_num<T, W>(f, e);
}

template <bool AXI, typename T>
__device__ __forceinline__ T inv_radius(int row)
{
    if constexpr (AXI) return T(1) / (T(row) + T(0.5));
    else return T(0);
}

// local coordinate (in a region with halo h) whose value stands in for the
// position l: the mirror node for wall / symmetry ghosts, else l itself
__device__ __forceinline__ int ghost_src(int l, int h, int o0, int n, int bc_lo, int lo, int hi)
{
    const int g = mirror_coord(o0 + l - h, n, bc_lo);
    return min(max(g - o0 + h, lo), hi);
}

template <typename T, int TX, int TY, int NT, bool AXI>
__global__ __launch_bounds__(NT) void twophase2d_kernel(Coef<T> c, State<T> in, State<T> out, int nbx)
{
    using S = Shape2P<TX, TY>;
    constexpr int PX = S::PX, MX = S::MX, RX = S::RX, DX = S::DX;
    __shared__ T sp[S::PXY];                          // phi^n, then mu*
    __shared__ T smu[S::MXY];                         // mu^n, then drho'
    __shared__ T sr[S::RXY], su[S::RXY], sv[S::RXY];  // drho, u, v
    __shared__ T sps[S::RXY];                         // phi*
    T* const sms = sp;
    T* const srn = smu;
    constexpr int NQ = (TX * TY + NT - 1) / NT;       // output nodes per thread
    T pcq[NQ], fsx[NQ], fsy[NQ];                      // phi^n and surface-tension force there

    const int lb = [&] {
        constexpr int NX = 8;
        const int nb = gridDim.x, b = blockIdx.x;
        const int per = nb / NX, rem = nb % NX;
        const int x = b % NX, i = b / NX;
        return x * per + min(x, rem) + i;
    }();
    const int by = lb / nbx, bx = lb - by * nbx;
    const int x0 = bx * TX, y0 = by * TY;
    const int nx = c.nx, ny = c.ny;
    const bool interior = (x0 >= 4) && (x0 + TX + 4 <= nx) && (y0 >= 4) && (y0 + TY + 4 <= ny);
    const bool mirror = !interior && c.nonperiodic;
    const int tid = threadIdx.x;

    // ---- stage phi (halo 4) and drho, u, v (halo 2); every load of the
    // thread is issued before its first LDS store so the latencies overlap
    {
        constexpr int NP = (S::PXY + NT - 1) / NT, NR = (S::RXY + NT - 1) / NT;
        T pv[NP], rv[NR], uv[NR], vv[NR];
        int fxs[NR], fys[NR];
        if (interior) {  // no ghost in either region: plain offsets
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int q = min(tid + i * NT, S::PXY - 1);
                const int ly = q / PX, lx = q - ly * PX;
                pv[i] = in.phi[(size_t)(y0 + ly - 4) * nx + (x0 + lx - 4)];
            }
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const int q = min(tid + i * NT, S::RXY - 1);
                const int ly = q / RX, lx = q - ly * RX;
                const size_t s = (size_t)(y0 + ly - 2) * nx + (x0 + lx - 2);
                rv[i] = in.r[s];
                uv[i] = in.u[s];
                vv[i] = in.v[s];
                fxs[i] = fys[i] = -1;
            }
        } else {
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int q = min(tid + i * NT, S::PXY - 1);
                const int ly = q / PX, lx = q - ly * PX;
                int fx, fy;
                const int sx = map_coord(x0 + lx - 4, nx, c.bc[0], 0, fx);
                const int sy = map_coord(y0 + ly - 4, ny, c.bc[2], 2, fy);
                pv[i] = in.phi[(size_t)sy * nx + sx];
                if (c.wet) {  // wetting rule across wall faces, x then y
                    if (fx >= 0) pv[i] = wet_ghost(pv[i], wet_b(c, fx));
                    if (fy >= 0) pv[i] = wet_ghost(pv[i], wet_b(c, fy));
                }
            }
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                const int q = min(tid + i * NT, S::RXY - 1);
                const int ly = q / RX, lx = q - ly * RX;
                const int sx = map_coord(x0 + lx - 2, nx, c.bc[0], 0, fxs[i]);
                const int sy = map_coord(y0 + ly - 2, ny, c.bc[2], 2, fys[i]);
                const size_t s = (size_t)sy * nx + sx;
                rv[i] = in.r[s];
                uv[i] = in.u[s];
                vv[i] = in.v[s];
            }
        }
#pragma unroll
        for (int i = 0; i < NP; ++i)
            if (tid + i * NT < S::PXY) sp[tid + i * NT] = pv[i];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int q = tid + i * NT;
            if (q < S::RXY) {
                T u = uv[i], v = vv[i];
                const int fx = fxs[i], fy = fys[i];
                if (fx >= 0) {
                    u = fmaT(c.fs[fx][0], u, c.fo[fx][0]);
                    v = fmaT(c.fs[fx][1], v, c.fo[fx][1]);
                }
                if (fy >= 0) {
                    u = fmaT(c.fs[fy][0], u, c.fo[fy][0]);
                    v = fmaT(c.fs[fy][1], v, c.fo[fy][1]);
                }
                sr[q] = rv[i];
                su[q] = u;
                sv[q] = v;
            }
        }
    }
    __syncthreads();

    // ---- mu^n on tile+3
#pragma unroll
    for (int q = tid; q < S::MXY; q += NT) {
        const int ly = q / MX, lx = q - ly * MX;
        int ex = lx + 1, ey = ly + 1;  // phi-region coordinates
        if (mirror) {
            ex = ghost_src(lx, 3, x0, nx, c.bc[0], 0, MX - 1) + 1;
            ey = ghost_src(ly, 3, y0, ny, c.bc[2], 0, S::MY - 1) + 1;
        }
        smu[q] = chem_a<T, PX, AXI>(c, sp, ey * PX + ex, inv_radius<AXI, T>(y0 + ey - 4));
    }
    __syncthreads();

    // ---- phi* on tile+2
#pragma unroll
    for (int q = tid; q < S::RXY; q += NT) {
        const int ly = q / RX, lx = q - ly * RX;
        int ex = lx, ey = ly;  // flow-region coordinates of the evaluation node
        if (mirror) {
            ex = ghost_src(lx, 2, x0, nx, c.bc[0], 0, RX - 1);
            ey = ghost_src(ly, 2, y0, ny, c.bc[2], 0, S::RY - 1);
        }
        const int ep = (ey + 2) * PX + (ex + 2);  // phi region
        const int em = (ey + 1) * MX + (ex + 1);  // mu region
        const int ef = ey * RX + ex;
        const T gxp = gisox_num<T, PX>(sp, ep), gyp = gisoy_num<T, PX>(sp, ep);
        const T adv = fmaT(su[ef], gxp, sv[ef] * gyp) * c.gi;
        const T rhs = fmaT(c.mob * c.li, lap_a<T, MX, AXI>(smu, em, inv_radius<AXI, T>(y0 + ey - 2)), -adv);
        T val = fmaT(c.dt, rhs, sp[ep]);
        if (mirror && c.wet) {  // a ghost position takes the wetting rule of its wall faces
            const int gx = x0 + lx - 2, gy = y0 + ly - 2;
            if (gx < 0) val = wet_ghost(val, c.wb[0]);
            if (gx >= nx) val = wet_ghost(val, c.wb[1]);
            if (gy < 0) val = wet_ghost(val, c.wb[2]);
            if (gy >= ny) val = wet_ghost(val, c.wb[3]);
        }
        sps[q] = val;
    }
    // phi^n and the surface-tension force -dt phi G_iso mu at this thread's
    // output nodes, while phi^n and mu^n are still in LDS
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const int q = min(tid + k * NT, TX * TY - 1);
        const int ly = q / TX, lx = q - ly * TX;
        const int ep = (ly + 4) * PX + (lx + 4);  // phi region
        const int em = (ly + 3) * MX + (lx + 3);  // mu region
        const T pc = sp[ep];
        pcq[k] = pc;
        fsx[k] = -c.dt * pc * (gisox_num<T, MX>(smu, em) * c.gi);
        fsy[k] = -c.dt * pc * (gisoy_num<T, MX>(smu, em) * c.gi);
    }
    __syncthreads();

    // ---- mu* on tile+1 (over phi^n) and drho' on tile+1 (over mu^n)
#pragma unroll
    for (int q = tid; q < S::DXY; q += NT) {
        const int ly = q / DX, lx = q - ly * DX;
        int ex = lx + 1, ey = ly + 1;  // phi*-region coordinates
        if (mirror) {
            ex = ghost_src(lx, 1, x0, nx, c.bc[0], 0, DX - 1) + 1;
            ey = ghost_src(ly, 1, y0, ny, c.bc[2], 0, S::DY - 1) + 1;
        }
        sms[q] = chem_a<T, RX, AXI>(c, sps, ey * RX + ex, inv_radius<AXI, T>(y0 + ey - 2));
    }
#pragma unroll
    for (int q = tid; q < S::DXY; q += NT) {
        const int ly = q / DX, lx = q - ly * DX;
        int ex = lx + 1, ey = ly + 1;  // flow-region coordinates
        if (mirror) {
            ex = ghost_src(lx, 1, x0, nx, c.bc[0], 0, DX - 1) + 1;
            ey = ghost_src(ly, 1, y0, ny, c.bc[2], 0, S::DY - 1) + 1;
        }
        const int e = ey * RX + ex;
        const T rc = sr[e];
        const T rE = sr[e + 1], rW = sr[e - 1], rN = sr[e + RX], rS = sr[e - RX];
        T div, lap;
        if constexpr (AXI) {  // cylindrical flux forms (kern_axisym.h)
            axi_continuity(c.rho0, T(y0 + ey - 2), inv_radius<AXI, T>(y0 + ey - 2), rc, rE, rW, rN, rS, su[e + 1],
                           su[e - 1], sv[e], sv[e + RX], sv[e - RX], div, lap);
        } else {
            div = mdiff(rE, su[e + 1], rW, su[e - 1], c.rho0) + mdiff(rN, sv[e + RX], rS, sv[e - RX], c.rho0);
            lap = ((rE + rW) + (rN + rS)) - T(4) * rc;
        }
        srn[q] = fmaT(-c.cg, div, fmaT(c.kr, lap, rc));
    }
    __syncthreads();

    // ---- outputs on the tile
    const T rho0 = c.rho0, cs2 = c.cs2;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const int q = tid + k * NT;
        if (q >= TX * TY) break;
        const int ly = q / TX, lx = q - ly * TX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= nx || gy >= ny) continue;
        const int e = (ly + 2) * RX + (lx + 2);   // flow / phi* region
        const int d = (ly + 1) * DX + (lx + 1);   // drho' / mu* region
        // flow
        const T rc = sr[e], uc = su[e], vc = sv[e];
        const T rE = sr[e + 1], rW = sr[e - 1], rN = sr[e + RX], rS = sr[e - RX];
        const T uE = su[e + 1], uW = su[e - 1], uN = su[e + RX], uS = su[e - RX];
        const T vE = sv[e + 1], vW = sv[e - 1], vN = sv[e + RX], vS = sv[e - RX];
        const T mxC = momc2(rc, uc, rho0), myC = momc2(rc, vc, rho0);
        const T mxE = momc2(rE, uE, rho0), mxW = momc2(rW, uW, rho0);
        const T mxN = momc2(rN, uN, rho0), mxS = momc2(rS, uS, rho0);
        const T myE = momc2(rE, vE, rho0), myW = momc2(rW, vW, rho0);
        const T myN = momc2(rN, vN, rho0), myS = momc2(rS, vS, rho0);
        const T rnC = srn[d];
        const T irc = inv_radius<AXI, T>(gy);
        T fxx, fyy, lpx, lpy;
        if constexpr (AXI) {  // cylindrical flux forms, hoop term, -m_r / r^2 (kern_axisym.h)
            axi_momentum(cs2, T(gy), irc, rc, rE, rW, rN, rS, uE, uW, vc, vN, vS, mxC, mxE, mxW, mxN, mxS, myC, myE,
                         myW, myN, myS, fxx, fyy, lpx, lpy);
        } else {
            fxx = (fmaT(mxE, uE, cs2 * rE) - fmaT(mxW, uW, cs2 * rW)) + (mxN * vN - mxS * vS);
            fyy = (myE * uE - myW * uW) + (fmaT(myN, vN, cs2 * rN) - fmaT(myS, vS, cs2 * rS));
            lpx = ((mxE + mxW) + (mxN + mxS)) - T(4) * mxC;
            lpy = ((myE + myW) + (myN + myS)) - T(4) * myC;
        }
        const T sx = (srn[d + 1] - srn[d - 1]) - (rE - rW);
        const T sy = (srn[d + DX] - srn[d - DX]) - (rN - rS);
        const T rho_n = rho0 + rnC;
        const T pc = pcq[k], fstx = fsx[k], fsty = fsy[k];
        T gx_ = c.gdt[0];
        if (c.fx) gx_ = fmaT(c.dt, c.fx[gy], gx_);
        const T dmx = fmaT(rho_n, gx_, fmaT(-c.ks, sx, fmaT(c.kv, lpx, fmaT(-c.cg, fxx, fstx))));
        const T dmy = fmaT(rho_n, c.gdt[1], fmaT(-c.ks, sy, fmaT(c.kv, lpy, fmaT(-c.cg, fyy, fsty))));
        const T drn = rnC - rc;
        const T inv = recipT(rho_n);
        // Cahn-Hilliard second stage
        const T gxs = gisox_num<T, RX>(sps, e), gys = gisoy_num<T, RX>(sps, e);
        const T adv = fmaT(uc, gxs, vc * gys) * c.gi;
        const T rhs = fmaT(c.mob * c.li, lap_a<T, DX, AXI>(sms, d, irc), -adv);
        const T phin = T(0.5) * fmaT(c.dt, rhs, pc + sps[e]);
        const size_t o = (size_t)gy * nx + gx;
        out.r[o] = rnC;
        out.u[o] = fmaT(fmaT(-uc, drn, dmx), inv, uc);
        out.v[o] = fmaT(fmaT(-vc, drn, dmy), inv, vc);
        out.phi[o] = phin;
    }
}

template <typename T, int TX, int TY, int NT, bool AXI>
static hipError_t launch2p_variant(const Coef<T>& c, const State<T>& in, const State<T>& out, hipStream_t s)
{
    const int nbx = (c.nx + TX - 1) / TX, nby = (c.ny + TY - 1) / TY;
    hipLaunchKernelGGL((twophase2d_kernel<T, TX, TY, NT, AXI>), dim3(nbx * nby), dim3(NT), 0, s, c, in, out, nbx);
    return hipGetLastError();
}

template <typename T, bool AXI>
static hipError_t launch2p(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile, hipStream_t s)
{
    switch (tile) {
        case 1: return launch2p_variant<T, 32, 8, 256, AXI>(c, in, out, s);
        case 2: return launch2p_variant<T, 64, 8, 256, AXI>(c, in, out, s);
        case 3: return launch2p_variant<T, 16, 16, 256, AXI>(c, in, out, s);
        default: return launch2p_variant<T, 32, 16, 256, AXI>(c, in, out, s);
    }
}

template <typename T>
hipError_t launch_twophase2d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile, hipStream_t s)
{
    return launch2p<T, false>(c, in, out, tile, s);
}

template <typename T>
hipError_t launch_twophase_axisym2d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile,
                                    hipStream_t s)
{
    return launch2p<T, true>(c, in, out, tile, s);
}

template hipError_t launch_twophase2d<float>(const Coef<float>&, const State<float>&, const State<float>&, int, hipStream_t);
template hipError_t launch_twophase2d<double>(const Coef<double>&, const State<double>&, const State<double>&, int, hipStream_t);
template hipError_t launch_twophase_axisym2d<float>(const Coef<float>&, const State<float>&, const State<float>&, int,
                                                    hipStream_t);
template hipError_t launch_twophase_axisym2d<double>(const Coef<double>&, const State<double>&, const State<double>&,
                                                     int, hipStream_t);

}  // namespace acm
