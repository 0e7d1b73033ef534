// 2D fused SMAME tile (continuity then momentum) shared by the single-case
// kernel and the batched kernels, so all produce identical bits for every
// node.  See kern_step.hip for the arithmetic.
#pragma once

#include "acm_internal.h"

namespace acm {

template <typename T>
__device__ __forceinline__ T momc(T r, T u, T rho0) { return fmaT(r, u, rho0 * u); }

template <int TX, int TY>
struct Shape2 {
    static constexpr int RX = TX + 4, RY = TY + 4, RXY = RX * RY;  // fields, halo 2
    static constexpr int DX = TX + 2, DY = TY + 2, DXY = DX * DY;  // drho', halo 1
};

template <typename T, int TX, int TY>
__host__ __device__ constexpr size_t tile2d_lds_bytes()
{
    return sizeof(T) * (3 * Shape2<TX, TY>::RXY + Shape2<TX, TY>::DXY);
}

// Centred difference of the momentum m = rho0 u + drho u between two nodes,
// split as rho0 (u_p - u_m) + (drho_p u_p - drho_m u_m): equal to m_p - m_m in
// exact arithmetic, but the two velocity values are subtracted before any
// rounding of m, so FP32 keeps the small density signal.
template <typename T>
__device__ __forceinline__ T mdiff(T rp, T up, T rm, T um, T rho0)
{
    return fmaT(rho0, up - um, fmaT(rp, up, -(rm * um)));
}

// Continuity update at R-region index e (2D), R-region row stride RX.
template <typename T>
__device__ __forceinline__ T rho_new_2d_at(const Coef<T>& c, const T* sr, const T* su, const T* sv, int e, int RX)
{
    const T rc = sr[e];
    const T rE = sr[e + 1], rW = sr[e - 1], rN = sr[e + RX], rS = sr[e - RX];
    const T div = mdiff(rE, su[e + 1], rW, su[e - 1], c.rho0) + mdiff(rN, sv[e + RX], rS, sv[e - RX], c.rho0);
    const T lap = ((rE + rW) + (rN + rS)) - T(4) * rc;
    return fmaT(-c.cg, div, fmaT(c.kr, lap, rc));
}
template <typename T, int RX>
__device__ __forceinline__ T rho_new_2d(const Coef<T>& c, const T* sr, const T* su, const T* sv, int e)
{
    return rho_new_2d_at<T>(c, sr, su, sv, e, RX);
}

// Stage fields (drho, u, v) of the (TX+4)x(TY+4) region into LDS.  Every
// load of the thread is issued before the first LDS store, so the memory
// latencies overlap instead of adding up.
template <typename T, int TX, int TY, int NT>
__device__ __forceinline__ void stage2d(const Coef<T>& c, const State<T>& in, int x0, int y0,
                                        bool interior, T* sr, T* su, T* sv)
{
    using S = Shape2<TX, TY>;
    constexpr int NIT = (S::RXY + NT - 1) / NT;
    T r[NIT], u[NIT], v[NIT];
    if (interior) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = min((int)threadIdx.x + it * NT, S::RXY - 1);
            const int ly = q / S::RX, lx = q - ly * S::RX;
            const size_t s = (size_t)(y0 + ly - 2) * c.nx + (x0 + lx - 2);
            r[it] = in.r[s];
            u[it] = in.u[s];
            v[it] = in.v[s];
        }
    } else {
        int fxs[NIT], fys[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = min((int)threadIdx.x + it * NT, S::RXY - 1);
            const int ly = q / S::RX, lx = q - ly * S::RX;
            const int sx = map_coord(x0 + lx - 2, c.nx, c.bc[0], 0, fxs[it]);
            const int sy = map_coord(y0 + ly - 2, c.ny, c.bc[2], 2, fys[it]);
            const size_t s = (size_t)sy * c.nx + sx;
            r[it] = in.r[s];
            u[it] = in.u[s];
            v[it] = in.v[s];
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int fx = fxs[it], fy = fys[it];
            if (fx >= 0) {
                u[it] = fmaT(c.fs[fx][0], u[it], c.fo[fx][0]);
                v[it] = fmaT(c.fs[fx][1], v[it], c.fo[fx][1]);
            }
            if (fy >= 0) {
                u[it] = fmaT(c.fs[fy][0], u[it], c.fo[fy][0]);
                v[it] = fmaT(c.fs[fy][1], v[it], c.fo[fy][1]);
            }
        }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int q = threadIdx.x + it * NT;
        if (q < S::RXY) {
            sr[q] = r[it];
            su[q] = u[it];
            sv[q] = v[it];
        }
    }
}

// drho' on the tile plus a one-node ring, into srn.
template <typename T, int TX, int TY, int NT>
__device__ __forceinline__ void rho_ring2d(const Coef<T>& c, int x0, int y0, bool interior,
                                           const T* sr, const T* su, const T* sv, T* srn)
{
    using S = Shape2<TX, TY>;
    for (int q = threadIdx.x; q < S::DXY; q += NT) {
        const int ly = q / S::DX, lx = q - ly * S::DX;
        int ex = lx + 1, ey = ly + 1;  // R-region coordinates
        if (!interior && c.nonperiodic) {
            // a wall / symmetry ghost takes the value of its mirror node
            const int gx = mirror_coord(x0 + lx - 1, c.nx, c.bc[0]);
            const int gy = mirror_coord(y0 + ly - 1, c.ny, c.bc[2]);
            ex = min(max(gx - x0 + 2, 1), S::DX);
            ey = min(max(gy - y0 + 2, 1), S::DY);
        }
        srn[q] = rho_new_2d<T, S::RX>(c, sr, su, sv, ey * S::RX + ex);
    }
}

// Momentum update of one node: R-region index e (row stride RX), drho'-region
// index d (row stride DX), grid row gy (for the per-row force).  Returns
// drho', u', v'.  Shared by the tile kernels, the batched kernels and the
// fused closure kernel, so all give identical bits.
template <typename T>
__device__ __forceinline__ void momentum_node2d_at(const Coef<T>& c, const T* sr, const T* su, const T* sv,
                                                   const T* srn, int e, int d, int gy, int RX, int DX, T& rn_out,
                                                   T& u_out, T& v_out)
{
    const T rc = sr[e], uc = su[e], vc = sv[e];
    const T rE = sr[e + 1], rW = sr[e - 1], rN = sr[e + RX], rS = sr[e - RX];
    const T uE = su[e + 1], uW = su[e - 1], uN = su[e + RX], uS = su[e - RX];
    const T vE = sv[e + 1], vW = sv[e - 1], vN = sv[e + RX], vS = sv[e - RX];
    const T rho0 = c.rho0, cs2 = c.cs2;
    const T mxC = momc(rc, uc, rho0), myC = momc(rc, vc, rho0);
    const T mxE = momc(rE, uE, rho0), mxW = momc(rW, uW, rho0);
    const T mxN = momc(rN, uN, rho0), mxS = momc(rS, uS, rho0);
    const T myE = momc(rE, vE, rho0), myW = momc(rW, vW, rho0);
    const T myN = momc(rN, vN, rho0), myS = momc(rS, vS, rho0);
    const T rnC = srn[d];
    const T rnE = srn[d + 1], rnW = srn[d - 1], rnN = srn[d + DX], rnS = srn[d - DX];
    // fluxes of Pi_ab = m_a u_b + cs^2 drho delta_ab
    const T fxx = (fmaT(mxE, uE, cs2 * rE) - fmaT(mxW, uW, cs2 * rW)) + (mxN * vN - mxS * vS);
    const T fyy = (myE * uE - myW * uW) + (fmaT(myN, vN, cs2 * rN) - fmaT(myS, vS, cs2 * rS));
    const T lx_ = ((mxE + mxW) + (mxN + mxS)) - T(4) * mxC;
    const T ly_ = ((myE + myW) + (myN + myS)) - T(4) * myC;
    const T sx = (rnE - rnW) - (rE - rW);
    const T sy = (rnN - rnS) - (rN - rS);
    const T rho_n = rho0 + rnC;
    T gx_ = c.gdt[0];
    if (c.fx) gx_ = fmaT(c.dt, c.fx[gy], gx_);
    const T dmx = fmaT(rho_n, gx_, fmaT(-c.ks, sx, fmaT(c.kv, lx_, -c.cg * fxx)));
    const T dmy = fmaT(rho_n, c.gdt[1], fmaT(-c.ks, sy, fmaT(c.kv, ly_, -c.cg * fyy)));
    const T drn = rnC - rc;
    const T inv = recipT(rho_n);
    rn_out = rnC;
    u_out = fmaT(fmaT(-uc, drn, dmx), inv, uc);
    v_out = fmaT(fmaT(-vc, drn, dmy), inv, vc);
}
template <typename T, int RX, int DX>
__device__ __forceinline__ void momentum_node2d(const Coef<T>& c, const T* sr, const T* su, const T* sv,
                                                const T* srn, int e, int d, int gy, T& rn_out, T& u_out, T& v_out)
{
    momentum_node2d_at<T>(c, sr, su, sv, srn, e, d, gy, RX, DX, rn_out, u_out, v_out);
}

// Momentum update and store for the nodes of the tile.
template <typename T, int TX, int TY, int NT>
__device__ __forceinline__ void momentum2d(const Coef<T>& c, const State<T>& out, int x0, int y0,
                                           const T* sr, const T* su, const T* sv, const T* srn)
{
    using S = Shape2<TX, TY>;
    for (int q = threadIdx.x; q < TX * TY; q += NT) {
        const int ly = q / TX, lx = q - ly * TX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= c.nx || gy >= c.ny) continue;
        T rn, un, vn;
        momentum_node2d<T, S::RX, S::DX>(c, sr, su, sv, srn, (ly + 2) * S::RX + (lx + 2), (ly + 1) * S::DX + (lx + 1),
                                         gy, rn, un, vn);
        const size_t o = (size_t)gy * c.nx + gx;
        out.r[o] = rn;
        out.u[o] = un;
        out.v[o] = vn;
    }
}

// One 2D tile: stage, drho' ring, momentum.  smem must hold
// tile2d_lds_bytes<T,TX,TY>() bytes.  Called by the single-case kernel and
// by the batched per-item kernel.
template <typename T, int TX, int TY, int NT>
__device__ __forceinline__ void tile2d(const Coef<T>& c, const State<T>& in, const State<T>& out,
                                       int x0, int y0, char* smem)
{
    using S = Shape2<TX, TY>;
    T* sr = reinterpret_cast<T*>(smem);
    T* su = sr + S::RXY;
    T* sv = su + S::RXY;
    T* srn = sv + S::RXY;
    const bool interior = (x0 >= 2) && (x0 + TX + 2 <= c.nx) && (y0 >= 2) && (y0 + TY + 2 <= c.ny);
    stage2d<T, TX, TY, NT>(c, in, x0, y0, interior, sr, su, sv);
    __syncthreads();
    rho_ring2d<T, TX, TY, NT>(c, x0, y0, interior, sr, su, sv, srn);
    __syncthreads();
    momentum2d<T, TX, TY, NT>(c, out, x0, y0, sr, su, sv, srn);
}

// Hardware places workgroup b on XCD (b mod 8); remap so that each XCD owns
// a contiguous range of logical tiles (neighbours share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    constexpr int NX = 8;
    const int per = nb / NX, rem = nb % NX;
    const int x = b % NX, i = b / NX;
    return x * per + min(x, rem) + i;
}

}  // namespace acm
