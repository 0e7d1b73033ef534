// Axisymmetric SMAME step (2D, single phase): x is the axial coordinate, y
// the radius, the -y face is the axis (a symmetry plane) and row j sits at
// r = (j + 1/2) dx.  Eqs. (2.10)-(2.11) are taken with the cylindrical
// divergence and Laplacian, (1/r) d_r(r f) and (1/r) d_r(r d_r f), in flux
// form with face radii r -+ dx/2 (the face value of a flux is the mean of its
// two nodes), and the radial momentum gains the hoop term of the divergence
// of Pi, -Pi_thth / r with Pi_thth = cs^2 drho (no swirl), and the
// -m_r / r^2 of the vector Laplacian (the radial sums are written out in
// kern_axisym.h and shared with the two-phase kernel).  Staging, ghosts and
// the per-node density update order are those of the 2D tile kernel.
#include <hip/hip_runtime.h>

#include "../../include/acm.h"
#include "acm_internal.h"
#include "kern_axisym.h"
#include "tile2d.h"

namespace acm {

namespace {

// drho' at R-region index e of a node on grid row gy
template <typename T, int RX>
__device__ __forceinline__ T rho_new_axi(const Coef<T>& c, const T* sr, const T* su, const T* sv, int e, int gy)
{
    const T g = T(gy), irc = T(1) / (T(gy) + T(0.5));
    const T rc = sr[e];
    T div, lap;
    axi_continuity(c.rho0, g, irc, rc, sr[e + 1], sr[e - 1], sr[e + RX], sr[e - RX], su[e + 1], su[e - 1], sv[e],
                   sv[e + RX], sv[e - RX], div, lap);
    return fmaT(-c.cg, div, fmaT(c.kr, lap, rc));
}

template <typename T, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void axisym2d_kernel(Coef<T> c, State<T> in, State<T> out, int nbx)
{
    using S = Shape2<TX, TY>;
    __shared__ __align__(16) char smem[tile2d_lds_bytes<T, TX, TY>()];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int by = lb / nbx, bx = lb - by * nbx;
    const int x0 = bx * TX, y0 = by * TY;
    T* sr = reinterpret_cast<T*>(smem);
    T* su = sr + S::RXY;
    T* sv = su + S::RXY;
    T* srn = sv + S::RXY;
    const bool interior = (x0 >= 2) && (x0 + TX + 2 <= c.nx) && (y0 >= 2) && (y0 + TY + 2 <= c.ny);
    stage2d<T, TX, TY, NT>(c, in, x0, y0, interior, sr, su, sv);
    __syncthreads();
    // drho' on the tile plus a one-node ring; a ghost position takes the
    // value of its mirror node (computed with the mirror node's radius)
    for (int q = threadIdx.x; q < S::DXY; q += NT) {
        const int ly = q / S::DX, lx = q - ly * S::DX;
        int ex = lx + 1, ey = ly + 1;
        if (!interior) {
            const int gx = mirror_coord(x0 + lx - 1, c.nx, c.bc[0]);
            const int gy = mirror_coord(y0 + ly - 1, c.ny, c.bc[2]);
            ex = min(max(gx - x0 + 2, 1), S::DX);
            ey = min(max(gy - y0 + 2, 1), S::DY);
        }
        srn[q] = rho_new_axi<T, S::RX>(c, sr, su, sv, ey * S::RX + ex, y0 + ey - 2);
    }
    __syncthreads();
    const T rho0 = c.rho0, cs2 = c.cs2;
    for (int q = threadIdx.x; q < TX * TY; q += NT) {
        const int ly = q / TX, lx = q - ly * TX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= c.nx || gy >= c.ny) continue;
        const int e = (ly + 2) * S::RX + (lx + 2), d = (ly + 1) * S::DX + (lx + 1);
        constexpr int RX = S::RX, DX = S::DX;
        const T g = T(gy), irc = T(1) / (T(gy) + T(0.5));
        const T rc = sr[e], uc = su[e], vc = sv[e];
        const T rE = sr[e + 1], rW = sr[e - 1], rN = sr[e + RX], rS = sr[e - RX];
        const T uE = su[e + 1], uW = su[e - 1], uN = su[e + RX], uS = su[e - RX];
        const T vE = sv[e + 1], vW = sv[e - 1], vN = sv[e + RX], vS = sv[e - RX];
        const T mxC = momc(rc, uc, rho0), myC = momc(rc, vc, rho0);
        const T mxE = momc(rE, uE, rho0), mxW = momc(rW, uW, rho0);
        const T mxN = momc(rN, uN, rho0), mxS = momc(rS, uS, rho0);
        const T myE = momc(rE, vE, rho0), myW = momc(rW, vW, rho0);
        const T myN = momc(rN, vN, rho0), myS = momc(rS, vS, rho0);
        const T rnC = srn[d];
        const T rnE = srn[d + 1], rnW = srn[d - 1], rnN = srn[d + DX], rnS = srn[d - DX];
        T fxx, fyy, lx_, ly_;
        axi_momentum(cs2, g, irc, rc, rE, rW, rN, rS, uE, uW, vc, vN, vS, mxC, mxE, mxW, mxN, mxS, myC, myE, myW, myN,
                     myS, fxx, fyy, lx_, ly_);
        const T sx = (rnE - rnW) - (rE - rW);
        const T sy = (rnN - rnS) - (rN - rS);
        const T rho_n = rho0 + rnC;
        T gx_ = c.gdt[0];
        if (c.fx) gx_ = fmaT(c.dt, c.fx[gy], gx_);
        const T dmx = fmaT(rho_n, gx_, fmaT(-c.ks, sx, fmaT(c.kv, lx_, -c.cg * fxx)));
        const T dmy = fmaT(rho_n, c.gdt[1], fmaT(-c.ks, sy, fmaT(c.kv, ly_, -c.cg * fyy)));
        const T drn = rnC - rc;
        const T inv = recipT(rho_n);
        const size_t o = (size_t)gy * c.nx + gx;
        out.r[o] = rnC;
        out.u[o] = fmaT(fmaT(-uc, drn, dmx), inv, uc);
        out.v[o] = fmaT(fmaT(-vc, drn, dmy), inv, vc);
    }
}

template <typename T, int TX, int TY, int NT>
hipError_t launch_variant(const Coef<T>& c, const State<T>& in, const State<T>& out, hipStream_t s)
{
    const int nbx = (c.nx + TX - 1) / TX, nby = (c.ny + TY - 1) / TY;
    hipLaunchKernelGGL((axisym2d_kernel<T, TX, TY, NT>), dim3(nbx * nby), dim3(NT), 0, s, c, in, out, nbx);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_axisym2d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile, hipStream_t s)
{
    // 32 x 16 is the fastest shape measured on a 4096 x 2048 pipe (55 us per
    // step against 56, 61 and 63 us for 64 x 8, 32 x 8 and 64 x 4)
    switch (tile) {
        case 1: return launch_variant<T, 32, 8, 256>(c, in, out, s);
        case 2: return launch_variant<T, 64, 8, 256>(c, in, out, s);
        case 4: return launch_variant<T, 64, 4, 256>(c, in, out, s);
        default: return launch_variant<T, 32, 16, 256>(c, in, out, s);
    }
}

template hipError_t launch_axisym2d<float>(const Coef<float>&, const State<float>&, const State<float>&, int,
                                           hipStream_t);
template hipError_t launch_axisym2d<double>(const Coef<double>&, const State<double>&, const State<double>&, int,
                                            hipStream_t);

}  // namespace acm
