// Launcher of the axisymmetric 2D step (kern_axisym.hip).  Not part of the
// public ABI.
#pragma once

#include "acm_internal.h"
#include "tile2d.h"

namespace acm {

// Radial parts of the cylindrical operators at a node on grid row g, with
// irc = 1 / (g + 1/2) (rows j - 1, j, j + 1 at radii (g, g + 1/2, g + 1) dx):
//   (1/r) d_r(r f)      = [g (f_N - f_S) + (f_C + f_N)] irc / (2 dx)
//   (1/r) d_r(r d_r f)  = [g (f_N + f_S - 2 f_C) + (f_N - f_C)] irc / dx^2
// (the face form with face radii r -+ dx/2, arranged so that FP32 keeps the
// centred difference).  Shared by the single- and two-phase kernels so both
// evaluate the same expressions.
template <typename T>
__device__ __forceinline__ T axi_div_r(T g, T irc, T diff_ns, T sum_cn)
{
    return fmaT(g, diff_ns, sum_cn) * irc;
}
template <typename T>
__device__ __forceinline__ T axi_lap_r(T g, T irc, T fC, T fN, T fS)
{
    return fmaT(g, (fN + fS) - T(2) * fC, fN - fC) * irc;
}

// Continuity (2.10) sums of the axisymmetric step: the divergence of m (in
// units of 1 / (2 dx)) and the Laplacian of drho (units of 1 / dx^2).
template <typename T>
__device__ __forceinline__ void axi_continuity(T rho0, T g, T irc, T rC, T rE, T rW, T rN, T rS, T uE, T uW, T vC,
                                               T vN, T vS, T& div, T& lap)
{
    const T myC = fmaT(rC, vC, rho0 * vC), myN = fmaT(rN, vN, rho0 * vN);
    div = mdiff(rE, uE, rW, uW, rho0) + axi_div_r(g, irc, mdiff(rN, vN, rS, vS, rho0), myC + myN);
    lap = ((rE + rW) - T(2) * rC) + axi_lap_r(g, irc, rC, rN, rS);
}

// Momentum (2.11) sums of the axisymmetric step at a node: fluxes of Pi
// (axial: d_x Pi_xx + (1/r) d_r(r Pi_xr); radial: d_x Pi_rx + (1/r) d_r(r
// Pi_rr) - Pi_thth / r, in units of 1 / (2 dx)) and vector Laplacians of m
// (units of 1 / dx^2, the radial one with -m_r / r^2).
template <typename T>
__device__ __forceinline__ void axi_momentum(T cs2, T g, T irc, T rC, T rE, T rW, T rN, T rS, T uE, T uW, T vC, T vN,
                                             T vS, T mxC, T mxE, T mxW, T mxN, T mxS, T myC, T myE, T myW, T myN,
                                             T myS, T& fxx, T& fyy, T& lpx, T& lpy)
{
    const T pxyC = mxC * vC, pxyN = mxN * vN, pxyS = mxS * vS;
    const T pyyC = fmaT(myC, vC, cs2 * rC), pyyN = fmaT(myN, vN, cs2 * rN), pyyS = fmaT(myS, vS, cs2 * rS);
    fxx = (fmaT(mxE, uE, cs2 * rE) - fmaT(mxW, uW, cs2 * rW)) + axi_div_r(g, irc, pxyN - pxyS, pxyC + pxyN);
    fyy = (myE * uE - myW * uW) + axi_div_r(g, irc, pyyN - pyyS, pyyC + pyyN) - T(2) * cs2 * rC * irc;
    lpx = ((mxE + mxW) - T(2) * mxC) + axi_lap_r(g, irc, mxC, mxN, mxS);
    lpy = ((myE + myW) - T(2) * myC) + axi_lap_r(g, irc, myC, myN, myS) - myC * irc * irc;
}

// One axisymmetric single-phase step (x axial, y radial, axis on the -y
// face); tile codes 1 32x8, 2 64x8, 4 64x4, else 32x16.
template <typename T>
hipError_t launch_axisym2d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile, hipStream_t s);

// Diagnostics of an axisymmetric state (kern_diag.hip): the reductions of
// launch_diag with every sum weighted by the node's radius (j + 1/2) dx / dx
// and the cylindrical divergence.
template <typename T>
hipError_t launch_diag_axisym(const Coef<T>& c, int two_phase, const State<T>& cur, const State<T>& prev,
                              int have_prev, double* partials, int nblocks, double* result, hipStream_t s);

// One axisymmetric two-phase step (kern_twophase.hip); tile codes as for the
// planar two-phase step.
template <typename T>
hipError_t launch_twophase_axisym2d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile,
                                    hipStream_t s);

}  // namespace acm
