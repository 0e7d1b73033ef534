// Adjoint (vector-Jacobian product) of the 2D SMAME step on a fully
// periodic grid, for training the learned closure through the solver.
//
// Forward step at node i, in the coefficient form of the step kernels
// (cg = dt/2dx, kr, kv, ks the SAT and viscous factors of Eqs. 2.10-2.11,
// gx = dt (g_x + f_x(row)), gy = dt g_y, rho = rho0 + drho, m = rho u):
//   r'   = r + kr L(r) - cg [(mx_E - mx_W) + (my_N - my_S)]
//   dmx  = -cg [(Pxx_E - Pxx_W) + (Pxy_N - Pxy_S)] + kv L(mx)
//          - ks [(r'_E - r'_W) - (r_E - r_W)] + rho' gx
//   dmy  likewise with Pyx, Pyy, gy;   u' = (mx + dmx) / rho',  v' = ...
//   Pxx = mx u + cs2 r, Pxy = mx v, Pyx = my u, Pyy = my v + cs2 r
// (L(f) = sum of the four neighbours - 4 f).  Given the cotangents
// (a_r', a_u', a_v') of the outputs, with bx = a_u'/rho', by = a_v'/rho':
//   A    = a_r' - (a_u' u' + a_v' v')/rho' + bx gx + by gy
//          + ks [(bx_E - bx_W) + (by_N - by_S)]            (cotangent of r')
//   aPxx = cg (bx_E - bx_W), aPxy = cg (bx_N - bx_S),
//   aPyx = cg (by_E - by_W), aPyy = cg (by_N - by_S)
//   amx  = cg (A_E - A_W) + bx + kv L(bx) + aPxx u + aPxy v
//   amy  = cg (A_N - A_S) + by + kv L(by) + aPyx u + aPyy v
//   a_r  = A + kr L(A) - ks [(bx_E - bx_W) + (by_N - by_S)] + cs2 (aPxx + aPyy)
//          + amx u + amy v
//   a_u  = rho amx + aPxx mx + aPyx my,   a_v = rho amy + aPxy mx + aPyy my
// The centred differences and the Laplacian are antisymmetric and symmetric
// on a periodic grid, which is what moves each neighbour difference from the
// forward's inputs onto the cotangents.  Like the forward it is a radius-2
// stencil: a tile stages (bx, by, the pointwise part of A) on a two-node
// ring in LDS, forms A on a one-node ring, then each node reads its own
// forward input q.
#include <hip/hip_runtime.h>

#include "../../include/acm.h"
#include "acm_internal.h"
#include "tile2d.h"

namespace acm {

namespace {

constexpr int ATX = 64, ATY = 4, ANT = 256;

// periodic index for -2 <= i < n + ATX + 2 (a tile's staging region may pass
// the far end of a grid narrower than the tile more than once)
__device__ __forceinline__ int pwrap(int i, int n) { return (int)(((long long)i + 2LL * n) % n); }

template <typename T>
__global__ __launch_bounds__(ANT) void step2d_adjoint_kernel(Coef<T> c, State<T> q, State<T> s, State<T> as,
                                                             State<T> aq, int nbx)
{
    constexpr int RX = ATX + 4, RY = ATY + 4, RXY = RX * RY;
    constexpr int DX = ATX + 2, DY = ATY + 2, DXY = DX * DY;
    __shared__ T sbx[RXY], sby[RXY], sp[RXY], sa[DXY];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int tby = lb / nbx, tbx = lb - tby * nbx;
    const int x0 = tbx * ATX, y0 = tby * ATY;
    const T rho0 = c.rho0;
    // cotangents of the momentum after the step, and the pointwise part of A
    for (int e = threadIdx.x; e < RXY; e += ANT) {
        const int ly = e / RX, lx = e - ly * RX;
        const int gx = pwrap(x0 + lx - 2, c.nx), gy = pwrap(y0 + ly - 2, c.ny);
        const size_t o = (size_t)gy * c.nx + gx;
        const T rn = s.r[o], un = s.u[o], vn = s.v[o];
        const T ar = as.r[o], au = as.u[o], av = as.v[o];
        const T inv = T(1) / (rho0 + rn);
        const T bx = au * inv, by = av * inv;
        T fxg = c.gdt[0];
        if (c.fx) fxg = fmaT(c.dt, c.fx[gy], fxg);
        sbx[e] = bx;
        sby[e] = by;
        sp[e] = fmaT(by, c.gdt[1], fmaT(bx, fxg, ar - (bx * un + by * vn)));
    }
    __syncthreads();
    for (int d = threadIdx.x; d < DXY; d += ANT) {
        const int ly = d / DX, lx = d - ly * DX;
        const int e = (ly + 1) * RX + (lx + 1);
        const T dbx = sbx[e + 1] - sbx[e - 1], dby = sby[e + RX] - sby[e - RX];
        sa[d] = fmaT(c.ks, dbx + dby, sp[e]);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ATX * ATY; t += ANT) {
        const int ly = t / ATX, lx = t - ly * ATX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= c.nx || gy >= c.ny) continue;
        const int e = (ly + 2) * RX + (lx + 2), d = (ly + 1) * DX + (lx + 1);
        const size_t o = (size_t)gy * c.nx + gx;
        const T r = q.r[o], u = q.u[o], v = q.v[o];
        const T rho = rho0 + r;
        const T mx = rho * u, my = rho * v;
        const T bxC = sbx[e], byC = sby[e];
        const T bxE = sbx[e + 1], bxW = sbx[e - 1], bxN = sbx[e + RX], bxS = sbx[e - RX];
        const T byE = sby[e + 1], byW = sby[e - 1], byN = sby[e + RX], byS = sby[e - RX];
        const T aC = sa[d], aE = sa[d + 1], aW = sa[d - 1], aN = sa[d + DX], aS = sa[d - DX];
        const T pxx = c.cg * (bxE - bxW), pxy = c.cg * (bxN - bxS);
        const T pyx = c.cg * (byE - byW), pyy = c.cg * (byN - byS);
        const T lbx = ((bxE + bxW) + (bxN + bxS)) - T(4) * bxC;
        const T lby = ((byE + byW) + (byN + byS)) - T(4) * byC;
        const T la = ((aE + aW) + (aN + aS)) - T(4) * aC;
        const T amx = fmaT(pxy, v, fmaT(pxx, u, fmaT(c.kv, lbx, fmaT(c.cg, aE - aW, bxC))));
        const T amy = fmaT(pyy, v, fmaT(pyx, u, fmaT(c.kv, lby, fmaT(c.cg, aN - aS, byC))));
        const T ar = fmaT(amy, v, fmaT(amx, u, fmaT(c.cs2, pxx + pyy,
                                                     fmaT(-c.ks, (bxE - bxW) + (byN - byS), fmaT(c.kr, la, aC)))));
        aq.r[o] = ar;
        aq.u[o] = fmaT(pyx, my, fmaT(pxx, mx, rho * amx));
        aq.v[o] = fmaT(pyy, my, fmaT(pxy, mx, rho * amy));
    }
}

}  // namespace

template <typename T>
hipError_t launch_adjoint2d(const Coef<T>& c, const State<T>& q, const State<T>& s, const State<T>& as,
                            const State<T>& aq, hipStream_t st)
{
    const int nbx = (c.nx + ATX - 1) / ATX, nby = (c.ny + ATY - 1) / ATY;
    hipLaunchKernelGGL((step2d_adjoint_kernel<T>), dim3(nbx * nby), dim3(ANT), 0, st, c, q, s, as, aq, nbx);
    return hipGetLastError();
}

template hipError_t launch_adjoint2d<float>(const Coef<float>&, const State<float>&, const State<float>&,
                                            const State<float>&, const State<float>&, hipStream_t);
template hipError_t launch_adjoint2d<double>(const Coef<double>&, const State<double>&, const State<double>&,
                                             const State<double>&, const State<double>&, hipStream_t);

}  // namespace acm
