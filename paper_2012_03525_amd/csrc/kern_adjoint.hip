// Adjoint (vector-Jacobian product) of the 2D SMAME step on planar grids
// with periodic, wall or symmetry faces, for training the learned closure
// through the solver.
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
//
// Walls and symmetry planes.  Outside the grid across such a face there are
// no outputs, so bx, by and A are zero there (instead of wrapped).  The
// forward reads one ghost layer, each ghost a function of the node it
// mirrors, i (its only neighbour inside): drho_g = drho_i, u_g = fs u_i + fo
// per component (2 u_w - u at a wall, the normal component negated at a
// symmetry plane), and rho'_g = rho'_i.  The transposed rules add to node i:
//   - the ghost's rho' is read by the SAT term of i: A_i += s ks bx_i (x
//     faces) or s ks by_i (y faces), s = +1 on a low face, -1 on a high one;
//   - the ghost's inputs are read by the stencils of i: the cotangents of
//     (drho_g, u_g, v_g) are the formulas above at the ghost position, where
//     only the neighbour i is nonzero, and they reach i through the ghost
//     rule: a_r += a_r(g), a_u += fs a_u(g), a_v += fs a_v(g).
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

// Cotangents of a ghost's inputs (drho_g, u_g, v_g) across face F (0..3:
// -x, +x, -y, +y; the ghost lies below its mirror node i on a low face,
// above on a high one), from i's bx, by and A (the only nonzero ones around
// the ghost), folded onto i through the face's ghost rule.
template <int F, typename T>
__device__ __forceinline__ void fold_ghost(const Coef<T>& c, T r, T u, T v, T bxC, T byC, T aC, T& ar, T& au, T& av)
{
    constexpr int AX = F / 2;
    const T sg = (F & 1) ? T(-1) : T(1);
    const T rho = c.rho0 + r;
    // the ghost's velocity and its derivative with respect to the mirror node's
    const T su = c.fs[F][0], sv = c.fs[F][1];
    const T ug = fmaT(su, u, c.fo[F][0]), vg = fmaT(sv, v, c.fo[F][1]);
    const T mx = rho * ug, my = rho * vg;
    const T d_bx = sg * bxC, d_by = sg * byC, d_a = sg * aC;  // neighbour differences at the ghost
    T amx, amy, arg, aug, avg;
    if constexpr (AX == 0) {
        const T pxx = c.cg * d_bx, pyx = c.cg * d_by;
        amx = fmaT(pxx, ug, fmaT(c.cg, d_a, c.kv * bxC));
        amy = fmaT(pyx, ug, c.kv * byC);
        arg = fmaT(amy, vg, fmaT(amx, ug, fmaT(c.cs2, pxx, fmaT(-c.ks, d_bx, c.kr * aC))));
        aug = fmaT(pyx, my, fmaT(pxx, mx, rho * amx));
        avg = rho * amy;
    } else {
        const T pxy = c.cg * d_bx, pyy = c.cg * d_by;
        amx = fmaT(pxy, vg, c.kv * bxC);
        amy = fmaT(pyy, vg, fmaT(c.cg, d_a, c.kv * byC));
        arg = fmaT(amy, vg, fmaT(amx, ug, fmaT(c.cs2, pyy, fmaT(-c.ks, d_by, c.kr * aC))));
        aug = rho * amx;
        avg = fmaT(pyy, my, fmaT(pxy, mx, rho * amy));
    }
    ar += arg;
    au = fmaT(su, aug, au);
    av = fmaT(sv, avg, av);
}

// NP: some face is a wall or a symmetry plane (the periodic build skips those checks)
template <typename T, bool NP>
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
    const bool px = !NP || c.bc[0] == BC_PERIODIC, py = !NP || c.bc[2] == BC_PERIODIC;
    // a position outside the grid across a wall or symmetry face holds no output
    auto outside = [&](int gx, int gy) {
        return (!px && (gx < 0 || gx >= c.nx)) || (!py && (gy < 0 || gy >= c.ny));
    };
    // cotangents of the momentum after the step, and the pointwise part of A
    for (int e = threadIdx.x; e < RXY; e += ANT) {
        const int ly = e / RX, lx = e - ly * RX;
        const int rx = x0 + lx - 2, ry = y0 + ly - 2;
        if (outside(rx, ry)) {
            sbx[e] = sby[e] = sp[e] = T(0);
            continue;
        }
        const int gx = px ? pwrap(rx, c.nx) : rx, gy = py ? pwrap(ry, c.ny) : ry;
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
    // A = cotangent of rho' at every node of the tile and its one-node ring
    for (int d = threadIdx.x; d < DXY; d += ANT) {
        const int ly = d / DX, lx = d - ly * DX;
        const int rx = x0 + lx - 1, ry = y0 + ly - 1;
        const int e = (ly + 1) * RX + (lx + 1);
        if (outside(rx, ry)) {
            sa[d] = T(0);
            continue;
        }
        const T dbx = sbx[e + 1] - sbx[e - 1], dby = sby[e + RX] - sby[e - RX];
        T A = fmaT(c.ks, dbx + dby, sp[e]);
        if (NP) {
            // rho' of a ghost is read by the SAT term of the node it mirrors
            if (!px && rx == 0) A = fmaT(c.ks, sbx[e], A);
            if (!px && rx == c.nx - 1) A = fmaT(-c.ks, sbx[e], A);
            if (!py && ry == 0) A = fmaT(c.ks, sby[e], A);
            if (!py && ry == c.ny - 1) A = fmaT(-c.ks, sby[e], A);
        }
        sa[d] = A;
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
        T ar = fmaT(amy, v, fmaT(amx, u, fmaT(c.cs2, pxx + pyy,
                                               fmaT(-c.ks, (bxE - bxW) + (byN - byS), fmaT(c.kr, la, aC)))));
        T au = fmaT(pyx, my, fmaT(pxx, mx, rho * amx));
        T av = fmaT(pyy, my, fmaT(pxy, mx, rho * amy));
        if (NP) {
            // the ghosts that mirror this node, face by face (-x, +x, -y, +y)
            if (!px && gx == 0) fold_ghost<0>(c, r, u, v, bxC, byC, aC, ar, au, av);
            if (!px && gx == c.nx - 1) fold_ghost<1>(c, r, u, v, bxC, byC, aC, ar, au, av);
            if (!py && gy == 0) fold_ghost<2>(c, r, u, v, bxC, byC, aC, ar, au, av);
            if (!py && gy == c.ny - 1) fold_ghost<3>(c, r, u, v, bxC, byC, aC, ar, au, av);
        }
        aq.r[o] = ar;
        aq.u[o] = au;
        aq.v[o] = av;
    }
}

}  // namespace

template <typename T>
hipError_t launch_adjoint2d(const Coef<T>& c, const State<T>& q, const State<T>& s, const State<T>& as,
                            const State<T>& aq, hipStream_t st)
{
    const int nbx = (c.nx + ATX - 1) / ATX, nby = (c.ny + ATY - 1) / ATY;
    if (c.nonperiodic)
        hipLaunchKernelGGL((step2d_adjoint_kernel<T, true>), dim3(nbx * nby), dim3(ANT), 0, st, c, q, s, as, aq, nbx);
    else
        hipLaunchKernelGGL((step2d_adjoint_kernel<T, false>), dim3(nbx * nby), dim3(ANT), 0, st, c, q, s, as, aq, nbx);
    return hipGetLastError();
}

template hipError_t launch_adjoint2d<float>(const Coef<float>&, const State<float>&, const State<float>&,
                                            const State<float>&, const State<float>&, hipStream_t);
template hipError_t launch_adjoint2d<double>(const Coef<double>&, const State<double>&, const State<double>&,
                                             const State<double>&, const State<double>&, hipStream_t);

}  // namespace acm
