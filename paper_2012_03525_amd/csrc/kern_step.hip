// Fused single-phase SMAME step kernels for gfx950 (2D LDS tiles, 3D
// 2.5D z-march).  One launch = one full step: continuity (Eq. 2.10), then
// momentum (Eq. 2.11) with the body force, using centred differences
// (Eqs. 2.12-2.13).  Boundary ghosts are produced while staging the tile.
//
// Arithmetic (per node, in the storage precision T):
//   m_a      = rho0 u_a + drho u_a                      (one fma)
//   drho'    = drho - cg sum_a (m_a(+a) - m_a(-a)) + kr L(drho)
//   dm_a     = -cg sum_b (Pi_ab(+b) - Pi_ab(-b)) + kv L(m_a)
//              - ks [(drho'(+a) - drho'(-a)) - (drho(+a) - drho(-a))]
//              + (rho0 + drho') dt g_a
//   Pi_ab    = m_a u_b + cs^2 drho delta_ab
//   u_a'     = u_a + (dm_a - u_a (drho' - drho)) / (rho0 + drho')
// The last line is (m_a + dm_a)/rho' rewritten as an increment so that FP32
// storage of u keeps the small per-step change to full relative precision.
// The code is compiled with -ffp-contract=off; every fma is explicit, so the
// per-node result does not depend on the tile shape or on the kernel that
// calls the tile function (the batched kernel relies on this).
#include "acm_internal.h"

namespace acm {

template <typename T>
__device__ __forceinline__ T momc(T r, T u, T rho0) { return fmaT(r, u, rho0 * u); }

// ===========================================================================
// 2D
// ===========================================================================
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

// Continuity update at R-region index e (2D).
template <typename T, int RX>
__device__ __forceinline__ T rho_new_2d(const Coef<T>& c, const T* sr, const T* su, const T* sv, int e)
{
    const T rc = sr[e];
    const T rE = sr[e + 1], rW = sr[e - 1], rN = sr[e + RX], rS = sr[e - RX];
    const T mE = momc(rE, su[e + 1], c.rho0), mW = momc(rW, su[e - 1], c.rho0);
    const T mN = momc(rN, sv[e + RX], c.rho0), mS = momc(rS, sv[e - RX], c.rho0);
    const T div = (mE - mW) + (mN - mS);
    const T lap = ((rE + rW) + (rN + rS)) - T(4) * rc;
    return fmaT(-c.cg, div, fmaT(c.kr, lap, rc));
}

// Stage fields (drho, u, v) of the (TX+4)x(TY+4) region into LDS.
template <typename T, int TX, int TY, int NT>
__device__ __forceinline__ void stage2d(const Coef<T>& c, const State<T>& in, int x0, int y0,
                                        bool interior, T* sr, T* su, T* sv)
{
    using S = Shape2<TX, TY>;
    for (int q = threadIdx.x; q < S::RXY; q += NT) {
        const int ly = q / S::RX, lx = q - ly * S::RX;
        const int gx = x0 + lx - 2, gy = y0 + ly - 2;
        T r, u, v;
        if (interior) {
            const size_t s = (size_t)gy * c.nx + gx;
            r = in.r[s];
            u = in.u[s];
            v = in.v[s];
        } else {
            int fx, fy;
            const int sx = map_coord(gx, c.nx, c.bc[0], 0, fx);
            const int sy = map_coord(gy, c.ny, c.bc[2], 2, fy);
            const size_t s = (size_t)sy * c.nx + sx;
            r = in.r[s];
            u = in.u[s];
            v = in.v[s];
            if (fx >= 0) {
                u = fmaT(c.fs[fx][0], u, c.fo[fx][0]);
                v = fmaT(c.fs[fx][1], v, c.fo[fx][1]);
            }
            if (fy >= 0) {
                u = fmaT(c.fs[fy][0], u, c.fo[fy][0]);
                v = fmaT(c.fs[fy][1], v, c.fo[fy][1]);
            }
        }
        sr[q] = r;
        su[q] = u;
        sv[q] = v;
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

// Momentum update and store for the nodes of the tile.
template <typename T, int TX, int TY, int NT>
__device__ __forceinline__ void momentum2d(const Coef<T>& c, const State<T>& out, int x0, int y0,
                                           const T* sr, const T* su, const T* sv, const T* srn)
{
    using S = Shape2<TX, TY>;
    constexpr int RX = S::RX, DX = S::DX;
    for (int q = threadIdx.x; q < TX * TY; q += NT) {
        const int ly = q / TX, lx = q - ly * TX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= c.nx || gy >= c.ny) continue;
        const int e = (ly + 2) * RX + (lx + 2);
        const int d = (ly + 1) * DX + (lx + 1);
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
        const size_t o = (size_t)gy * c.nx + gx;
        out.r[o] = rnC;
        out.u[o] = fmaT(fmaT(-uc, drn, dmx), inv, uc);
        out.v[o] = fmaT(fmaT(-vc, drn, dmy), inv, vc);
    }
}

// One 2D tile: stage, drho' ring, momentum.  smem must hold
// tile2d_lds_bytes<T,TX,TY>() bytes.  Called by the single-case kernel and
// by the batched persistent kernel.
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

template <typename T, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void step2d_kernel(Coef<T> c, State<T> in, State<T> out, int nbx)
{
    __shared__ __align__(16) char smem[tile2d_lds_bytes<T, TX, TY>()];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int by = lb / nbx, bx = lb - by * nbx;
    tile2d<T, TX, TY, NT>(c, in, out, bx * TX, by * TY, smem);
}

template <typename T, int TX, int TY, int NT>
static hipError_t launch2d_variant(const Coef<T>& c, const State<T>& in, const State<T>& out, hipStream_t s)
{
    const int nbx = (c.nx + TX - 1) / TX, nby = (c.ny + TY - 1) / TY;
    hipLaunchKernelGGL((step2d_kernel<T, TX, TY, NT>), dim3(nbx * nby), dim3(NT), 0, s, c, in, out, nbx);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step2d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile, hipStream_t s)
{
    switch (tile) {
        case 1: return launch2d_variant<T, 32, 8, 256>(c, in, out, s);
        case 2: return launch2d_variant<T, 64, 8, 256>(c, in, out, s);
        case 3: return launch2d_variant<T, 16, 16, 256>(c, in, out, s);
        case 4: return launch2d_variant<T, 128, 4, 256>(c, in, out, s);
        case 5: return launch2d_variant<T, 32, 16, 256>(c, in, out, s);
        default: return launch2d_variant<T, 64, 4, 256>(c, in, out, s);
    }
}

template hipError_t launch_step2d<float>(const Coef<float>&, const State<float>&, const State<float>&, int, hipStream_t);
template hipError_t launch_step2d<double>(const Coef<double>&, const State<double>&, const State<double>&, int, hipStream_t);

// ===========================================================================
// 3D: 2.5D march along z.  A workgroup owns a TX x TY column of nodes and a
// chunk of ZC planes.  Four input planes (with a two-node in-plane halo) are
// resident in LDS as a ring; drho' is computed one plane ahead on the tile
// plus a one-node ring, so every node's drho' is formed exactly once per
// workgroup.  Plane k+3 is fetched into registers while plane k is computed.
// ===========================================================================
template <int TX, int TY>
struct Shape3 {
    static constexpr int RX = TX + 4, RY = TY + 4, RXY = RX * RY;
    static constexpr int DX = TX + 2, DY = TY + 2, DXY = DX * DY;
    static constexpr int NT = TX * TY;
    static constexpr int NL = (RXY + NT - 1) / NT;  // plane points staged per thread
};

// drho' at R-index e of plane slot (cur), with the planes below / above.
template <typename T, int RX>
__device__ __forceinline__ T rho_new_3d(const Coef<T>& c, const T* r0, const T* u0, const T* v0,
                                        const T* rD, const T* wD, const T* rU, const T* wU, int e)
{
    const T rc = r0[e];
    const T rE = r0[e + 1], rW = r0[e - 1], rN = r0[e + RX], rS = r0[e - RX];
    const T rUp = rU[e], rDn = rD[e];
    const T mE = momc(rE, u0[e + 1], c.rho0), mW = momc(rW, u0[e - 1], c.rho0);
    const T mN = momc(rN, v0[e + RX], c.rho0), mS = momc(rS, v0[e - RX], c.rho0);
    const T mU = momc(rUp, wU[e], c.rho0), mD = momc(rDn, wD[e], c.rho0);
    const T div = ((mE - mW) + (mN - mS)) + (mU - mD);
    const T lap = (((rE + rW) + (rN + rS)) + (rUp + rDn)) - T(6) * rc;
    return fmaT(-c.cg, div, fmaT(c.kr, lap, rc));
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void step3d_kernel(Coef<T> c, State<T> in, State<T> out, int zc,
                                                          int nbx, int nby)
{
    using S = Shape3<TX, TY>;
    constexpr int RX = S::RX, RXY = S::RXY, DX = S::DX, DXY = S::DXY, NT = S::NT, NL = S::NL;
    __shared__ T sr[4][RXY], su[4][RXY], sv[4][RXY], sw[4][RXY];
    __shared__ T sd[2][DXY];

    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = lb % nbx;
    const int t1 = lb / nbx;
    const int by = t1 % nby, bz = t1 / nby;
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = bz * zc;
    const int z1 = min(z0 + zc, c.nz);
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const size_t plane = (size_t)nx * ny;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int gx = x0 + tx, gy = y0 + ty;
    const bool active = (gx < nx) && (gy < ny);
    const int eo = (ty + 2) * RX + (tx + 2);  // own node in R coordinates
    const int dO = (ty + 1) * DX + (tx + 1);  // own node in D coordinates
    const bool inplane_interior = (x0 >= 2) && (x0 + TX + 2 <= nx) && (y0 >= 2) && (y0 + TY + 2 <= ny);
    const bool zperiodic = (c.bc[4] == BC_PERIODIC);

    // per-thread staging map: in-plane source offset and crossed faces
    int soff[NL];
    signed char sfx[NL], sfy[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int q = tid + i * NT;
        const int qq = q < RXY ? q : 0;
        const int ly = qq / RX, lx = qq - ly * RX;
        int fx, fy;
        const int sx = map_coord(x0 + lx - 2, nx, c.bc[0], 0, fx);
        const int sy = map_coord(y0 + ly - 2, ny, c.bc[2], 2, fy);
        soff[i] = sy * nx + sx;
        sfx[i] = (signed char)fx;
        sfy[i] = (signed char)fy;
    }
    // drho' ring positions (mirror substitution for wall / symmetry ghosts)
    int dsrc[(DXY + NT - 1) / NT];
#pragma unroll
    for (int i = 0; i < (DXY + NT - 1) / NT; ++i) {
        const int q = tid + i * NT;
        const int qq = q < DXY ? q : 0;
        const int ly = qq / DX, lx = qq - ly * DX;
        int ex = lx + 1, ey = ly + 1;
        if (!inplane_interior && c.nonperiodic) {
            const int mx = mirror_coord(x0 + lx - 1, nx, c.bc[0]);
            const int my = mirror_coord(y0 + ly - 1, ny, c.bc[2]);
            ex = min(max(mx - x0 + 2, 1), DX);
            ey = min(max(my - y0 + 2, 1), S::DY);
        }
        dsrc[i] = ey * RX + ex;
    }

    T pr[NL], pu[NL], pv[NL], pw[NL];
    // fetch plane gz into registers (ghost planes mapped, velocity rules applied)
    auto fetch = [&](int gz) {
        int fz;
        const int sz = map_coord(gz, nz, c.bc[4], 4, fz);
        const size_t base = (size_t)sz * plane;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            if (tid + i * NT < RXY) {
                const size_t s = base + soff[i];
                pr[i] = in.r[s];
                pu[i] = in.u[s];
                pv[i] = in.v[s];
                pw[i] = in.w[s];
                if (c.nonperiodic) {
                    const int f0 = sfx[i], f1 = sfy[i];
                    if (f0 >= 0) {
                        pu[i] = fmaT(c.fs[f0][0], pu[i], c.fo[f0][0]);
                        pv[i] = fmaT(c.fs[f0][1], pv[i], c.fo[f0][1]);
                        pw[i] = fmaT(c.fs[f0][2], pw[i], c.fo[f0][2]);
                    }
                    if (f1 >= 0) {
                        pu[i] = fmaT(c.fs[f1][0], pu[i], c.fo[f1][0]);
                        pv[i] = fmaT(c.fs[f1][1], pv[i], c.fo[f1][1]);
                        pw[i] = fmaT(c.fs[f1][2], pw[i], c.fo[f1][2]);
                    }
                    if (fz >= 0) {
                        pu[i] = fmaT(c.fs[fz][0], pu[i], c.fo[fz][0]);
                        pv[i] = fmaT(c.fs[fz][1], pv[i], c.fo[fz][1]);
                        pw[i] = fmaT(c.fs[fz][2], pw[i], c.fo[fz][2]);
                    }
                }
            }
        }
    };
    auto store = [&](int slot) {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int q = tid + i * NT;
            if (q < RXY) {
                sr[slot][q] = pr[i];
                su[slot][q] = pu[i];
                sv[slot][q] = pv[i];
                sw[slot][q] = pw[i];
            }
        }
    };
    // drho' of plane p (slot sp) on the tile + ring into sd[dslot]
    auto ring = [&](int p, int dslot) {
        const int s0 = p & 3, sD = (p - 1) & 3, sU = (p + 1) & 3;
#pragma unroll
        for (int i = 0; i < (DXY + NT - 1) / NT; ++i) {
            const int q = tid + i * NT;
            if (q < DXY)
                sd[dslot][q] = rho_new_3d<T, RX>(c, sr[s0], su[s0], sv[s0], sr[sD], sw[sD], sr[sU], sw[sU],
                                                 dsrc[i]);
        }
    };

    // ---- prologue: planes z0-2 .. z0+1, drho'(z0-1) own node, drho'(z0) ring
    for (int p = z0 - 2; p <= z0 + 1; ++p) {
        fetch(p);
        store(p & 3);
    }
    fetch(z0 + 2);  // in flight during the prologue compute
    __syncthreads();
    ring(z0, z0 & 1);
    T rn_prev = T(0);
    if (zperiodic || z0 > 0) {
        // drho'(z0-1) at the own node (planes z0-2, z0-1, z0 are resident)
        const int p = z0 - 1;
        rn_prev = rho_new_3d<T, RX>(c, sr[p & 3], su[p & 3], sv[p & 3], sr[(p - 1) & 3], sw[(p - 1) & 3],
                                    sr[(p + 1) & 3], sw[(p + 1) & 3], eo);
    }
    __syncthreads();
    if (!(zperiodic || z0 > 0)) rn_prev = sd[z0 & 1][dO];  // wall / symmetry at z = 0: mirror
    // own-node values of plane z0-1
    T r_prev = sr[(z0 - 1) & 3][eo], u_prev = su[(z0 - 1) & 3][eo];
    T v_prev = sv[(z0 - 1) & 3][eo], w_prev = sw[(z0 - 1) & 3][eo];

    const T rho0 = c.rho0, cs2 = c.cs2;
    for (int k = z0; k < z1; ++k) {
        store((k + 2) & 3);  // plane k+2 (its slot held plane k-2)
        if (k + 3 <= z1 + 1) fetch(k + 3);
        __syncthreads();
        const bool upper_ghost = (!zperiodic) && (k + 1 >= nz);
        if (!upper_ghost) ring(k + 1, (k + 1) & 1);
        __syncthreads();

        const int s0 = k & 3, sU = (k + 1) & 3;
        const T* r0 = sr[s0];
        const T* u0 = su[s0];
        const T* v0 = sv[s0];
        const T* w0 = sw[s0];
        const T* dc = sd[k & 1];
        const T rc = r0[eo], uc = u0[eo], vc = v0[eo], wc = w0[eo];
        const T rnC = dc[dO];
        const T rn_next = upper_ghost ? rnC : sd[(k + 1) & 1][dO];
        if (active) {
            const int e = eo;
            const T rE = r0[e + 1], rW = r0[e - 1], rN = r0[e + RX], rS = r0[e - RX];
            const T rU = sr[sU][e], rD = r_prev;
            const T uE = u0[e + 1], uW = u0[e - 1], uN = u0[e + RX], uS = u0[e - RX];
            const T vE = v0[e + 1], vW = v0[e - 1], vN = v0[e + RX], vS = v0[e - RX];
            const T wE = w0[e + 1], wW = w0[e - 1], wN = w0[e + RX], wS = w0[e - RX];
            const T uU = su[sU][e], vU = sv[sU][e], wU = sw[sU][e];
            const T uD = u_prev, vD = v_prev, wD = w_prev;

            const T mxC = momc(rc, uc, rho0), myC = momc(rc, vc, rho0), mzC = momc(rc, wc, rho0);
            const T mxE = momc(rE, uE, rho0), myE = momc(rE, vE, rho0), mzE = momc(rE, wE, rho0);
            const T mxW = momc(rW, uW, rho0), myW = momc(rW, vW, rho0), mzW = momc(rW, wW, rho0);
            const T mxN = momc(rN, uN, rho0), myN = momc(rN, vN, rho0), mzN = momc(rN, wN, rho0);
            const T mxS = momc(rS, uS, rho0), myS = momc(rS, vS, rho0), mzS = momc(rS, wS, rho0);
            const T mxU = momc(rU, uU, rho0), myU = momc(rU, vU, rho0), mzU = momc(rU, wU, rho0);
            const T mxD = momc(rD, uD, rho0), myD = momc(rD, vD, rho0), mzD = momc(rD, wD, rho0);

            const T fxx = ((fmaT(mxE, uE, cs2 * rE) - fmaT(mxW, uW, cs2 * rW)) + (mxN * vN - mxS * vS)) +
                          (mxU * wU - mxD * wD);
            const T fyy = ((myE * uE - myW * uW) + (fmaT(myN, vN, cs2 * rN) - fmaT(myS, vS, cs2 * rS))) +
                          (myU * wU - myD * wD);
            const T fzz = ((mzE * uE - mzW * uW) + (mzN * vN - mzS * vS)) +
                          (fmaT(mzU, wU, cs2 * rU) - fmaT(mzD, wD, cs2 * rD));
            const T lpx = (((mxE + mxW) + (mxN + mxS)) + (mxU + mxD)) - T(6) * mxC;
            const T lpy = (((myE + myW) + (myN + myS)) + (myU + myD)) - T(6) * myC;
            const T lpz = (((mzE + mzW) + (mzN + mzS)) + (mzU + mzD)) - T(6) * mzC;
            const T sx = (dc[dO + 1] - dc[dO - 1]) - (rE - rW);
            const T sy = (dc[dO + DX] - dc[dO - DX]) - (rN - rS);
            const T sz = (rn_next - rn_prev) - (rU - rD);
            const T rho_n = rho0 + rnC;
            T gx_ = c.gdt[0];
            if (c.fx) gx_ = fmaT(c.dt, c.fx[gy], gx_);
            const T dmx = fmaT(rho_n, gx_, fmaT(-c.ks, sx, fmaT(c.kv, lpx, -c.cg * fxx)));
            const T dmy = fmaT(rho_n, c.gdt[1], fmaT(-c.ks, sy, fmaT(c.kv, lpy, -c.cg * fyy)));
            const T dmz = fmaT(rho_n, c.gdt[2], fmaT(-c.ks, sz, fmaT(c.kv, lpz, -c.cg * fzz)));
            const T drn = rnC - rc;
            const T inv = recipT(rho_n);
            const size_t o = (size_t)k * plane + (size_t)gy * nx + gx;
            out.r[o] = rnC;
            out.u[o] = fmaT(fmaT(-uc, drn, dmx), inv, uc);
            out.v[o] = fmaT(fmaT(-vc, drn, dmy), inv, vc);
            out.w[o] = fmaT(fmaT(-wc, drn, dmz), inv, wc);
        }
        r_prev = rc;
        u_prev = uc;
        v_prev = vc;
        w_prev = wc;
        rn_prev = rnC;
    }
}

template <typename T, int TX, int TY>
static hipError_t launch3d_variant(const Coef<T>& c, const State<T>& in, const State<T>& out, int zc,
                                   hipStream_t s)
{
    const int nbx = (c.nx + TX - 1) / TX, nby = (c.ny + TY - 1) / TY, nbz = (c.nz + zc - 1) / zc;
    hipLaunchKernelGGL((step3d_kernel<T, TX, TY>), dim3(nbx * nby * nbz), dim3(TX * TY), 0, s, c, in, out, zc,
                       nbx, nby);
    return hipGetLastError();
}

// tile codes (3D): low byte = in-plane shape, upper bits = z chunk / 16
template <typename T>
hipError_t launch_step3d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile, hipStream_t s)
{
    int zc = (tile >> 8) * 16;
    if (zc <= 0) zc = 64;
    if (zc > c.nz) zc = c.nz;
    switch (tile & 0xff) {
        case 1: return launch3d_variant<T, 32, 8>(c, in, out, zc, s);
        case 2: return launch3d_variant<T, 64, 8>(c, in, out, zc, s);
        case 3: return launch3d_variant<T, 32, 4>(c, in, out, zc, s);
        case 4: return launch3d_variant<T, 64, 2>(c, in, out, zc, s);
        default: return launch3d_variant<T, 64, 4>(c, in, out, zc, s);
    }
}

template hipError_t launch_step3d<float>(const Coef<float>&, const State<float>&, const State<float>&, int, hipStream_t);
template hipError_t launch_step3d<double>(const Coef<double>&, const State<double>&, const State<double>&, int, hipStream_t);

}  // namespace acm
