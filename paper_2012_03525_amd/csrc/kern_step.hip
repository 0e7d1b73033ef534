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
#include <type_traits>

#include "acm_internal.h"
#include "step3d.h"
#include "tile2d.h"

namespace acm {

// ===========================================================================
// 2D (tile function in tile2d.h)
// ===========================================================================
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
// chunk of ZC planes.  NS input planes (with a two-node in-plane halo) are
// resident in LDS as a ring; drho' is computed one plane ahead on the tile
// plus a one-node ring, so every node's drho' is formed exactly once per
// workgroup.  Plane k+4 is fetched into registers while plane k is computed.
// NS = 4 keeps the plane being written clear of the planes being read (two
// barriers per plane); NS = 3 takes 3/4 of the LDS and a third barrier
// before a slot is overwritten.
//
// GEN = false is the fast path for fully periodic boxes (nz >= 2) with rho0 = 1: no
// ghost transforms, m = u + drho u.  GEN = true handles every boundary type,
// any rho0 and the per-node surface-tension force of two-phase runs.  Both evaluate the same expressions, so a periodic rho0 = 1
// case gives identical bits on either path.
// ===========================================================================
template <int TX, int TY, int RPT>
struct Shape3 {
    static constexpr int RX = TX + 4, RY = TY + 4, RXY = RX * RY;
    static constexpr int DX = TX + 2, DY = TY + 2, DXY = DX * DY;
    // the drho' ring is stored with the staged region's row stride RX (the
    // last two columns of each row unused), so a wave's lanes walk
    // consecutive LDS words instead of wrapping to the next DX-wide row
    static constexpr int SDXY = RX * DY;
    static constexpr int NT = TX * TY / RPT;        // threads; each owns RPT rows of one column
    static constexpr int YS = TY / RPT;             // row stride between a thread's rows
    static constexpr int NL = (RXY + NT - 1) / NT;  // plane points staged per thread
    static constexpr int ND = (SDXY + NT - 1) / NT;  // drho' slots per thread
};

// WPE > 0 asks the compiler for at least WPE waves per SIMD (a register
// budget of 512 / WPE VGPRs); 0 leaves the budget to the compiler.
template <typename T, int TX, int TY, int RPT, bool GEN, bool WIDE, int NS, int WPE = 0>
__global__ __launch_bounds__(TX * TY / RPT) __attribute__((amdgpu_waves_per_eu(WPE))) void step3d_kernel(Coef<T> c, State<T> in, State<T> out, int zc,
                                                                int nbx, int nby)
{
    using S = Shape3<TX, TY, RPT>;
    constexpr int RX = S::RX, RXY = S::RXY, DX = S::DX, SDXY = S::SDXY, NT = S::NT, NL = S::NL, ND = S::ND;
    constexpr int YS = S::YS;
    static_assert(NS == 3 || NS == 4, "three or four resident planes");
    // plane p lives in slot (p - z0) mod NS; the loop body is unrolled over P
    // planes so that every slot, register set and drho' buffer is fixed at
    // compile time
    constexpr int P = NS == 4 ? 4 : 6;
    __shared__ T sr[NS][RXY], su[NS][RXY], sv[NS][RXY], sw[NS][RXY];
    __shared__ T sd[2][SDXY];
    // ghost velocity rules u_a = gs[0][f][a] u_a + gs[1][f][a] per crossed
    // face f, looked up per lane from LDS (GEN only)
    __shared__ T gs[2][6][3];

    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = lb % nbx;
    const int t1 = lb / nbx;
    const int by = t1 % nby, bz = t1 / nby;
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = bz * zc;
    const int z1 = min(z0 + zc, c.nz);
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const unsigned pbytes = plane * (unsigned)sizeof(T);
    const unsigned fbytes = WIDE ? 0u : pbytes * (unsigned)nz;  // below 2^31 unless WIDE
    const int tid = threadIdx.x;
    const int tx = tid % TX, tyb = tid / TX;
    const int gx = x0 + tx;
    const bool inplane_interior = (x0 >= 2) && (x0 + TX + 2 <= nx) && (y0 >= 2) && (y0 + TY + 2 <= ny);
    const bool zperiodic = GEN ? (c.bc[4] == BC_PERIODIC) : true;

    // per-thread staging map: in-plane byte offset and crossed faces.
    // Padding lanes (q >= RXY) load a valid duplicate and skip the LDS store.
    unsigned voff[NL];
    signed char sfx[NL], sfy[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int q = tid + i * NT;
        const int qq = q < RXY ? q : tid;
        const int ly = qq / RX, lx = qq - ly * RX;
        int fx, fy;
        const int sx = map_coord(x0 + lx - 2, nx, c.bc[0], 0, fx);
        const int sy = map_coord(y0 + ly - 2, ny, c.bc[2], 2, fy);
        voff[i] = ((unsigned)sy * (unsigned)nx + (unsigned)sx) * (unsigned)sizeof(T);
        sfx[i] = (signed char)fx;
        sfy[i] = (signed char)fy;
    }
    // drho' ring positions (mirror substitution for wall / symmetry ghosts)
    int dsrc[ND];
    bool dval[ND];  // the slot holds a ring point
#pragma unroll
    for (int i = 0; i < ND; ++i) {
        const int q = tid + i * NT;
        dval[i] = q < SDXY && q % RX < DX;
        const int qq = dval[i] ? q : 0;
        const int ly = qq / RX, lx = qq - ly * RX;
        int ex = lx + 1, ey = ly + 1;
        if (GEN && !inplane_interior && c.nonperiodic) {
            const int mx = mirror_coord(x0 + lx - 1, nx, c.bc[0]);
            const int my = mirror_coord(y0 + ly - 1, ny, c.bc[2]);
            ex = min(max(mx - x0 + 2, 1), DX);
            ey = min(max(my - y0 + 2, 1), S::DY);
        }
        dsrc[i] = ey * RX + ex;
    }
    // output byte offsets of the thread's nodes (same in every plane).  A
    // lane outside the grid (ragged tile) computes like the others but gets
    // the descriptor size as its offset, so the range check drops its stores
    // (no branch around the stores: the memory-counter waits stay exact).
    unsigned ooff[RPT], oidx[RPT];
    T fxr[RPT];  // per-row x force, dt excluded
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int gy = y0 + tyb + r * YS;
        const bool act = (gx < nx) && (gy < ny);
        oidx[r] = act ? (unsigned)gy * (unsigned)nx + (unsigned)gx : 0u;
        ooff[r] = act ? oidx[r] * (unsigned)sizeof(T) : (WIDE ? pbytes : fbytes);
        fxr[r] = c.fx ? c.fx[min(gy, ny - 1)] : T(0);
    }

    if constexpr (GEN) {
        if (tid < 18) {
            gs[0][tid / 3][tid % 3] = c.fs[tid / 3][tid % 3];
            gs[1][tid / 3][tid % 3] = c.fo[tid / 3][tid % 3];
        }
        __syncthreads();
    }
    auto ghost = [&](int f, T& u, T& v, T& w) {
        u = fmaT(gs[0][f][0], u, gs[1][f][0]);
        v = fmaT(gs[0][f][1], v, gs[1][f][1]);
        w = fmaT(gs[0][f][2], w, gs[1][f][2]);
    };

    T pr[2][NL], pu[2][NL], pv[2][NL], pw[2][NL];
    int pfz0 = -1, pfz1 = -1;  // z face crossed by the plane in register set 0 / 1
    // fetch plane gz into register set b (ghost planes mapped)
    auto fetch = [&](int gz, auto bset) {
        constexpr int b = decltype(bset)::value;
        int sz;
        if constexpr (GEN) {
            int fz;
            sz = map_coord(gz, nz, c.bc[4], 4, fz);
            if constexpr (b == 0) pfz0 = fz;
            else pfz1 = fz;
        } else {
            sz = gz < 0 ? gz + nz : (gz >= nz ? gz - nz : gz);  // periodic z, nz >= 2
        }
        const PlaneAccess<WIDE, T> pa(in, sz, plane, pbytes, fbytes);
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            pr[b][i] = bload((T*)nullptr, pa.r, voff[i], pa.soff);
            pu[b][i] = bload((T*)nullptr, pa.u, voff[i], pa.soff);
            pv[b][i] = bload((T*)nullptr, pa.v, voff[i], pa.soff);
            pw[b][i] = bload((T*)nullptr, pa.w, voff[i], pa.soff);
        }
    };
    // register set b into LDS slot; the ghost velocity rules are applied here,
    // when the loads have long arrived, rather than right after issuing them
    auto store = [&](auto slotc, auto bset) {
        constexpr int slot = decltype(slotc)::value;
        constexpr int b = decltype(bset)::value;
        if constexpr (GEN) {
            if (c.nonperiodic) {
                const int fz = b == 0 ? pfz0 : pfz1;
#pragma unroll
                for (int i = 0; i < NL; ++i) {
                    // faces crossed in x, then y, then z order
                    if (sfx[i] >= 0) ghost(sfx[i], pu[b][i], pv[b][i], pw[b][i]);
                    if (sfy[i] >= 0) ghost(sfy[i], pu[b][i], pv[b][i], pw[b][i]);
                    if (fz >= 0) ghost(fz, pu[b][i], pv[b][i], pw[b][i]);
                }
            }
        }
        // A padding lane (q >= RXY) holds the value of position tid, which the
        // same thread also writes as its element 0: it writes that value there
        // again instead of branching around the store.
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int q = tid + i * NT;
            const int e = ((i + 1) * NT <= RXY || q < RXY) ? q : tid;
            sr[slot][e] = pr[b][i];
            su[slot][e] = pu[b][i];
            sv[slot][e] = pv[b][i];
            sw[slot][e] = pw[b][i];
        }
    };
    // drho' of the plane in slot s0 (below sD, above sU) on the tile + ring into sd[ds]
    auto ring = [&](auto s0c, auto sDc, auto sUc, auto dsc) {
        constexpr int s0 = decltype(s0c)::value, sD = decltype(sDc)::value, sU = decltype(sUc)::value;
        constexpr int ds = decltype(dsc)::value;
#pragma unroll
        for (int i = 0; i < ND; ++i) {
            const int q = tid + i * NT;
            if (dval[i])
                sd[ds][q] = rho_new_3d<GEN, T, RX>(c, sr[s0], su[s0], sv[s0], sr[sD], sw[sD], sr[sU], sw[sU],
                                                   dsrc[i]);
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;

    // ---- prologue: planes z0-1 .. z0+1 resident and drho'(z0) on the ring,
    // planes z0+2 and z0+3 in flight in register sets 0 and 1
    T rn_prev[RPT], r_prev[RPT], u_prev[RPT], v_prev[RPT], w_prev[RPT];
    // drho'(z0-1) at the own nodes and the level-n values of plane z0-1
    auto own_below = [&](auto sMc, auto sDc, auto sUc) {
        constexpr int sM = decltype(sMc)::value, sD = decltype(sDc)::value, sU = decltype(sUc)::value;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int eo = (tyb + r * YS + 2) * RX + (tx + 2);
            rn_prev[r] = T(0);
            if (zperiodic || z0 > 0)  // planes z0-2, z0-1, z0 are resident
                rn_prev[r] = rho_new_3d<GEN, T, RX>(c, sr[sM], su[sM], sv[sM], sr[sD], sw[sD], sr[sU], sw[sU], eo);
            r_prev[r] = sr[sM][eo];
            u_prev[r] = su[sM][eo];
            v_prev[r] = sv[sM][eo];
            w_prev[r] = sw[sM][eo];
        }
    };
    fetch(z0 - 2, I0{});
    fetch(z0 - 1, I1{});
    if constexpr (NS == 4) {
        store(I2{}, I0{});
        store(I3{}, I1{});
        fetch(z0, I0{});
        fetch(z0 + 1, I1{});
        store(I0{}, I0{});
        store(I1{}, I1{});
        fetch(z0 + 2, I0{});
        fetch(z0 + 3, I1{});
        __syncthreads();
        ring(I0{}, I3{}, I1{}, I0{});
        own_below(I3{}, I2{}, I0{});
    } else {
        store(I1{}, I0{});
        store(I2{}, I1{});
        fetch(z0, I0{});
        fetch(z0 + 1, I1{});
        store(I0{}, I0{});
        fetch(z0 + 2, I0{});
        __syncthreads();
        own_below(I2{}, I1{}, I0{});
        __syncthreads();  // plane z0+1 replaces plane z0-2
        store(I1{}, I1{});
        fetch(z0 + 3, I1{});
        __syncthreads();
        ring(I0{}, I2{}, I1{}, I0{});
    }
    __syncthreads();
    if (!(zperiodic || z0 > 0)) {  // wall / symmetry at z = 0: drho'(-1) is the mirror value
#pragma unroll
        for (int r = 0; r < RPT; ++r) rn_prev[r] = sd[0][(tyb + r * YS + 1) * RX + (tx + 1)];
    }

    const T rho0 = c.rho0, cs2 = c.cs2;
    // one plane; J = k mod 4 fixes every LDS slot and register set at compile time
    auto iterate = [&](int k, auto jc) {
        constexpr int J = decltype(jc)::value;
        constexpr int s0 = J % NS, sU = (J + 1) % NS, s2 = (J + 2) % NS;
        using BS = std::integral_constant<int, J & 1>;
        if constexpr (NS == 3) __syncthreads();  // slot s2 held plane k-1, read by the previous plane
        const size_t ob = (size_t)k * plane;
        // two-phase: surface-tension force phi G_iso mu of this plane, loaded
        // before the prefetch so that waiting for it leaves the prefetch in flight
        T fst[3][RPT];
        if constexpr (GEN) {
            if (c.fst[0]) {
#pragma unroll
                for (int r = 0; r < RPT; ++r)
#pragma unroll
                    for (int a = 0; a < 3; ++a) fst[a][r] = c.fst[a][ob + oidx[r]];
            }
        }
        store(std::integral_constant<int, s2>{}, BS{});  // plane k+2 (its slot held plane k-2)
        fetch(min(k + 4, z1 + 1), BS{});  // past the chunk: plane z1+1 again (cached)
        __syncthreads();
        const bool upper_ghost = (!zperiodic) && (k + 1 >= nz);
        if (!upper_ghost)
            ring(std::integral_constant<int, sU>{}, std::integral_constant<int, s0>{},
                 std::integral_constant<int, s2>{}, std::integral_constant<int, (J + 1) & 1>{});
        __syncthreads();

        const T* r0 = sr[s0];
        const T* u0 = su[s0];
        const T* v0 = sv[s0];
        const T* w0 = sw[s0];
        const T* dc = sd[J & 1];
        const T* dn = sd[(J + 1) & 1];
        const PlaneAccess<WIDE, T> po(out, k, plane, pbytes, fbytes);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int ty = tyb + r * YS;
            const int e = (ty + 2) * RX + (tx + 2);
            const int dO = (ty + 1) * RX + (tx + 1);
            const T rc = r0[e], uc = u0[e], vc = v0[e], wc = w0[e];
            const T rnC = dc[dO];
            const T rn_next = upper_ghost ? rnC : dn[dO];
            const T rE = r0[e + 1], rW = r0[e - 1], rN = r0[e + RX], rS = r0[e - RX];
            const T rU = sr[sU][e], rD = r_prev[r];
            const T uE = u0[e + 1], uW = u0[e - 1], uN = u0[e + RX], uS = u0[e - RX];
            const T vE = v0[e + 1], vW = v0[e - 1], vN = v0[e + RX], vS = v0[e - RX];
            const T wE = w0[e + 1], wW = w0[e - 1], wN = w0[e + RX], wS = w0[e - RX];
            const T uU = su[sU][e], vU = sv[sU][e], wU = sw[sU][e];
            const T uD = u_prev[r], vD = v_prev[r], wD = w_prev[r];

            const T mxC = mom3<GEN>(rc, uc, rho0), myC = mom3<GEN>(rc, vc, rho0), mzC = mom3<GEN>(rc, wc, rho0);
            const T mxE = mom3<GEN>(rE, uE, rho0), myE = mom3<GEN>(rE, vE, rho0), mzE = mom3<GEN>(rE, wE, rho0);
            const T mxW = mom3<GEN>(rW, uW, rho0), myW = mom3<GEN>(rW, vW, rho0), mzW = mom3<GEN>(rW, wW, rho0);
            const T mxN = mom3<GEN>(rN, uN, rho0), myN = mom3<GEN>(rN, vN, rho0), mzN = mom3<GEN>(rN, wN, rho0);
            const T mxS = mom3<GEN>(rS, uS, rho0), myS = mom3<GEN>(rS, vS, rho0), mzS = mom3<GEN>(rS, wS, rho0);
            const T mxU = mom3<GEN>(rU, uU, rho0), myU = mom3<GEN>(rU, vU, rho0), mzU = mom3<GEN>(rU, wU, rho0);
            const T mxD = mom3<GEN>(rD, uD, rho0), myD = mom3<GEN>(rD, vD, rho0), mzD = mom3<GEN>(rD, wD, rho0);

            // centred differences of drho (pressure term and density SAT share them)
            const T gxr = rE - rW, gyr = rN - rS, gzr = rU - rD;
            const T fxx = fmaT(cs2, gxr, ((mxE * uE - mxW * uW) + (mxN * vN - mxS * vS)) + (mxU * wU - mxD * wD));
            const T fyy = fmaT(cs2, gyr, ((myE * uE - myW * uW) + (myN * vN - myS * vS)) + (myU * wU - myD * wD));
            const T fzz = fmaT(cs2, gzr, ((mzE * uE - mzW * uW) + (mzN * vN - mzS * vS)) + (mzU * wU - mzD * wD));
            const T lpx = fmaT(T(-6), mxC, ((mxE + mxW) + (mxN + mxS)) + (mxU + mxD));
            const T lpy = fmaT(T(-6), myC, ((myE + myW) + (myN + myS)) + (myU + myD));
            const T lpz = fmaT(T(-6), mzC, ((mzE + mzW) + (mzN + mzS)) + (mzU + mzD));
            const T sx = (dc[dO + 1] - dc[dO - 1]) - gxr;
            const T sy = (dc[dO + RX] - dc[dO - RX]) - gyr;
            const T sz = (rn_next - rn_prev[r]) - gzr;
            const T rho_n = rho0 + rnC;
            T gx_ = c.gdt[0];
            if (c.fx) gx_ = fmaT(c.dt, fxr[r], gx_);
            T dmx = fmaT(rho_n, gx_, fmaT(-c.ks, sx, fmaT(c.kv, lpx, -c.cg * fxx)));
            T dmy = fmaT(rho_n, c.gdt[1], fmaT(-c.ks, sy, fmaT(c.kv, lpy, -c.cg * fyy)));
            T dmz = fmaT(rho_n, c.gdt[2], fmaT(-c.ks, sz, fmaT(c.kv, lpz, -c.cg * fzz)));
            if constexpr (GEN) {
                if (c.fst[0]) {  // -dt phi G_iso mu
                    dmx = fmaT(-c.dt, fst[0][r], dmx);
                    dmy = fmaT(-c.dt, fst[1][r], dmy);
                    dmz = fmaT(-c.dt, fst[2][r], dmz);
                }
            }
            const T drn = rnC - rc;
            const T inv = recipT(rho_n);
            bstore(rnC, po.r, ooff[r], po.soff);
            bstore(fmaT(fmaT(-uc, drn, dmx), inv, uc), po.u, ooff[r], po.soff);
            bstore(fmaT(fmaT(-vc, drn, dmy), inv, vc), po.v, ooff[r], po.soff);
            bstore(fmaT(fmaT(-wc, drn, dmz), inv, wc), po.w, ooff[r], po.soff);
            r_prev[r] = rc;
            u_prev[r] = uc;
            v_prev[r] = vc;
            w_prev[r] = wc;
            rn_prev[r] = rnC;
        }
    };
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    int k = z0;
    for (; k + P - 1 < z1; k += P) {
        iterate(k, I0{});
        iterate(k + 1, I1{});
        iterate(k + 2, I2{});
        iterate(k + 3, I3{});
        if constexpr (P == 6) {
            iterate(k + 4, I4{});
            iterate(k + 5, I5{});
        }
    }
    if (k < z1) iterate(k, I0{});
    if (k + 1 < z1) iterate(k + 1, I1{});
    if (k + 2 < z1) iterate(k + 2, I2{});
    if constexpr (P == 6) {
        if (k + 3 < z1) iterate(k + 3, I3{});
        if (k + 4 < z1) iterate(k + 4, I4{});
    }
}

// the fully periodic fast path applies (rho0 = 1, no per-node force)
template <typename T>
static bool fast3d(const Coef<T>& c)
{
    return !c.nonperiodic && c.rho0 == T(1) && !c.fst[0] && c.nz >= 2;
}

// a shape that only the fast path uses (its wall path would not fit the
// register file at two waves per SIMD)
template <typename T, int TX, int TY, int RPT, int NS>
static hipError_t launch3d_fast(const Coef<T>& c, const State<T>& in, const State<T>& out, int zc, hipStream_t s)
{
    const int nbx = (c.nx + TX - 1) / TX, nby = (c.ny + TY - 1) / TY, nbz = (c.nz + zc - 1) / zc;
    const bool wide = (size_t)c.nx * c.ny * c.nz * sizeof(T) >= (size_t(1) << 31);
    const dim3 grid(nbx * nby * nbz), block(TX * TY / RPT);
    if (!wide)
        hipLaunchKernelGGL((step3d_kernel<T, TX, TY, RPT, false, false, NS>), grid, block, 0, s, c, in, out, zc, nbx, nby);
    else
        hipLaunchKernelGGL((step3d_kernel<T, TX, TY, RPT, false, true, NS>), grid, block, 0, s, c, in, out, zc, nbx, nby);
    return hipGetLastError();
}

// The FP32 wall path of the 8-row, one-row-per-thread shapes asks for four
// waves per SIMD (128 VGPRs, two 8-wave workgroups per CU): at 64 x 8 it
// would otherwise take 144 VGPRs and one workgroup per CU, 20 % slower on a
// walled 256^3 grid, for an 8-byte spill.  (The 4-row shapes would spill
// over 100 bytes per lane under the same cap and keep their budget.)
template <typename T, int TX, int TY, int RPT, int NS = 4>
static hipError_t launch3d_variant(const Coef<T>& c, const State<T>& in, const State<T>& out, int zc,
                                   hipStream_t s)
{
    constexpr int WG = (sizeof(T) == 4 && RPT == 1 && TY == 8) ? 4 : 0;
    const int nbx = (c.nx + TX - 1) / TX, nby = (c.ny + TY - 1) / TY, nbz = (c.nz + zc - 1) / zc;
    const bool fast = fast3d(c);
    const bool wide = (size_t)c.nx * c.ny * c.nz * sizeof(T) >= (size_t(1) << 31);
    const dim3 grid(nbx * nby * nbz), block(TX * TY / RPT);
    if (fast && !wide)
        hipLaunchKernelGGL((step3d_kernel<T, TX, TY, RPT, false, false, NS>), grid, block, 0, s, c, in, out, zc, nbx, nby);
    else if (fast)
        hipLaunchKernelGGL((step3d_kernel<T, TX, TY, RPT, false, true, NS>), grid, block, 0, s, c, in, out, zc, nbx, nby);
    else if (!wide)
        hipLaunchKernelGGL((step3d_kernel<T, TX, TY, RPT, true, false, NS, WG>), grid, block, 0, s, c, in, out, zc, nbx,
                           nby);
    else
        hipLaunchKernelGGL((step3d_kernel<T, TX, TY, RPT, true, true, NS, WG>), grid, block, 0, s, c, in, out, zc, nbx,
                           nby);
    return hipGetLastError();
}

// Default launch shape: 64 x 8 columns with two rows per thread and 64-plane
// chunks.  The 2.5D march gives one workgroup per (column, z chunk), so a
// 96^3 grid at 64 x 8 x 64 would keep only 48 workgroups busy: shorten the
// chunk, then the tile, until the launch has at least two workgroups per CU
// (the choice never changes results).  Chunks go down to 4 planes, below the
// 16-plane steps a tile code can name: on a 96^3 walled grid 32 x 8 columns
// with 4-plane chunks (864 workgroups) take the two-phase step from 63.8 to
// 51.8 us against 32 x 4 columns with 16-plane chunks.
struct Launch3 {
    int code, zc;
};
static Launch3 small_grid_shape(int nx, int ny, int nz, bool fp64)
{
    static int ncu = 0;
    if (ncu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            ncu = 256;
    }
    struct Cand {
        int code, tx, ty, zc;
    };
    static const Cand f32c[] = {{13, 64, 8, 64}, {2, 64, 8, 32}, {2, 64, 8, 16},
                                {1, 32, 8, 16},  {1, 32, 8, 8},  {1, 32, 8, 4}};
    static const Cand f64c[] = {{1, 32, 8, 64}, {1, 32, 8, 32}, {1, 32, 8, 16}, {1, 32, 8, 8}, {1, 32, 8, 4}};
    const Cand* cs = fp64 ? f64c : f32c;
    const int nc = fp64 ? 5 : 6;
    for (int i = 0; i < nc; ++i) {
        const long nb = (long)((nx + cs[i].tx - 1) / cs[i].tx) * ((ny + cs[i].ty - 1) / cs[i].ty) *
                        ((nz + cs[i].zc - 1) / cs[i].zc);
        if (nb >= 2L * ncu || i == nc - 1) return {cs[i].code, cs[i].zc};
    }
    return {0, 64};
}

// Chunk length of the default whole-row launch (6-wave, 4-row bands): the
// march of a chunk of zc planes costs about zc + 4 plane iterations (two
// planes of lead-in and the halo planes), and the launch takes
// ceil(workgroups / CUs) such rounds; the chunk with the fewest plane
// iterations in total wins (64 on 256^3: 256 workgroups, one per CU).
static int rows_default_chunk(int ny, int nz)
{
    static int ncu = 0;
    if (ncu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            ncu = 256;
    }
    static const int cand[] = {4, 8, 12, 16, 24, 32, 48, 64, 96, 128};
    const long nby = (ny + 3) / 4;
    int best = 64;
    long best_cost = -1;
    for (int zc : cand) {
        if (zc > nz && zc != cand[0]) break;
        const long nb = nby * ((nz + zc - 1) / zc);
        const long cost = ((nb + ncu - 1) / ncu) * (long)(std::min(zc, nz) + 4);
        if (best_cost < 0 || cost < best_cost) best_cost = cost, best = zc;
    }
    return best;
}

// tile codes (3D): low byte = in-plane shape, upper bits = z chunk / 16
template <typename T>
hipError_t launch_step3d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile, hipStream_t s)
{
    if (tile == 0 && step3d_rows_ok(c) && c.ny >= 8) {
        // whole x rows per wave: the fastest shape where it applies
        const hipError_t e = launch_step3d_rows<T>(c, in, out, 16, rows_default_chunk(c.ny, c.nz), s);
        if (e != hipErrorInvalidValue) return e;
    }
    int zc;
    if (tile == 0) {
        const Launch3 d = small_grid_shape(c.nx, c.ny, c.nz, sizeof(T) == 8);
        tile = d.code;
        zc = d.zc;
    } else {
        zc = (tile >> 8) * 16;
        if (zc <= 0) zc = 64;
    }
    if (zc > c.nz) zc = c.nz;
    int shape = tile & 0xff;
    if ((shape == 16 || shape == 17 || shape == 19) && step3d_rows_ok(c)) {
        const hipError_t e = launch_step3d_rows<T>(c, in, out, shape, zc, s);
        if (e != hipErrorInvalidValue) return e;
        shape = 0;  // grid too small for the band height: the default shape
    }
    if constexpr (sizeof(T) == 8) {
        // FP64 keeps one row per thread and moderate tiles (LDS and registers)
        switch (shape) {
            case 3: return launch3d_variant<T, 32, 4, 1>(c, in, out, zc, s);
            case 4: return launch3d_variant<T, 64, 4, 1>(c, in, out, zc, s);
            default: return launch3d_variant<T, 32, 8, 1>(c, in, out, zc, s);
        }
    } else {
        switch (shape) {
            case 1: return launch3d_variant<T, 32, 8, 1>(c, in, out, zc, s);
            case 2: return launch3d_variant<T, 64, 8, 1>(c, in, out, zc, s);
            case 3: return launch3d_variant<T, 32, 4, 1>(c, in, out, zc, s);
            case 4: return launch3d_variant<T, 64, 4, 1>(c, in, out, zc, s);
            case 5: return launch3d_variant<T, 64, 16, 2>(c, in, out, zc, s);
            case 7: return launch3d_variant<T, 32, 16, 2>(c, in, out, zc, s);
            case 9: return launch3d_variant<T, 128, 4, 1>(c, in, out, zc, s);
            case 12: return launch3d_variant<T, 128, 8, 1>(c, in, out, zc, s);
            // periodic fast path: two rows per thread (256 threads) and a
            // three-plane ring (44 KB of LDS, 197 VGPRs), 5 % faster than one
            // row per thread at 256^3; other grids: 64 x 8, one row per thread
            case 13:
                if (fast3d(c)) return launch3d_fast<T, 64, 8, 2, 3>(c, in, out, zc, s);
                return launch3d_variant<T, 64, 8, 1>(c, in, out, zc, s);
            default: return launch3d_variant<T, 64, 8, 1>(c, in, out, zc, s);
        }
    }
}

template hipError_t launch_step3d<float>(const Coef<float>&, const State<float>&, const State<float>&, int, hipStream_t);
template hipError_t launch_step3d<double>(const Coef<double>&, const State<double>&, const State<double>&, int, hipStream_t);

}  // namespace acm
