// Two SMAME steps per launch on fully periodic 3D boxes (the one-step fast
// path's conditions: rho0 = 1, no per-node force).  A 2.5D march along z
// forms level n+1 on the tile plus a two-node ring, keeps it in LDS, and from
// it level n+2 on the tile, so HBM sees one read of level n and one write of
// level n+2 per node: half the traffic of two one-step launches, for about
// 1.3x their arithmetic (level n+1 is formed on (TX+4)(TY+4) nodes per
// TX*TY outputs).  Every value comes from rho_new_3d and momentum3d, the
// expressions of the one-step kernel in the same order, so a launch here
// equals two one-step launches bit for bit.
//
// In-plane regions around a TX x TY tile:
//   A  level n on the tile + 4 ring      staged from HBM, 3-plane LDS ring
//   B  drho' on the tile + 3 ring        3 planes
//   C  level n+1 on the tile + 2 ring    3-plane LDS ring
//   D  drho'' on the tile + 1 ring       3 planes
// One iteration forms level n+1 on plane k1 (stage 1) and level n+2 on plane
// k2 = k1 - 2 (stage 2) with four barriers; level-n planes k1 + 3 .. k1 + 5
// are in flight in registers meanwhile.  The plane below the one being
// updated (level n at the stage-1 nodes, level n+1 at the own node) and its
// drho' / drho'' stay in registers, as in the one-step march.
//
// Selected by tile codes 14 and 15 only.  On a 256^3 grid it takes 318 us per
// launch (159 us per step) against 133-137 us per one-step launch: the four
// level-n+1 fields on the grown tile take LDS that holds the CU to eight
// waves (two per SIMD), too few to hide the LDS latency of the larger
// per-node work, so halving the HBM traffic does not pay.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "acm_internal.h"
#include "step3d.h"

namespace acm {

namespace {

// All four regions share the row stride AX of region A, so that a wave's
// lanes walk consecutive LDS words (no bank conflicts where a narrower region
// would wrap to its next row) and the index of a point in one region is its
// index in another plus a constant; the columns past a region's width are
// left idle.
template <int TX, int TY>
struct ShapeP {
    static constexpr int AX = TX + 8;
    static constexpr int AXY = AX * (TY + 8), BXY = AX * (TY + 6), CXY = AX * (TY + 4), DXY = AX * (TY + 2);
    static constexpr int BW = TX + 6, CW = TX + 4, DW = TX + 2;  // valid columns of B, C, D
    static constexpr int NT = TX * TY;                           // one output column per thread
    static constexpr int NA = (AXY + NT - 1) / NT, NB = (BXY + NT - 1) / NT;
    static constexpr int NC = (CXY + NT - 1) / NT, ND = (DXY + NT - 1) / NT;
};

template <typename T>
constexpr size_t pair_lds_bytes(int tx, int ty)
{
    return sizeof(T) * (size_t)(tx + 8) * (12 * (ty + 8) + 3 * (ty + 6) + 12 * (ty + 4) + 3 * (ty + 2));
}

__device__ __forceinline__ int pwrap(int g, int n)
{
    g %= n;
    return g < 0 ? g + n : g;
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void step3d_pair_kernel(Coef<T> c, State<T> in, State<T> out, int zc, int nbx,
                                                             int nby)
{
    using S = ShapeP<TX, TY>;
    constexpr int AX = S::AX, AXY = S::AXY, BXY = S::BXY, CXY = S::CXY, DXY = S::DXY, NT = S::NT;
    constexpr int NA = S::NA, NB = S::NB, NC = S::NC, ND = S::ND;
    static_assert(pair_lds_bytes<T>(TX, TY) <= 160 * 1024, "LDS");
    __shared__ T ar[3][AXY], au[3][AXY], av[3][AXY], aw[3][AXY];
    __shared__ T bd[3][BXY];
    __shared__ T cr[3][CXY], cu[3][CXY], cv[3][CXY], cw[3][CXY];
    __shared__ T dd[3][DXY];

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
    const unsigned fbytes = pbytes * (unsigned)nz;  // below 2^31 (checked by the launcher)
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;

    // staging map of region A (periodic images); padding lanes load a valid
    // duplicate and skip the LDS store
    unsigned voff[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int q = tid + i * NT;
        const int qq = q < AXY ? q : tid;
        const int ly = qq / AX, lx = qq - ly * AX;
        const int sx = pwrap(x0 + lx - 4, nx), sy = pwrap(y0 + ly - 4, ny);
        voff[i] = ((unsigned)sy * (unsigned)nx + (unsigned)sx) * (unsigned)sizeof(T);
    }
    // slots of regions B, C and D held by this thread, and whether each is a
    // point of its region; the point at B (C, D) index q sits at A index
    // q + AX + 1 (q + 2 AX + 2, and B index q + AX + 1; C index q + AX + 1)
    bool vB[NB], vC[NC], vD[ND];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int q = tid + i * NT;
        vB[i] = q < BXY && q % AX < S::BW;
    }
    T fx1[NC];  // the row's x force at the stage-1 nodes
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const int q = tid + i * NT;
        vC[i] = q < CXY && q % AX < S::CW;
        fx1[i] = c.fx ? c.fx[pwrap(y0 + min(q, CXY - 1) / AX - 2, ny)] : T(0);
    }
#pragma unroll
    for (int i = 0; i < ND; ++i) {
        const int q = tid + i * NT;
        vD[i] = q < DXY && q % AX < S::DW;
    }
    // the own node: C and D indices, output byte offset (a lane outside the
    // grid gets the descriptor size, so the range check drops its stores)
    const int e2 = (ty + 2) * AX + tx + 2, d2 = (ty + 1) * AX + tx + 1;
    const int gx = x0 + tx, gy = y0 + ty;
    const bool act = gx < nx && gy < ny;
    const unsigned ooff = act ? ((unsigned)gy * (unsigned)nx + (unsigned)gx) * (unsigned)sizeof(T) : fbytes;
    const T fx2 = c.fx ? c.fx[min(gy, ny - 1)] : T(0);

    // three register sets: level-n plane k1 + 5 is fetched while plane k1 + 2
    // is stored, so a load has three iterations to arrive
    T pr[3][NA], pu[3][NA], pv[3][NA], pw[3][NA];
    auto fetch = [&](int gz, auto bset) {
        constexpr int b = decltype(bset)::value;
        const PlaneAccess<false, T> pa(in, pwrap(gz, nz), plane, pbytes, fbytes);
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            pr[b][i] = bload((T*)nullptr, pa.r, voff[i], pa.soff);
            pu[b][i] = bload((T*)nullptr, pa.u, voff[i], pa.soff);
            pv[b][i] = bload((T*)nullptr, pa.v, voff[i], pa.soff);
            pw[b][i] = bload((T*)nullptr, pa.w, voff[i], pa.soff);
        }
    };
    auto store = [&](int s, auto bset) {
        constexpr int b = decltype(bset)::value;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int q = tid + i * NT;
            if ((i + 1) * NT <= AXY || q < AXY) {
                ar[s][q] = pr[b][i];
                au[s][q] = pu[b][i];
                av[s][q] = pv[b][i];
                aw[s][q] = pw[b][i];
            }
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    // drho' of the level-n plane in slot s0 (below sD, above sU) on region B
    auto ring_b = [&](int s0, int sD, int sU, int db) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int q = tid + i * NT;
            if (vB[i])
                bd[db][q] = rho_new_3d<false, T, AX>(c, ar[s0], au[s0], av[s0], ar[sD], aw[sD], ar[sU], aw[sU],
                                                     q + AX + 1);
        }
    };
    // drho'' of the level-(n+1) plane in slot s0 on region D
    auto ring_d = [&](int s0, int sD, int sU, int dq) {
#pragma unroll
        for (int i = 0; i < ND; ++i) {
            const int q = tid + i * NT;
            if (vD[i])
                dd[dq][q] = rho_new_3d<false, T, AX>(c, cr[s0], cu[s0], cv[s0], cr[sD], cw[sD], cr[sU], cw[sU],
                                                     q + AX + 1);
        }
    };

    // stage-1 registers: level n one plane below, and its drho'
    T d1r[NC], d1u[NC], d1v[NC], d1w[NC], n1D[NC];
    // stage-2 registers: level n+1 one plane below the own node, and its drho''
    T d2r = T(0), d2u = T(0), d2v = T(0), d2w = T(0), n2D = T(0);

    // level-n plane p, its drho', and level n+1 and drho'' of plane p sit in
    // slot (p - z0 + 2) mod 3 of their rings; the loop is unrolled three
    // times so that every slot and register set is fixed at compile time
    fetch(z0 - 4, I0{});
    store(1, I0{});
    fetch(z0 - 3, I0{});
    store(2, I0{});
    fetch(z0 - 2, I0{});
    store(0, I0{});
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const int e = (vC[i] ? tid + i * NT : 0) + 2 * AX + 2;
        n1D[i] = rho_new_3d<false, T, AX>(c, ar[2], au[2], av[2], ar[1], aw[1], ar[0], aw[0], e);
        d1r[i] = ar[2][e];
        d1u[i] = au[2][e];
        d1v[i] = av[2][e];
        d1w[i] = aw[2][e];
    }
    __syncthreads();  // plane z0-1 replaces plane z0-4
    fetch(z0 - 1, I0{});
    store(1, I0{});
    __syncthreads();
    ring_b(0, 2, 1, 0);  // drho'(z0-2)
    fetch(z0, I0{});
    fetch(z0 + 1, I1{});
    fetch(z0 + 2, I2{});
    __syncthreads();  // the first store replaces plane z0-3, read just above

    // iteration k1 = z0 - 2 + j has J = j mod 3: plane k1 in slot J, and it
    // stores register set J
    auto iter = [&](int k1, auto jc) {
        constexpr int J = decltype(jc)::value;
        constexpr int sa = J, sa1 = (J + 1) % 3, sa2 = (J + 2) % 3;  // planes k1, k1+1, k1+2
        constexpr int sam1 = sa2, sam2 = sa1;                        // planes k1-1, k1-2
        constexpr int sb = sa, sb1 = sa1;
        store(sa2, jc);  // level n, plane k1+2
        fetch(min(k1 + 5, z1 + 3), jc);
        __syncthreads();
        ring_b(sa1, sa, sa2, sb1);  // drho'(k1+1)
        __syncthreads();
        // stage 1: level n+1 on region C of plane k1
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const int q = tid + i * NT;
            if (vC[i]) {
                const int e = q + 2 * AX + 2, b = q + AX + 1;
                const T* r0 = ar[sa];
                const T* u0 = au[sa];
                const T* v0 = av[sa];
                const T* w0 = aw[sa];
                const Pt3<T> C{r0[e], u0[e], v0[e], w0[e]};
                const Pt3<T> E{r0[e + 1], u0[e + 1], v0[e + 1], w0[e + 1]};
                const Pt3<T> W{r0[e - 1], u0[e - 1], v0[e - 1], w0[e - 1]};
                const Pt3<T> N{r0[e + AX], u0[e + AX], v0[e + AX], w0[e + AX]};
                const Pt3<T> Sn{r0[e - AX], u0[e - AX], v0[e - AX], w0[e - AX]};
                const Pt3<T> U{ar[sa1][e], au[sa1][e], av[sa1][e], aw[sa1][e]};
                const Pt3<T> D{d1r[i], d1u[i], d1v[i], d1w[i]};
                const T* dc = bd[sb];
                const T rnC = dc[b];
                T ro, uo, vo, wo;
                momentum3d<false, T>(c, C, E, W, N, Sn, U, D, rnC, dc[b + 1], dc[b - 1], dc[b + AX], dc[b - AX],
                                     bd[sb1][b], n1D[i], fx1[i], false, T(0), T(0), T(0), ro, uo, vo, wo);
                cr[sa][q] = ro;
                cu[sa][q] = uo;
                cv[sa][q] = vo;
                cw[sa][q] = wo;
                d1r[i] = C.r;
                d1u[i] = C.u;
                d1v[i] = C.v;
                d1w[i] = C.w;
                n1D[i] = rnC;
            }
        }
        __syncthreads();
        if (k1 >= z0) ring_d(sam1, sam2, sa, sam1);  // drho''(k1-1) from level n+1 planes k1-2 .. k1
        __syncthreads();
        if (k1 == z0 + 1) {  // level n+1 of plane z0-1 at the own node
            d2r = cr[sam2][e2];
            d2u = cu[sam2][e2];
            d2v = cv[sam2][e2];
            d2w = cw[sam2][e2];
            n2D = dd[sam2][d2];
        } else if (k1 >= z0 + 2) {
            // stage 2: level n+2 at the own node of plane k2 = k1 - 2
            const int k2 = k1 - 2;
            const T* r0 = cr[sam2];
            const T* u0 = cu[sam2];
            const T* v0 = cv[sam2];
            const T* w0 = cw[sam2];
            const int e = e2;
            const Pt3<T> C{r0[e], u0[e], v0[e], w0[e]};
            const Pt3<T> E{r0[e + 1], u0[e + 1], v0[e + 1], w0[e + 1]};
            const Pt3<T> W{r0[e - 1], u0[e - 1], v0[e - 1], w0[e - 1]};
            const Pt3<T> N{r0[e + AX], u0[e + AX], v0[e + AX], w0[e + AX]};
            const Pt3<T> Sn{r0[e - AX], u0[e - AX], v0[e - AX], w0[e - AX]};
            const Pt3<T> U{cr[sam1][e], cu[sam1][e], cv[sam1][e], cw[sam1][e]};
            const Pt3<T> D{d2r, d2u, d2v, d2w};
            const T* dc = dd[sam2];  // drho''(k2)
            const T rnC = dc[d2];
            T ro, uo, vo, wo;
            momentum3d<false, T>(c, C, E, W, N, Sn, U, D, rnC, dc[d2 + 1], dc[d2 - 1], dc[d2 + AX], dc[d2 - AX],
                                 dd[sam1][d2], n2D, fx2, false, T(0), T(0), T(0), ro, uo, vo, wo);
            const PlaneAccess<false, T> po(out, k2, plane, pbytes, fbytes);
            bstore(ro, po.r, ooff, po.soff);
            bstore(uo, po.u, ooff, po.soff);
            bstore(vo, po.v, ooff, po.soff);
            bstore(wo, po.w, ooff, po.soff);
            d2r = C.r;
            d2u = C.u;
            d2v = C.v;
            d2w = C.w;
            n2D = rnC;
        }
    };
    int k1 = z0 - 2;
    for (; k1 + 2 <= z1 + 1; k1 += 3) {
        iter(k1, I0{});
        iter(k1 + 1, I1{});
        iter(k1 + 2, I2{});
    }
    if (k1 <= z1 + 1) iter(k1, I0{});
    if (k1 + 1 <= z1 + 1) iter(k1 + 1, I1{});
}

template <typename T, int TX, int TY>
hipError_t launch_pair(const Coef<T>& c, const State<T>& in, const State<T>& out, int zc, hipStream_t s)
{
    const int nbx = (c.nx + TX - 1) / TX, nby = (c.ny + TY - 1) / TY, nbz = (c.nz + zc - 1) / zc;
    hipLaunchKernelGGL((step3d_pair_kernel<T, TX, TY>), dim3(nbx * nby * nbz), dim3(TX * TY), 0, s, c, in, out, zc,
                       nbx, nby);
    return hipGetLastError();
}

}  // namespace

template <typename T>
bool step3d_pair_ok(const Coef<T>& c, int tile)
{
    const int shape = tile & 0xff;
    if (shape != 14 && shape != 15) return false;
    if (sizeof(T) == 8 && shape == 14) return false;
    return c.nz >= 2 && !c.nonperiodic && c.rho0 == T(1) && !c.fst[0] &&
           (size_t)c.nx * c.ny * c.nz * sizeof(T) < (size_t(1) << 31);
}

// tile codes: 14 = 64 x 8 (FP32), 15 = 32 x 8; bits 8+ = z chunk / 16.  The
// default chunk is the longest (128, 64, 32 or 16 planes) that still gives
// every CU a workgroup.
template <typename T>
hipError_t launch_step3d_pair(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile, hipStream_t s)
{
    const int shape = tile & 0xff;
    const int tx = shape == 14 ? 64 : 32, ty = 8;
    int zc = (tile >> 8) * 16;
    if (zc <= 0) {
        static int ncu = 0;
        if (ncu == 0) {
            int dev = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
                ncu = 256;
        }
        const long cols = (long)((c.nx + tx - 1) / tx) * ((c.ny + ty - 1) / ty);
        zc = 16;
        for (int z : {128, 64, 32}) {
            if (cols * ((c.nz + z - 1) / z) >= ncu) {
                zc = z;
                break;
            }
        }
    }
    if (zc > c.nz) zc = c.nz;
    if constexpr (sizeof(T) == 8) return launch_pair<T, 32, 8>(c, in, out, zc, s);
    else {
        if (shape == 14) return launch_pair<T, 64, 8>(c, in, out, zc, s);
        return launch_pair<T, 32, 8>(c, in, out, zc, s);
    }
}

template bool step3d_pair_ok<float>(const Coef<float>&, int);
template bool step3d_pair_ok<double>(const Coef<double>&, int);
template hipError_t launch_step3d_pair<float>(const Coef<float>&, const State<float>&, const State<float>&, int,
                                              hipStream_t);
template hipError_t launch_step3d_pair<double>(const Coef<double>&, const State<double>&, const State<double>&, int,
                                               hipStream_t);

}  // namespace acm
