// Two-phase SMAME step in 3D for gfx950: the flow update with the
// surface-tension force and the Cahn-Hilliard equation (Eq. 2.14) by Heun's
// method, as three launches per step (Sec. 2, two-phase paragraphs):
//   1. mu      = 4 a phi (phi^2 - 1) - kappa L_iso phi on the tile and its ring,
//      then F_a = phi G_iso,a mu;  phi* = phi + dt (M L_iso mu - u_a G_iso,a phi)
//   2. flow    = single-phase 3D step (Eqs. 2.10-2.11) with -dt F_a added to the momentum
//   3. mu*     = mu(phi*) on the tile and its ring,
//      then phi^{n+1} = (phi + phi* + dt (M L_iso mu* - u_a G_iso,a phi*)) / 2
// u is u^n in both Heun stages.  Isotropic stencils with D3Q19 weights:
//   G_iso,a f = [2 (f_{+a} - f_{-a}) + sum_{b != a} (f_{+a+b} + f_{+a-b} - f_{-a+b} - f_{-a-b})] / (12 dx)
//   L_iso f   = [2 (sum of the 6 face neighbours) + (sum of the 12 edge neighbours) - 24 f] / (6 dx^2)
// Ghosts: mu is mirrored across walls and symmetry planes (no flux); phi
// and phi* are mirrored, then take the wetting rule of each crossed wall
// face (x, y, z order).  One thread per node; phi is staged per workgroup in
// LDS with a two-node halo, mu is formed in LDS on the tile plus a one-node
// ring (a wall or symmetry ghost takes the value of its mirror node, a
// periodic ghost is formed from wrapped data and equals its image), so mu
// never goes through global memory.
#include "acm_internal.h"

namespace acm {

namespace {

// value of a scalar field at node (i, j, k), which may lie one layer outside
// the grid; WET applies the wetting rule across wall faces, with the face's
// coefficient from the table wbt (LDS: a per-lane lookup there costs no
// scratch memory, unlike one into the kernel arguments)
template <bool WET, typename T>
__device__ __forceinline__ T at(const Coef<T>& c, const T* __restrict__ f, int i, int j, int k, const T* wbt)
{
    int fx, fy, fz;
    const int si = map_coord(i, c.nx, c.bc[0], 0, fx);
    const int sj = map_coord(j, c.ny, c.bc[2], 2, fy);
    const int sk = map_coord(k, c.nz, c.bc[4], 4, fz);
    T v = f[((size_t)sk * c.ny + sj) * c.nx + si];
    if constexpr (WET) {
        if (c.wet) {
            if (fx >= 0) v = wet_ghost(v, wbt[fx]);
            if (fy >= 0) v = wet_ghost(v, wbt[fy]);
            if (fz >= 0) v = wet_ghost(v, wbt[fz]);
        }
    }
    return v;
}

// numerators (the 1/(12 dx) and 1/(6 dx^2) factors are applied by the caller)
template <typename T>
__device__ __forceinline__ T lap_num(const T n[3][3][3])
{
    const T ax = ((n[2][1][1] + n[0][1][1]) + (n[1][2][1] + n[1][0][1])) + (n[1][1][2] + n[1][1][0]);
    const T xy = (n[2][2][1] + n[2][0][1]) + (n[0][2][1] + n[0][0][1]);
    const T xz = (n[2][1][2] + n[2][1][0]) + (n[0][1][2] + n[0][1][0]);
    const T yz = (n[1][2][2] + n[1][2][0]) + (n[1][0][2] + n[1][0][0]);
    return fmaT(T(2), ax, (xy + xz) + yz) - T(24) * n[1][1][1];
}
template <typename T>
__device__ __forceinline__ T gx_num(const T n[3][3][3])
{
    const T e = ((n[2][2][1] + n[2][0][1]) - (n[0][2][1] + n[0][0][1])) +
                ((n[2][1][2] + n[2][1][0]) - (n[0][1][2] + n[0][1][0]));
    return fmaT(T(2), n[2][1][1] - n[0][1][1], e);
}
template <typename T>
__device__ __forceinline__ T gy_num(const T n[3][3][3])
{
    const T e = ((n[2][2][1] + n[0][2][1]) - (n[2][0][1] + n[0][0][1])) +
                ((n[1][2][2] + n[1][2][0]) - (n[1][0][2] + n[1][0][0]));
    return fmaT(T(2), n[1][2][1] - n[1][0][1], e);
}
template <typename T>
__device__ __forceinline__ T gz_num(const T n[3][3][3])
{
    const T e = ((n[2][1][2] + n[0][1][2]) - (n[2][1][0] + n[0][1][0])) +
                ((n[1][2][2] + n[1][0][2]) - (n[1][2][0] + n[1][0][0]));
    return fmaT(T(2), n[1][1][2] - n[1][1][0], e);
}

// Workgroup tile BX x BY x BZ nodes; R region = the tile plus a one-node
// ring (mu), P region = the tile plus two nodes (phi, ghost rules applied
// while staging), so a node's neighbours come from LDS instead of 19
// separate global loads.
// Threads BX x BY x TZ; each owns ZR nodes of its column, TZ planes apart,
// so the staged halo is shared by twice the nodes (the tile is BZ = TZ ZR deep).
constexpr int BX = 32, BY = 4, TZ = 4, ZR = 2, BZ = TZ * ZR, NTH = BX * BY * TZ;
constexpr int RX = BX + 2, RY = BY + 2, RZ = BZ + 2, RXYZ = RX * RY * RZ;

// halo-2 region of a staged phi field and the D3Q19 neighbourhood of LDS
// index e in a region of row length SX and plane height SY
constexpr int PX = BX + 4, PY = BY + 4, PZ = BZ + 4, PXYZ = PX * PY * PZ;

template <int SX, int SY, typename T>
__device__ __forceinline__ void nb19at(const T* s, int e, T n[3][3][3])
{
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if ((dx != 0) + (dy != 0) + (dz != 0) == 3) continue;
                n[1 + dx][1 + dy][1 + dz] = s[e + dx + SX * (dy + SY * dz)];
            }
}

template <bool WET, typename T>
__device__ __forceinline__ void stage_halo2(const Coef<T>& c, const T* __restrict__ f, int i0, int j0, int k0, T* s,
                                            const T* wbt)
{
    const int tid = threadIdx.x + BX * (threadIdx.y + BY * threadIdx.z);
    constexpr int NIT = (PXYZ + NTH - 1) / NTH;
    T v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int q = min(tid + it * NTH, PXYZ - 1);
        const int lz = q / (PX * PY), r = q - lz * (PX * PY), ly = r / PX, lx = r - ly * PX;
        v[it] = at<WET>(c, f, i0 + lx - 2, j0 + ly - 2, k0 + lz - 2, wbt);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it)
        if (tid + it * NTH < PXYZ) s[tid + it * NTH] = v[it];
}

// mu on the tile plus a one-node ring (R region) from phi staged with halo 2
template <typename T>
__device__ __forceinline__ void mu_ring(const Coef<T>& c, int i0, int j0, int k0, const T* sp, T* sm)
{
    const int tid = threadIdx.x + BX * (threadIdx.y + BY * threadIdx.z);
    for (int q = tid; q < RXYZ; q += NTH) {
        const int lz = q / (RX * RY), r = q - lz * (RX * RY), ly = r / RX, lx = r - ly * RX;
        // source node: the mirror node for a wall / symmetry ghost, else the position itself
        int sx = i0 + lx - 1, sy = j0 + ly - 1, sz = k0 + lz - 1;
        if (c.nonperiodic) {
            sx = mirror_coord(sx, c.nx, c.bc[0]);
            sy = mirror_coord(sy, c.ny, c.bc[2]);
            sz = mirror_coord(sz, c.nz, c.bc[4]);
        }
        // P-region coordinates, clamped (only ragged positions no output reads can leave the range)
        const int px = min(max(sx - i0 + 2, 1), PX - 2), py = min(max(sy - j0 + 2, 1), PY - 2);
        const int pz = min(max(sz - k0 + 2, 1), PZ - 2);
        T n[3][3][3];
        nb19at<PX, PY>(sp, px + PX * (py + PY * pz), n);
        const T p = n[1][1][1];
        sm[q] = fmaT(c.a4 * p, fmaT(p, p, T(-1)), -c.kap6 * lap_num(n));
    }
}

// the wetting coefficients of the six faces into LDS (constant indices only)
template <typename T>
__device__ __forceinline__ void wet_table(const Coef<T>& c, T* wbt)
{
    if (threadIdx.x + threadIdx.y + threadIdx.z == 0) {
        wbt[0] = c.wb[0];
        wbt[1] = c.wb[1];
        wbt[2] = c.wb[2];
        wbt[3] = c.wb[3];
        wbt[4] = c.wb[4];
        wbt[5] = c.wb[5];
    }
    __syncthreads();
}

struct Node {
    int i, j, k;
    bool in;
};
// the thread's r-th node (r < ZR) and its local z in the tile
template <typename T>
__device__ __forceinline__ Node my_node(const Coef<T>& c, int r)
{
    Node n;
    n.i = blockIdx.x * BX + threadIdx.x;
    n.j = blockIdx.y * BY + threadIdx.y;
    n.k = blockIdx.z * BZ + threadIdx.z + TZ * r;
    n.in = n.i < c.nx && n.j < c.ny && n.k < c.nz;
    return n;
}

// mu of phi on the tile and its ring, then F_a = phi G_iso,a mu and
// phi* = phi + dt (M L_iso mu - u_a G_iso,a phi)
template <typename T>
__global__ __launch_bounds__(NTH) void stage1_kernel(Coef<T> c, State<T> in, T* __restrict__ fx,
                                                     T* __restrict__ fy, T* __restrict__ fz, T* __restrict__ phis)
{
    __shared__ T sp[PXYZ], sm[RXYZ], wbt[6];
    const int i0 = blockIdx.x * BX, j0 = blockIdx.y * BY, k0 = blockIdx.z * BZ;
    wet_table(c, wbt);
    stage_halo2<true>(c, in.phi, i0, j0, k0, sp, wbt);
    __syncthreads();
    mu_ring(c, i0, j0, k0, sp, sm);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ZR; ++r) {
        const Node d = my_node(c, r);
        if (!d.in) continue;
        const int lz = threadIdx.z + TZ * r;
        const size_t o = ((size_t)d.k * c.ny + d.j) * c.nx + d.i;
        T m[3][3][3], p[3][3][3];
        nb19at<RX, RY>(sm, (threadIdx.x + 1) + RX * ((threadIdx.y + 1) + RY * (lz + 1)), m);
        nb19at<PX, PY>(sp, (threadIdx.x + 2) + PX * ((threadIdx.y + 2) + PY * (lz + 2)), p);
        const T pc = p[1][1][1];
        fx[o] = pc * (gx_num(m) * c.gi);
        fy[o] = pc * (gy_num(m) * c.gi);
        fz[o] = pc * (gz_num(m) * c.gi);
        const T adv = fmaT(in.u[o], gx_num(p), fmaT(in.v[o], gy_num(p), in.w[o] * gz_num(p))) * c.gi;
        const T rhs = fmaT(c.mob * c.li, lap_num(m), -adv);
        phis[o] = fmaT(c.dt, rhs, pc);
    }
}

// mu* of phi* on the tile and its ring, then
// phi^{n+1} = (phi + phi* + dt (M L_iso mu* - u_a G_iso,a phi*)) / 2
template <typename T>
__global__ __launch_bounds__(NTH) void stage2_kernel(Coef<T> c, State<T> in, const T* __restrict__ phis,
                                                     T* __restrict__ phi_out)
{
    __shared__ T sp[PXYZ], sm[RXYZ], wbt[6];
    const int i0 = blockIdx.x * BX, j0 = blockIdx.y * BY, k0 = blockIdx.z * BZ;
    wet_table(c, wbt);
    stage_halo2<true>(c, phis, i0, j0, k0, sp, wbt);
    __syncthreads();
    mu_ring(c, i0, j0, k0, sp, sm);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ZR; ++r) {
        const Node d = my_node(c, r);
        if (!d.in) continue;
        const int lz = threadIdx.z + TZ * r;
        const size_t o = ((size_t)d.k * c.ny + d.j) * c.nx + d.i;
        T m[3][3][3], p[3][3][3];
        nb19at<RX, RY>(sm, (threadIdx.x + 1) + RX * ((threadIdx.y + 1) + RY * (lz + 1)), m);
        nb19at<PX, PY>(sp, (threadIdx.x + 2) + PX * ((threadIdx.y + 2) + PY * (lz + 2)), p);
        const T adv = fmaT(in.u[o], gx_num(p), fmaT(in.v[o], gy_num(p), in.w[o] * gz_num(p))) * c.gi;
        const T rhs = fmaT(c.mob * c.li, lap_num(m), -adv);
        phi_out[o] = T(0.5) * fmaT(c.dt, rhs, in.phi[o] + p[1][1][1]);
    }
}

}  // namespace

template <typename T>
hipError_t launch_twophase3d(const Coef<T>& c, const State<T>& in, const State<T>& out, T* scratch, int tile,
                             hipStream_t s)
{
    const size_t n = (size_t)c.nx * c.ny * c.nz;
    T* phis = scratch;
    T* f[3] = {scratch + n, scratch + 2 * n, scratch + 3 * n};
    const dim3 block(BX, BY, TZ), grid((c.nx + BX - 1) / BX, (c.ny + BY - 1) / BY, (c.nz + BZ - 1) / BZ);
    hipLaunchKernelGGL(stage1_kernel<T>, grid, block, 0, s, c, in, f[0], f[1], f[2], phis);
    Coef<T> cf = c;
    for (int a = 0; a < 3; ++a) cf.fst[a] = f[a];
    hipError_t e = launch_step3d<T>(cf, in, out, tile, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(stage2_kernel<T>, grid, block, 0, s, c, in, phis, out.phi);
    return hipGetLastError();
}

template hipError_t launch_twophase3d<float>(const Coef<float>&, const State<float>&, const State<float>&, float*,
                                             int, hipStream_t);
template hipError_t launch_twophase3d<double>(const Coef<double>&, const State<double>&, const State<double>&,
                                              double*, int, hipStream_t);

}  // namespace acm
