// Two-phase SMAME step in 3D for gfx950: the flow update with the
// surface-tension force and the Cahn-Hilliard equation (Eq. 2.14) by Heun's
// method, as five launches per step (Sec. 2, two-phase paragraphs):
//   1. mu      = 4 a phi (phi^2 - 1) - kappa L_iso phi
//   2. F_a     = phi G_iso,a mu;  phi* = phi + dt (M L_iso mu - u_a G_iso,a phi)
//   3. flow    = single-phase 3D step (Eqs. 2.10-2.11) with -dt F_a added to the momentum
//   4. mu*     = mu(phi*)
//   5. phi^{n+1} = (phi + phi* + dt (M L_iso mu* - u_a G_iso,a phi*)) / 2
// u is u^n in both Heun stages.  Isotropic stencils with D3Q19 weights:
//   G_iso,a f = [2 (f_{+a} - f_{-a}) + sum_{b != a} (f_{+a+b} + f_{+a-b} - f_{-a+b} - f_{-a-b})] / (12 dx)
//   L_iso f   = [2 (sum of the 6 face neighbours) + (sum of the 12 edge neighbours) - 24 f] / (6 dx^2)
// Ghosts: mu is mirrored across walls and symmetry planes (no flux); phi
// and phi* are mirrored, then take the wetting rule of each crossed wall
// face (x, y, z order).  One thread per node; each stencil field is staged
// per workgroup in LDS with its halo.
#include "acm_internal.h"

namespace acm {

namespace {

// value of a scalar field at node (i, j, k), which may lie one layer outside
// the grid; WET applies the wetting rule across wall faces
template <bool WET, typename T>
__device__ __forceinline__ T at(const Coef<T>& c, const T* __restrict__ f, int i, int j, int k)
{
    int fx, fy, fz;
    const int si = map_coord(i, c.nx, c.bc[0], 0, fx);
    const int sj = map_coord(j, c.ny, c.bc[2], 2, fy);
    const int sk = map_coord(k, c.nz, c.bc[4], 4, fz);
    T v = f[((size_t)sk * c.ny + sj) * c.nx + si];
    if constexpr (WET) {
        if (c.wet) {
            if (fx >= 0) v = wet_ghost(v, wet_b(c, fx));
            if (fy >= 0) v = wet_ghost(v, wet_b(c, fy));
            if (fz >= 0) v = wet_ghost(v, wet_b(c, fz));
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

// Workgroup tile BX x BY x BZ nodes; each field a kernel reads with its
// 19-point stencil is staged once per workgroup in LDS with a one-node halo
// (ghost rules applied while staging), so a node's neighbours come from LDS
// instead of 19 separate global loads.
constexpr int BX = 32, BY = 4, BZ = 4, NTH = BX * BY * BZ;
constexpr int RX = BX + 2, RY = BY + 2, RZ = BZ + 2, RXYZ = RX * RY * RZ;

template <bool WET, typename T>
__device__ __forceinline__ void stage(const Coef<T>& c, const T* __restrict__ f, int i0, int j0, int k0, T* s)
{
    const int tid = threadIdx.x + BX * (threadIdx.y + BY * threadIdx.z);
    constexpr int NIT = (RXYZ + NTH - 1) / NTH;
    T v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {  // every load before the first LDS store
        const int q = min(tid + it * NTH, RXYZ - 1);
        const int lz = q / (RX * RY), r = q - lz * (RX * RY), ly = r / RX, lx = r - ly * RX;
        v[it] = at<WET>(c, f, i0 + lx - 1, j0 + ly - 1, k0 + lz - 1);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it)
        if (tid + it * NTH < RXYZ) s[tid + it * NTH] = v[it];
}

// the D3Q19 neighbourhood of the thread's node from a staged region
template <typename T>
__device__ __forceinline__ void nb19(const T* s, T n[3][3][3])
{
    const int e = (threadIdx.x + 1) + RX * ((threadIdx.y + 1) + RY * (threadIdx.z + 1));
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if ((dx != 0) + (dy != 0) + (dz != 0) == 3) continue;  // corners are not part of the stencil
                n[1 + dx][1 + dy][1 + dz] = s[e + dx + RX * (dy + RY * dz)];
            }
}

struct Node {
    int i, j, k;
    bool in;
};
template <typename T>
__device__ __forceinline__ Node my_node(const Coef<T>& c)
{
    Node n;
    n.i = blockIdx.x * BX + threadIdx.x;
    n.j = blockIdx.y * BY + threadIdx.y;
    n.k = blockIdx.z * BZ + threadIdx.z;
    n.in = n.i < c.nx && n.j < c.ny && n.k < c.nz;
    return n;
}

// mu = 4 a phi (phi^2 - 1) - kappa L_iso phi
template <typename T>
__global__ __launch_bounds__(NTH) void chem3_kernel(Coef<T> c, const T* __restrict__ phi, T* __restrict__ mu)
{
    __shared__ T sp[RXYZ];
    stage<true>(c, phi, blockIdx.x * BX, blockIdx.y * BY, blockIdx.z * BZ, sp);
    __syncthreads();
    const Node d = my_node(c);
    if (!d.in) return;
    T n[3][3][3];
    nb19(sp, n);
    const T p = n[1][1][1];
    mu[((size_t)d.k * c.ny + d.j) * c.nx + d.i] = fmaT(c.a4 * p, fmaT(p, p, T(-1)), -c.kap6 * lap_num(n));
}

// F_a = phi G_iso,a mu and phi* = phi + dt (M L_iso mu - u_a G_iso,a phi)
template <typename T>
__global__ __launch_bounds__(NTH) void stage1_kernel(Coef<T> c, State<T> in, const T* __restrict__ mu,
                                                     T* __restrict__ fx, T* __restrict__ fy, T* __restrict__ fz,
                                                     T* __restrict__ phis)
{
    __shared__ T sm[RXYZ], sp[RXYZ];
    stage<false>(c, mu, blockIdx.x * BX, blockIdx.y * BY, blockIdx.z * BZ, sm);
    stage<true>(c, in.phi, blockIdx.x * BX, blockIdx.y * BY, blockIdx.z * BZ, sp);
    __syncthreads();
    const Node d = my_node(c);
    if (!d.in) return;
    const size_t o = ((size_t)d.k * c.ny + d.j) * c.nx + d.i;
    T m[3][3][3], p[3][3][3];
    nb19(sm, m);
    nb19(sp, p);
    const T pc = p[1][1][1];
    fx[o] = pc * (gx_num(m) * c.gi);
    fy[o] = pc * (gy_num(m) * c.gi);
    fz[o] = pc * (gz_num(m) * c.gi);
    const T adv = fmaT(in.u[o], gx_num(p), fmaT(in.v[o], gy_num(p), in.w[o] * gz_num(p))) * c.gi;
    const T rhs = fmaT(c.mob * c.li, lap_num(m), -adv);
    phis[o] = fmaT(c.dt, rhs, pc);
}

// phi^{n+1} = (phi + phi* + dt (M L_iso mu* - u_a G_iso,a phi*)) / 2
template <typename T>
__global__ __launch_bounds__(NTH) void stage2_kernel(Coef<T> c, State<T> in, const T* __restrict__ phis,
                                                     const T* __restrict__ mus, T* __restrict__ phi_out)
{
    __shared__ T sm[RXYZ], sp[RXYZ];
    stage<false>(c, mus, blockIdx.x * BX, blockIdx.y * BY, blockIdx.z * BZ, sm);
    stage<true>(c, phis, blockIdx.x * BX, blockIdx.y * BY, blockIdx.z * BZ, sp);
    __syncthreads();
    const Node d = my_node(c);
    if (!d.in) return;
    const size_t o = ((size_t)d.k * c.ny + d.j) * c.nx + d.i;
    T m[3][3][3], p[3][3][3];
    nb19(sm, m);
    nb19(sp, p);
    const T adv = fmaT(in.u[o], gx_num(p), fmaT(in.v[o], gy_num(p), in.w[o] * gz_num(p))) * c.gi;
    const T rhs = fmaT(c.mob * c.li, lap_num(m), -adv);
    phi_out[o] = T(0.5) * fmaT(c.dt, rhs, in.phi[o] + p[1][1][1]);
}

}  // namespace

template <typename T>
hipError_t launch_twophase3d(const Coef<T>& c, const State<T>& in, const State<T>& out, T* scratch, int tile,
                             hipStream_t s)
{
    const size_t n = (size_t)c.nx * c.ny * c.nz;
    T* mu = scratch;
    T* phis = scratch + n;
    T* f[3] = {scratch + 2 * n, scratch + 3 * n, scratch + 4 * n};
    const dim3 block(BX, BY, BZ), grid((c.nx + BX - 1) / BX, (c.ny + BY - 1) / BY, (c.nz + BZ - 1) / BZ);
    hipLaunchKernelGGL(chem3_kernel<T>, grid, block, 0, s, c, in.phi, mu);
    hipLaunchKernelGGL(stage1_kernel<T>, grid, block, 0, s, c, in, mu, f[0], f[1], f[2], phis);
    Coef<T> cf = c;
    for (int a = 0; a < 3; ++a) cf.fst[a] = f[a];
    hipError_t e = launch_step3d<T>(cf, in, out, tile, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(chem3_kernel<T>, grid, block, 0, s, c, phis, mu);
    hipLaunchKernelGGL(stage2_kernel<T>, grid, block, 0, s, c, in, phis, mu, out.phi);
    return hipGetLastError();
}

template hipError_t launch_twophase3d<float>(const Coef<float>&, const State<float>&, const State<float>&, float*,
                                             int, hipStream_t);
template hipError_t launch_twophase3d<double>(const Coef<double>&, const State<double>&, const State<double>&,
                                              double*, int, hipStream_t);

}  // namespace acm
