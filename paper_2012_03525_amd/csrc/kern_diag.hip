// Diagnostics of a state: FP64 two-stage deterministic reductions.
// Stage 1: each workgroup walks a fixed grid-stride set of nodes and reduces
// its partials in LDS with a fixed tree; stage 2: one workgroup reduces the
// per-workgroup partials in a fixed order.  No atomics, so the result is
// bitwise reproducible run to run.
//
// Quantities (index: meaning), all accumulated in FP64:
//  0 sum drho            1-3 sum rho u_a        4 sum |u|^2
//  5 max | |u| - |u_prev| |   (steady-state test of Sec. 3.2)
//  6 max |u|             7 sum |omega|^2 (centred vorticity, Eq. 3.4)
//  8 sum div^2           9 max |div|   (centred divergence of u)
// 10 sum phi            11 nonfinite flag (max)
// Axisymmetric runs (AXI) weight the sums by the node's radius (j + 1/2), in
// units of dx (the host scales by 2 pi dx^3 or divides by the summed
// weights), and take the divergence in the cylindrical face form of the step.
#include "acm_internal.h"
#include "kern_axisym.h"

namespace acm {

__device__ __forceinline__ bool is_max_slot(int q) { return q == 5 || q == 6 || q == 9 || q == 11; }

template <typename T>
__device__ __forceinline__ void load_vel(const Coef<T>& c, int dim, const State<T>& s, int gx, int gy, int gz,
                                         double& u, double& v, double& w)
{
    int fx, fy, fz = -1;
    const int sx = map_coord(gx, c.nx, c.bc[0], 0, fx);
    const int sy = map_coord(gy, c.ny, c.bc[2], 2, fy);
    const int sz = (dim == 3) ? map_coord(gz, c.nz, c.bc[4], 4, fz) : 0;
    const size_t o = ((size_t)sz * c.ny + sy) * c.nx + sx;
    T qu = s.u[o], qv = s.v[o], qw = dim == 3 ? s.w[o] : T(0);
    if (fx >= 0) ghost_velocity(c, fx, qu, qv, qw);
    if (fy >= 0) ghost_velocity(c, fy, qu, qv, qw);
    if (fz >= 0) ghost_velocity(c, fz, qu, qv, qw);
    u = (double)qu;
    v = (double)qv;
    w = (double)qw;
}

template <typename T, bool AXI>
__global__ __launch_bounds__(256) void diag_partial_kernel(Coef<T> c, int dim, int two_phase, State<T> cur,
                                                           State<T> prev, int have_prev, double* partials)
{
    double acc[NDIAG];
    for (int q = 0; q < NDIAG; ++q) acc[q] = 0.0;
    const size_t n = (size_t)c.nx * c.ny * (dim == 3 ? c.nz : 1);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int gx = (int)(i % c.nx);
        const size_t t = i / c.nx;
        const int gy = (int)(t % c.ny);
        const int gz = (int)(t / c.ny);
        const double r = (double)cur.r[i];
        const double u = (double)cur.u[i], v = (double)cur.v[i];
        const double w = dim == 3 ? (double)cur.w[i] : 0.0;
        const double rho = (double)c.rho0 + r;
        const double cv = AXI ? (double)gy + 0.5 : 1.0;  // node weight
        acc[0] += r * cv;
        acc[1] += rho * u * cv;
        acc[2] += rho * v * cv;
        acc[3] += rho * w * cv;
        const double q2 = u * u + v * v + w * w;
        acc[4] += q2 * cv;
        const double mag = sqrt(q2);
        acc[6] = fmax(acc[6], mag);
        if (have_prev) {
            const double pu = (double)prev.u[i], pv = (double)prev.v[i];
            const double pw = dim == 3 ? (double)prev.w[i] : 0.0;
            acc[5] = fmax(acc[5], fabs(mag - sqrt(pu * pu + pv * pv + pw * pw)));
        }
        // centred derivatives d_b u_a (times 2 dx)
        double d[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        double vN = 0.0;
        {
            double a0, a1, a2, b0, b1, b2;
            load_vel(c, dim, cur, gx + 1, gy, gz, a0, a1, a2);
            load_vel(c, dim, cur, gx - 1, gy, gz, b0, b1, b2);
            d[0][0] = a0 - b0;
            d[1][0] = a1 - b1;
            d[2][0] = a2 - b2;
            load_vel(c, dim, cur, gx, gy + 1, gz, a0, a1, a2);
            vN = a1;
            load_vel(c, dim, cur, gx, gy - 1, gz, b0, b1, b2);
            d[0][1] = a0 - b0;
            d[1][1] = a1 - b1;
            d[2][1] = a2 - b2;
            if (dim == 3) {
                load_vel(c, dim, cur, gx, gy, gz + 1, a0, a1, a2);
                load_vel(c, dim, cur, gx, gy, gz - 1, b0, b1, b2);
                d[0][2] = a0 - b0;
                d[1][2] = a1 - b1;
                d[2][2] = a2 - b2;
            }
        }
        double om2;
        if (dim == 2) {
            const double oz = d[1][0] - d[0][1];
            om2 = oz * oz;
        } else {
            const double ox = d[2][1] - d[1][2], oy = d[0][2] - d[2][0], oz = d[1][0] - d[0][1];
            om2 = ox * ox + oy * oy + oz * oz;
        }
        acc[7] += om2 * cv;  // scaled by 1/(2 dx)^2 on the host
        // (times 2 dx) cylindrical: d_z u_z + [g (v_N - v_S) + (v_C + v_N)] / (g + 1/2)
        const double dv = AXI ? d[0][0] + ((double)gy * d[1][1] + (v + vN)) / cv : d[0][0] + d[1][1] + d[2][2];
        acc[8] += dv * dv * cv;
        acc[9] = fmax(acc[9], fabs(dv));
        double ph = 0.0;
        if (two_phase) {
            ph = (double)cur.phi[i];
            acc[10] += ph * cv;
        }
        const double chk = r + u + v + w + ph;
        if (!isfinite(chk)) acc[11] = 1.0;
    }
    // block tree reduction (fixed order)
    __shared__ double red[256];
    for (int q = 0; q < NDIAG; ++q) {
        red[threadIdx.x] = acc[q];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                const double a = red[threadIdx.x], b = red[threadIdx.x + s];
                red[threadIdx.x] = is_max_slot(q) ? fmax(a, b) : a + b;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) partials[(size_t)blockIdx.x * NDIAG + q] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void diag_final_kernel(const double* partials, int nblocks, double* result)
{
    __shared__ double red[256];
    for (int q = 0; q < NDIAG; ++q) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += 256) {
            const double x = partials[(size_t)b * NDIAG + q];
            a = is_max_slot(q) ? fmax(a, x) : a + x;
        }
        red[threadIdx.x] = a;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                const double x = red[threadIdx.x], y = red[threadIdx.x + s];
                red[threadIdx.x] = is_max_slot(q) ? fmax(x, y) : x + y;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) result[q] = red[0];
        __syncthreads();
    }
}

template <typename T, bool AXI>
hipError_t launch_diag_impl(const Coef<T>& c, int dim, int two_phase, const State<T>& cur, const State<T>& prev,
                            int have_prev, double* partials, int nblocks, double* result, hipStream_t s)
{
    hipLaunchKernelGGL((diag_partial_kernel<T, AXI>), dim3(nblocks), dim3(256), 0, s, c, dim, two_phase, cur, prev,
                       have_prev, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, result);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diag(const Coef<T>& c, int dim, int two_phase, const State<T>& cur, const State<T>& prev,
                       int have_prev, double* partials, int nblocks, double* result, hipStream_t s)
{
    return launch_diag_impl<T, false>(c, dim, two_phase, cur, prev, have_prev, partials, nblocks, result, s);
}

template <typename T>
hipError_t launch_diag_axisym(const Coef<T>& c, int two_phase, const State<T>& cur, const State<T>& prev,
                              int have_prev, double* partials, int nblocks, double* result, hipStream_t s)
{
    return launch_diag_impl<T, true>(c, 2, two_phase, cur, prev, have_prev, partials, nblocks, result, s);
}

template hipError_t launch_diag_axisym<float>(const Coef<float>&, int, const State<float>&, const State<float>&, int,
                                              double*, int, double*, hipStream_t);
template hipError_t launch_diag_axisym<double>(const Coef<double>&, int, const State<double>&, const State<double>&,
                                               int, double*, int, double*, hipStream_t);

template hipError_t launch_diag<float>(const Coef<float>&, int, int, const State<float>&, const State<float>&, int,
                                       double*, int, double*, hipStream_t);
template hipError_t launch_diag<double>(const Coef<double>&, int, int, const State<double>&, const State<double>&,
                                        int, double*, int, double*, hipStream_t);

}  // namespace acm
