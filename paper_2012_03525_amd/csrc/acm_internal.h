// Internal declarations of libacm: device-side coefficient block, boundary
// mapping helpers and kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace acm {

enum : int { BC_PERIODIC = 0, BC_WALL = 1, BC_SYMMETRY = 2 };

// Coefficients of one SMAME step, folded on the host from the problem
// statement so that the kernels only multiply and add.
template <typename T>
struct Coef {
    int nx, ny, nz;
    int bc[6];
    int nonperiodic;   // any face is a wall or symmetry plane
    T rho0;
    T cg;              // dt / (2 dx): centred difference times dt
    T cs2;             // cs^2
    T kr;              // sat_rho * cs^2 dt^2 / (2 dx^2)      (Eq. 2.10 SAT)
    T kv;              // nu dt / dx^2                         (viscous term)
    T ks;              // sat_mom (nu + cs^2 dt / 2) / (2 dx)  (Eq. 2.11 SAT)
    T gdt[3];          // dt g
    T dt;
    T fs[6][3];        // ghost velocity = fs * mirror + fo, per crossed face
    T fo[6][3];
    const T* fx;       // per-row x force (ny values) or null
    // two-phase
    T a4;              // 4 a, a = 3 sigma / (4 W)
    T kap6;            // kappa / (6 dx^2)
    T mob;             // M
    T gi;              // 1 / (12 dx)   isotropic gradient
    T li;              // 1 / (6 dx^2)  isotropic Laplacian
    T wb[6];           // wall faces: dx (2/W) cos(contact angle); 0 elsewhere
    int wet;           // any nonzero wb
    const T* fst[3];   // 3D two-phase: phi G_iso mu per node (subtracted times dt), or null
};

template <typename T>
struct State {
    T* r;
    T* u;
    T* v;
    T* w;
    T* phi;
};

// Map a possibly out-of-range coordinate onto its source node.  face is set
// to the crossed face index (lo = 2*axis, hi = 2*axis+1) for a wall or a
// symmetry plane, -1 otherwise.  Points more than one reflection away (only
// reached by ragged tiles, never used by an output) are clamped in range.
__device__ __forceinline__ int map_coord(int g, int n, int bc_lo, int face_lo, int& face)
{
    face = -1;
    if (g < 0) {
        if (bc_lo == BC_PERIODIC) {
            g += n;
            if (g < 0) g = ((g % n) + n) % n;
        } else {
            face = face_lo;
            g = -1 - g;
            if (g >= n) g = n - 1;
        }
    } else if (g >= n) {
        if (bc_lo == BC_PERIODIC) {
            g -= n;
            if (g >= n) g %= n;
        } else {
            face = face_lo + 1;
            g = 2 * n - 1 - g;
            if (g < 0) g = 0;
        }
    }
    return g;
}

// Position whose rho^{n+1} stands in for a ghost position: the mirror node
// for a wall / symmetry face, the position itself otherwise (a periodic
// ghost is computed from wrapped data and equals its image bit for bit).
__device__ __forceinline__ int mirror_coord(int g, int n, int bc_lo)
{
    if (bc_lo == BC_PERIODIC) return g;
    if (g < 0) return -1 - g;
    if (g >= n) return 2 * n - 1 - g;
    return g;
}

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) { return fma(a, b, c); }

// 1 / rho for the velocity update.  FP32 uses the hardware reciprocal: it
// only scales the (small) increment u^{n+1} - u^n, so its 1-ulp error is
// far below the storage rounding of u.
__device__ __forceinline__ float recipT(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recipT(double x) { return 1.0 / x; }

// Order parameter of a ghost node across a wall face with wetting (Sec. 2):
// (phi_m - phi_g)/dx = -(2/W) cos(theta) (1 - phi_w^2), phi_w = (phi_g + phi_m)/2
// the value at the halfway wall.  With b = dx (2/W) cos(theta) the wall value
// solves b s^2 + 2 s - (2 phi_m + b) = 0; the root that tends to phi_m as
// b -> 0 is taken in the cancellation-free form below; b = 0 gives phi_m.
// The ghost is phi_m + 2 (s - phi_m) with the offset s - phi_m taken at phi_m
// clamped to the bulk values [-1, 1] (the offset vanishes there): a value
// beyond +-1 is mirrored, b = 0 mirrors every value, and the root stays real
// for |b| <= 1 when phi overshoots 1 next to a wall with cos(theta) near -1.
template <typename T>
__device__ __forceinline__ T wet_ghost(T m, T b)
{
    const T mc = fmin(fmax(m, T(-1)), T(1));
    const T q = fmaT(T(2), mc, b);
    const T s = q / (T(1) + sqrt(fmaT(b, q, T(1))));
    return fmaT(T(2), s - mc, m);
}

// wb of the crossed face f (per-lane value: selected, not indexed)
template <typename T>
__device__ __forceinline__ T wet_b(const Coef<T>& c, int f)
{
    T b = c.wb[0];
#pragma unroll
    for (int k = 1; k < 6; ++k) b = f == k ? c.wb[k] : b;
    return b;
}

// Velocity of a ghost node from its mirror node across face f (0..5):
// u_a = fs[f][a] u_a + fo[f][a].  f differs between lanes, so the six faces
// are selected explicitly instead of indexing the coefficient arrays with a
// per-lane value (which would copy the coefficients to scratch memory).
template <typename T>
__device__ __forceinline__ void ghost_velocity(const Coef<T>& c, int f, T& u, T& v, T& w)
{
    T s[3], o[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s[a] = c.fs[0][a];
        o[a] = c.fo[0][a];
#pragma unroll
        for (int k = 1; k < 6; ++k) {
            s[a] = f == k ? c.fs[k][a] : s[a];
            o[a] = f == k ? c.fo[k][a] : o[a];
        }
    }
    u = fmaT(s[0], u, o[0]);
    v = fmaT(s[1], v, o[1]);
    w = fmaT(s[2], w, o[2]);
}

// ---------------------------------------------------------------------------
// launchers (kern_step.hip, kern_twophase.hip, kern_diag.hip)
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_step2d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile,
                         hipStream_t s);
template <typename T>
hipError_t launch_step3d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile,
                         hipStream_t s);
// Two 3D steps in one launch (in -> out holds level n+2) on fully periodic
// boxes with rho0 = 1 and fields below 2 GiB, selected by tile codes 14 and
// 15; step3d_pair_ok says whether the configuration and tile code allow it
// (kern_step_pair.hip).
template <typename T>
bool step3d_pair_ok(const Coef<T>& c, int tile);
template <typename T>
hipError_t launch_step3d_pair(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile,
                              hipStream_t s);
// 3D step with whole x rows per wave (kern_step3d_rows.hip): FP32 fully
// periodic boxes with rho0 = 1 and nx in {64, 128, 256}; shape 16..19
// selects the band height, zc the planes per chunk.  step3d_rows_ok says
// whether the configuration allows it.
template <typename T>
bool step3d_rows_ok(const Coef<T>& c);
template <typename T>
hipError_t launch_step3d_rows(const Coef<T>& c, const State<T>& in, const State<T>& out, int shape, int zc,
                              hipStream_t s);
template <typename T>
hipError_t launch_twophase2d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile,
                             hipStream_t s);
// 3D two-phase step: scratch holds 4 fields of nx*ny*nz values (phi* and
// phi G_iso mu per axis), owned by the caller
template <typename T>
hipError_t launch_twophase3d(const Coef<T>& c, const State<T>& in, const State<T>& out, T* scratch, int tile,
                             hipStream_t s);

// adjoint of one 2D single-phase step on a fully periodic grid (kern_adjoint.hip):
// aq = (dS/dq)^T as at state q, with s = S(q)
template <typename T>
hipError_t launch_adjoint2d(const Coef<T>& c, const State<T>& q, const State<T>& s, const State<T>& as,
                            const State<T>& aq, hipStream_t st);

// number of FP64 quantities reduced by the diagnostics kernel
constexpr int NDIAG = 14;
template <typename T>
hipError_t launch_diag(const Coef<T>& c, int dim, int two_phase, const State<T>& cur,
                       const State<T>& prev, int have_prev, double* partials, int nblocks,
                       double* result, hipStream_t s);

}  // namespace acm
