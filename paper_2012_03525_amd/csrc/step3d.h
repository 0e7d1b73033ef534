// Per-node pieces of the 3D single-phase step shared by the one-step z-march
// (kern_step.hip) and the two-step z-march (kern_step_pair.hip): the
// momentum, the continuity update drho' (Eq. 2.10), the momentum update of
// Eq. (2.11) at one node, and buffer-resource access to whole planes.  Both
// kernels evaluate the same expressions in the same order, so a node's new
// state does not depend on which kernel computed it.
#pragma once

#include "acm_internal.h"
#include "tile2d.h"

namespace acm {

template <bool GEN, typename T>
__device__ __forceinline__ T mom3(T r, T u, T rho0)
{
    if constexpr (GEN) return fmaT(r, u, rho0 * u);
    else return fmaT(r, u, u);
}

// drho' of one node (Eq. 2.10) from drho at the node and its six
// neighbours and the momentum component of each neighbour along its axis:
// (u, drho) east / west, (v, drho) north / south, (w, drho) up / down.
// The momentum differences use the split form of mdiff (tile2d.h).
template <bool GEN, typename T>
__device__ __forceinline__ T rho_new_pt(const Coef<T>& c, T rc, T rE, T uE, T rW, T uW, T rN, T vN, T rS, T vS,
                                        T rUp, T wUp, T rDn, T wDn)
{
    const T rho0 = GEN ? c.rho0 : T(1);
    const T div = (mdiff(rE, uE, rW, uW, rho0) + mdiff(rN, vN, rS, vS, rho0)) + mdiff(rUp, wUp, rDn, wDn, rho0);
    const T lap = (((rE + rW) + (rN + rS)) + (rUp + rDn)) - T(6) * rc;
    return fmaT(-c.cg, div, fmaT(c.kr, lap, rc));
}

// drho' at R-index e of plane slot (cur), with the planes below / above.
template <bool GEN, typename T, int RX>
__device__ __forceinline__ T rho_new_3d(const Coef<T>& c, const T* r0, const T* u0, const T* v0,
                                        const T* rD, const T* wD, const T* rU, const T* wU, int e)
{
    return rho_new_pt<GEN, T>(c, r0[e], r0[e + 1], u0[e + 1], r0[e - 1], u0[e - 1], r0[e + RX], v0[e + RX],
                              r0[e - RX], v0[e - RX], rU[e], wU[e], rD[e], wD[e]);
}

// Buffer-resource access for the z-march: 32-bit lane byte offsets within a
// plane, fixed for the whole march, plus a uniform plane offset.  A field
// below 2 GiB gets one descriptor for the march and the plane's byte offset
// in the scalar offset operand, so moving to the next plane costs one scalar
// multiply; a larger field (WIDE) gets a descriptor per field and plane.
// The hardware range-checks every access against the descriptor's size.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(float*, __amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
__device__ __forceinline__ double bload(double*, __amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
// streaming (non-temporal) store: the new state is not re-read in this step
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, soff, 2);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff)
{
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, soff, 2);
}

// the four field descriptors of one plane (WIDE) or of the whole field, and
// the scalar byte offset of plane z
template <bool WIDE, typename T>
struct PlaneAccess {
    __amdgpu_buffer_rsrc_t r, u, v, w;
    unsigned soff;
    __device__ __forceinline__ PlaneAccess(const State<T>& f, int z, unsigned plane, unsigned pbytes,
                                           unsigned fbytes)
    {
        if constexpr (WIDE) {
            const size_t base = (size_t)z * plane;
            r = plane_rsrc(f.r + base, pbytes);
            u = plane_rsrc(f.u + base, pbytes);
            v = plane_rsrc(f.v + base, pbytes);
            w = plane_rsrc(f.w + base, pbytes);
            soff = 0u;
        } else {
            r = plane_rsrc(f.r, fbytes);
            u = plane_rsrc(f.u, fbytes);
            v = plane_rsrc(f.v, fbytes);
            w = plane_rsrc(f.w, fbytes);
            soff = (unsigned)z * pbytes;
        }
    }
};

// level-n values of one node
template <typename T>
struct Pt3 {
    T r, u, v, w;
};

// Momentum update (Eq. 2.11) of one node from the level-n values of the node
// (C) and of its six neighbours, drho' at the node and at its neighbours, the
// row's x force (used when c.fx is set) and, on the general path, the
// per-node surface-tension force phi G_iso mu (fs, when has_fs).  Returns the
// new drho, u, v, w.
template <bool GEN, typename T>
__device__ __forceinline__ void momentum3d(const Coef<T>& c, const Pt3<T>& C, const Pt3<T>& E, const Pt3<T>& W,
                                           const Pt3<T>& N, const Pt3<T>& S, const Pt3<T>& U, const Pt3<T>& D,
                                           T rnC, T rnE, T rnW, T rnN, T rnS, T rnU, T rnD, T fxrow,
                                           bool has_fs, T fs0, T fs1, T fs2, T& ro, T& uo, T& vo, T& wo)
{
    const T rho0 = c.rho0, cs2 = c.cs2;
    const T mxC = mom3<GEN>(C.r, C.u, rho0), myC = mom3<GEN>(C.r, C.v, rho0), mzC = mom3<GEN>(C.r, C.w, rho0);
    const T mxE = mom3<GEN>(E.r, E.u, rho0), myE = mom3<GEN>(E.r, E.v, rho0), mzE = mom3<GEN>(E.r, E.w, rho0);
    const T mxW = mom3<GEN>(W.r, W.u, rho0), myW = mom3<GEN>(W.r, W.v, rho0), mzW = mom3<GEN>(W.r, W.w, rho0);
    const T mxN = mom3<GEN>(N.r, N.u, rho0), myN = mom3<GEN>(N.r, N.v, rho0), mzN = mom3<GEN>(N.r, N.w, rho0);
    const T mxS = mom3<GEN>(S.r, S.u, rho0), myS = mom3<GEN>(S.r, S.v, rho0), mzS = mom3<GEN>(S.r, S.w, rho0);
    const T mxU = mom3<GEN>(U.r, U.u, rho0), myU = mom3<GEN>(U.r, U.v, rho0), mzU = mom3<GEN>(U.r, U.w, rho0);
    const T mxD = mom3<GEN>(D.r, D.u, rho0), myD = mom3<GEN>(D.r, D.v, rho0), mzD = mom3<GEN>(D.r, D.w, rho0);

    // centred differences of drho (pressure term and density SAT share them)
    const T gxr = E.r - W.r, gyr = N.r - S.r, gzr = U.r - D.r;
    const T fxx = fmaT(cs2, gxr, ((mxE * E.u - mxW * W.u) + (mxN * N.v - mxS * S.v)) + (mxU * U.w - mxD * D.w));
    const T fyy = fmaT(cs2, gyr, ((myE * E.u - myW * W.u) + (myN * N.v - myS * S.v)) + (myU * U.w - myD * D.w));
    const T fzz = fmaT(cs2, gzr, ((mzE * E.u - mzW * W.u) + (mzN * N.v - mzS * S.v)) + (mzU * U.w - mzD * D.w));
    const T lpx = fmaT(T(-6), mxC, ((mxE + mxW) + (mxN + mxS)) + (mxU + mxD));
    const T lpy = fmaT(T(-6), myC, ((myE + myW) + (myN + myS)) + (myU + myD));
    const T lpz = fmaT(T(-6), mzC, ((mzE + mzW) + (mzN + mzS)) + (mzU + mzD));
    const T sx = (rnE - rnW) - gxr;
    const T sy = (rnN - rnS) - gyr;
    const T sz = (rnU - rnD) - gzr;
    const T rho_n = rho0 + rnC;
    T gx_ = c.gdt[0];
    if (c.fx) gx_ = fmaT(c.dt, fxrow, gx_);
    T dmx = fmaT(rho_n, gx_, fmaT(-c.ks, sx, fmaT(c.kv, lpx, -c.cg * fxx)));
    T dmy = fmaT(rho_n, c.gdt[1], fmaT(-c.ks, sy, fmaT(c.kv, lpy, -c.cg * fyy)));
    T dmz = fmaT(rho_n, c.gdt[2], fmaT(-c.ks, sz, fmaT(c.kv, lpz, -c.cg * fzz)));
    if constexpr (GEN) {
        if (has_fs) {  // -dt phi G_iso mu
            dmx = fmaT(-c.dt, fs0, dmx);
            dmy = fmaT(-c.dt, fs1, dmy);
            dmz = fmaT(-c.dt, fs2, dmz);
        }
    }
    const T drn = rnC - C.r;
    const T inv = recipT(rho_n);
    ro = rnC;
    uo = fmaT(fmaT(-C.u, drn, dmx), inv, C.u);
    vo = fmaT(fmaT(-C.v, drn, dmy), inv, C.v);
    wo = fmaT(fmaT(-C.w, drn, dmz), inv, C.w);
}

}  // namespace acm
