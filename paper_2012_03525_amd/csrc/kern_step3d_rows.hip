// 3D single-phase SMAME step on fully periodic boxes with whole x rows per
// wave (FP32, rho0 = 1, nx = 64, 128 or 256).
//
// One launch = one step: continuity (Eq. 2.10) then momentum (Eq. 2.11)
// with the body force, centred differences (Eqs. 2.12-2.13), the same
// per-node expressions as the other 3D kernels (rho_new_pt, momentum3d in
// step3d.h), so every launch shape gives the same bits.
//
// Layout of the work:
//  * A wave owns one complete x row: lane l holds the VX = nx / 64
//    consecutive nodes 4l..4l+VX-1, loaded and stored with one VX-wide
//    buffer access per field (16-byte accesses for nx = 256, so a wave moves
//    a whole 1 KiB row per instruction).  x neighbours are the lane's own
//    registers or come from the adjacent lane through a wave-wide DPP
//    rotation, which also closes the periodic row.
//  * A workgroup of NW waves owns a band of TY = NW - 2 rows and marches it
//    through a chunk of planes.  Waves 1..TY hold the band's rows; waves 0
//    and NW-1 hold the rows just outside (the one-row ring on which drho'
//    must also be known) and, for drho' there, the density and v of the row
//    beyond.  Each wave keeps its own row's planes k-1 .. k+2 in registers
//    (z neighbours never touch LDS) and fetches plane k+3 while plane k is
//    computed.
//  * LDS carries only the exchange between rows: drho and v of plane k+1
//    (rows -2 .. TY+1, for drho'(k+1)) and of plane k (for the momentum of
//    plane k), and u, w, drho' of plane k (rows -1 .. TY).  Two barriers per
//    plane: one before a plane's rows are written, one after.
//
// Iteration k (output plane k): issue the loads of plane k+3; barrier; write
// this wave's row of plane k+1 (drho, v) and of plane k (u, w, drho');
// barrier; drho'(k+1) on the wave's row; the band's waves form the momentum
// of plane k and store it.  The march starts two planes below the chunk so
// that drho' of the plane below is known when the chunk's first plane is
// formed.
#include <type_traits>

#include "acm_internal.h"
#include "step3d.h"

namespace acm {

// Planes fetched ahead of the one whose drho' is formed next: one plane is
// about 1.7 us of march on 256^3, enough to cover the load latency (a depth
// of two measured the same).
constexpr int ROWS_PREFETCH = 1;

namespace {

// wave-wide rotations by one lane (DPP): every lane receives the value of
// the lane below (lane 0 that of lane 63) or of the lane above (lane 63
// that of lane 0)
__device__ __forceinline__ float from_lane_below(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x13C, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_lane_above(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x134, 0xF, 0xF, false));
}

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// The buffer builtins return integer vectors; they are bit-cast whole to
// float vectors before any element is read (reading elements of the integer
// vector directly was compiled into a one-dword load broadcast to every
// element by this toolchain).
template <int VX>
__device__ __forceinline__ void row_load(float (&d)[VX], __amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff)
{
    if constexpr (VX == 4) {
        const f32x4 q = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0));
        d[0] = q[0];
        d[1] = q[1];
        d[2] = q[2];
        d[3] = q[3];
    } else if constexpr (VX == 2) {
        const f32x2 q = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
        d[0] = q[0];
        d[1] = q[1];
    } else {
        d[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    }
}

// streaming store (the new state is not read again in this step)
template <int VX>
__device__ __forceinline__ void row_store(const float (&d)[VX], __amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff)
{
    if constexpr (VX == 4) {
        const f32x4 q = {d[0], d[1], d[2], d[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, q), r, off, soff, 2);
    } else if constexpr (VX == 2) {
        const f32x2 q = {d[0], d[1]};
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, q), r, off, soff, 2);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, d[0]), r, off, soff, 2);
    }
}

template <int VX>
__device__ __forceinline__ void lds_put(float* p, const float (&d)[VX])
{
    if constexpr (VX == 4) *reinterpret_cast<float4*>(p) = make_float4(d[0], d[1], d[2], d[3]);
    else if constexpr (VX == 2) *reinterpret_cast<float2*>(p) = make_float2(d[0], d[1]);
    else p[0] = d[0];
}

template <int VX>
__device__ __forceinline__ void lds_get(float (&d)[VX], const float* p)
{
    if constexpr (VX == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        d[0] = q.x;
        d[1] = q.y;
        d[2] = q.z;
        d[3] = q.w;
    } else if constexpr (VX == 2) {
        const float2 q = *reinterpret_cast<const float2*>(p);
        d[0] = q.x;
        d[1] = q.y;
    } else {
        d[0] = p[0];
    }
}

// the lane's VX nodes of one row of one plane
template <int VX>
struct RowSet {
    float r[VX], u[VX], v[VX], w[VX];
};

// x neighbours of a lane's nodes: e[j] = value at node j + 1, o[j] at j - 1
template <int VX>
__device__ __forceinline__ void x_neighbours(const float (&f)[VX], float (&e)[VX], float (&o)[VX])
{
#pragma unroll
    for (int j = 0; j < VX; ++j) {
        e[j] = (j + 1 < VX) ? f[j + 1] : 0.f;
        o[j] = (j > 0) ? f[j - 1] : 0.f;
    }
    e[VX - 1] = from_lane_above(f[0]);
    o[0] = from_lane_below(f[VX - 1]);
}

}  // namespace

template <int VX, int NW>
struct Rows3 {
    static constexpr int TY = NW - 2;     // rows of the band
    static constexpr int NX = 64 * VX;    // row length (nx)
    static constexpr int NRR = TY + 4;    // rows -2 .. TY+1 (drho, v)
    static constexpr int NUR = TY + 2;    // rows -1 .. TY (u, w, drho')
    static constexpr size_t lds_bytes = (size_t)(2 * 2 * NRR + 3 * NUR) * NX * sizeof(float);
};

template <int VX, int NW, bool WIDE, int PD>
__global__ __launch_bounds__(NW * 64) void step3d_rows_kernel(Coef<float> c, State<float> in, State<float> out,
                                                               int zc, int nby)
{
    using S = Rows3<VX, NW>;
    constexpr int TY = S::TY, NX = S::NX, NRR = S::NRR, NUR = S::NUR;
    // the 10-wave band (80 KB of LDS) measured 2-4x slower and did not repeat
    // the other shapes' bits at 256^3; shapes stay within 64 KB
    static_assert(S::lds_bytes <= 65536, "row kernel shapes stay within 64 KB of LDS");
    // sR[q][f][row + 2][x]: drho (f = 0) and v (f = 1) of the plane with
    // relative parity q; sU[f][row + 1][x]: u, w, drho' of the momentum plane
    __shared__ __align__(16) float sR[2][2][NRR][NX];
    __shared__ __align__(16) float sU[3][NUR][NX];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int by = lb % nby, bz = lb / nby;
    const int y0 = by * TY, z0 = bz * zc;
    const int z1 = min(z0 + zc, c.nz);
    const int ny = c.ny, nz = c.nz;
    const unsigned plane = (unsigned)NX * (unsigned)ny;
    const unsigned pbytes = plane * 4u;
    const unsigned fbytes = WIDE ? 0u : pbytes * (unsigned)nz;  // below 2^31 unless WIDE
    const int ry = wave - 1;  // this wave's row in the band, -1 .. TY
    const bool ring = (wave == 0) || (wave == NW - 1);
    const int orow = (wave == 0) ? -2 : TY + 1;  // a ring wave's row beyond the ring
    auto wrapy = [&](int y) { return y < 0 ? y + ny : (y >= ny ? y - ny : y); };  // overhang <= 2 < ny
    const unsigned xoff = (unsigned)(VX * lane) * 4u;
    const unsigned voff = (unsigned)wrapy(y0 + ry) * (unsigned)NX * 4u + xoff;
    const unsigned ovoff = (unsigned)wrapy(y0 + orow) * (unsigned)NX * 4u + xoff;
    // a band row past ny (ragged last band) computes on wrapped data and
    // stores out of the descriptor's range, which the hardware drops
    const unsigned stoff = (!ring && y0 + ry < ny) ? voff : (WIDE ? pbytes : fbytes);
    const float fxrow = c.fx ? c.fx[wrapy(y0 + ry)] : 0.f;

    float* const sRrow0 = &sR[0][0][ry + 2][VX * lane];   // + q * (2 NRR NX) + f * (NRR NX)
    float* const sOrow0 = &sR[0][0][orow + 2][VX * lane];
    float* const sUrow = &sU[0][ry + 1][VX * lane];       // + f * (NUR NX)
    constexpr int QS = 2 * NRR * NX, FS = NRR * NX, US = NUR * NX;

    auto plane_of = [&](int p) { return p < 0 ? p + nz : (p >= nz ? p - nz : p); };  // nz >= 2

    // planes k-1 .. k+2 resident, k+3 .. k+2+PD in flight, by (p - k0) mod NF
    constexpr int NF = 4 + PD;
    RowSet<VX> F[NF];
    float O[2][2][VX];     // ring waves: drho, v of the row beyond, by (p - k0) mod 2
    float dD[VX], dC[VX];  // drho' of planes k-1 and k on the wave's row

    auto fetch = [&](int p, RowSet<VX>& d) {
        const PlaneAccess<WIDE, float> pa(in, plane_of(p), plane, pbytes, fbytes);
        row_load<VX>(d.r, pa.r, voff, pa.soff);
        row_load<VX>(d.u, pa.u, voff, pa.soff);
        row_load<VX>(d.v, pa.v, voff, pa.soff);
        row_load<VX>(d.w, pa.w, voff, pa.soff);
    };
    auto fetch_outer = [&](int p, float (&d)[2][VX]) {
        const PlaneAccess<WIDE, float> pa(in, plane_of(p), plane, pbytes, fbytes);
        row_load<VX>(d[0], pa.r, ovoff, pa.soff);
        row_load<VX>(d[1], pa.v, ovoff, pa.soff);
    };

    const int k0 = z0 - 2;
#pragma unroll
    for (int i = 0; i < 2 + PD; ++i)
        if (i < 3 || k0 + i <= z1 + 1) fetch(k0 + i, F[i]);
    if (ring) fetch_outer(k0 + 1, O[1]);
#pragma unroll
    for (int j = 0; j < VX; ++j) dD[j] = dC[j] = 0.f;

    // one plane; J = (k - k0) mod NU fixes every register set and LDS slot
    auto iterate = [&](int k, auto jc) {
        constexpr int J = decltype(jc)::value;
        RowSet<VX>& C = F[J % NF];
        RowSet<VX>& D = F[(J + NF - 1) % NF];
        RowSet<VX>& U = F[(J + 1) % NF];
        RowSet<VX>& P = F[(J + 2) % NF];
        RowSet<VX>& Q = F[(J + 2 + PD) % NF];
        constexpr int qk = J & 1, qu = (J + 1) & 1;  // relative parity of planes k and k+1
        if (k + 2 + PD <= z1 + 1) fetch(k + 2 + PD, Q);
        if (ring && k + 2 <= z1) fetch_outer(k + 2, O[qk]);
        __syncthreads();  // every wave is done with plane k-1's rows and with plane k's ring
        // rows of plane k+1 for drho'(k+1), of plane k for the momentum
        lds_put<VX>(sRrow0 + qu * QS, U.r);
        lds_put<VX>(sRrow0 + qu * QS + FS, U.v);
        if (ring) {
            lds_put<VX>(sOrow0 + qu * QS, O[qu][0]);
            lds_put<VX>(sOrow0 + qu * QS + FS, O[qu][1]);
        }
        lds_put<VX>(sUrow, C.u);
        lds_put<VX>(sUrow + US, C.w);
        lds_put<VX>(sUrow + 2 * US, dC);
        __syncthreads();

        // drho'(k+1) on the wave's row
        float dU[VX];
        {
            float rN[VX], vN[VX], rS[VX], vS[VX], rE[VX], rW[VX], uE[VX], uW[VX];
            lds_get<VX>(rN, sRrow0 + qu * QS + NX);
            lds_get<VX>(vN, sRrow0 + qu * QS + FS + NX);
            lds_get<VX>(rS, sRrow0 + qu * QS - NX);
            lds_get<VX>(vS, sRrow0 + qu * QS + FS - NX);
            x_neighbours<VX>(U.r, rE, rW);
            x_neighbours<VX>(U.u, uE, uW);
#pragma unroll
            for (int j = 0; j < VX; ++j)
                dU[j] = rho_new_pt<false, float>(c, U.r[j], rE[j], uE[j], rW[j], uW[j], rN[j], vN[j], rS[j], vS[j],
                                                 P.r[j], P.w[j], C.r[j], C.w[j]);
        }

        if (!ring && k >= z0) {
            // momentum of plane k on the wave's row
            Pt3<float> Cn[VX], En[VX], Wn[VX], Nn[VX], Sn[VX], Un[VX], Dn[VX];
            float dE[VX], dW[VX], dN[VX], dS[VX];
            {
                float e[VX], o[VX];
                x_neighbours<VX>(C.r, e, o);
#pragma unroll
                for (int j = 0; j < VX; ++j) En[j].r = e[j], Wn[j].r = o[j];
                x_neighbours<VX>(C.u, e, o);
#pragma unroll
                for (int j = 0; j < VX; ++j) En[j].u = e[j], Wn[j].u = o[j];
                x_neighbours<VX>(C.v, e, o);
#pragma unroll
                for (int j = 0; j < VX; ++j) En[j].v = e[j], Wn[j].v = o[j];
                x_neighbours<VX>(C.w, e, o);
#pragma unroll
                for (int j = 0; j < VX; ++j) En[j].w = e[j], Wn[j].w = o[j];
                x_neighbours<VX>(dC, dE, dW);
            }
            {
                float t[VX];
                lds_get<VX>(t, sRrow0 + qk * QS + NX);
#pragma unroll
                for (int j = 0; j < VX; ++j) Nn[j].r = t[j];
                lds_get<VX>(t, sRrow0 + qk * QS + FS + NX);
#pragma unroll
                for (int j = 0; j < VX; ++j) Nn[j].v = t[j];
                lds_get<VX>(t, sRrow0 + qk * QS - NX);
#pragma unroll
                for (int j = 0; j < VX; ++j) Sn[j].r = t[j];
                lds_get<VX>(t, sRrow0 + qk * QS + FS - NX);
#pragma unroll
                for (int j = 0; j < VX; ++j) Sn[j].v = t[j];
                lds_get<VX>(t, sUrow + NX);
#pragma unroll
                for (int j = 0; j < VX; ++j) Nn[j].u = t[j];
                lds_get<VX>(t, sUrow + US + NX);
#pragma unroll
                for (int j = 0; j < VX; ++j) Nn[j].w = t[j];
                lds_get<VX>(t, sUrow - NX);
#pragma unroll
                for (int j = 0; j < VX; ++j) Sn[j].u = t[j];
                lds_get<VX>(t, sUrow + US - NX);
#pragma unroll
                for (int j = 0; j < VX; ++j) Sn[j].w = t[j];
                lds_get<VX>(dN, sUrow + 2 * US + NX);
                lds_get<VX>(dS, sUrow + 2 * US - NX);
            }
            float ro[VX], uo[VX], vo[VX], wo[VX];
#pragma unroll
            for (int j = 0; j < VX; ++j) {
                Cn[j] = Pt3<float>{C.r[j], C.u[j], C.v[j], C.w[j]};
                Un[j] = Pt3<float>{U.r[j], U.u[j], U.v[j], U.w[j]};
                Dn[j] = Pt3<float>{D.r[j], D.u[j], D.v[j], D.w[j]};
                momentum3d<false, float>(c, Cn[j], En[j], Wn[j], Nn[j], Sn[j], Un[j], Dn[j], dC[j], dE[j], dW[j],
                                         dN[j], dS[j], dU[j], dD[j], fxrow, false, 0.f, 0.f, 0.f, ro[j], uo[j],
                                         vo[j], wo[j]);
            }
            const PlaneAccess<WIDE, float> po(out, k, plane, pbytes, fbytes);
            row_store<VX>(ro, po.r, stoff, po.soff);
            row_store<VX>(uo, po.u, stoff, po.soff);
            row_store<VX>(vo, po.v, stoff, po.soff);
            row_store<VX>(wo, po.w, stoff, po.soff);
        }
#pragma unroll
        for (int j = 0; j < VX; ++j) {
            dD[j] = dC[j];
            dC[j] = dU[j];
        }
    };

    // unrolled over NU planes (a multiple of NF and of the LDS parity 2);
    // explicit calls keep every register set in registers
    constexpr int NU = (NF % 2 == 0) ? NF : 2 * NF;
    static_assert(NU <= 10, "prefetch depth 1, 2 or 4");
    int k = k0;
#define ROWS_IT(j) \
    if constexpr ((j) < NU) iterate(k + (j), std::integral_constant<int, (j)>{});
#define ROWS_TAIL(j) \
    if constexpr ((j) < NU - 1) {                                      \
        if (k + (j) < z1) iterate(k + (j), std::integral_constant<int, (j)>{}); \
    }
    for (; k + NU - 1 < z1; k += NU) {
        ROWS_IT(0) ROWS_IT(1) ROWS_IT(2) ROWS_IT(3) ROWS_IT(4) ROWS_IT(5) ROWS_IT(6) ROWS_IT(7) ROWS_IT(8) ROWS_IT(9)
    }
    ROWS_TAIL(0) ROWS_TAIL(1) ROWS_TAIL(2) ROWS_TAIL(3) ROWS_TAIL(4) ROWS_TAIL(5) ROWS_TAIL(6) ROWS_TAIL(7) ROWS_TAIL(8)
#undef ROWS_IT
#undef ROWS_TAIL
}

// The row kernel applies: FP32 fully periodic box with rho0 = 1 and no
// per-node force, nx one of 64, 128, 256, ny >= 3 (the ring rows must be
// distinct from the band's rows on a small grid: ny >= TY + 2 is checked by
// the launcher), nz >= 2.
template <typename T>
bool step3d_rows_ok(const Coef<T>& c)
{
    if constexpr (sizeof(T) != 4) {
        return false;
    } else {
        return !c.nonperiodic && c.rho0 == T(1) && !c.fst[0] && c.nz >= 2 && c.ny >= 4 &&
               (c.nx == 64 || c.nx == 128 || c.nx == 256);
    }
}

template <int VX, int NW>
static hipError_t launch_rows(const Coef<float>& c, const State<float>& in, const State<float>& out, int zc,
                              hipStream_t s)
{
    constexpr int TY = NW - 2;
    constexpr int PD = ROWS_PREFETCH;
    if (c.ny < TY + 4) return hipErrorInvalidValue;
    const int nby = (c.ny + TY - 1) / TY, nbz = (c.nz + zc - 1) / zc;
    const bool wide = (size_t)c.nx * c.ny * c.nz * sizeof(float) >= (size_t(1) << 31);
    if (!wide)
        hipLaunchKernelGGL((step3d_rows_kernel<VX, NW, false, PD>), dim3(nby * nbz), dim3(NW * 64), 0, s, c, in, out,
                           zc, nby);
    else
        hipLaunchKernelGGL((step3d_rows_kernel<VX, NW, true, PD>), dim3(nby * nbz), dim3(NW * 64), 0, s, c, in, out,
                           zc, nby);
    return hipGetLastError();
}

template <int NW>
static hipError_t launch_rows_nw(const Coef<float>& c, const State<float>& in, const State<float>& out, int zc,
                                 hipStream_t s)
{
    switch (c.nx) {
        case 64: return launch_rows<1, NW>(c, in, out, zc, s);
        case 128: return launch_rows<2, NW>(c, in, out, zc, s);
        default: return launch_rows<4, NW>(c, in, out, zc, s);
    }
}

// shape: 16 -> 6 waves (4-row bands), 17 -> 8 waves (6 rows), 19 -> 4 waves
// (2 rows); zc planes per chunk
template <typename T>
hipError_t launch_step3d_rows(const Coef<T>& c, const State<T>& in, const State<T>& out, int shape, int zc,
                              hipStream_t s)
{
    if constexpr (sizeof(T) != 4) {
        return hipErrorInvalidValue;
    } else {
        if (!step3d_rows_ok(c)) return hipErrorInvalidValue;
        switch (shape) {
            case 17: return launch_rows_nw<8>(c, in, out, zc, s);
            case 19: return launch_rows_nw<4>(c, in, out, zc, s);
            default: return launch_rows_nw<6>(c, in, out, zc, s);
        }
    }
}

template bool step3d_rows_ok<float>(const Coef<float>&);
template bool step3d_rows_ok<double>(const Coef<double>&);
template hipError_t launch_step3d_rows<float>(const Coef<float>&, const State<float>&, const State<float>&, int, int,
                                              hipStream_t);
template hipError_t launch_step3d_rows<double>(const Coef<double>&, const State<double>&, const State<double>&, int,
                                               int, hipStream_t);

}  // namespace acm
