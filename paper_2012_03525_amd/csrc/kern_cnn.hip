// Learned-closure network on gfx950: per-layer 3x3 convolutions as implicit
// GEMMs on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) for training, the weight gradient as an MFMA reduction over
// pixels, a one-launch whole-network inference kernel (16x16x32 bf16 MFMA,
// all layers of a tile in LDS) for the closure run, and the element-wise
// pieces (input packing, loss gradient, correction, Adam, box filter,
// bilinear prolongation).
//
// Layouts (all device memory, caller-owned unless stated):
//   activations  bf16 [H][W][C], channel fastest; C = 16 (padded 3-channel
//                input / output) or 32
//   weights      bf16 [9][C_out][C_in], tap t = (dy+1)*3 + (dx+1)
//   bias, grads  fp32
// Convolution: y[p][o] = b[o] + sum_{t,i} w[t][o][i] x[p + off(t)][i] with
// circular (periodic) wrap.  MFMA operand mapping: v_mfma_f32_16x16x32_bf16
// has A[i][k] in lane i + 16*(k/8), element k%8, and B[k][n] in lane
// n + 16*(k/8); v_mfma_f32_16x16x16_bf16 (used where K is only 16) has
// A[i][k] in lane i + 16*(k/4), element k%4, and B[k][n] in lane
// n + 16*(k/4); both give D[i][n] in lane n + 16*(i/4), element i%4.  Both
// issue at the same rate, so K = 32 halves the instruction count.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>

#include "../../include/acm.h"
#include "acm_internal.h"
#include "tile2d.h"

namespace acm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;

// float -> bf16, round to nearest even, by the hardware conversion
// (v_cvt_pk_bf16_f32 converts two values per instruction)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16_t f2bf(float f) { return __builtin_bit_cast(bf16_t, (__bf16)f); }
__device__ __forceinline__ unsigned f2bf2(float lo, float hi)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, bf16x2v));
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

enum : int { CONV_RELU = 0, CONV_RAW = 1, CONV_MASK = 2 };

// ---------------------------------------------------------------------------
// forward convolution: workgroup tile TR rows x 32 columns, 4 waves; wave w
// owns TR/4 rows, i.e. TR/2 groups of 16 pixels, whose accumulators are
// advanced together so consecutive MFMAs are independent.  The weights of
// the layer are fetched into registers (MFMA B operands) before the input
// tile (with a one-pixel circular halo) is staged in LDS, so both loads are
// in flight together.
// MODE: CONV_RELU   y = bf16(relu(conv + b))
//       CONV_RAW    y = fp32(conv + b)
//       CONV_MASK   y = bf16(conv * (mask > 0))   (data gradient through ReLU)
// ---------------------------------------------------------------------------
// Operands of the K = 32 (CIN a multiple of 32) or K = 16 (CIN = 16) product:
// KW channels per lane, lane group lg holding channels KW lg .. KW lg + KW - 1
// of a block of 4 KW.
template <int CIN>
struct ConvK {
    static constexpr int KW = CIN % 32 == 0 ? 8 : 4;  // channels per lane
    static constexpr int KB = 4 * KW;                 // channels per product
    static constexpr int KS = CIN / KB;               // products per tap
    typedef typename std::conditional<KW == 8, bf16x8s, bf16x4>::type op;
    static __device__ __forceinline__ f32x4 mfma(const op& a, const op& b, const f32x4& c)
    {
        if constexpr (KW == 8)
            return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8v, a),
                                                           __builtin_bit_cast(bf16x8v, b), c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
};

template <int CIN, int COUT, int MODE, int TR = 4>
__global__ __launch_bounds__(256) void conv3x3_kernel(int H, int W, const bf16_t* __restrict__ x,
                                                      const bf16_t* __restrict__ w, const float* __restrict__ bias,
                                                      const bf16_t* __restrict__ mask, void* __restrict__ y)
{
    using K = ConvK<CIN>;
    using op = typename K::op;
    constexpr int TC = 32, IR = TR + 2, IC = TC + 2;
    constexpr int KS = K::KS, KB = K::KB, KW = K::KW, NH = COUT / 16, CH4 = CIN / 4;
    constexpr int NG = TR / 2;  // 16-pixel groups per wave
    __shared__ __align__(16) bf16_t sx[IR * IC * CIN];
    const int tiles_x = W / TC;
    const int x0 = (blockIdx.x % tiles_x) * TC, y0 = (blockIdx.x / tiles_x) * TR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lg = lane >> 4;
    op bw[9][KS][NH];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int nh = 0; nh < NH; ++nh)
                bw[t][ks][nh] = *reinterpret_cast<const op*>(w + ((size_t)(t * COUT + nh * 16 + l16) * CIN +
                                                                 ks * KB + lg * KW));
    {
        constexpr int TOT = IR * IC * CH4;
        constexpr int NIT = (TOT + 255) / 256;
        uint2 v[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {  // all loads first, then the LDS stores
            const int q = min((int)threadIdx.x + it * 256, TOT - 1);
            const int c4 = q % CH4, pix = q / CH4;
            const int r = pix / IC, cc = pix - r * IC;
            const int gy = wrap(y0 + r - 1, H), gx = wrap(x0 + cc - 1, W);
            v[it] = *reinterpret_cast<const uint2*>(x + ((size_t)gy * W + gx) * CIN + c4 * 4);
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = threadIdx.x + it * 256;
            if (q < TOT) {
                const int c4 = q % CH4, pix = q / CH4;
                *reinterpret_cast<uint2*>(sx + pix * CIN + c4 * 4) = v[it];
            }
        }
    }
    __syncthreads();
    f32x4 acc[NG][NH];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int nh = 0; nh < NH; ++nh) acc[g][nh] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int dy = t / 3 - 1, dx = t % 3 - 1;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            op a[NG];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int r = (TR / 4) * wave + (g >> 1), c0 = (g & 1) * 16;
                const int pix = (r + 1 + dy) * IC + (c0 + l16 + 1 + dx);
                a[g] = *reinterpret_cast<const op*>(sx + pix * CIN + ks * KB + lg * KW);
            }
#pragma unroll
            for (int g = 0; g < NG; ++g)
#pragma unroll
                for (int nh = 0; nh < NH; ++nh) acc[g][nh] = K::mfma(a[g], bw[t][ks][nh], acc[g][nh]);
        }
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int r = (TR / 4) * wave + (g >> 1), c0 = (g & 1) * 16;
        const int py = y0 + r;
#pragma unroll
        for (int nh = 0; nh < NH; ++nh) {
            const int co = nh * 16 + l16;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int px = x0 + c0 + 4 * lg + j;
                const size_t o = ((size_t)py * W + px) * COUT + co;
                float val = acc[g][nh][j];
                if constexpr (MODE == CONV_RELU) {
                    val = fmaxf(val + bias[co], 0.f);
                    static_cast<bf16_t*>(y)[o] = f2bf(val);
                } else if constexpr (MODE == CONV_RAW) {
                    static_cast<float*>(y)[o] = val + bias[co];
                } else {
                    const bf16_t m = mask[o];
                    const bool pos = (m & 0x8000u) == 0 && (m & 0x7FFFu) != 0;
                    static_cast<bf16_t*>(y)[o] = f2bf(pos ? val : 0.f);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[t][o][i] = sum_p g[p][o] x[p + off(t)][i], db[o] = sum_p g[p][o]
// Workgroup tile 4 rows x 64 columns; x (with halo) and g are staged in LDS
// channel-major so that eight consecutive pixels of one channel are one
// operand of a K = 32 product over pixels.  The 16x16 output tiles
// (tap, o-block, i-block) are dealt to the waves by tap row: a wave owns the
// three taps dx = -1, 0, 1 of a (dy, o-block, i-block), whose x operands are
// the same 10 halfwords of a channel row shifted by 0, 1 and 2, so one
// 16-byte and one 4-byte load serve all three.  The partial sums of every
// workgroup go to a workspace reduced in a fixed order.
// ---------------------------------------------------------------------------
constexpr int WG_TR = 4, WG_TC = 64;

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(int H, int W, const bf16_t* __restrict__ x,
                                                         const bf16_t* __restrict__ g, float* __restrict__ partial)
{
    // channel rows of x: columns x0-1 .. x0+64 and padding; of g: columns x0 .. x0+63
    // and padding (row strides of 144 bytes)
    constexpr int XR = WG_TR + 2, XC = WG_TC + 8, GC = WG_TC + 8;
    __shared__ __align__(16) bf16_t sxT[XR][CIN][XC];
    __shared__ __align__(16) bf16_t sgT[WG_TR][COUT][GC];
    const int tiles_x = W / WG_TC;
    const int x0 = (blockIdx.x % tiles_x) * WG_TC, y0 = (blockIdx.x / tiles_x) * WG_TR;
    for (int q = threadIdx.x; q < XR * (WG_TC + 2) * CIN; q += 256) {
        const int ci = q % CIN, pix = q / CIN;
        const int r = pix / (WG_TC + 2), cc = pix - r * (WG_TC + 2);
        const int gy = wrap(y0 + r - 1, H), gx = wrap(x0 + cc - 1, W);
        sxT[r][ci][cc] = x[((size_t)gy * W + gx) * CIN + ci];
    }
    for (int q = threadIdx.x; q < WG_TR * WG_TC * COUT; q += 256) {
        const int co = q % COUT, pix = q / COUT;
        const int r = pix / WG_TC, cc = pix - r * WG_TC;
        sgT[r][co][cc] = g[((size_t)(y0 + r) * W + x0 + cc) * COUT + co];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lg = lane >> 4;
    constexpr int OB = COUT / 16, IB = CIN / 16;
    constexpr int NTRI = 3 * OB * IB;      // (dy, o-block, i-block) triples
    constexpr int PER = (NTRI + 3) / 4;    // triples per wave
    f32x4 acc[PER][3];
#pragma unroll
    for (int s = 0; s < PER; ++s)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) acc[s][dx] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int r = 0; r < WG_TR; ++r) {
#pragma unroll 1
        for (int kc = 0; kc < WG_TC / 32; ++kc) {
            const int c0 = kc * 32 + 8 * lg;  // this lane's eight pixels: columns c0 .. c0 + 7
#pragma unroll
            for (int s = 0; s < PER; ++s) {
                const int tr = wave + 4 * s;
                if (tr < NTRI) {
                    const int dy = tr / (OB * IB) - 1, rem = tr % (OB * IB);
                    const int ob = rem / IB, ib = rem % IB;
                    // A[i = o][k = pixel]
                    const bf16x8v a = *reinterpret_cast<const bf16x8v*>(&sgT[r][ob * 16 + l16][c0]);
                    // B[k = pixel][n = i] for dx = -1, 0, 1: x columns c0 + dx .. c0 + dx + 7,
                    // i.e. halfwords 0..7, 1..8 and 2..9 of the row from column c0 - 1
                    const bf16_t* row = &sxT[r + 1 + dy][ib * 16 + l16][c0];
                    const uint4 lo = *reinterpret_cast<const uint4*>(row);
                    const unsigned hi = *reinterpret_cast<const unsigned*>(row + 8);
                    const uint4 mid = {__builtin_amdgcn_alignbyte(lo.y, lo.x, 2), __builtin_amdgcn_alignbyte(lo.z, lo.y, 2),
                                       __builtin_amdgcn_alignbyte(lo.w, lo.z, 2), __builtin_amdgcn_alignbyte(hi, lo.w, 2)};
                    const uint4 up = {lo.y, lo.z, lo.w, hi};
                    acc[s][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8v, lo), acc[s][0], 0, 0, 0);
                    acc[s][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8v, mid), acc[s][1], 0, 0, 0);
                    acc[s][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8v, up), acc[s][2], 0, 0, 0);
                }
            }
        }
    }
    float* part = partial + (size_t)blockIdx.x * (9 * COUT * CIN + COUT);
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const int tr = wave + 4 * s;
        if (tr < NTRI) {
            const int dyi = tr / (OB * IB), rem = tr % (OB * IB);
            const int ob = rem / IB, ib = rem % IB;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int tap = 3 * dyi + dx;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int o = ob * 16 + 4 * lg + j, i = ib * 16 + l16;
                    part[((size_t)tap * COUT + o) * CIN + i] = acc[s][dx][j];
                }
            }
        }
    }
    if ((int)threadIdx.x < COUT) {
        float sb = 0.f;
        for (int r = 0; r < WG_TR; ++r)
            for (int c = 0; c < WG_TC; ++c) sb += bf2f(sgT[r][threadIdx.x][c]);
        part[9 * COUT * CIN + threadIdx.x] = sb;
    }
}

// fixed-order sum of the per-workgroup partials: out[e] = sum_b partial[b][e]
// (acc: out[e] += that sum).  A workgroup takes 64 consecutive elements;
// wave s of its RP_SEG waves sums the blocks b = s, s + RP_SEG, ... in
// increasing b (64 consecutive floats of a partial row per load), and the
// RP_SEG segment sums are added in increasing s: a fixed order for any
// launch, with RP_SEG independent load streams per element.
constexpr int RP_SEG = 16;
__global__ __launch_bounds__(64 * RP_SEG) void reduce_partials_kernel(const float* __restrict__ partial, int nblk,
                                                                      int n, float* __restrict__ dw,
                                                                      float* __restrict__ db, int nw, int acc)
{
    __shared__ float seg[RP_SEG][64];
    const int lane = threadIdx.x & 63, sgi = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    float s = 0.f;
    if (e < n) {
        int b = sgi;
        // four loads in flight per lane; the sum stays in increasing b
        for (; b + 3 * RP_SEG < nblk; b += 4 * RP_SEG) {
            const float v0 = partial[(size_t)b * n + e], v1 = partial[(size_t)(b + RP_SEG) * n + e];
            const float v2 = partial[(size_t)(b + 2 * RP_SEG) * n + e], v3 = partial[(size_t)(b + 3 * RP_SEG) * n + e];
            s = (((s + v0) + v1) + v2) + v3;
        }
        for (; b < nblk; b += RP_SEG) s += partial[(size_t)b * n + e];
    }
    seg[sgi][lane] = s;
    __syncthreads();
    if (sgi == 0 && e < n) {
        float t = seg[0][lane];
        for (int k = 1; k < RP_SEG; ++k) t += seg[k][lane];
        float* dst = e < nw ? &dw[e] : &db[e - nw];
        *dst = acc ? *dst + t : t;
    }
}

// wt[t][i][o] = w[8 - t][o][i]: weights of the transposed convolution
__global__ void transpose_weights_kernel(int cin, int cout, const bf16_t* __restrict__ w, bf16_t* __restrict__ wt)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= 9 * cin * cout) return;
    const int t = e / (cin * cout), rem = e % (cin * cout);
    const int i = rem / cout, o = rem % cout;
    wt[e] = w[((size_t)(8 - t) * cout + o) * cin + i];
}

// normalised network input: a0[p][c] = bf16(s_c q_c[p]) for c < 3, zero above
__global__ void pack_input_kernel(int n, const float* __restrict__ r, const float* __restrict__ u,
                                  const float* __restrict__ v, float s0, float s1, float s2, bf16_t* __restrict__ a0)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    bf16_t out[16];
    out[0] = f2bf(r[p] * s0);
    out[1] = f2bf(u[p] * s1);
    out[2] = f2bf(v[p] * s2);
    for (int c = 3; c < 16; ++c) out[c] = 0;
    uint4* dst = reinterpret_cast<uint4*>(a0 + (size_t)p * 16);
    dst[0] = *reinterpret_cast<uint4*>(&out[0]);
    dst[1] = *reinterpret_cast<uint4*>(&out[8]);
}

// correction: q_c[p] += d_c raw[p][c]
__global__ void apply_correction_kernel(int n, const float* __restrict__ raw, float d0, float d1, float d2,
                                        float* __restrict__ r, float* __restrict__ u, float* __restrict__ v)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const float* o = raw + (size_t)p * 16;
    r[p] = fmaf(d0, o[0], r[p]);
    u[p] = fmaf(d1, o[1], u[p]);
    v[p] = fmaf(d2, o[2], v[p]);
}

// loss: target residual t_c = (target_c - base_c) / d_c; e = raw_c - t_c;
// grad[p][c] = bf16(2 e / (3 n)) (zero for padded channels); per-block sum of e^2
// Channels with a zero output scale take no part in the loss: their error
// and gradient are zero (w = 0) and nact counts the others.
struct LossChannels {
    float id[3];  // 1 / out_scale, or 0 for an excluded channel
    float w[3];   // 1 or 0
    int nact;
};

__global__ __launch_bounds__(256) void loss_grad_kernel(int n, const float* __restrict__ raw,
                                                        const float* __restrict__ b0, const float* __restrict__ b1,
                                                        const float* __restrict__ b2, const float* __restrict__ t0,
                                                        const float* __restrict__ t1, const float* __restrict__ t2,
                                                        LossChannels lc, bf16_t* __restrict__ grad,
                                                        double* __restrict__ partial)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    double se = 0.0;
    if (p < n) {
        const float* o = raw + (size_t)p * 16;
        const float e0 = lc.w[0] * (o[0] - (t0[p] - b0[p]) * lc.id[0]);
        const float e1 = lc.w[1] * (o[1] - (t1[p] - b1[p]) * lc.id[1]);
        const float e2 = lc.w[2] * (o[2] - (t2[p] - b2[p]) * lc.id[2]);
        se = (double)e0 * e0 + (double)e1 * e1 + (double)e2 * e2;
        const float k = 2.f / ((float)lc.nact * (float)n);
        bf16_t out[16];
        out[0] = f2bf(k * e0);
        out[1] = f2bf(k * e1);
        out[2] = f2bf(k * e2);
        for (int c = 3; c < 16; ++c) out[c] = 0;
        uint4* dst = reinterpret_cast<uint4*>(grad + (size_t)p * 16);
        dst[0] = *reinterpret_cast<uint4*>(&out[0]);
        dst[1] = *reinterpret_cast<uint4*>(&out[8]);
    }
    __shared__ double red[256];
    red[threadIdx.x] = se;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out = sum_b partial[b] / count: thread t sums b = t, t + 64, ... in
// increasing b, then thread 0 adds the 64 sums in increasing t (fixed order)
__global__ __launch_bounds__(64) void loss_final_kernel(const double* __restrict__ partial, int nblk, double count,
                                                        double* __restrict__ out)
{
    __shared__ double part[64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += partial[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t = part[0];
    for (int k = 1; k < 64; ++k) t += part[k];
    out[0] = t / count;
}

// loss of a state against its target, for training through several steps:
// e_c = (q_c - t_c) / d_c on the active channels; adj_c += k e_c / d_c with
// k = 2 weight / (n_active n); per-block sum of e^2
__global__ __launch_bounds__(256) void state_loss_kernel(int n, const float* __restrict__ q0,
                                                         const float* __restrict__ q1, const float* __restrict__ q2,
                                                         const float* __restrict__ t0, const float* __restrict__ t1,
                                                         const float* __restrict__ t2, LossChannels lc, float k,
                                                         float* __restrict__ a0, float* __restrict__ a1,
                                                         float* __restrict__ a2, double* __restrict__ partial)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    double se = 0.0;
    if (p < n) {
        const float e0 = lc.w[0] * (q0[p] - t0[p]) * lc.id[0];
        const float e1 = lc.w[1] * (q1[p] - t1[p]) * lc.id[1];
        const float e2 = lc.w[2] * (q2[p] - t2[p]) * lc.id[2];
        se = (double)e0 * e0 + (double)e1 * e1 + (double)e2 * e2;
        a0[p] = fmaf(k * e0, lc.id[0], a0[p]);
        a1[p] = fmaf(k * e1, lc.id[1], a1[p]);
        a2[p] = fmaf(k * e2, lc.id[2], a2[p]);
    }
    __shared__ double red[256];
    red[threadIdx.x] = se;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// divergence penalty of a correction: d = G.(a - b) (centred, periodic, in
// grid units); per-block sum of d^2; adj_a += k G^T d and adj_b -= k G^T d
// with k = 2 weight / n.  G^T d at a node is ((d_W - d_E) / 2, (d_S - d_N) / 2),
// each neighbour's d formed from the four differences around it.
__device__ __forceinline__ float dcorr(const float* __restrict__ a, const float* __restrict__ b, size_t o)
{
    return a[o] - b[o];
}

__device__ __forceinline__ float div_at(int nx, int ny, int x, int y, const float* __restrict__ au,
                                        const float* __restrict__ bu, const float* __restrict__ av,
                                        const float* __restrict__ bv)
{
    const int xe = x + 1 == nx ? 0 : x + 1, xw = x == 0 ? nx - 1 : x - 1;
    const int yn = y + 1 == ny ? 0 : y + 1, ys = y == 0 ? ny - 1 : y - 1;
    const size_t row = (size_t)y * nx;
    return 0.5f * ((dcorr(au, bu, row + xe) - dcorr(au, bu, row + xw)) +
                   (dcorr(av, bv, (size_t)yn * nx + x) - dcorr(av, bv, (size_t)ys * nx + x)));
}

__global__ __launch_bounds__(256) void div_penalty_kernel(int nx, int ny, const float* __restrict__ au,
                                                          const float* __restrict__ av, const float* __restrict__ bu,
                                                          const float* __restrict__ bv, float k,
                                                          float* __restrict__ gau, float* __restrict__ gav,
                                                          float* __restrict__ gbu, float* __restrict__ gbv,
                                                          double* __restrict__ partial)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    double se = 0.0;
    if (p < nx * ny) {
        const int y = p / nx, x = p - y * nx;
        const int xe = x + 1 == nx ? 0 : x + 1, xw = x == 0 ? nx - 1 : x - 1;
        const int yn = y + 1 == ny ? 0 : y + 1, ys = y == 0 ? ny - 1 : y - 1;
        const float d = div_at(nx, ny, x, y, au, bu, av, bv);
        se = (double)d * d;
        const float gu = 0.5f * (div_at(nx, ny, xw, y, au, bu, av, bv) - div_at(nx, ny, xe, y, au, bu, av, bv));
        const float gv = 0.5f * (div_at(nx, ny, x, ys, au, bu, av, bv) - div_at(nx, ny, x, yn, au, bu, av, bv));
        gau[p] = fmaf(k, gu, gau[p]);
        gav[p] = fmaf(k, gv, gav[p]);
        if (gbu) {
            gbu[p] = fmaf(-k, gu, gbu[p]);
            gbv[p] = fmaf(-k, gv, gbv[p]);
        }
    }
    __shared__ double red[256];
    red[threadIdx.x] = se;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out += scale * (fixed-order sum of the partials)
__global__ void loss_accumulate_kernel(const double* __restrict__ partial, int nblk, double scale,
                                       double* __restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[b];
    out[0] += s * scale;
}

// Adam (Kingma & Ba) with bias correction; p16 (optional) receives bf16(p)
__global__ void adam_kernel(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, bf16_t* __restrict__ p16, float lr, float b1, float b2, float eps,
                            float c1, float c2)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float ge = g[e];
    const float me = fmaf(b1, m[e], (1.f - b1) * ge);
    const float ve = fmaf(b2, v[e], (1.f - b2) * ge * ge);
    m[e] = me;
    v[e] = ve;
    const float pe = p[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
    p[e] = pe;
    if (p16) p16[e] = f2bf(pe);
}

__global__ void to_bf16_kernel(size_t n, const float* __restrict__ s, bf16_t* __restrict__ d)
{
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) d[e] = f2bf(s[e]);
}

// box filter: coarse node (I, J) averages fine nodes (rI..rI+r-1, rJ..rJ+r-1)
template <typename T>
__global__ void box_filter_kernel(int nxc, int nyc, int r, const T* __restrict__ f, T* __restrict__ c)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nxc * nyc) return;
    const int J = e / nxc, I = e - J * nxc;
    const int nxf = nxc * r;
    double s = 0.0;
    for (int b = 0; b < r; ++b)
        for (int a = 0; a < r; ++a) s += (double)f[(size_t)(J * r + b) * nxf + I * r + a];
    c[e] = (T)(s / (double)(r * r));
}

// periodic bilinear prolongation; coarse node I sits at fine coordinate r I + (r-1)/2
template <typename T>
__global__ void prolong_kernel(int nxc, int nyc, int r, const T* __restrict__ c, T* __restrict__ f)
{
    const int nxf = nxc * r, nyf = nyc * r;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nxf * nyf) return;
    const int j = e / nxf, i = e - j * nxf;
    const double sx = (i - 0.5 * (r - 1)) / r, sy = (j - 0.5 * (r - 1)) / r;
    const int ix = (int)floor(sx), iy = (int)floor(sy);
    const double tx = sx - ix, ty = sy - iy;
    const int x0 = (ix % nxc + nxc) % nxc, x1 = (x0 + 1) % nxc;
    const int y0 = (iy % nyc + nyc) % nyc, y1 = (y0 + 1) % nyc;
    const double a = (double)c[(size_t)y0 * nxc + x0] * (1 - tx) + (double)c[(size_t)y0 * nxc + x1] * tx;
    const double b = (double)c[(size_t)y1 * nxc + x0] * (1 - tx) + (double)c[(size_t)y1 * nxc + x1] * tx;
    f[e] = (T)(a * (1 - ty) + b * ty);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
constexpr int CONV_TR = 4;  // rows per workgroup tile (two workgroups per CU at 256 x 256)

template <int CIN, int COUT, int MODE>
hipError_t launch_conv(int H, int W, const bf16_t* x, const bf16_t* w, const float* b, const bf16_t* mask, void* y,
                       hipStream_t s)
{
    hipLaunchKernelGGL((conv3x3_kernel<CIN, COUT, MODE, CONV_TR>), dim3((W / 32) * (H / CONV_TR)), dim3(256), 0, s, H,
                       W, x, w, b, mask, y);
    return hipGetLastError();
}

hipError_t conv_dispatch(int H, int W, int cin, int cout, int mode, const void* x, const void* w, const float* b,
                         const void* mask, void* y, hipStream_t s)
{
    const bf16_t* xx = static_cast<const bf16_t*>(x);
    const bf16_t* ww = static_cast<const bf16_t*>(w);
    const bf16_t* mm = static_cast<const bf16_t*>(mask);
    if (cin == 16 && cout == 32 && mode == CONV_RELU) return launch_conv<16, 32, CONV_RELU>(H, W, xx, ww, b, mm, y, s);
    if (cin == 32 && cout == 32 && mode == CONV_RELU) return launch_conv<32, 32, CONV_RELU>(H, W, xx, ww, b, mm, y, s);
    if (cin == 32 && cout == 16 && mode == CONV_RAW) return launch_conv<32, 16, CONV_RAW>(H, W, xx, ww, b, mm, y, s);
    if (cin == 16 && cout == 32 && mode == CONV_MASK) return launch_conv<16, 32, CONV_MASK>(H, W, xx, ww, b, mm, y, s);
    if (cin == 32 && cout == 32 && mode == CONV_MASK) return launch_conv<32, 32, CONV_MASK>(H, W, xx, ww, b, mm, y, s);
    if (cin == 32 && cout == 32 && mode == CONV_RAW) return launch_conv<32, 32, CONV_RAW>(H, W, xx, ww, b, mm, y, s);
    if (cin == 16 && cout == 32 && mode == CONV_RAW) return launch_conv<16, 32, CONV_RAW>(H, W, xx, ww, b, mm, y, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Whole-network inference on one 16x16 output tile per workgroup:
//   q_out = q_in + D f(N q_in).
// Layer l (0..4) is evaluated on the tile grown by 4 - l nodes on every side,
// so the five-node receptive field is covered without exchanging data between
// workgroups (the ring is recomputed by the neighbours).  Weights of every
// layer and two activation buffers live in LDS.
// The MFMA roles are transposed with respect to conv3x3_kernel: A = weights
// (16 output channels x 32 inputs), B = activations (32 inputs x 16 pixels),
// so each lane's accumulator holds four consecutive output channels of one
// pixel and is written back as one 8-byte LDS store.  v_mfma_f32_16x16x32_bf16
// pairs element e of lane (i, g) in A with element e of lane (n, g) in B, so
// loading A and B with the same k order gives the product for any layout of
// k inside a lane.  The first layer is an im2col product: taps 0..7 with
// their 3 channels and a zero pad make K = 32, tap 8 a second K = 32 product
// with zero weights past its channels, instead of nine K = 16 products.
//
// LDS layout.  Every activation buffer has the row pitch of layer 0's output
// (P = 24 slots of 32 channels, 64 bytes): layer l's output position (y, x)
// is slot q = 24 y + x, and its input for tap (dy, dx) is slot q + 25 + 24 dy
// + dx of the previous buffer, so a group of 16 consecutive slots reads 16
// consecutive slots for every tap.  Layer l >= 1 computes whole pitch rows,
// the columns past its width included (their values are never read by a
// column inside the width: 1.17x the MFMA work of layers 1..4 in exchange for
// reads without row breaks).  The four 16-byte chunks of a 64-byte row
// (slot, or weight row) are stored in the order c ^ ((row >> 1) & 3): on
// gfx950 sixteen lanes reading chunk lg of 16 consecutive rows then hit
// distinct banks (measured: 4.7 cycles per ds_read_b128 per CU against 8.3
// unswizzled, and 12 with a row break inside the group).
// ---------------------------------------------------------------------------
namespace fused {
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
constexpr int T = 16;                     // output tile side
constexpr int NT = 512;                   // threads per workgroup
constexpr int NW = NT / 64;               // waves
constexpr int P = T + 8;                  // slot pitch of every activation buffer (layer 0's output side, 24)
constexpr int SI = T + 10;                // staged input side (26)
constexpr int SLOT = 32;                  // halfwords per slot (32 channels)
constexpr int W0A = 32 * 32;              // layer 0, taps 0..7 as im2col: [o][k], k = 4 t + c
constexpr int W0 = W0A + 32 * 4;          // then tap 8: [o][c]
constexpr int WL = 9 * 32 * 32;           // layers 1..3: [t][o][i]
constexpr int W4 = 9 * 16 * 32;           // layer 4: [t][o][i]
constexpr int OW1 = W0, OW2 = OW1 + WL, OW3 = OW2 + WL, OW4 = OW3 + WL, WTOT = OW4 + W4;
constexpr int PAD = 32;                   // slots past a buffer's last row, read by the last columns only
constexpr int BA = (P * P + PAD) * SLOT;        // outputs of layers 0 and 2
constexpr int BB = ((P - 2) * P + PAD) * SLOT;  // outputs of layers 1 and 3; the staged input before them
constexpr int LDS_HALF = WTOT + BA + BB;
constexpr int NBIAS = 4 * 32 + 16;        // biases of the five layers, in order
static_assert(SI * SI * 4 <= BB, "input fits in buffer B");
// 256-byte aligned buffers: the bank pattern of a swizzled row depends on the address modulo 256
static_assert(OW1 % 128 == 0 && WTOT % 128 == 0 && BA % 128 == 0, "256-byte aligned buffers");

struct Args {
    const float* qi[3];  // state after the coarse step (read only)
    float* qo[3];        // corrected state
    float s[3], d[3];    // input and output channel scales
    const bf16_t* w[ACM_CNN_LAYERS];
    const float* b[ACM_CNN_LAYERS];
};

// halfword offset of 16-byte chunk c (channels 8 c .. 8 c + 7) of 64-byte row r
__device__ __forceinline__ int chunk_at(int r, int c) { return r * SLOT + 8 * (c ^ ((r >> 1) & 3)); }

__device__ __forceinline__ bf16x8 lds8(const bf16_t* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ __forceinline__ uint2 pack4(float a, float b, float c, float d) { return uint2{f2bf2(a, b), f2bf2(c, d)}; }

// bf16(relu(x)) of four values: rounding keeps the sign, so the ReLU is
// taken after the conversion, as a signed 16-bit maximum with 0 on each
// half (a negative value or -0 has its top bit set).  Equal to converting
// relu(x) for every value but NaN.
__device__ __forceinline__ unsigned relu2(float a, float b)
{
    const s16x2 h = __builtin_bit_cast(s16x2, f2bf2(a, b));
    return __builtin_bit_cast(unsigned, __builtin_elementwise_max(h, s16x2{0, 0}));
}
__device__ __forceinline__ uint2 relu4(const f32x4& v) { return uint2{relu2(v[0], v[1]), relu2(v[2], v[3])}; }

// Offset (halfwords) of the 8-byte store of output channels 16 nh + 4 lg ..
// + 3 of slot l16 (a group starts at a multiple of 16 slots, which leaves
// (slot >> 1) & 3 unchanged).
__device__ __forceinline__ int store_off(int l16, int lg, int nh)
{
    return chunk_at(l16, 2 * nh + (lg >> 1)) + 4 * (lg & 1);
}

// Weights of a 32-input-channel layer with NH blocks of 16 output channels
// as MFMA A operands: wa[t][nh] holds output channel 16 nh + l16, inputs
// 8 lg .. 8 lg + 7 of tap t.
template <int NH>
__device__ __forceinline__ void load_weights(const bf16_t* wl, bf16x8 (&wa)[9][NH])
{
    const int lane = threadIdx.x & 63, l16 = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nh = 0; nh < NH; ++nh) wa[t][nh] = lds8(wl + chunk_at((t * NH + nh) * 16 + l16, lg));
}

// One 32-input-channel layer with output width SO (rows of P slots, SO of
// them computed), NH blocks of 16 output channels, weights in wa.  Not LAST:
// bias + ReLU into `out`; LAST: the lanes holding channels 0..3 of a slot
// inside the tile apply the correction, to the uncorrected state read from
// sq in LDS (SQ) or from a.qi.  bias is in LDS.  Wave w takes the groups w,
// w + NW, ...; the operands of the next group are loaded before the products
// of the current one.  After its last group the wave loads the weights of
// the next layer (wl_next, NHN blocks) into wn, while slower waves finish.
template <int SO, int PI, int NH, bool LAST, bool SQ, int NHN>
__device__ __forceinline__ void layer32(const bf16x8 (&wa)[9][NH], const float* bias,
                                        const bf16_t* __restrict__ in, bf16_t* __restrict__ out, const Args& a,
                                        int gx0, int gy0, int W, const float* sq, const bf16_t* wl_next,
                                        bf16x8 (&wn)[9][NHN > 0 ? NHN : 1])
{
    // slots q = PI y + x of the input's pitch; the last group may pass the
    // last row (those slots, like the columns x >= SO, are not stored)
    constexpr int NG = (SO * PI + 15) / 16, KMAX = (NG + NW - 1) / NW;
    static_assert(PI == SO + 2, "the input is the previous layer's compact output");
    static_assert(16 * NG + 2 * PI + 2 <= (SO + 2) * PI + PAD, "reads stay inside the input buffer");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, lg = lane >> 4;
    const int K = (NG - wave + NW - 1) / NW;  // groups of this wave
    f32x4 bb[NH];
#pragma unroll
    for (int nh = 0; nh < NH; ++nh) bb[nh] = *reinterpret_cast<const f32x4*>(bias + nh * 16 + 4 * lg);
    // per-tap input offsets of this lane, relative to the group's first slot
    int kt[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) kt[t] = chunk_at(l16 + (PI + 1) + (t / 3 - 1) * PI + (t % 3 - 1), lg);
    auto load = [&](int g, bf16x8(&x)[9]) {
#pragma unroll
        for (int t = 0; t < 9; ++t) x[t] = lds8(in + g * 16 * SLOT + kt[t]);
    };
    // products and epilogue of group g
    auto group = [&](int g, const bf16x8(&x)[9]) {
        const int q = 16 * g + l16, y = q / PI, xq = q - y * PI;
        if constexpr (!LAST) {
            // the accumulators start from the bias, so acc = conv + b
            f32x4 acc[NH];
#pragma unroll
            for (int nh = 0; nh < NH; ++nh) acc[nh] = bb[nh];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
#pragma unroll
                for (int nh = 0; nh < NH; ++nh)
                    acc[nh] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t][nh], x[t], acc[nh], 0, 0, 0);
            }
            // compact output: slot SO y + x, the pitch of the next layer's input
            if (xq < SO && y < SO) {
                const int so = SO * y + xq;
#pragma unroll
                for (int nh = 0; nh < NH; ++nh)
                    *reinterpret_cast<uint2*>(out + chunk_at(so, 2 * nh + (lg >> 1)) + 4 * (lg & 1)) = relu4(acc[nh]);
            }
        } else {
            static_assert(NH == 1 && NHN == 0, "one block of output channels in the last layer");
            // two independent chains (taps 0..4 from the bias, taps 5..8 from 0)
            f32x4 c0 = bb[0], c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 5; ++t) {
                c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t][0], x[t], c0, 0, 0, 0);
                if (t + 5 < 9) c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t + 5][0], x[t + 5], c1, 0, 0, 0);
            }
            if (lg == 0 && xq < T && y < T) {
                const size_t o = (size_t)(gy0 + y) * W + (gx0 + xq);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    // the uncorrected state: from LDS when the kernel ran the step itself
                    const float v = SQ ? sq[c * T * T + y * T + xq] : a.qi[c][o];
                    a.qo[c][o] = a.d[c] != 0.f ? fmaf(a.d[c], c0[c] + c1[c], v) : v;
                }
            }
        }
    };
    bf16x8 xb[2][9];
    load(wave, xb[0]);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k < K) {
            // all loads of the next group are issued before this group's products
            if (k + 1 < KMAX && k + 1 < K) load(wave + (k + 1) * NW, xb[(k + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
            group(wave + k * NW, xb[k & 1]);
        }
    }
    if constexpr (NHN > 0) load_weights<NHN>(wl_next, wn);
}

// Layer 0 on one group of 16 output slots (all inside the 24-wide output):
// staged input (side SI, 4 halfwords per node: 3 channels and a zero) ->
// slots of buffer A.  Lane group lg holds k = 8 lg .. 8 lg + 7, i.e. taps
// 2 lg and 2 lg + 1 with their four halfwords, two 8-byte loads; tap 8 is a
// second product (below).
// Tap 8 is a second K = 32 product whose weights are zero outside elements
// 0..3 of lane group 0: a chain of v_mfma_f32_16x16x16_bf16 and
// v_mfma_f32_16x16x32_bf16 on one accumulator issued back to back gives
// wrong accumulators on gfx950 (measured; the compiler inserts no wait
// states between them), while same-instruction chains are forwarded.
struct Layer0 {
    bf16x8 wa0, wa1, wc0, wc1;
    f32x4 bb0, bb1;
    int offa, offb, l16, lg;
    __device__ __forceinline__ f32x4 mfma(const bf16x8& w, const bf16x8& wc, const bf16x8& x, const bf16x8& x8,
                                          const f32x4& b) const
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x, __builtin_amdgcn_mfma_f32_16x16x32_bf16(wc, x8, b, 0, 0, 0),
                                                       0, 0, 0);
    }
};

// STEP: the kernel first runs the SMAME step itself (fully periodic grids):
// it stages the state before the step on the (SI + 4)^2 region in the space
// of buffer A, forms drho' on the (SI + 2)^2 ring, and the momentum update on
// the SI^2 input region of layer 0, with the same per-node functions as the
// step kernels (tile2d.h), so the result equals a step launch followed by
// the correction launch bit for bit.  The tile's own uncorrected values stay
// in LDS for the epilogue.
constexpr int RS = SI + 4, NRS = RS * RS;  // staged state region (30^2)
constexpr int DS = SI + 2, NDS = DS * DS;  // drho' region (28^2)
static_assert((3 * NRS + NDS) * 4 <= BA * 2, "step staging fits in buffer A");
constexpr int SQ_HALF = 3 * T * T * 2;     // centre values, FP32, in halfwords

// One workgroup per CU (LDS), i.e. two waves per SIMD: up to 256 VGPRs a lane.
template <bool STEP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 2))) void cnn_fused_kernel(
    int H, int W, Args a, Coef<float> cf, State<float> qs)
{
    __shared__ __align__(16) bf16_t lds[LDS_HALF + (STEP ? SQ_HALF : 0)];
    // biases of the five layers, then the per-row force of the SI input rows
    __shared__ __align__(16) float sbf[NBIAS + 32];
    bf16_t* const sw = lds;
    bf16_t* const sa = lds + WTOT;
    bf16_t* const sb = sa + BA;
    float* const sfx = sbf + NBIAS;
    const int tiles_x = W / T;
    // each XCD takes a contiguous run of tiles, so most halo nodes were written through its own L2
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int gx0 = (lb % tiles_x) * T, gy0 = (lb / tiles_x) * T;
    const int tid = threadIdx.x;

    // ---- staging.  Loads in the order they are needed: the input region
    // (the state), the force rows, the biases and the layer-0 im2col weights,
    // then the weights of layers 1..4 (straight copies).  The latter stay in
    // registers until layer 0 has been computed, so their latency hides
    // behind the step and layer 0.
    constexpr int NI = SI * SI;
    constexpr int NQ = STEP ? NRS : NI, IQ = (NQ + NT - 1) / NT;
    constexpr int QS = STEP ? RS : SI, QH = STEP ? 7 : 5;  // staged side and halo
    const float* const q0p = STEP ? qs.r : a.qi[0];
    const float* const q1p = STEP ? qs.u : a.qi[1];
    const float* const q2p = STEP ? qs.v : a.qi[2];
    float q0[IQ], q1[IQ], q2[IQ];
#pragma unroll
    for (int i = 0; i < IQ; ++i) {
        const int e = min(tid + i * NT, NQ - 1);
        const int r = e / QS, c = e - r * QS;
        const size_t src = (size_t)wrap(gy0 - QH + r, H) * W + wrap(gx0 - QH + c, W);
        q0[i] = q0p[src];
        q1[i] = q1p[src];
        q2[i] = q2p[src];
    }
    const int fr = tid - NBIAS;  // force row handled by this thread
    float fv = 0.f;
    if (STEP && cf.fx && fr >= 0 && fr < SI) fv = cf.fx[wrap(gy0 - 5 + fr, H)];
    float bv = 0.f;
    if (tid < NBIAS) {
        // per-lane layer index: select the pointer instead of indexing the argument array
        const int l = tid >> 5;
        const float* bp = l == 0 ? a.b[0] : l == 1 ? a.b[1] : l == 2 ? a.b[2] : l == 3 ? a.b[3] : a.b[4];
        bv = bp[tid - 32 * l];
    }
    constexpr int I0 = (W0 + NT - 1) / NT;  // layer-0 entries per thread
    bf16_t w0v[I0];
#pragma unroll
    for (int i = 0; i < I0; ++i) {
        const int e = tid + i * NT;
        // taps 0..7: [o][4 t + c]; tap 8: [o][c]; c = 3 is the zero padding
        const int o = e < W0A ? e >> 5 : (e - W0A) >> 2;
        const int t = e < W0A ? (e & 31) >> 2 : 8, c = e & 3;
        w0v[i] = e < W0 && c < 3 ? a.w[0][(t * 32 + o) * 16 + c] : bf16_t(0);
    }
    // layers 1..4 are contiguous in LDS: chunk e (16 bytes) of that span
    // comes from layer 1 + e / NV; thread tid moves chunks tid + j NT.  The
    // chunks are named values, not an array, so that they stay in registers
    // across the loops in between.
    constexpr int NV = WL / 8, NVT = (3 * WL + W4) / 8;  // 16-byte chunks per layer 1..3, in total
    static_assert(NVT <= 8 * NT && NVT > 7 * NT, "eight chunks per thread");
    auto wchunk = [&](int j) {
        const int e = min(tid + j * NT, NVT - 1), l = e / NV;
        const bf16_t* src = l == 0 ? a.w[1] : l == 1 ? a.w[2] : l == 2 ? a.w[3] : a.w[4];
        return reinterpret_cast<const uint4*>(src)[e - l * NV];
    };
    const uint4 wc0 = wchunk(0), wc1 = wchunk(1), wc2 = wchunk(2), wc3 = wchunk(3);
    const uint4 wc4 = wchunk(4), wc5 = wchunk(5), wc6 = wchunk(6), wc7 = wchunk(7);
#pragma unroll
    for (int i = 0; i < I0; ++i) {
        const int e = tid + i * NT;
        if (e < W0A)
            sw[chunk_at(e >> 5, (e & 31) >> 3) + (e & 7)] = w0v[i];
        else if (e < W0)
            sw[e] = w0v[i];
    }
    if (tid < NBIAS) sbf[tid] = bv;
    if (STEP && fr >= 0 && fr < SI) sfx[fr] = fv;
    if constexpr (STEP) {
        float* const sr = reinterpret_cast<float*>(sa);
        float* const su = sr + NRS;
        float* const sv = su + NRS;
        float* const srn = sv + NRS;
        float* const sq = reinterpret_cast<float*>(lds + LDS_HALF);
#pragma unroll
        for (int i = 0; i < IQ; ++i) {
            const int e = tid + i * NT;
            if (e < NRS) {
                sr[e] = q0[i];
                su[e] = q1[i];
                sv[e] = q2[i];
            }
        }
        __syncthreads();
        // nodes tid and tid + NT.  Waves with a second node compute both in
        // straight-line code (the second at a clamped index, stored only when
        // inside the region) so their LDS reads overlap; the others one.
        static_assert(NDS <= 2 * NT && NI <= 2 * NT, "two nodes per thread");
        const int wave = tid >> 6;
        {
            auto node = [&](int q) {
                q = min(q, NDS - 1);
                const int ly = q / DS, lx = q - ly * DS;
                return rho_new_2d<float, RS>(cf, sr, su, sv, (ly + 1) * RS + (lx + 1));
            };
            if (64 * wave + NT < NDS) {
                const float r0 = node(tid), r1 = node(tid + NT);
                srn[tid] = r0;
                if (tid + NT < NDS) srn[tid + NT] = r1;
            } else {
                srn[tid] = node(tid);
            }
        }
        __syncthreads();
        // the force of input row ly from LDS (same values as the step kernels read)
        Coef<float> cl = cf;
        if (cf.fx) cl.fx = sfx;
        float rn[2], un[2], vn[2];
        auto mnode = [&](int q, int i) {
            q = min(q, NI - 1);
            const int ly = q / SI, lx = q - ly * SI;
            momentum_node2d<float, RS, DS>(cl, sr, su, sv, srn, (ly + 2) * RS + (lx + 2), (ly + 1) * DS + (lx + 1),
                                           ly, rn[i], un[i], vn[i]);
        };
        const bool two = 64 * wave + NT < NI;  // wave-uniform
        if (two) {
            mnode(tid, 0);
            mnode(tid + NT, 1);
        } else {
            mnode(tid, 0);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int q = tid + i * NT;
            if (q < NI && (i == 0 || two)) {
                const int ly = q / SI, lx = q - ly * SI;
                *reinterpret_cast<uint2*>(sb + 4 * q) = pack4(rn[i] * a.s[0], un[i] * a.s[1], vn[i] * a.s[2], 0.f);
                const int cy = ly - 5, cx = lx - 5;
                if (cy >= 0 && cy < T && cx >= 0 && cx < T) {
                    sq[cy * T + cx] = rn[i];
                    sq[T * T + cy * T + cx] = un[i];
                    sq[2 * T * T + cy * T + cx] = vn[i];
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < IQ; ++i) {
            const int e = tid + i * NT;
            if (e < NI)
                *reinterpret_cast<uint2*>(sb + 4 * e) = pack4(q0[i] * a.s[0], q1[i] * a.s[1], q2[i] * a.s[2], 0.f);
        }
    }
    __syncthreads();

    // ---- layer 0: staged input (buffer B) -> buffer A, 36 groups
    {
        constexpr int NG = P * P / 16;
        static_assert(P * P % 16 == 0, "layer 0 has whole groups");
        const int lane = tid & 63, wave = tid >> 6;
        Layer0 L;
        L.l16 = lane & 15;
        L.lg = lane >> 4;
        const int ta = 2 * L.lg, tb = 2 * L.lg + 1;
        L.offa = ((ta / 3 - 1) * SI + (ta % 3 - 1)) * 4;
        L.offb = ((tb / 3 - 1) * SI + (tb % 3 - 1)) * 4;
        constexpr int off8 = (SI + 1) * 4;
        L.wa0 = lds8(sw + chunk_at(L.l16, L.lg));
        L.wa1 = lds8(sw + chunk_at(16 + L.l16, L.lg));
        // tap-8 weights: elements 0..3 of lane group 0 (channels 0..2 and the zero pad), zero elsewhere
        auto w8 = [&](int o) {
            const uint2 h = *reinterpret_cast<const uint2*>(sw + W0A + o * 4);
            return __builtin_bit_cast(bf16x8, L.lg == 0 ? uint4{h.x, h.y, 0u, 0u} : uint4{0u, 0u, 0u, 0u});
        };
        L.wc0 = w8(L.l16);
        L.wc1 = w8(16 + L.l16);
        L.bb0 = *reinterpret_cast<const f32x4*>(sbf + 4 * L.lg);
        L.bb1 = *reinterpret_cast<const f32x4*>(sbf + 16 + 4 * L.lg);
        const int so0 = store_off(L.l16, L.lg, 0), so1 = store_off(L.l16, L.lg, 1);
        auto input = [&](int g, bf16x8& x, bf16x8& x8) {
            const int p = 16 * g + L.l16, py = p / P, px = p - py * P;
            const int base = ((py + 1) * SI + (px + 1)) * 4;
            const uint2 xa = *reinterpret_cast<const uint2*>(sb + base + L.offa);
            const uint2 xb = *reinterpret_cast<const uint2*>(sb + base + L.offb);
            const uint2 xc = *reinterpret_cast<const uint2*>(sb + base + off8);
            x = __builtin_bit_cast(bf16x8, uint4{xa.x, xa.y, xb.x, xb.y});
            x8 = __builtin_bit_cast(bf16x8, uint4{xc.x, xc.y, xc.x, xc.y});  // elements 4..7 meet zero weights
        };
        // the wave's groups (wave, wave + NW, ...) in pairs: the operands of
        // the next pair are loaded before the products of this one, and the
        // weight stores of layers 1..4 go between the first loads and the
        // first products (LDS is idle otherwise)
        constexpr int KMAX = (NG + NW - 1) / NW, PM = (KMAX + 1) / 2;
        const int K = (NG - wave + NW - 1) / NW;
        bf16x8 x[2][2], y[2][2];
        auto in_pair = [&](int pr, int buf) {
            input(wave + 2 * pr * NW, x[buf][0], y[buf][0]);
            if (2 * pr + 1 < K) input(wave + (2 * pr + 1) * NW, x[buf][1], y[buf][1]);
        };
        in_pair(0, 0);
        {
            // weights of layers 1..4, chunk e of row e / 4 at its swizzled place
            uint4* const d = reinterpret_cast<uint4*>(sw + OW1);
            auto put = [&](int j, const uint4& v) {
                const int e = tid + j * NT;
                if (e < NVT) d[(e & ~3) | ((e & 3) ^ ((e >> 3) & 3))] = v;
            };
            put(0, wc0);
            put(1, wc1);
            put(2, wc2);
            put(3, wc3);
            put(4, wc4);
            put(5, wc5);
            put(6, wc6);
            put(7, wc7);
        }
#pragma unroll
        for (int pr = 0; pr < PM; ++pr) {
            if (2 * pr < K) {
                const int bf = pr & 1;
                if (pr + 1 < PM && 2 * (pr + 1) < K) in_pair(pr + 1, bf ^ 1);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (2 * pr + h < K) {
                        const int g = wave + (2 * pr + h) * NW;
                        const f32x4 c0 = L.mfma(L.wa0, L.wc0, x[bf][h], y[bf][h], L.bb0);
                        const f32x4 c1 = L.mfma(L.wa1, L.wc1, x[bf][h], y[bf][h], L.bb1);
                        *reinterpret_cast<uint2*>(sa + g * 16 * SLOT + so0) = relu4(c0);
                        *reinterpret_cast<uint2*>(sa + g * 16 * SLOT + so1) = relu4(c1);
                    }
                }
            }
        }
    }
    __syncthreads();
    const float* const sq = reinterpret_cast<const float*>(lds + LDS_HALF);
    bf16x8 w1[9][2], w2[9][2], w3[9][2], w4[9][1], wnone[9][1];
    load_weights<2>(sw + OW1, w1);
    layer32<P - 2, P, 2, false, false, 2>(w1, sbf + 32, sa, sb, a, gx0, gy0, W, sq, sw + OW2, w2);
    __syncthreads();
    layer32<P - 4, P - 2, 2, false, false, 2>(w2, sbf + 64, sb, sa, a, gx0, gy0, W, sq, sw + OW3, w3);
    __syncthreads();
    layer32<P - 6, P - 4, 2, false, false, 1>(w3, sbf + 96, sa, sb, a, gx0, gy0, W, sq, sw + OW4, w4);
    __syncthreads();
    // last layer: output width 16 = the tile; (gx0, gy0) is its origin
    layer32<T, P - 6, 1, true, STEP, 0>(w4, sbf + 128, sb, nullptr, a, gx0, gy0, W, sq, nullptr, wnone);
}
}  // namespace fused

hipError_t launch_fused(int H, int W, const fused::Args& a, hipStream_t s)
{
    if (H % fused::T || W % fused::T) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fused::cnn_fused_kernel<false>, dim3((W / fused::T) * (H / fused::T)), dim3(fused::NT), 0, s,
                       H, W, a, Coef<float>{}, State<float>{});
    return hipGetLastError();
}

// SMAME step of the state qs and the correction in one launch (fully
// periodic grids); a.qi is not read.
hipError_t launch_fused_step(int H, int W, const fused::Args& a, const Coef<float>& c, const State<float>& qs,
                             hipStream_t s)
{
    if (H % fused::T || W % fused::T || c.nonperiodic) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fused::cnn_fused_kernel<true>, dim3((W / fused::T) * (H / fused::T)), dim3(fused::NT), 0, s,
                       H, W, a, c, qs);
    return hipGetLastError();
}

}  // namespace acm

using namespace acm;

namespace acm {
void set_error(const std::string& msg);
acm_status api_validate(const acm_config* c, std::string& err);
double api_max_amplification(const acm_config& c);
template <typename T>
Coef<T> api_make_coef(const acm_config& c, const void* force_x);
}  // namespace acm

namespace {
acm_status cfail(acm_status s, const std::string& m)
{
    set_error(m);
    return s;
}
acm_status chip(hipError_t e, const char* what)
{
    if (e == hipSuccess) return ACM_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorInvalidValue ? ACM_EINVAL : ACM_EHIP;
}
bool grid_ok(int nx, int ny) { return nx > 0 && ny > 0 && nx % 64 == 0 && ny % 8 == 0; }
// per-pixel kernels index pixels with int
bool pixels_ok(int nx, int ny) { return nx > 0 && ny > 0 && (int64_t)nx * ny <= INT32_MAX - 256; }
int blocks_for(size_t n) { return (int)((n + 255) / 256); }
}  // namespace

// Device scratch of acm_cnn_loss_noalloc: the per-workgroup partial sums of
// the loss, one double per 256 pixels.  Each GPU holds its own copy for the
// life of the process.  In host code `scratch` names a host-side stand-in,
// not device memory: kernels get the address that hipGetSymbolAddress
// returns for the current device, taken once per device.
static __device__ __align__(256) double scratch[ACM_LOSS_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[MAX_DEVICES] = {};

acm_status static_scratch_ptr(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return chip(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return cfail(ACM_EINVAL, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return chip(e, "hipGetSymbolAddress(scratch)");
        if (!p) return cfail(ACM_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return ACM_OK;
}
}  // namespace

extern "C" {

acm_status acm_cnn_layer_shape(int32_t layer, int32_t* cin, int32_t* cout)
{
    static const int ci[ACM_CNN_LAYERS] = {16, 32, 32, 32, 32};
    static const int co[ACM_CNN_LAYERS] = {32, 32, 32, 32, 16};
    if (layer < 0 || layer >= ACM_CNN_LAYERS) return cfail(ACM_EINVAL, "layer out of range");
    if (cin) *cin = ci[layer];
    if (cout) *cout = co[layer];
    return ACM_OK;
}

acm_status acm_cnn_conv(int32_t nx, int32_t ny, int32_t cin, int32_t cout, int32_t mode, const void* x, const void* w,
                        const float* bias, const void* mask, void* y, void* stream)
{
    if (!grid_ok(nx, ny)) return cfail(ACM_EINVAL, "network grids need nx % 64 == 0 and ny % 8 == 0");
    if (!x || !w || !y || (mode != CONV_MASK && !bias) || (mode == CONV_MASK && !mask))
        return cfail(ACM_EINVAL, "NULL pointer");
    return chip(conv_dispatch(ny, nx, cin, cout, mode, x, w, bias, mask, y, static_cast<hipStream_t>(stream)),
                "unsupported (cin, cout, mode) or launch failure");
}

size_t acm_cnn_wgrad_workspace(int32_t nx, int32_t ny, int32_t cin, int32_t cout)
{
    if (!grid_ok(nx, ny)) return 0;
    const size_t nblk = (size_t)(nx / WG_TC) * (ny / WG_TR);
    return nblk * (size_t)(9 * cout * cin + cout) * sizeof(float);
}

static acm_status wgrad_impl(int32_t nx, int32_t ny, int32_t cin, int32_t cout, const void* x, const void* g,
                             float* workspace, float* dw, float* db, void* stream, int acc)
{
    if (!grid_ok(nx, ny)) return cfail(ACM_EINVAL, "network grids need nx % 64 == 0 and ny % 8 == 0");
    if (!x || !g || !workspace || !dw || !db) return cfail(ACM_EINVAL, "NULL pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nblk = (nx / WG_TC) * (ny / WG_TR);
    const bf16_t* xx = static_cast<const bf16_t*>(x);
    const bf16_t* gg = static_cast<const bf16_t*>(g);
    if (cin == 16 && cout == 32)
        hipLaunchKernelGGL((conv_wgrad_kernel<16, 32>), dim3(nblk), dim3(256), 0, s, ny, nx, xx, gg, workspace);
    else if (cin == 32 && cout == 32)
        hipLaunchKernelGGL((conv_wgrad_kernel<32, 32>), dim3(nblk), dim3(256), 0, s, ny, nx, xx, gg, workspace);
    else if (cin == 32 && cout == 16)
        hipLaunchKernelGGL((conv_wgrad_kernel<32, 16>), dim3(nblk), dim3(256), 0, s, ny, nx, xx, gg, workspace);
    else
        return cfail(ACM_EINVAL, "unsupported (cin, cout)");
    acm_status st = chip(hipGetLastError(), "wgrad launch");
    if (st != ACM_OK) return st;
    const int n = 9 * cout * cin + cout;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((n + 63) / 64), dim3(64 * RP_SEG), 0, s, workspace, nblk, n, dw,
                       db, 9 * cout * cin, acc);
    return chip(hipGetLastError(), "reduce launch");
}

acm_status acm_cnn_wgrad(int32_t nx, int32_t ny, int32_t cin, int32_t cout, const void* x, const void* g,
                         float* workspace, float* dw, float* db, void* stream)
{
    return wgrad_impl(nx, ny, cin, cout, x, g, workspace, dw, db, stream, 0);
}

acm_status acm_cnn_wgrad_add(int32_t nx, int32_t ny, int32_t cin, int32_t cout, const void* x, const void* g,
                             float* workspace, float* dw, float* db, void* stream)
{
    return wgrad_impl(nx, ny, cin, cout, x, g, workspace, dw, db, stream, 1);
}

acm_status acm_cnn_transpose(int32_t cin, int32_t cout, const void* w, void* wt, void* stream)
{
    if (!w || !wt || cin <= 0 || cout <= 0) return cfail(ACM_EINVAL, "bad transpose arguments");
    hipLaunchKernelGGL(transpose_weights_kernel, dim3(blocks_for((size_t)9 * cin * cout)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), cin, cout, static_cast<const bf16_t*>(w),
                       static_cast<bf16_t*>(wt));
    return chip(hipGetLastError(), "transpose launch");
}

acm_status acm_cnn_pack(int32_t nx, int32_t ny, const float* drho, const float* u, const float* v,
                        const float* in_scale, void* a0, void* stream)
{
    if (!drho || !u || !v || !in_scale || !a0 || !pixels_ok(nx, ny)) return cfail(ACM_EINVAL, "bad pack arguments");
    const int n = nx * ny;
    hipLaunchKernelGGL(pack_input_kernel, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, drho,
                       u, v, in_scale[0], in_scale[1], in_scale[2], static_cast<bf16_t*>(a0));
    return chip(hipGetLastError(), "pack launch");
}

acm_status acm_cnn_apply(int32_t nx, int32_t ny, const float* raw, const float* out_scale, float* drho, float* u,
                         float* v, void* stream)
{
    if (!raw || !out_scale || !drho || !u || !v || !pixels_ok(nx, ny)) return cfail(ACM_EINVAL, "bad apply arguments");
    const int n = nx * ny;
    hipLaunchKernelGGL(apply_correction_kernel, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       n, raw, out_scale[0], out_scale[1], out_scale[2], drho, u, v);
    return chip(hipGetLastError(), "apply launch");
}

size_t acm_cnn_loss_workspace(int32_t nx, int32_t ny) { return (size_t)blocks_for((size_t)nx * ny) * sizeof(double); }

static acm_status loss_impl(int32_t nx, int32_t ny, const float* raw, const float* const* base,
                            const float* const* target, const float* out_scale, void* grad, double* workspace,
                            double* loss, void* stream)
{
    const int n = nx * ny;
    const int nb = blocks_for(n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    LossChannels lc{};
    for (int c = 0; c < 3; ++c) {
        if (!(out_scale[c] >= 0.f) || !std::isfinite(out_scale[c])) return cfail(ACM_EINVAL, "out_scale must be >= 0");
        lc.w[c] = out_scale[c] > 0.f ? 1.f : 0.f;
        lc.id[c] = out_scale[c] > 0.f ? 1.f / out_scale[c] : 0.f;
        lc.nact += out_scale[c] > 0.f;
    }
    if (lc.nact == 0) return cfail(ACM_EINVAL, "every output channel is excluded");
    hipLaunchKernelGGL(loss_grad_kernel, dim3(nb), dim3(256), 0, s, n, raw, base[0], base[1], base[2], target[0],
                       target[1], target[2], lc, static_cast<bf16_t*>(grad), workspace);
    acm_status st = chip(hipGetLastError(), "loss launch");
    if (st != ACM_OK) return st;
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, s, workspace, nb, (double)lc.nact * n, loss);
    return chip(hipGetLastError(), "loss final launch");
}

acm_status acm_cnn_loss(int32_t nx, int32_t ny, const float* raw, const float* const* base, const float* const* target,
                        const float* out_scale, void* grad, double* workspace, double* loss, void* stream)
{
    if (!raw || !base || !target || !out_scale || !grad || !workspace || !loss) return cfail(ACM_EINVAL, "NULL pointer");
    if (!pixels_ok(nx, ny)) return cfail(ACM_EINVAL, "bad grid");
    return loss_impl(nx, ny, raw, base, target, out_scale, grad, workspace, loss, stream);
}

acm_status acm_cnn_loss_noalloc(int32_t nx, int32_t ny, const float* raw, const float* const* base,
                                const float* const* target, const float* out_scale, void* grad, double* loss,
                                void* stream)
{
    if (!raw || !base || !target || !out_scale || !grad || !loss) return cfail(ACM_EINVAL, "NULL pointer");
    if (!pixels_ok(nx, ny)) return cfail(ACM_EINVAL, "bad grid");
    if ((size_t)blocks_for((size_t)nx * ny) > ACM_LOSS_SCRATCH_DOUBLES)
        return cfail(ACM_EINVAL, "grid of " + std::to_string((long long)nx * ny) +
                                     " pixels exceeds the static scratch (at most " +
                                     std::to_string((long long)ACM_LOSS_SCRATCH_DOUBLES * 256) + " pixels)");
    double* ws = nullptr;
    const acm_status st = static_scratch_ptr(&ws);
    if (st != ACM_OK) return st;
    return loss_impl(nx, ny, raw, base, target, out_scale, grad, ws, loss, stream);
}

acm_status acm_cnn_state_loss(int32_t nx, int32_t ny, const float* const* q, const float* const* target,
                              const float* out_scale, float weight, float* const* adj, double* workspace,
                              double* loss, void* stream)
{
    if (!q || !target || !out_scale || !adj || !workspace || !loss) return cfail(ACM_EINVAL, "NULL pointer");
    if (!pixels_ok(nx, ny)) return cfail(ACM_EINVAL, "bad grid");
    for (int c = 0; c < 3; ++c)
        if (!q[c] || !target[c] || !adj[c]) return cfail(ACM_EINVAL, "NULL field");
    if (!std::isfinite(weight)) return cfail(ACM_EINVAL, "weight must be finite");
    LossChannels lc{};
    for (int c = 0; c < 3; ++c) {
        if (!(out_scale[c] >= 0.f) || !std::isfinite(out_scale[c])) return cfail(ACM_EINVAL, "out_scale must be >= 0");
        lc.w[c] = out_scale[c] > 0.f ? 1.f : 0.f;
        lc.id[c] = out_scale[c] > 0.f ? 1.f / out_scale[c] : 0.f;
        lc.nact += out_scale[c] > 0.f;
    }
    if (lc.nact == 0) return cfail(ACM_EINVAL, "every output channel is excluded");
    const int n = nx * ny;
    const int nb = blocks_for(n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float k = 2.f * weight / ((float)lc.nact * (float)n);
    hipLaunchKernelGGL(state_loss_kernel, dim3(nb), dim3(256), 0, s, n, q[0], q[1], q[2], target[0], target[1],
                       target[2], lc, k, adj[0], adj[1], adj[2], workspace);
    acm_status st = chip(hipGetLastError(), "state loss launch");
    if (st != ACM_OK) return st;
    hipLaunchKernelGGL(loss_accumulate_kernel, dim3(1), dim3(64), 0, s, workspace, nb,
                       (double)weight / ((double)lc.nact * n), loss);
    return chip(hipGetLastError(), "state loss final launch");
}

acm_status acm_cnn_div_penalty(int32_t nx, int32_t ny, const float* const* a, const float* const* b, float weight,
                               float* const* adj_a, float* const* adj_b, double* workspace, double* loss,
                               void* stream)
{
    if (!a || !b || !adj_a || !workspace || !loss) return cfail(ACM_EINVAL, "NULL pointer");
    if (nx < 3 || ny < 3 || !pixels_ok(nx, ny)) return cfail(ACM_EINVAL, "grid needs nx, ny >= 3");
    if (!a[0] || !a[1] || !b[0] || !b[1] || !adj_a[0] || !adj_a[1]) return cfail(ACM_EINVAL, "NULL field");
    if (adj_b && (!adj_b[0] || !adj_b[1])) return cfail(ACM_EINVAL, "NULL field");
    if (!std::isfinite(weight)) return cfail(ACM_EINVAL, "weight must be finite");
    const int n = nx * ny;
    const int nb = blocks_for(n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(div_penalty_kernel, dim3(nb), dim3(256), 0, s, nx, ny, a[0], a[1], b[0], b[1],
                       2.f * weight / (float)n, adj_a[0], adj_a[1], adj_b ? adj_b[0] : nullptr,
                       adj_b ? adj_b[1] : nullptr, workspace);
    acm_status st = chip(hipGetLastError(), "divergence penalty launch");
    if (st != ACM_OK) return st;
    hipLaunchKernelGGL(loss_accumulate_kernel, dim3(1), dim3(64), 0, s, workspace, nb, (double)weight / n, loss);
    return chip(hipGetLastError(), "divergence penalty final launch");
}

acm_status acm_cnn_adam(int64_t n, float* p, const float* g, float* m, float* v, void* p16, float lr, float b1,
                        float b2, float eps, int64_t t, void* stream)
{
    if (n <= 0 || !p || !g || !m || !v || t < 1) return cfail(ACM_EINVAL, "bad Adam arguments");
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for((size_t)n)), dim3(256), 0, static_cast<hipStream_t>(stream), (int)n,
                       p, g, m, v, static_cast<bf16_t*>(p16), lr, b1, b2, eps, c1, c2);
    return chip(hipGetLastError(), "adam launch");
}

acm_status acm_cnn_to_bf16(size_t n, const float* src, void* dst, void* stream)
{
    if (!src || !dst) return cfail(ACM_EINVAL, "NULL pointer");
    if (n == 0) return ACM_OK;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, src,
                       static_cast<bf16_t*>(dst));
    return chip(hipGetLastError(), "to_bf16 launch");
}

acm_status acm_filter_box(int32_t nxf, int32_t nyf, int32_t factor, int32_t precision, const acm_fields* fine,
                          const acm_fields* coarse, void* stream)
{
    if (!fine || !coarse || factor < 1 || nxf % factor || nyf % factor) return cfail(ACM_EINVAL, "bad filter arguments");
    const int nxc = nxf / factor, nyc = nyf / factor;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* const src[3] = {fine->drho, fine->u, fine->v};
    void* const dst[3] = {coarse->drho, coarse->u, coarse->v};
    for (int k = 0; k < 3; ++k) {
        if (!src[k] || !dst[k]) return cfail(ACM_EINVAL, "NULL field");
        if (precision == ACM_F64)
            hipLaunchKernelGGL((box_filter_kernel<double>), dim3(blocks_for((size_t)nxc * nyc)), dim3(256), 0, s, nxc,
                               nyc, factor, static_cast<const double*>(src[k]), static_cast<double*>(dst[k]));
        else
            hipLaunchKernelGGL((box_filter_kernel<float>), dim3(blocks_for((size_t)nxc * nyc)), dim3(256), 0, s, nxc,
                               nyc, factor, static_cast<const float*>(src[k]), static_cast<float*>(dst[k]));
    }
    return chip(hipGetLastError(), "filter launch");
}

acm_status acm_prolong_bilinear(int32_t nxc, int32_t nyc, int32_t factor, int32_t precision, const acm_fields* coarse,
                                const acm_fields* fine, void* stream)
{
    if (!fine || !coarse || factor < 1 || nxc < 1 || nyc < 1) return cfail(ACM_EINVAL, "bad prolongation arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nf = (size_t)nxc * nyc * factor * factor;
    void* const src[3] = {coarse->drho, coarse->u, coarse->v};
    void* const dst[3] = {fine->drho, fine->u, fine->v};
    for (int k = 0; k < 3; ++k) {
        if (!src[k] || !dst[k]) return cfail(ACM_EINVAL, "NULL field");
        if (precision == ACM_F64)
            hipLaunchKernelGGL((prolong_kernel<double>), dim3(blocks_for(nf)), dim3(256), 0, s, nxc, nyc, factor,
                               static_cast<const double*>(src[k]), static_cast<double*>(dst[k]));
        else
            hipLaunchKernelGGL((prolong_kernel<float>), dim3(blocks_for(nf)), dim3(256), 0, s, nxc, nyc, factor,
                               static_cast<const float*>(src[k]), static_cast<float*>(dst[k]));
    }
    return chip(hipGetLastError(), "prolongation launch");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// closure inference: per coarse step, the SMAME step then the network
// correction, captured as HIP graphs of `chunk` steps.
// ---------------------------------------------------------------------------
struct acm_closure {
    acm_config cfg;
    acm_fields set[2];
    const void* force_x = nullptr;
    const void* w[ACM_CNN_LAYERS];
    const float* b[ACM_CNN_LAYERS];
    float in_scale[3], out_scale[3];
    float* tmp[3] = {nullptr, nullptr, nullptr};  // uncorrected state after the coarse step (workspace)
    hipStream_t stream = nullptr, cap = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int chunk = 100;
    int which = 0;
    int64_t step = 0;
    int use_net = 1;
    int two_launch = 0;  // 1: step kernel then correction kernel even on periodic grids
    Coef<float> coef;
};

namespace {

fused::Args fused_args(const acm_closure* h, const float* const* qi, float* const* qo)
{
    fused::Args a;
    for (int c = 0; c < 3; ++c) {
        a.qi[c] = qi[c];
        a.qo[c] = qo[c];
        a.s[c] = h->in_scale[c];
        a.d[c] = h->out_scale[c];
    }
    for (int l = 0; l < ACM_CNN_LAYERS; ++l) {
        a.w[l] = static_cast<const bf16_t*>(h->w[l]);
        a.b[l] = h->b[l];
    }
    return a;
}

// one coarse step: SMAME step into the scratch state, then the network
// correction into the other buffer set (plain step straight into it when
// the network is off)
hipError_t closure_step(acm_closure* h, int from, hipStream_t s)
{
    const acm_fields& in = h->set[from];
    const acm_fields& out = h->set[1 - from];
    const State<float> si{static_cast<float*>(in.drho), static_cast<float*>(in.u), static_cast<float*>(in.v), nullptr,
                          nullptr};
    const State<float> so{static_cast<float*>(out.drho), static_cast<float*>(out.u), static_cast<float*>(out.v),
                          nullptr, nullptr};
    if (!h->use_net) return launch_step2d<float>(h->coef, si, so, h->cfg.tile, s);
    float* const qo[3] = {so.r, so.u, so.v};
    if (!h->coef.nonperiodic && !h->two_launch)  // step and correction in one launch
        return launch_fused_step(h->cfg.ny, h->cfg.nx, fused_args(h, h->tmp, qo), h->coef, si, s);
    const State<float> st{h->tmp[0], h->tmp[1], h->tmp[2], nullptr, nullptr};
    hipError_t e = launch_step2d<float>(h->coef, si, st, h->cfg.tile, s);
    if (e != hipSuccess) return e;
    return launch_fused(h->cfg.ny, h->cfg.nx, fused_args(h, h->tmp, qo), s);
}

}  // namespace

extern "C" {

size_t acm_closure_workspace(int32_t nx, int32_t ny)
{
    if (nx <= 0 || ny <= 0) return 0;
    return (size_t)nx * ny * 3 * sizeof(float);  // the uncorrected state (drho, u, v)
}

acm_status acm_cnn_correct(int32_t nx, int32_t ny, const acm_fields* in, const acm_fields* out,
                           const void* const* weights, const float* const* biases, const float* in_scale,
                           const float* out_scale, void* stream)
{
    if (nx < fused::T || ny < fused::T || nx % fused::T || ny % fused::T)
        return cfail(ACM_EINVAL, "fused inference needs nx and ny multiples of 16");
    if (!in || !out || !weights || !biases || !in_scale || !out_scale) return cfail(ACM_EINVAL, "NULL pointer");
    fused::Args a;
    const void* const qi[3] = {in->drho, in->u, in->v};
    void* const qo[3] = {out->drho, out->u, out->v};
    for (int c = 0; c < 3; ++c) {
        if (!qi[c] || !qo[c]) return cfail(ACM_EINVAL, "NULL field");
        for (int k = 0; k < 3; ++k)
            if (qi[c] == qo[k]) return cfail(ACM_EINVAL, "in and out fields must be distinct");
        a.qi[c] = static_cast<const float*>(qi[c]);
        a.qo[c] = static_cast<float*>(qo[c]);
        a.s[c] = in_scale[c];
        a.d[c] = out_scale[c];
    }
    for (int l = 0; l < ACM_CNN_LAYERS; ++l) {
        if (!weights[l] || !biases[l]) return cfail(ACM_EINVAL, "NULL layer parameters");
        a.w[l] = static_cast<const bf16_t*>(weights[l]);
        a.b[l] = biases[l];
    }
    return chip(launch_fused(ny, nx, a, static_cast<hipStream_t>(stream)), "fused inference launch");
}

acm_status acm_closure_init(const acm_config* cfg, const acm_fields* a, const acm_fields* b, const void* force_x,
                            const void* const* weights, const float* const* biases, const float* in_scale,
                            const float* out_scale, void* workspace, int32_t chunk, void* stream, acm_closure** out)
{
    if (!out) return cfail(ACM_EINVAL, "out is NULL");
    *out = nullptr;
    std::string err;
    if (api_validate(cfg, err) != ACM_OK) return cfail(ACM_EINVAL, err);
    if (cfg->dim != 2 || cfg->two_phase || cfg->axisym || cfg->precision != ACM_F32)
        return cfail(ACM_EINVAL, "the closure runs 2D single-phase planar FP32 coarse grids");
    if (cfg->nx < fused::T || cfg->ny < fused::T || cfg->nx % fused::T || cfg->ny % fused::T)
        return cfail(ACM_EINVAL, "closure grids need nx and ny multiples of 16");
    if (!a || !b || !a->drho || !a->u || !a->v || !b->drho || !b->u || !b->v || !weights || !biases || !in_scale ||
        !out_scale || !workspace)
        return cfail(ACM_EINVAL, "NULL pointer");
    if (chunk < 0 || chunk % 2) return cfail(ACM_EINVAL, "chunk must be even");
    if (!cfg->allow_unstable && api_max_amplification(*cfg) > 1.0 + 1e-12)
        return cfail(ACM_EUNSTABLE, "coarse step fails the linear stability check");
    acm_closure* h = new (std::nothrow) acm_closure();
    if (!h) return cfail(ACM_EINVAL, "out of host memory");
    h->cfg = *cfg;
    h->set[0] = *a;
    h->set[1] = *b;
    h->force_x = force_x;
    for (int l = 0; l < ACM_CNN_LAYERS; ++l) {
        h->w[l] = weights[l];
        h->b[l] = biases[l];
        if (!h->w[l] || !h->b[l]) {
            delete h;
            return cfail(ACM_EINVAL, "NULL layer parameters");
        }
    }
    for (int c = 0; c < 3; ++c) {
        h->in_scale[c] = in_scale[c];
        h->out_scale[c] = out_scale[c];
    }
    const size_t n = (size_t)cfg->nx * cfg->ny;
    for (int c = 0; c < 3; ++c) h->tmp[c] = static_cast<float*>(workspace) + c * n;
    h->chunk = chunk > 0 ? chunk : 100;
    h->stream = static_cast<hipStream_t>(stream);
    h->coef = api_make_coef<float>(*cfg, force_x);
    hipError_t e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete h;
        return chip(e, "stream create");
    }
    *out = h;
    return ACM_OK;
}

acm_status acm_closure_set_network(acm_closure* h, int32_t enabled)
{
    if (!h) return cfail(ACM_EINVAL, "closure is NULL");
    if (enabled < 0 || enabled > 2) return cfail(ACM_EINVAL, "enabled must be 0, 1 or 2");
    const int use_net = enabled ? 1 : 0, two_launch = enabled == 2 ? 1 : 0;
    if (use_net != h->use_net || two_launch != h->two_launch) {  // the captured graphs are stale
        for (int p = 0; p < 2; ++p)
            if (h->exec[p]) {
                (void)hipGraphExecDestroy(h->exec[p]);
                h->exec[p] = nullptr;
            }
    }
    h->use_net = use_net;
    h->two_launch = two_launch;
    return ACM_OK;
}

acm_status acm_closure_run(acm_closure* h, int64_t nsteps)
{
    if (!h || nsteps < 0) return cfail(ACM_EINVAL, "bad closure run arguments");
    while (nsteps >= h->chunk) {
        const int p = h->which;
        if (!h->exec[p]) {
            hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return chip(e, "capture");
            for (int i = 0; i < h->chunk && e == hipSuccess; ++i) e = closure_step(h, (p + i) & 1, h->cap);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(h->cap, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return chip(e != hipSuccess ? e : e2, "closure capture");
            }
            e = hipGraphInstantiate(&h->exec[p], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return chip(e, "closure instantiate");
        }
        acm_status st = chip(hipGraphLaunch(h->exec[p], h->stream), "closure graph launch");
        if (st != ACM_OK) return st;
        h->step += h->chunk;
        nsteps -= h->chunk;
    }
    for (int64_t i = 0; i < nsteps; ++i) {
        acm_status st = chip(closure_step(h, h->which, h->stream), "closure step");
        if (st != ACM_OK) return st;
        h->which ^= 1;
        h->step += 1;
    }
    return ACM_OK;
}

acm_status acm_closure_current(const acm_closure* h, int32_t* which, int64_t* step)
{
    if (!h) return cfail(ACM_EINVAL, "closure is NULL");
    if (which) *which = h->which;
    if (step) *step = h->step;
    return ACM_OK;
}

void acm_closure_destroy(acm_closure* h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (int p = 0; p < 2; ++p)
        if (h->exec[p]) (void)hipGraphExecDestroy(h->exec[p]);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    delete h;
}

}  // extern "C"
