// Batched independent 2D cases in one launch per step.
//
// Every active (case, tile) pair is an item of a device table.  Mode 0
// (default): one workgroup per item slot (the item capacity), slots past the
// active count exit at once, and the hardware dispatcher keeps as many items
// in flight as occupancy allows.  Mode 1: a persistent grid (CUs x occupancy
// workgroups) pops ranges of `grab` items from an atomic counter, one range
// ahead, and loads the next item's fields into registers while it computes
// the current one, so its own load latency overlaps its arithmetic; the tile
// shape is a run-time value there, so one loop serves every case.  The last
// workgroup to finish resets the counter for the next launch.  Both modes
// apply the node updates of the single-case kernel (tile2d.h) to the same
// staged values, so each case's result is bitwise equal to running it
// alone.  A
// chunk of steps is captured once as a HIP graph (the item table and its
// length live in device memory, so the graph survives changes of the active
// set); after each chunk a health kernel reduces max|u| and a non-finite
// flag per case, and the host retires finished or diverged cases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/acm.h"
#include "acm_internal.h"
#include "tile2d.h"

namespace acm {

template <typename T>
struct BatchCaseDev {
    Coef<T> c;
    State<T> s[2];
    int tile;
    int tw, th;          // tile width (a power of two) and height
    unsigned mrx, mdx;   // division by the staged and drho' row strides (div_magic)
};

// tile shapes of the 2D kernels (same numbering as launch_step2d)
constexpr int NTILE2D = 6;
constexpr int TILE_W[NTILE2D] = {64, 32, 64, 16, 128, 32};
constexpr int TILE_H[NTILE2D] = {4, 8, 8, 16, 4, 16};

// q / d == (q * div_magic(d)) >> 20 for every index q of a staged region:
// with m = ceil(2^20 / d) the product overshoots q / d by less than
// q / 2^20 < 1 / d, which never reaches the next integer.  Checked at compile
// time for every tile shape below.
constexpr unsigned div_magic(int d) { return ((1u << 20) + (unsigned)d - 1u) / (unsigned)d; }
constexpr bool div_magic_exact()
{
    for (int t = 0; t < NTILE2D; ++t) {
        const int rx = TILE_W[t] + 4, rxy = rx * (TILE_H[t] + 4), dx = TILE_W[t] + 2;
        for (int q = 0; q < rxy; ++q) {
            if ((int)((q * div_magic(rx)) >> 20) != q / rx) return false;
            if ((int)((q * div_magic(dx)) >> 20) != q / dx) return false;
        }
    }
    return true;
}
static_assert(div_magic_exact(), "row division by multiply and shift");

template <typename T>
constexpr size_t batch_lds_bytes()
{
    size_t m = tile2d_lds_bytes<T, 64, 4>();
    m = std::max(m, tile2d_lds_bytes<T, 32, 8>());
    m = std::max(m, tile2d_lds_bytes<T, 64, 8>());
    m = std::max(m, tile2d_lds_bytes<T, 16, 16>());
    m = std::max(m, tile2d_lds_bytes<T, 128, 4>());
    m = std::max(m, tile2d_lds_bytes<T, 32, 16>());
    return m;
}

// the tile function of one item (the case's tile variant)
template <typename T>
__device__ __forceinline__ void batch_item(const BatchCaseDev<T>& bc, int4 it, int parity, char* smem)
{
    const State<T> in = bc.s[parity], out = bc.s[parity ^ 1];
    switch (bc.tile) {
        case 1: tile2d<T, 32, 8, 256>(bc.c, in, out, it.y * 32, it.z * 8, smem); break;
        case 2: tile2d<T, 64, 8, 256>(bc.c, in, out, it.y * 64, it.z * 8, smem); break;
        case 3: tile2d<T, 16, 16, 256>(bc.c, in, out, it.y * 16, it.z * 16, smem); break;
        case 4: tile2d<T, 128, 4, 256>(bc.c, in, out, it.y * 128, it.z * 4, smem); break;
        case 5: tile2d<T, 32, 16, 256>(bc.c, in, out, it.y * 32, it.z * 16, smem); break;
        default: tile2d<T, 64, 4, 256>(bc.c, in, out, it.y * 64, it.z * 4, smem); break;
    }
}

// ---- mode 1: the tile shape as run-time values --------------------------

// One item's tile; every member is wave-uniform.
struct ItemTile {
    int x0, y0, tx, ty;  // origin and size of the tile
    int rx, rxy;         // staged region: halo 2, row stride rx, rxy values
    int dx, dxy;         // drho' region: halo 1
    unsigned mrx, mdx;
    int interior;        // no node of the staged region is a ghost
};

template <typename T>
__device__ __forceinline__ ItemTile item_tile(const BatchCaseDev<T>& bc, int4 it)
{
    ItemTile g;
    g.tx = bc.tw;
    g.ty = bc.th;
    g.x0 = it.y * g.tx;
    g.y0 = it.z * g.ty;
    g.rx = g.tx + 4;
    g.rxy = g.rx * (g.ty + 4);
    g.dx = g.tx + 2;
    g.dxy = g.dx * (g.ty + 2);
    g.mrx = bc.mrx;
    g.mdx = bc.mdx;
    g.interior = (g.x0 >= 2) && (g.x0 + g.tx + 2 <= bc.c.nx) && (g.y0 >= 2) && (g.y0 + g.ty + 2 <= bc.c.ny);
    return g;
}

// Source node of staged index q, with the wall / symmetry face it crosses
// in x and in y (-1: none), as stage2d maps it.
template <typename T>
__device__ __forceinline__ size_t stage_source(const Coef<T>& c, const ItemTile& g, int q, int& fx, int& fy)
{
    const int ly = (int)(((unsigned)q * g.mrx) >> 20), lx = q - ly * g.rx;
    if (g.interior) {
        fx = fy = -1;
        return (size_t)(g.y0 + ly - 2) * c.nx + (g.x0 + lx - 2);
    }
    const int sx = map_coord(g.x0 + lx - 2, c.nx, c.bc[0], 0, fx);
    const int sy = map_coord(g.y0 + ly - 2, c.ny, c.bc[2], 2, fy);
    return (size_t)sy * c.nx + sx;
}

// A value known to be the same in every lane, held in scalar registers: a
// per-lane choice between such values stays a register select (the
// compiler would otherwise turn a choice between two loads into one vector
// load from a per-lane address, whose wait would also cover the prefetch).
__device__ __forceinline__ float uni(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uni(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The ghost rule u_g = fs u + fo of the crossed x face (0, 1) and y face
// (2, 3), as stage2d applies it.
template <typename T>
struct GhostUV {
    T s[4][2], o[4][2];
};
template <typename T>
__device__ __forceinline__ GhostUV<T> ghost_factors(const Coef<T>& c)
{
    GhostUV<T> h;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            h.s[f][a] = uni(c.fs[f][a]);
            h.o[f][a] = uni(c.fo[f][a]);
        }
    return h;
}
template <typename T>
__device__ __forceinline__ void ghost_uv(const GhostUV<T>& h, int fx, int fy, T& u, T& v)
{
    if (fx >= 0) {
        const int f = fx == 0 ? 0 : 1;
        u = fmaT(f == 0 ? h.s[0][0] : h.s[1][0], u, f == 0 ? h.o[0][0] : h.o[1][0]);
        v = fmaT(f == 0 ? h.s[0][1] : h.s[1][1], v, f == 0 ? h.o[0][1] : h.o[1][1]);
    }
    if (fy >= 0) {
        const int f = fy == 2 ? 2 : 3;
        u = fmaT(f == 2 ? h.s[2][0] : h.s[3][0], u, f == 2 ? h.o[2][0] : h.o[3][0]);
        v = fmaT(f == 2 ? h.s[2][1] : h.s[3][1], v, f == 2 ? h.o[2][1] : h.o[3][1]);
    }
}

// Staged values held in registers between their loads and their LDS
// stores: NPF per thread cover regions of up to 1024 values; the rest (only
// the 128 x 4 tile has more) are loaded when the item is stored.
constexpr int NPF = 4;
template <typename T>
struct ItemRegs {
    T r[NPF], u[NPF], v[NPF];
};

template <typename T>
__device__ __forceinline__ void item_load(const Coef<T>& c, const State<T>& in, const ItemTile& g, ItemRegs<T>& p)
{
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
        if (i * 256 >= g.rxy) break;  // wave-uniform
        const int q = min((int)threadIdx.x + i * 256, g.rxy - 1);
        int fx, fy;
        const size_t s = stage_source(c, g, q, fx, fy);
        p.r[i] = in.r[s];
        p.u[i] = in.u[s];
        p.v[i] = in.v[s];
    }
}

template <typename T>
__device__ __forceinline__ void item_store(const Coef<T>& c, const State<T>& in, const ItemTile& g,
                                           const ItemRegs<T>& p, T* sr, T* su, T* sv)
{
    const GhostUV<T> h = ghost_factors(c);
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
        const int q = threadIdx.x + i * 256;
        if (q < g.rxy) {
            T u = p.u[i], v = p.v[i];
            if (!g.interior) {
                int fx, fy;
                (void)stage_source(c, g, q, fx, fy);
                ghost_uv(h, fx, fy, u, v);
            }
            sr[q] = p.r[i];
            su[q] = u;
            sv[q] = v;
        }
    }
    for (int q = threadIdx.x + NPF * 256; q < g.rxy; q += 256) {
        int fx, fy;
        const size_t s = stage_source(c, g, q, fx, fy);
        const T r = in.r[s];
        T u = in.u[s], v = in.v[s];
        ghost_uv(h, fx, fy, u, v);
        sr[q] = r;
        su[q] = u;
        sv[q] = v;
    }
}

// drho' on the tile plus a one-node ring (as rho_ring2d), then the momentum
// update and stores of the tile's nodes (as momentum2d).
template <typename T>
__device__ __forceinline__ void item_ring(const Coef<T>& c, const ItemTile& g, const T* sr, const T* su,
                                          const T* sv, T* srn)
{
    for (int q = threadIdx.x; q < g.dxy; q += 256) {
        const int ly = (int)(((unsigned)q * g.mdx) >> 20), lx = q - ly * g.dx;
        int ex = lx + 1, ey = ly + 1;
        if (!g.interior && c.nonperiodic) {
            const int gx = mirror_coord(g.x0 + lx - 1, c.nx, c.bc[0]);
            const int gy = mirror_coord(g.y0 + ly - 1, c.ny, c.bc[2]);
            ex = min(max(gx - g.x0 + 2, 1), g.dx);
            ey = min(max(gy - g.y0 + 2, 1), g.ty + 2);
        }
        srn[q] = rho_new_2d_at<T>(c, sr, su, sv, ey * g.rx + ex, g.rx);
    }
}

// Momentum update of the tile's nodes (as momentum2d), at most two per
// thread (every tile has at most 512 nodes).  The results stay in registers
// and are stored during the next item, before that item's successor is
// prefetched: stores count on the same in-order counter as loads, so stores
// issued after the prefetch would make the wait for the prefetched values
// wait for them as well.
constexpr int max_tile_nodes()
{
    int m = 0;
    for (int t = 0; t < NTILE2D; ++t) m = TILE_W[t] * TILE_H[t] > m ? TILE_W[t] * TILE_H[t] : m;
    return m;
}
static_assert(max_tile_nodes() <= 2 * 256, "two nodes per thread");

template <typename T>
struct ItemOut {
    T r[2], u[2], v[2];
    int o[2];  // grid index of the node, -1: none
};

template <typename T>
__device__ __forceinline__ void item_momentum(const Coef<T>& c, const ItemTile& g, const T* sr, const T* su,
                                              const T* sv, const T* srn, ItemOut<T>& res)
{
    const int sh = __builtin_ctz((unsigned)g.tx);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int q = threadIdx.x + i * 256;
        const int ly = q >> sh, lx = q & (g.tx - 1);
        const int gx = g.x0 + lx, gy = g.y0 + ly;
        res.o[i] = -1;
        if (q < g.tx * g.ty && gx < c.nx && gy < c.ny) {
            momentum_node2d_at<T>(c, sr, su, sv, srn, (ly + 2) * g.rx + (lx + 2), (ly + 1) * g.dx + (lx + 1), gy,
                                  g.rx, g.dx, res.r[i], res.u[i], res.v[i]);
            res.o[i] = gy * c.nx + gx;
        }
    }
}

template <typename T>
__device__ __forceinline__ void item_write(const State<T>& out, const ItemOut<T>& res)
{
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        if (res.o[i] >= 0) {
            out.r[res.o[i]] = res.r[i];
            out.u[res.o[i]] = res.u[i];
            out.v[res.o[i]] = res.v[i];
        }
    }
}

// Mode 1: persistent workgroups.  The active items are split into one
// contiguous range per XCD group (workgroup b runs on XCD b mod 8, so
// neighbouring tiles of a case meet in that XCD's L2).  Within its group's
// range a workgroup first takes a fixed share, every Gx-th item from its
// own index (Gx workgroups in the group; the shares cover half the range),
// and then claims the rest `grab` items at a time from the group's counter:
// workgroups of one launch run at unequal speeds (later-dispatched waves
// lose issue priority), which only the claimed half can even out.  A claim is issued one range
// ahead (register `pend` of thread 0) and published through LDS when the
// current range runs out; the next item's fields are loaded into registers
// while the current item computes, and each item's results are stored
// during the item after it.  Counters sit 128 bytes apart
// (QSTRIDE ints); queue[QDONE] counts the workgroups that have left, and the
// last one resets every counter for the next launch.
constexpr int QGROUPS = 8, QSTRIDE = 32, QDONE = QGROUPS * QSTRIDE;
constexpr size_t QUEUE_BYTES = (QDONE + 1) * sizeof(int);

// The case records and the item table do not change during a launch; read
// through the constant address space they stay scalar loads inside the loop
// (through a generic pointer the compiler cannot rule out that this
// launch's stores reach them, and reads them with vector loads whose waits
// would also wait for the prefetched fields).  The host pass, which only
// checks the kernel body, has no such address space.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using ConstCases = const __attribute__((address_space(4))) BatchCaseDev<T>*;
using ConstItems = const __attribute__((address_space(4))) int4*;
#else
template <typename T>
using ConstCases = const BatchCaseDev<T>*;
using ConstItems = const int4*;
#endif

// Registers capped for eight (FP32) or four (FP64) waves per SIMD: at 69
// VGPRs the occupancy query reported seven FP32 workgroups per CU while the
// hardware kept six resident, so a grid sized from the query ran its last
// workgroups as a second round.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 4))) void batch_step_kernel(const BatchCaseDev<T>* __restrict__ cases_g,
                                                          const int4* __restrict__ items_g,
                                                          const int* __restrict__ nitems, int* queue, int parity,
                                                          int grab)
{
    __shared__ __align__(16) char smem[batch_lds_bytes<T>()];
    __shared__ int s_first, s_next;
    const ConstCases<T> cases = (ConstCases<T>)cases_g;
    const ConstItems items = (ConstItems)items_g;
    const int n = *nitems;
    const int tid = threadIdx.x;
    const int G = gridDim.x, b = blockIdx.x;
    const int ng = min(QGROUPS, G), x = b % ng, j = b / ng;
    const int gx = (G - x + ng - 1) / ng;                   // workgroups in group x
    const int lo = (int)((long long)n * x / ng), hi = (int)((long long)n * (x + 1) / ng);
    const int k = (hi - lo) / (2 * gx);                      // fixed share: half the range
    const int tb = lo + k * gx;                              // first claimed item
    int* const qx = queue + x * QSTRIDE;
    int t = lo + j, stride = gx, end = tb;
    int pend = 0;
    if (tid == 0) pend = atomicAdd(qx, grab);
    if (t >= end) {  // no fixed share: take the first claim now
        if (tid == 0) s_first = pend;
        __syncthreads();
        t = tb + __builtin_amdgcn_readfirstlane(s_first);
        stride = 1;
        end = min(t + grab, hi);
        if (t < hi && tid == 0) pend = atomicAdd(qx, grab);
    }
    if (t < end) {
        const BatchCaseDev<T>* bc = cases + items[t].x;
        ItemTile g = item_tile(*bc, items[t]);
        ItemRegs<T> p;
        item_load(bc->c, bc->s[parity], g, p);
        const BatchCaseDev<T>* bcw = bc;  // case of the results held in `res`
        ItemOut<T> res;
        res.o[0] = res.o[1] = -1;
        for (;;) {
            const bool inrange = t + stride < end;
            int tn = t + stride;
            const BatchCaseDev<T>* bcn = bc;
            ItemTile gn = g;
            if (inrange) {  // the next item is known: read its records while this one's values arrive
                const int4 itn = items[tn];
                bcn = cases + itn.x;
                gn = item_tile(*bcn, itn);
            } else if (tid == 0) {
                s_next = pend;
            }
            T* sr = reinterpret_cast<T*>(smem);
            T* su = sr + g.rxy;
            T* sv = su + g.rxy;
            T* srn = sv + g.rxy;
            item_store(bc->c, bc->s[parity], g, p, sr, su, sv);
            __syncthreads();
            if (!inrange) {
                tn = tb + __builtin_amdgcn_readfirstlane(s_next);
                stride = 1;
                end = min(tn + grab, hi);
                if (tn < hi) {
                    if (tid == 0) pend = atomicAdd(qx, grab);
                    const int4 itn = items[tn];
                    bcn = cases + itn.x;
                    gn = item_tile(*bcn, itn);
                }
            }
            const bool more = tn < end;
            item_write(bcw->s[parity ^ 1], res);  // the previous item's results
            if (more)  // the next item's loads are in flight during this item's arithmetic
                item_load(bcn->c, bcn->s[parity], gn, p);
            item_ring(bc->c, g, sr, su, sv, srn);
            __syncthreads();
            item_momentum(bc->c, g, sr, su, sv, srn, res);
            bcw = bc;
            if (!more) break;
            __syncthreads();  // the next item reuses the LDS tile
            t = tn;
            bc = bcn;
            g = gn;
        }
        item_write(bcw->s[parity ^ 1], res);
    }
    if (tid == 0) {
        const int d = atomicAdd(&queue[QDONE], 1);
        if (d == G - 1) {  // every workgroup has left the loop: reset for the next launch
            for (int q = 0; q < QGROUPS; ++q) queue[q * QSTRIDE] = 0;
            queue[QDONE] = 0;
        }
    }
}

// Mode 0: one workgroup per active item; slots past the active count exit.
template <typename T>
__global__ __launch_bounds__(256) void batch_grid_kernel(const BatchCaseDev<T>* __restrict__ cases,
                                                          const int4* __restrict__ items,
                                                          const int* __restrict__ nitems, int parity)
{
    __shared__ __align__(16) char smem[batch_lds_bytes<T>()];
    const int n = *nitems;
    if ((int)blockIdx.x >= n) return;
    // a bijection of the active slots that gives each XCD a contiguous run of
    // items (neighbouring tiles of a case), so their halos meet in its L2
    const int t = xcd_remap(blockIdx.x, n);
    const int4 it = items[t];
    batch_item<T>(cases[it.x], it, parity, smem);
}

// One workgroup per active case: max |u| and a non-finite flag.
template <typename T>
__global__ __launch_bounds__(256) void batch_health_kernel(const BatchCaseDev<T>* __restrict__ cases,
                                                            const int* __restrict__ active, int parity,
                                                            double* health)
{
    const int ci = active[blockIdx.x];
    const BatchCaseDev<T>& bc = cases[ci];
    const State<T> s = bc.s[parity];
    const size_t n = (size_t)bc.c.nx * bc.c.ny;
    double m = 0.0;
    int bad = 0;
    for (size_t i = threadIdx.x; i < n; i += 256) {
        const double u = (double)s.u[i], v = (double)s.v[i], r = (double)s.r[i];
        const double q = u * u + v * v;
        if (!isfinite(q + r)) bad = 1;
        else m = fmax(m, q);
    }
    __shared__ double red[256];
    __shared__ int rbad[256];
    red[threadIdx.x] = m;
    rbad[threadIdx.x] = bad;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
            rbad[threadIdx.x] |= rbad[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        health[2 * ci] = sqrt(red[0]);
        health[2 * ci + 1] = (double)rbad[0];
    }
}

}  // namespace acm

using namespace acm;

// defined in api.hip
namespace acm {
void set_error(const std::string& msg);
acm_status api_validate(const acm_config* c, std::string& err);
double api_max_amplification(const acm_config& c);
template <typename T>
Coef<T> api_make_coef(const acm_config& c, const void* force_x);
}  // namespace acm

namespace {
acm_status bfail(acm_status s, const std::string& m)
{
    set_error(m);
    return s;
}
}  // namespace

struct acm_batch {
    int n = 0;
    int precision = ACM_F32;
    int chunk = 500;
    int blocks = 0;
    int grab = 2;
    int mode = 0;   // 0 one workgroup per item, 1 persistent work queue
    double umax_limit = 0.3;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    // device tables, carved from the caller's scratch (batch_layout)
    void* dcases = nullptr;   // BatchCaseDev<T>[n]
    int4* ditems = nullptr;
    int* dnitems = nullptr;
    int* dqueue = nullptr;
    int* dactive = nullptr;
    double* dhealth = nullptr;
    std::vector<int4> hitems;
    int hnitems = 0;
    std::vector<int> hactive;
    std::vector<double> hhealth;
    size_t max_items = 0;
    std::vector<int> tile, nx, ny, state;
    std::vector<int64_t> nsteps, done;
    std::vector<double> done_ms, umax;
    hipEvent_t ev_start = nullptr, ev_chunk = nullptr;
    bool started = false;
    double elapsed_ms = 0.0;
    int64_t lups = 0;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Items of one case: (tiles in x) * (tiles in y) of its tile variant; for
// tile -1 the largest count over the variants, so the scratch size does not
// depend on the autotuner's choice.
size_t case_items(int nx, int ny, int tile)
{
    size_t m = 0;
    for (int t = 0; t < NTILE2D; ++t) {
        if (tile >= 0 && t != tile) continue;
        m = std::max(m, (size_t)((nx + TILE_W[t] - 1) / TILE_W[t]) * ((ny + TILE_H[t] - 1) / TILE_H[t]));
    }
    return m;
}

// Layout of the batch's device tables in the caller's scratch, each part
// 256-byte aligned: case records, item table, item count, queue counters,
// active list, health pairs.
struct BatchLayout {
    size_t cases, items, nitems, queue, active, health, total;
};

BatchLayout batch_layout(int ncases, size_t max_items, int precision)
{
    const size_t rec = precision == ACM_F64 ? sizeof(BatchCaseDev<double>) : sizeof(BatchCaseDev<float>);
    BatchLayout L{};
    L.cases = 0;
    L.items = L.cases + align256(rec * (size_t)ncases);
    L.nitems = L.items + align256(sizeof(int4) * std::max<size_t>(1, max_items));
    L.queue = L.nitems + 256;
    L.active = L.queue + align256(QUEUE_BYTES);
    L.health = L.active + align256(sizeof(int) * (size_t)ncases);
    L.total = L.health + align256(2 * sizeof(double) * (size_t)ncases);
    return L;
}

template <typename T>
hipError_t upload_cases(acm_batch* b, const acm_batch_case* cases)
{
    std::vector<BatchCaseDev<T>> h(b->n);
    for (int i = 0; i < b->n; ++i) {
        h[i].c = api_make_coef<T>(cases[i].cfg, cases[i].force_x);
        const acm_fields* f[2] = {&cases[i].a, &cases[i].b};
        for (int s = 0; s < 2; ++s)
            h[i].s[s] = State<T>{static_cast<T*>(f[s]->drho), static_cast<T*>(f[s]->u), static_cast<T*>(f[s]->v),
                                 nullptr, nullptr};
        h[i].tile = b->tile[i];
        h[i].tw = TILE_W[b->tile[i]];
        h[i].th = TILE_H[b->tile[i]];
        h[i].mrx = div_magic(TILE_W[b->tile[i]] + 4);
        h[i].mdx = div_magic(TILE_W[b->tile[i]] + 2);
    }
    hipError_t e = hipMemcpyAsync(b->dcases, h.data(), sizeof(BatchCaseDev<T>) * b->n, hipMemcpyHostToDevice,
                                  b->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(b->stream);  // h is released on return
}

template <typename T>
hipError_t launch_batch_step(acm_batch* b, int parity, hipStream_t s)
{
    if (b->mode == 0)
        hipLaunchKernelGGL((batch_grid_kernel<T>), dim3((unsigned)std::max<size_t>(1, b->max_items)), dim3(256), 0,
                           s, static_cast<const BatchCaseDev<T>*>(b->dcases), b->ditems, b->dnitems, parity);
    else
        hipLaunchKernelGGL((batch_step_kernel<T>), dim3(b->blocks), dim3(256), 0, s,
                           static_cast<const BatchCaseDev<T>*>(b->dcases), b->ditems, b->dnitems, b->dqueue,
                           parity, b->grab);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_health(acm_batch* b, int nact, hipStream_t s)
{
    hipLaunchKernelGGL((batch_health_kernel<T>), dim3(nact), dim3(256), 0, s,
                       static_cast<const BatchCaseDev<T>*>(b->dcases), b->dactive, 0, b->dhealth);
    return hipGetLastError();
}

template <typename T>
int occupancy_blocks()
{
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_step_kernel<T>, 256, 0) != hipSuccess) return 0;
    return std::max(1, ncu * std::max(1, per));
}

// Tile variants chosen by the autotuner, per (nx, ny, precision), for the
// life of the process.
std::mutex g_tune_mutex;
std::map<std::tuple<int, int, int, int>, int> g_tune_cache;  // (nx, ny, precision, mode) -> tile

acm_status build_graph(acm_batch* b)
{
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(ACM_EHIP, std::string("capture: ") + hipGetErrorString(e));
    for (int i = 0; i < b->chunk; ++i) {
        e = (b->precision == ACM_F64) ? launch_batch_step<double>(b, i & 1, b->cap)
                                      : launch_batch_step<float>(b, i & 1, b->cap);
        if (e != hipSuccess) break;
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(ACM_EHIP, std::string("batch capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return bfail(ACM_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
    return ACM_OK;
}

}  // namespace

namespace {
acm_status autotune_shape(int nx, int ny, int precision, int copies, int steps, void* scratch, size_t scratch_bytes,
                          void* stream, double* ms_per_tile, int32_t* best, int mode);

bool tuned_tile(int nx, int ny, int precision, int mode, int* tile)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    const auto it = g_tune_cache.find(std::make_tuple(nx, ny, precision, mode));
    if (it == g_tune_cache.end()) return false;
    *tile = it->second;
    return true;
}

// checks shared by acm_batch_scratch_bytes and acm_batch_init
acm_status check_cases(const acm_batch_case* cases, int32_t ncases, const acm_batch_opts* opts, size_t* max_items)
{
    if (!cases || ncases <= 0) return bfail(ACM_EINVAL, "cases / ncases invalid");
    const int prec = cases[0].cfg.precision;
    if (opts && opts->chunk > 0 && opts->chunk % 2) return bfail(ACM_EINVAL, "chunk must be even");
    if (opts && opts->mode != 0 && opts->mode != 1) return bfail(ACM_EINVAL, "mode must be 0 or 1");
    size_t items = 0;
    for (int i = 0; i < ncases; ++i) {
        const acm_batch_case& k = cases[i];
        std::string err;
        if (api_validate(&k.cfg, err) != ACM_OK) return bfail(ACM_EINVAL, "case " + std::to_string(i) + ": " + err);
        if (k.cfg.dim != 2 || k.cfg.two_phase || k.cfg.axisym)
            return bfail(ACM_EINVAL, "batched cases are 2D single-phase planar");
        if (k.cfg.precision != prec) return bfail(ACM_EINVAL, "every case of a batch needs the same precision");
        if (k.tile < -1 || k.tile >= NTILE2D) return bfail(ACM_EINVAL, "tile must be -1..5");
        items += case_items(k.cfg.nx, k.cfg.ny, k.tile);
    }
    if (max_items) *max_items = items;
    return ACM_OK;
}
}

extern "C" {

size_t acm_batch_scratch_bytes(const acm_batch_case* cases, int32_t ncases, const acm_batch_opts* opts)
{
    set_error("");
    size_t items = 0;
    if (check_cases(cases, ncases, opts, &items) != ACM_OK) return 0;
    return batch_layout(ncases, items, cases[0].cfg.precision).total;
}

acm_status acm_batch_tuned_tile(int32_t nx, int32_t ny, int32_t precision, int32_t mode, int32_t* tile)
{
    if (!tile) return bfail(ACM_EINVAL, "tile is NULL");
    int t = 0;
    if (!tuned_tile(nx, ny, precision, mode, &t)) return bfail(ACM_ESTATE, "grid shape not tuned");
    *tile = t;
    return ACM_OK;
}

acm_status acm_batch_set_tuned_tile(int32_t nx, int32_t ny, int32_t precision, int32_t mode, int32_t tile)
{
    if (nx < 4 || ny < 4 || (precision != ACM_F32 && precision != ACM_F64) || (mode != 0 && mode != 1) || tile < 0 ||
        tile >= NTILE2D)
        return bfail(ACM_EINVAL, "set_tuned_tile: bad arguments");
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[std::make_tuple((int)nx, (int)ny, (int)precision, (int)mode)] = tile;
    return ACM_OK;
}

acm_status acm_batch_init(const acm_batch_case* cases, int32_t ncases, const acm_batch_opts* opts, void* scratch,
                          size_t scratch_bytes, void* stream, acm_batch** out)
{
    set_error("");
    if (!out) return bfail(ACM_EINVAL, "out is NULL");
    *out = nullptr;
    size_t items_bound = 0;
    acm_status cst = check_cases(cases, ncases, opts, &items_bound);
    if (cst != ACM_OK) return cst;
    const int prec = cases[0].cfg.precision;
    const int chunk = (opts && opts->chunk > 0) ? opts->chunk : 500;
    const int mode = opts ? opts->mode : 0;
    const BatchLayout L = batch_layout(ncases, items_bound, prec);
    if (!scratch) return bfail(ACM_EINVAL, "scratch is NULL (acm_batch_scratch_bytes gives its size)");
    if (reinterpret_cast<uintptr_t>(scratch) % 256 != 0) return bfail(ACM_EINVAL, "scratch must be 256-byte aligned");
    if (scratch_bytes < L.total)
        return bfail(ACM_EINVAL, "scratch holds " + std::to_string(scratch_bytes) + " bytes, the batch needs " +
                                     std::to_string(L.total));
    for (int i = 0; i < ncases; ++i) {
        const acm_batch_case& k = cases[i];
        if (!k.a.drho || !k.a.u || !k.a.v || !k.b.drho || !k.b.u || !k.b.v)
            return bfail(ACM_EINVAL, "case " + std::to_string(i) + ": missing field pointers");
        if (k.nsteps <= 0) return bfail(ACM_EINVAL, "nsteps must be positive");
        if (!k.cfg.allow_unstable && api_max_amplification(k.cfg) > 1.0 + 1e-12)
            return bfail(ACM_EUNSTABLE, "case " + std::to_string(i) + " fails the linear stability check");
    }
    // tile -1: the autotuner's choice for the case's shape (acm_batch_autotune)
    std::vector<int> tiles(ncases);
    for (int i = 0; i < ncases; ++i) {
        tiles[i] = cases[i].tile;
        if (tiles[i] >= 0) continue;
        int t = 0;
        if (!tuned_tile(cases[i].cfg.nx, cases[i].cfg.ny, prec, mode, &t))
            return bfail(ACM_ESTATE, "case " + std::to_string(i) + ": grid shape " + std::to_string(cases[i].cfg.nx) +
                                         " x " + std::to_string(cases[i].cfg.ny) +
                                         " is not tuned for this precision and launch mode (acm_batch_autotune)");
        tiles[i] = t;
    }
    acm_batch* b = new (std::nothrow) acm_batch();
    if (!b) return bfail(ACM_EINVAL, "out of host memory");
    b->n = ncases;
    b->precision = prec;
    b->chunk = chunk;
    b->grab = (opts && opts->grab > 0) ? opts->grab : 2;
    b->mode = mode;
    b->umax_limit = (opts && opts->umax_limit > 0) ? opts->umax_limit : 0.3;
    b->stream = static_cast<hipStream_t>(stream);
    b->tile.resize(ncases);
    b->nx.resize(ncases);
    b->ny.resize(ncases);
    b->state.assign(ncases, 0);
    b->nsteps.resize(ncases);
    b->done.assign(ncases, 0);
    b->done_ms.assign(ncases, -1.0);
    b->umax.assign(ncases, 0.0);
    for (int i = 0; i < ncases; ++i) {
        b->tile[i] = tiles[i];
        b->nx[i] = cases[i].cfg.nx;
        b->ny[i] = cases[i].cfg.ny;
        b->nsteps[i] = ((cases[i].nsteps + chunk - 1) / chunk) * chunk;
        b->max_items += case_items(b->nx[i], b->ny[i], tiles[i]);
    }
    char* base = static_cast<char*>(scratch);
    b->dcases = base + L.cases;
    b->ditems = reinterpret_cast<int4*>(base + L.items);
    b->dnitems = reinterpret_cast<int*>(base + L.nitems);
    b->dqueue = reinterpret_cast<int*>(base + L.queue);
    b->dactive = reinterpret_cast<int*>(base + L.active);
    b->dhealth = reinterpret_cast<double*>(base + L.health);
    b->hitems.resize(std::max<size_t>(1, b->max_items));
    b->hactive.resize(ncases);
    b->hhealth.resize(2 * (size_t)ncases);
    // queue counters start at zero (outside any graph; the persistent kernel
    // resets them itself after every launch)
    hipError_t e = hipMemsetAsync(b->dqueue, 0, QUEUE_BYTES, b->stream);
    if (e == hipSuccess) e = (prec == ACM_F64) ? upload_cases<double>(b, cases) : upload_cases<float>(b, cases);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&b->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&b->ev_chunk);
    if (e != hipSuccess) {
        acm_batch_destroy(b);
        return bfail(ACM_EHIP, std::string("batch set-up: ") + hipGetErrorString(e));
    }
    b->blocks = (opts && opts->blocks > 0) ? opts->blocks
                                           : (prec == ACM_F64 ? occupancy_blocks<double>() : occupancy_blocks<float>());
    if (b->blocks <= 0) {
        acm_batch_destroy(b);
        return bfail(ACM_EHIP, "could not size the persistent grid");
    }
    acm_status st = build_graph(b);
    if (st != ACM_OK) {
        acm_batch_destroy(b);
        return st;
    }
    *out = b;
    return ACM_OK;
}

acm_status acm_batch_run(acm_batch* b, int32_t max_chunks, int32_t* active_left)
{
    if (!b) return bfail(ACM_EINVAL, "batch is NULL");
    hipError_t e;
    if (!b->started) {
        e = hipEventRecord(b->ev_start, b->stream);
        if (e != hipSuccess) return bfail(ACM_EHIP, "event record");
        b->started = true;
    }
    int chunks = 0;
    for (;;) {
        // active set and its item table (case-major order)
        int nact = 0;
        size_t nit = 0;
        int64_t chunk_lups = 0;
        for (int i = 0; i < b->n; ++i) {
            if (b->state[i] != 0) continue;
            b->hactive[nact++] = i;
            const int t = b->tile[i];
            const int tx = (b->nx[i] + TILE_W[t] - 1) / TILE_W[t], ty = (b->ny[i] + TILE_H[t] - 1) / TILE_H[t];
            for (int y = 0; y < ty; ++y)
                for (int x = 0; x < tx; ++x) b->hitems[nit++] = make_int4(i, x, y, 0);
            chunk_lups += (int64_t)b->nx[i] * b->ny[i] * b->chunk;
        }
        if (active_left) *active_left = nact;
        if (nact == 0 || (max_chunks >= 0 && chunks >= max_chunks)) break;
        b->hnitems = (int)nit;
        e = hipMemcpyAsync(b->ditems, b->hitems.data(), sizeof(int4) * nit, hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->dnitems, &b->hnitems, sizeof(int), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->dactive, b->hactive.data(), sizeof(int) * nact, hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
        if (e == hipSuccess)
            e = (b->precision == ACM_F64) ? launch_health<double>(b, nact, b->stream)
                                          : launch_health<float>(b, nact, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->hhealth.data(), b->dhealth, 2 * sizeof(double) * b->n, hipMemcpyDeviceToHost,
                               b->stream);
        if (e == hipSuccess) e = hipEventRecord(b->ev_chunk, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return bfail(ACM_EHIP, std::string("batch chunk: ") + hipGetErrorString(e));
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, b->ev_start, b->ev_chunk);
        if (e != hipSuccess) return bfail(ACM_EHIP, std::string("batch timing: ") + hipGetErrorString(e));
        b->elapsed_ms = ms;
        b->lups += chunk_lups;
        for (int a = 0; a < nact; ++a) {
            const int i = b->hactive[a];
            b->done[i] += b->chunk;
            b->umax[i] = b->hhealth[2 * i];
            const bool bad = b->hhealth[2 * i + 1] != 0.0 || !(b->umax[i] <= b->umax_limit);
            if (bad) {
                b->state[i] = 2;
                b->done_ms[i] = ms;
            } else if (b->done[i] >= b->nsteps[i]) {
                b->state[i] = 1;
                b->done_ms[i] = ms;
            }
        }
        ++chunks;
    }
    return ACM_OK;
}

acm_status acm_batch_status(const acm_batch* b, int32_t i, acm_batch_case_status* out)
{
    if (!b || !out || i < 0 || i >= b->n) return bfail(ACM_EINVAL, "bad batch status query");
    out->steps_done = b->done[i];
    out->state = b->state[i];
    out->which = 0;  // chunks have an even number of steps: the state is back in set a
    out->done_ms = b->done_ms[i];
    out->umax = b->umax[i];
    return ACM_OK;
}

acm_status acm_batch_timing(const acm_batch* b, double* total_ms, int64_t* lattice_updates)
{
    if (!b) return bfail(ACM_EINVAL, "batch is NULL");
    if (total_ms) *total_ms = b->elapsed_ms;
    if (lattice_updates) *lattice_updates = b->lups;
    return ACM_OK;
}

void acm_batch_destroy(acm_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->ev_start) (void)hipEventDestroy(b->ev_start);
    if (b->ev_chunk) (void)hipEventDestroy(b->ev_chunk);
    delete b;
}

size_t acm_batch_autotune_scratch_bytes(int32_t nx, int32_t ny, int32_t precision, int32_t copies)
{
    set_error("");
    if (nx < 4 || ny < 4 || copies <= 0 || (precision != ACM_F32 && precision != ACM_F64)) {
        set_error("autotune: bad arguments");
        return 0;
    }
    const size_t es = precision == ACM_F64 ? 8 : 4;
    return align256((size_t)nx * ny * es * 6 * (size_t)copies) +
           batch_layout(copies, case_items(nx, ny, -1) * (size_t)copies, precision).total;
}

acm_status acm_batch_autotune(int32_t nx, int32_t ny, int32_t precision, int32_t mode, int32_t copies, int32_t steps,
                              void* scratch, size_t scratch_bytes, void* stream, double* ms_per_tile, int32_t* best)
{
    if (nx < 4 || ny < 4 || copies <= 0 || steps <= 0 || steps % 2 || !ms_per_tile || !best)
        return bfail(ACM_EINVAL, "autotune: bad arguments");
    if (precision != ACM_F32 && precision != ACM_F64) return bfail(ACM_EINVAL, "autotune: precision");
    if (mode != 0 && mode != 1) return bfail(ACM_EINVAL, "autotune: mode must be 0 or 1");
    const size_t need = acm_batch_autotune_scratch_bytes(nx, ny, precision, copies);
    if (!scratch || reinterpret_cast<uintptr_t>(scratch) % 256 != 0 || scratch_bytes < need)
        return bfail(ACM_EINVAL, "autotune: scratch must be 256-byte aligned and hold " + std::to_string(need) +
                                     " bytes");
    acm_status st = autotune_shape(nx, ny, precision, copies, steps, scratch, scratch_bytes, stream, ms_per_tile, best,
                                   mode);
    if (st != ACM_OK) return st;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[std::make_tuple((int)nx, (int)ny, (int)precision, (int)mode)] = *best;
    return ACM_OK;
}

}  // extern "C"

namespace {
acm_status autotune_shape(int nx, int ny, int precision, int copies, int steps, void* scratch, size_t scratch_bytes,
                          void* stream, double* ms_per_tile, int32_t* best, int mode)
{
    const size_t es = precision == ACM_F64 ? 8 : 4;
    const size_t field = (size_t)nx * ny * es;
    const size_t fields_bytes = align256(field * 6 * (size_t)copies);
    char* mem = static_cast<char*>(scratch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemsetAsync(mem, 0, field * 6 * (size_t)copies, s);
    if (e != hipSuccess) return bfail(ACM_EHIP, std::string("autotune clear: ") + hipGetErrorString(e));
    std::vector<acm_batch_case> cs(copies);
    for (int i = 0; i < copies; ++i) {
        acm_batch_case& k = cs[i];
        std::memset(&k, 0, sizeof k);
        k.cfg.dim = 2;
        k.cfg.nx = nx;
        k.cfg.ny = ny;
        k.cfg.nz = 1;
        k.cfg.dx = k.cfg.dt = 1.0;
        k.cfg.nu = 0.05;
        k.cfg.rho0 = 1.0;
        k.cfg.sat_rho = k.cfg.sat_mom = 1.0;
        k.cfg.precision = precision;
        k.cfg.allow_unstable = 1;  // nu = 0.05 is inside the linear bound; skip the per-copy check
        char* base = mem + (size_t)i * 6 * field;
        k.a = acm_fields{base, base + field, base + 2 * field, nullptr, nullptr};
        k.b = acm_fields{base + 3 * field, base + 4 * field, base + 5 * field, nullptr, nullptr};
        k.nsteps = steps;
    }
    acm_status st = ACM_OK;
    double bestv = 1e300;
    *best = 0;
    for (int t = 0; t < NTILE2D && st == ACM_OK; ++t) {
        for (auto& k : cs) k.tile = t;
        acm_batch_opts o{};
        o.chunk = steps;
        o.mode = mode;
        acm_batch* b = nullptr;
        st = acm_batch_init(cs.data(), copies, &o, mem + fields_bytes, scratch_bytes - fields_bytes, stream, &b);
        if (st != ACM_OK) break;
        st = acm_batch_run(b, 1, nullptr);  // warm-up chunk
        const auto t0 = std::chrono::steady_clock::now();
        if (st == ACM_OK) {
            for (int i = 0; i < copies; ++i) b->state[i] = 0, b->done[i] = 0;
            st = acm_batch_run(b, 1, nullptr);
        }
        const auto t1 = std::chrono::steady_clock::now();
        acm_batch_destroy(b);
        ms_per_tile[t] = std::chrono::duration<double, std::milli>(t1 - t0).count() / steps;
        if (ms_per_tile[t] < bestv) {
            bestv = ms_per_tile[t];
            *best = t;
        }
    }
    (void)hipStreamSynchronize(s);
    return st;
}
}  // namespace
