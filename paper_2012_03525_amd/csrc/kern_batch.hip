// Batched independent 2D cases in one launch per step.
//
// Every active (case, tile) pair is an item of a device table.  Mode 0
// (default): one workgroup per item slot (the item capacity), slots past the
// active count exit at once, and the hardware dispatcher keeps as many items
// in flight as occupancy allows.  Mode 1: a persistent grid (CUs x occupancy
// workgroups) pops items `grab` at a time from an atomic counter; the last
// workgroup to finish resets the counter for the next launch.  A persistent
// workgroup waits out each item's load latency in turn, which the dispatcher
// hides in mode 0 (1.5x faster on the 512-case sweep).  Both run
// the same tile function as the single-case kernel (tile2d.h), so each
// case's result is bitwise equal to running it alone.  A
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
};

// tile shapes of the 2D kernels (same numbering as launch_step2d)
constexpr int NTILE2D = 6;
constexpr int TILE_W[NTILE2D] = {64, 32, 64, 16, 128, 32};
constexpr int TILE_H[NTILE2D] = {4, 8, 8, 16, 4, 16};

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

template <typename T>
__global__ __launch_bounds__(256) void batch_step_kernel(const BatchCaseDev<T>* __restrict__ cases,
                                                          const int4* __restrict__ items,
                                                          const int* __restrict__ nitems, int* queue, int parity,
                                                          int grab)
{
    __shared__ __align__(16) char smem[batch_lds_bytes<T>()];
    __shared__ int s_first;
    const int n = *nitems;
    for (;;) {
        if (threadIdx.x == 0) s_first = atomicAdd(&queue[0], grab);
        __syncthreads();
        const int first = s_first;
        __syncthreads();
        if (first >= n) break;
        const int last = min(first + grab, n);
        for (int t = first; t < last; ++t) {
            const int4 it = items[t];
            batch_item<T>(cases[it.x], it, parity, smem);
            __syncthreads();  // the next item reuses the LDS tile
        }
    }
    if (threadIdx.x == 0) {
        const int d = atomicAdd(&queue[1], 1);
        if (d == (int)gridDim.x - 1) {  // every workgroup has left the loop: reset for the next launch
            queue[0] = 0;
            queue[1] = 0;
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
    int grab = 4;
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
    L.active = L.queue + 256;
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
    b->grab = (opts && opts->grab > 0) ? opts->grab : 4;
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
    hipError_t e = hipMemsetAsync(b->dqueue, 0, 2 * sizeof(int), b->stream);
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
