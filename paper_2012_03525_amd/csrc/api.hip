// C ABI of libacm (declared in include/acm.h): validation, the linear
// stability guard, HIP-graph run loop and diagnostics.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/acm.h"
#include "acm_internal.h"
#include "kern_axisym.h"

using namespace acm;

namespace {

thread_local std::string g_err;

acm_status fail(acm_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

acm_status hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return ACM_EHIP;
}

double sound_speed(const acm_config& c) { return c.cs > 0 ? c.cs : c.dx / (c.dt * std::sqrt(3.0)); }

// Spectral radius of the step linearised about rest (Eqs. 2.10-2.13 in
// Fourier space).  With s_a = sin(k_a dx)/dx, |s|^2 = sum s_a^2 and
// lambda = sum (2 - 2 cos k_a dx)/dx^2, the density and the momentum
// component along s evolve by
//   [ 1 - A lambda              , -i dt |s|                      ]
//   [ i |s| (A B lambda - dt cs^2), 1 - nu dt lambda - B dt |s|^2 ]
// (A = sat_rho cs^2 dt^2 / 2, B = sat_mom (nu + cs^2 dt / 2)); the other
// momentum components decay by 1 - nu dt lambda.
double max_amplification(const acm_config& c)
{
    const double cs = sound_speed(c), cs2 = cs * cs, dt = c.dt, dx = c.dx, nu = c.nu;
    const double A = c.sat_rho * 0.5 * cs2 * dt * dt;
    const double B = c.sat_mom * (nu + 0.5 * cs2 * dt);
    const int D = c.dim;
    const int nk = (D == 3) ? 33 : 129;
    const double pi = 3.14159265358979323846;
    double worst = 0.0;
    const int nz = (D == 3) ? nk : 1;
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < nk; ++iy)
            for (int ix = 0; ix < nk; ++ix) {
                const double k[3] = {pi * ix / (nk - 1), pi * iy / (nk - 1), D == 3 ? pi * iz / (nk - 1) : 0.0};
                double lam = 0.0, s2 = 0.0;
                for (int a = 0; a < D; ++a) {
                    lam += (2.0 - 2.0 * std::cos(k[a])) / (dx * dx);
                    const double sa = std::sin(k[a]) / dx;
                    s2 += sa * sa;
                }
                const double s = std::sqrt(s2);
                using cd = std::complex<double>;
                const cd a11 = 1.0 - A * lam, a12 = cd(0, -dt * s);
                const cd a21 = cd(0, s * (A * B * lam - dt * cs2)), a22 = 1.0 - nu * dt * lam - B * dt * s2;
                const cd tr = a11 + a22, det = a11 * a22 - a12 * a21;
                const cd disc = std::sqrt(tr * tr / 4.0 - det);
                const double l1 = std::abs(tr / 2.0 + disc), l2 = std::abs(tr / 2.0 - disc);
                const double lt = std::abs(1.0 - nu * dt * lam);
                worst = std::fmax(worst, std::fmax(std::fmax(l1, l2), lt));
            }
    return worst;
}

// Heun stability number of the bulk Cahn-Hilliard mode: linearised about
// phi = +-1, mu = 8 a phi' - kappa L phi', so the growth symbol is
// -dt M lambda (8 a + kappa lambda); the isotropic Laplacian reaches
// lambda = 16 / (3 dx^2) at the checkerboard mode.  Heun is stable for <= 2.
double che_number(const acm_config& c)
{
    if (!c.two_phase) return 0.0;
    const double a = 3.0 * c.sigma / (4.0 * c.width), kappa = 3.0 * c.sigma * c.width / 8.0;
    const double lam = 16.0 / (3.0 * c.dx * c.dx);
    return c.dt * c.mobility * lam * (8.0 * a + kappa * lam);
}

// Layout of the caller's scratch buffer, each part 256-byte aligned: the
// diagnostics partial sums (NDIAG doubles per reduction workgroup), the
// NDIAG final sums, and for 3D two-phase runs four fields of intermediates
// (phi* and phi G_iso mu per axis).
struct ScratchLayout {
    int diag_blocks;
    size_t partials, result, fields, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

ScratchLayout scratch_layout(const acm_config& c)
{
    ScratchLayout L{};
    const double n = (double)c.nx * c.ny * (c.dim == 3 ? c.nz : 1);
    L.diag_blocks = (int)std::fmin(2048.0, std::fmax(1.0, std::ceil(n / 256.0)));
    L.partials = 0;
    L.result = align256(sizeof(double) * NDIAG * (size_t)L.diag_blocks);
    L.fields = L.result + align256(sizeof(double) * NDIAG);
    L.total = L.fields;
    if (c.two_phase && c.dim == 3)
        L.total += align256((size_t)n * 4 * (c.precision == ACM_F64 ? sizeof(double) : sizeof(float)));
    return L;
}

acm_status validate(const acm_config* c)
{
    if (!c) return fail(ACM_EINVAL, "config is NULL");
    if (c->dim != 2 && c->dim != 3) return fail(ACM_EINVAL, "dim must be 2 or 3");
    const int minn = c->two_phase ? 8 : 4;
    if (c->nx < minn || c->ny < minn || (c->dim == 3 && c->nz < minn))
        return fail(ACM_EINVAL, "every axis needs at least " + std::to_string(minn) + " nodes");
    if ((double)c->nx * c->ny * (c->dim == 3 ? c->nz : 1) > 4.0e9)
        return fail(ACM_EINVAL, "grid larger than 4e9 nodes");
    if (c->dim == 3 && (double)c->nx * c->ny * (c->precision == ACM_F64 ? 8 : 4) >= 2147483648.0)
        return fail(ACM_EINVAL, "3D plane (nx * ny values) of 2 GiB or more");
    if (!(c->dx > 0) || !(c->dt > 0)) return fail(ACM_EINVAL, "dx and dt must be positive");
    if (!(c->nu >= 0)) return fail(ACM_EINVAL, "nu must be non-negative");
    if (!(c->rho0 > 0)) return fail(ACM_EINVAL, "rho0 must be positive");
    if (c->two_phase && (!(c->width > 0) || !(c->sigma >= 0) || !(c->mobility >= 0)))
        return fail(ACM_EINVAL, "two-phase needs width > 0, sigma >= 0, mobility >= 0");
    for (int f = 0; f < 6; ++f)
        if (!(c->wet_cos[f] >= -1.0 && c->wet_cos[f] <= 1.0))
            return fail(ACM_EINVAL, "wet_cos must lie in [-1, 1]");
    if (c->precision != ACM_F64 && c->precision != ACM_F32) return fail(ACM_EINVAL, "unknown precision");
    if (c->axisym != 0 && c->axisym != 1) return fail(ACM_EINVAL, "axisym must be 0 or 1");
    if (c->axisym && (c->dim != 2 || c->bc[2] != ACM_BC_SYMMETRY))
        return fail(ACM_EINVAL, "axisymmetric runs are 2D with the axis (-y face) a symmetry plane");
    const int nf = c->dim == 3 ? 6 : 4;
    for (int f = 0; f < nf; ++f) {
        if (c->bc[f] < 0 || c->bc[f] > 2) return fail(ACM_EINVAL, "unknown boundary type");
        if (c->bc[f] == ACM_BC_WALL && c->wall_u[f][f / 2] != 0.0)
            return fail(ACM_EINVAL, "wall velocity must be tangential");
    }
    for (int a = 0; a < nf; a += 2)
        if ((c->bc[a] == ACM_BC_PERIODIC) != (c->bc[a + 1] == ACM_BC_PERIODIC))
            return fail(ACM_EINVAL, "a periodic face needs a periodic opposite face");
    if (c->graph_chunk < 0 || (c->graph_chunk % 2) != 0) return fail(ACM_EINVAL, "graph_chunk must be even");
    return ACM_OK;
}

template <typename T>
Coef<T> make_coef(const acm_config& c, const void* force_x)
{
    Coef<T> k{};
    k.nx = c.nx;
    k.ny = c.ny;
    k.nz = c.dim == 3 ? c.nz : 1;
    const int nf = c.dim == 3 ? 6 : 4;
    k.nonperiodic = 0;
    for (int f = 0; f < 6; ++f) {
        k.bc[f] = (f < nf) ? c.bc[f] : ACM_BC_PERIODIC;
        if (k.bc[f] != ACM_BC_PERIODIC) k.nonperiodic = 1;
        for (int a = 0; a < 3; ++a) {
            if (k.bc[f] == ACM_BC_WALL) {
                k.fs[f][a] = T(-1);
                k.fo[f][a] = T(2.0 * c.wall_u[f][a]);
            } else if (k.bc[f] == ACM_BC_SYMMETRY) {
                k.fs[f][a] = (a == f / 2) ? T(-1) : T(1);
                k.fo[f][a] = T(0);
            } else {
                k.fs[f][a] = T(1);
                k.fo[f][a] = T(0);
            }
        }
    }
    const double cs = sound_speed(c), cs2 = cs * cs, dt = c.dt, dx = c.dx;
    k.rho0 = T(c.rho0);
    k.cg = T(dt / (2.0 * dx));
    k.cs2 = T(cs2);
    k.kr = T(c.sat_rho * 0.5 * cs2 * dt * dt / (dx * dx));
    k.kv = T(c.nu * dt / (dx * dx));
    k.ks = T(c.sat_mom * (c.nu + 0.5 * cs2 * dt) / (2.0 * dx));
    for (int a = 0; a < 3; ++a) k.gdt[a] = T(dt * c.g[a]);
    k.dt = T(dt);
    k.fx = static_cast<const T*>(force_x);
    if (c.two_phase) {
        const double a = 3.0 * c.sigma / (4.0 * c.width), kappa = 3.0 * c.sigma * c.width / 8.0;
        k.a4 = T(4.0 * a);
        k.kap6 = T(kappa / (6.0 * dx * dx));
        k.mob = T(c.mobility);
        k.gi = T(1.0 / (12.0 * dx));
        k.li = T(1.0 / (6.0 * dx * dx));
        for (int f = 0; f < nf; ++f)
            if (k.bc[f] == ACM_BC_WALL && c.wet_cos[f] != 0.0) {
                k.wb[f] = T(dx * (2.0 / c.width) * c.wet_cos[f]);
                k.wet = 1;
            }
    }
    return k;
}

}  // namespace

namespace acm {
// shared with the batched entry points (kern_batch.hip)
void set_error(const std::string& msg) { g_err = msg; }
acm_status api_validate(const acm_config* c, std::string& err)
{
    const acm_status s = validate(c);
    err = g_err;
    return s;
}
double api_max_amplification(const acm_config& c) { return max_amplification(c); }
template <typename T>
Coef<T> api_make_coef(const acm_config& c, const void* force_x)
{
    return make_coef<T>(c, force_x);
}
template Coef<float> api_make_coef<float>(const acm_config&, const void*);
template Coef<double> api_make_coef<double>(const acm_config&, const void*);
}  // namespace acm

struct acm_handle {
    acm_config cfg;
    acm_fields set[2];
    const void* force_x = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    int which = 0;
    int64_t step = 0;
    int chunk = 64;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    // tile codes 14 / 15 on 3D periodic boxes: acm_run advances two steps
    // per launch
    bool pair = false;
    hipGraphExec_t exec_pair[2] = {nullptr, nullptr};
    // carved from the caller's scratch buffer (acm_scratch_bytes)
    double* partials = nullptr;
    double* result = nullptr;
    void* fields = nullptr;  // 3D two-phase intermediates (4 fields)
    double host[NDIAG];      // diagnostics read-back
    int diag_blocks = 0;
    Coef<float> cf;
    Coef<double> cd;
};

namespace {

template <typename T>
State<T> state_of(const acm_fields& f)
{
    return State<T>{static_cast<T*>(f.drho), static_cast<T*>(f.u), static_cast<T*>(f.v), static_cast<T*>(f.w),
                    static_cast<T*>(f.phi)};
}

template <typename T>
hipError_t launch_typed(const acm_handle* h, const Coef<T>& c, int from, hipStream_t s)
{
    const State<T> in = state_of<T>(h->set[from]);
    const State<T> out = state_of<T>(h->set[1 - from]);
    if (h->cfg.two_phase && h->cfg.dim == 3)
        return launch_twophase3d<T>(c, in, out, static_cast<T*>(h->fields), h->cfg.tile, s);
    if (h->cfg.two_phase && h->cfg.axisym) return launch_twophase_axisym2d<T>(c, in, out, h->cfg.tile, s);
    if (h->cfg.two_phase) return launch_twophase2d<T>(c, in, out, h->cfg.tile, s);
    if (h->cfg.dim == 3) return launch_step3d<T>(c, in, out, h->cfg.tile, s);
    if (h->cfg.axisym) return launch_axisym2d<T>(c, in, out, h->cfg.tile, s);
    return launch_step2d<T>(c, in, out, h->cfg.tile, s);
}

hipError_t launch_one(const acm_handle* h, int from, hipStream_t s)
{
    if (h->cfg.precision == ACM_F64) return launch_typed<double>(h, h->cd, from, s);
    return launch_typed<float>(h, h->cf, from, s);
}

// two steps from set `from` into the other set
hipError_t launch_pair(const acm_handle* h, int from, hipStream_t s)
{
    if (h->cfg.precision == ACM_F64)
        return launch_step3d_pair<double>(h->cd, state_of<double>(h->set[from]), state_of<double>(h->set[1 - from]),
                                          h->cfg.tile, s);
    return launch_step3d_pair<float>(h->cf, state_of<float>(h->set[from]), state_of<float>(h->set[1 - from]),
                                     h->cfg.tile, s);
}

// a graph of chunk steps from set `parity`: chunk one-step launches, or
// chunk / 2 two-step launches
acm_status build_graph(acm_handle* h, int parity, bool pair)
{
    hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    const int nl = pair ? h->chunk / 2 : h->chunk;
    for (int i = 0; i < nl; ++i) {
        e = pair ? launch_pair(h, (parity + i) & 1, h->cap) : launch_one(h, (parity + i) & 1, h->cap);
        if (e != hipSuccess) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(h->cap, &g);
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(e, "kernel launch during capture");
        }
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->cap, &g);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t* slot = pair ? &h->exec_pair[parity] : &h->exec[parity];
    e = hipGraphInstantiate(slot, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *slot = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    return ACM_OK;
}

}  // namespace

extern "C" {

const char* acm_last_error(void) { return g_err.c_str(); }

const char* acm_version(void) { return "acm 0.1 (gfx950)"; }

acm_status acm_stability(const acm_config* cfg, double* max_amp, double* che)
{
    acm_status st = validate(cfg);
    if (st != ACM_OK) return st;
    if (max_amp) *max_amp = max_amplification(*cfg);
    if (che) *che = che_number(*cfg);
    return ACM_OK;
}

size_t acm_scratch_bytes(const acm_config* cfg)
{
    g_err.clear();
    if (validate(cfg) != ACM_OK) return 0;
    return scratch_layout(*cfg).total;
}

acm_status acm_init(const acm_config* cfg, const acm_fields* a, const acm_fields* b, const void* force_x,
                    void* scratch, size_t scratch_bytes, void* stream, acm_handle** out)
{
    g_err.clear();
    if (!out) return fail(ACM_EINVAL, "out is NULL");
    *out = nullptr;
    acm_status st = validate(cfg);
    if (st != ACM_OK) return st;
    if (!a || !b) return fail(ACM_EINVAL, "field sets are NULL");
    const acm_fields* sets[2] = {a, b};
    for (int s = 0; s < 2; ++s) {
        const acm_fields* f = sets[s];
        if (!f->drho || !f->u || !f->v) return fail(ACM_EINVAL, "drho, u and v are required");
        if (cfg->dim == 3 && !f->w) return fail(ACM_EINVAL, "w is required in 3D");
        if (cfg->two_phase && !f->phi) return fail(ACM_EINVAL, "phi is required for two-phase runs");
    }
    const ScratchLayout L = scratch_layout(*cfg);
    if (!scratch) return fail(ACM_EINVAL, "scratch is NULL (acm_scratch_bytes gives its size)");
    if (reinterpret_cast<uintptr_t>(scratch) % 256 != 0) return fail(ACM_EINVAL, "scratch must be 256-byte aligned");
    if (scratch_bytes < L.total)
        return fail(ACM_EINVAL, "scratch holds " + std::to_string(scratch_bytes) + " bytes, the configuration needs " +
                                    std::to_string(L.total));
    if (!cfg->allow_unstable) {
        const double amp = max_amplification(*cfg);
        if (amp > 1.0 + 1e-12) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "linearised step amplifies by %.6f > 1 (set allow_unstable to run anyway)",
                          amp);
            return fail(ACM_EUNSTABLE, buf);
        }
        const double z = che_number(*cfg);
        if (z > 2.0) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "Cahn-Hilliard stability number %.4f > 2", z);
            return fail(ACM_EUNSTABLE, buf);
        }
    }
    acm_handle* h = new (std::nothrow) acm_handle();
    if (!h) return fail(ACM_EINVAL, "out of host memory");
    h->cfg = *cfg;
    h->set[0] = *a;
    h->set[1] = *b;
    h->force_x = force_x;
    h->stream = static_cast<hipStream_t>(stream);
    h->chunk = cfg->graph_chunk > 0 ? cfg->graph_chunk : 64;
    h->cf = make_coef<float>(*cfg, force_x);
    h->cd = make_coef<double>(*cfg, force_x);
    char* base = static_cast<char*>(scratch);
    h->partials = reinterpret_cast<double*>(base + L.partials);
    h->result = reinterpret_cast<double*>(base + L.result);
    h->fields = (cfg->two_phase && cfg->dim == 3) ? base + L.fields : nullptr;
    h->diag_blocks = L.diag_blocks;
    if (cfg->dim == 3 && !cfg->two_phase)
        h->pair = cfg->precision == ACM_F64 ? step3d_pair_ok<double>(h->cd, cfg->tile)
                                            : step3d_pair_ok<float>(h->cf, cfg->tile);
    hipError_t e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    // capture the chunk graphs of both parities now, so that no run call
    // pays for (or times) a capture
    for (int p = 0; p < 2 && st == ACM_OK; ++p) {
        st = build_graph(h, p, false);
        if (st == ACM_OK && h->pair) st = build_graph(h, p, true);
    }
    if (st != ACM_OK) {
        const std::string msg = g_err;
        acm_destroy(h);
        return fail(st, msg);
    }
    *out = h;
    return ACM_OK;
}

acm_status acm_step(acm_handle* h)
{
    if (!h) return fail(ACM_EINVAL, "handle is NULL");
    hipError_t e = launch_one(h, h->which, h->stream);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    h->which ^= 1;
    h->step += 1;
    return ACM_OK;
}

acm_status acm_run(acm_handle* h, int64_t nsteps)
{
    if (!h) return fail(ACM_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(ACM_EINVAL, "nsteps must be >= 0");
    if (h->pair && nsteps >= 3) {
        // two steps per launch; the run ends with a one-step launch, so the
        // other set holds the state one step back, as after one-step runs
        while (nsteps > h->chunk) {
            hipError_t e = hipGraphLaunch(h->exec_pair[h->which], h->stream);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
            h->which ^= (h->chunk / 2) & 1;
            h->step += h->chunk;
            nsteps -= h->chunk;
        }
        while (nsteps >= 3) {
            hipError_t e = launch_pair(h, h->which, h->stream);
            if (e != hipSuccess) return hip_fail(e, "step launch");
            h->which ^= 1;
            h->step += 2;
            nsteps -= 2;
        }
    }
    while (nsteps >= h->chunk) {
        hipError_t e = hipGraphLaunch(h->exec[h->which], h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        h->step += h->chunk;  // chunk is even: the parity is unchanged
        nsteps -= h->chunk;
    }
    for (int64_t i = 0; i < nsteps; ++i) {
        acm_status st = acm_step(h);
        if (st != ACM_OK) return st;
    }
    return ACM_OK;
}

acm_status acm_diagnostics(acm_handle* h, acm_diag* out)
{
    if (!h || !out) return fail(ACM_EINVAL, "NULL argument");
    const acm_config& c = h->cfg;
    hipError_t e;
    const int have_prev = h->step > 0 ? 1 : 0;
    if (c.axisym && c.precision == ACM_F64)
        e = launch_diag_axisym<double>(h->cd, c.two_phase, state_of<double>(h->set[h->which]),
                                       state_of<double>(h->set[1 - h->which]), have_prev, h->partials,
                                       h->diag_blocks, h->result, h->stream);
    else if (c.axisym)
        e = launch_diag_axisym<float>(h->cf, c.two_phase, state_of<float>(h->set[h->which]),
                                      state_of<float>(h->set[1 - h->which]), have_prev, h->partials,
                                      h->diag_blocks, h->result, h->stream);
    else if (c.precision == ACM_F64)
        e = launch_diag<double>(h->cd, c.dim, c.two_phase, state_of<double>(h->set[h->which]),
                                state_of<double>(h->set[1 - h->which]), have_prev, h->partials, h->diag_blocks,
                                h->result, h->stream);
    else
        e = launch_diag<float>(h->cf, c.dim, c.two_phase, state_of<float>(h->set[h->which]),
                               state_of<float>(h->set[1 - h->which]), have_prev, h->partials, h->diag_blocks,
                               h->result, h->stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostics launch");
    e = hipMemcpyAsync(h->host, h->result, sizeof(double) * NDIAG, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const double* r = h->host;
    // planar: node sums times dx^D, means over the node count; axisymmetric:
    // sums of (j + 1/2) x value times 2 pi dx^3 (cell volume 2 pi r dx^2),
    // means over the summed weights nx ny^2 / 2
    const double pi = 3.14159265358979323846;
    const double dxd = c.axisym ? 2.0 * pi * c.dx * c.dx * c.dx : (c.dim == 3 ? c.dx * c.dx * c.dx : c.dx * c.dx);
    const double n = c.axisym ? 0.5 * (double)c.nx * c.ny * c.ny : (double)c.nx * c.ny * (c.dim == 3 ? c.nz : 1);
    const double inv2dx = 1.0 / (2.0 * c.dx);
    out->mass = r[0] * dxd;
    out->mom[0] = r[1] * dxd;
    out->mom[1] = r[2] * dxd;
    out->mom[2] = r[3] * dxd;
    out->ke = 0.5 * r[4] * dxd;
    out->dumax = r[5];
    out->umax = r[6];
    out->enstrophy = r[7] * inv2dx * inv2dx / (2.0 * n);
    out->energy = r[4] / (2.0 * n);
    out->div_rms = std::sqrt(r[8] / n) * inv2dx;
    out->div_max = r[9] * inv2dx;
    out->phi_sum = c.axisym ? r[10] * dxd : r[10];
    out->nonfinite = r[11] != 0.0 ? 1 : 0;
    out->step = h->step;
    out->which = h->which;
    if (out->nonfinite) return fail(ACM_ENONFINITE, "state holds a NaN or Inf");
    return ACM_OK;
}

acm_status acm_current(const acm_handle* h, int32_t* which, int64_t* step)
{
    if (!h) return fail(ACM_EINVAL, "handle is NULL");
    if (which) *which = h->which;
    if (step) *step = h->step;
    return ACM_OK;
}

acm_status acm_set_current(acm_handle* h, int32_t which, int64_t step)
{
    if (!h) return fail(ACM_EINVAL, "handle is NULL");
    if (which != 0 && which != 1) return fail(ACM_EINVAL, "which must be 0 or 1");
    if (step < 0) return fail(ACM_EINVAL, "step must be >= 0");
    h->which = which;
    h->step = step;
    return ACM_OK;
}

acm_status acm_step_adjoint(acm_handle* h, const acm_fields* q, const acm_fields* s, const acm_fields* adj_s,
                            const acm_fields* adj_q)
{
    if (!h || !q || !s || !adj_s || !adj_q) return fail(ACM_EINVAL, "NULL argument");
    if (h->cfg.dim != 2 || h->cfg.two_phase || h->cfg.axisym)
        return fail(ACM_EINVAL, "the adjoint step covers planar 2D single-phase runs");
    const acm_fields* all[4] = {q, s, adj_s, adj_q};
    for (const acm_fields* f : all)
        if (!f->drho || !f->u || !f->v) return fail(ACM_EINVAL, "NULL field");
    const void* outs[3] = {adj_q->drho, adj_q->u, adj_q->v};
    for (const void* o : outs)
        for (int k = 0; k < 3; ++k) {
            const void* ins[3] = {all[k]->drho, all[k]->u, all[k]->v};
            for (const void* in : ins)
                if (o == in) return fail(ACM_EINVAL, "adj_q must not alias q, s or adj_s");
        }
    hipError_t e;
    if (h->cfg.precision == ACM_F64)
        e = launch_adjoint2d<double>(h->cd, state_of<double>(*q), state_of<double>(*s), state_of<double>(*adj_s),
                                     state_of<double>(*adj_q), h->stream);
    else
        e = launch_adjoint2d<float>(h->cf, state_of<float>(*q), state_of<float>(*s), state_of<float>(*adj_s),
                                    state_of<float>(*adj_q), h->stream);
    return e == hipSuccess ? ACM_OK : hip_fail(e, "adjoint launch");
}

void acm_destroy(acm_handle* h)
{
    if (!h) return;
    if (h->stream || h->cap) (void)hipStreamSynchronize(h->stream);
    for (int p = 0; p < 2; ++p) {
        if (h->exec[p]) (void)hipGraphExecDestroy(h->exec[p]);
        if (h->exec_pair[p]) (void)hipGraphExecDestroy(h->exec_pair[p]);
    }
    if (h->cap) (void)hipStreamDestroy(h->cap);
    delete h;
}

}  // extern "C"
