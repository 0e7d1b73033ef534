"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  FP64 builds must agree to relative L2 <= 1e-12; the
FP32 build (drho storage) to <= 2e-5 on u and <= 1e-4 on drho after 1000
steps of the 2D Taylor-Green case.  FP32 inputs are rounded to FP32 first
and the oracle starts from exactly those values."""
import math

import numpy as np
import pytest

from paper_2012_03525_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def acm_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2012_03525_amd import acm
    acm.lib()
    return acm


def rel_l2(a, b):
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / max(den, 1e-300))


def rel_l2_vec(g, o, keys):
    """Relative L2 of a vector field (components stacked): the FP32 error of
    a component that is nearly zero is measured against the velocity scale."""
    num = sum(float(np.sum((g[k] - o[k]) ** 2)) for k in keys)
    den = sum(float(np.sum(o[k] ** 2)) for k in keys)
    return math.sqrt(num / max(den, 1e-300))


def to_f32(st):
    return {k: v.astype(np.float32).astype(np.float64) for k, v in st.items()}


def oparams(orc, cfg):
    bc = list(cfg.bc)
    wu = [[cfg.wall_u[f][a] for a in range(3)] for f in range(6)]
    cs = cfg.cs if cfg.cs > 0 else cfg.dx / (cfg.dt * math.sqrt(3))
    return orc.Params(dim=cfg.dim, nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, dx=cfg.dx, dt=cfg.dt, nu=cfg.nu, cs=cs,
                      rho0=cfg.rho0, sat_rho=cfg.sat_rho, sat_mom=cfg.sat_mom, g=list(cfg.g), bc=bc, wall_u=wu,
                      two_phase=bool(cfg.two_phase), sigma=cfg.sigma, width=cfg.width, mobility=cfg.mobility,
                      wet_cos=[cfg.wet_cos[f] for f in range(6)])


def run_both(acm, orc, cfg, st, nsteps, force_x=None, use_run=True):
    s = acm.Solver(cfg, st, force_x=force_x)
    if use_run:
        s.run(nsteps)
    else:
        for _ in range(nsteps):
            s.step()
    g = s.state()
    s.close()
    o = orc.run(oparams(orc, cfg), st, nsteps, force_x_row=force_x)
    return g, o


# --- the 2D Taylor-Green case: 64^2, u0 = 0.01, nu = 0.01, 1000 steps -------
def tgv64():
    return inputs.tgv2d(64, 0.01, seed=20201206, noise=1e-6)


def test_tgv2d_fp64_parity(acm_mod, orc):
    cfg = acm_mod.make_config(2, 64, 64, nu=0.01, precision="f64")
    g, o = run_both(acm_mod, orc, cfg, tgv64(), 1000)
    for k in ("drho", "u", "v"):
        assert rel_l2(g[k], o[k]) <= 1e-12, k


def test_tgv2d_fp32_parity(acm_mod, orc):
    cfg = acm_mod.make_config(2, 64, 64, nu=0.01, precision="f32")
    st = to_f32(tgv64())
    g, o = run_both(acm_mod, orc, cfg, st, 1000)
    eu, ev, er = rel_l2(g["u"], o["u"]), rel_l2(g["v"], o["v"]), rel_l2(g["drho"], o["drho"])
    print(f"fp32 rel L2 after 1000 steps: u {eu:.3e} v {ev:.3e} drho {er:.3e}")
    assert eu <= 2e-5 and ev <= 2e-5
    assert er <= 1e-4


def test_graph_run_equals_single_steps(acm_mod):
    """acm_run (captured graphs of graph_chunk steps) is bitwise equal to
    the same number of acm_step calls."""
    st = to_f32(tgv64())
    cfg = acm_mod.make_config(2, 64, 64, nu=0.01, precision="f32", graph_chunk=8)
    a = acm_mod.Solver(cfg, st)
    a.run(37)
    b = acm_mod.Solver(cfg, st)
    for _ in range(37):
        b.step()
    sa, sb = a.state(), b.state()
    assert a.current() == b.current() == (1, 37)
    for k in sa:
        assert np.array_equal(sa[k], sb[k])


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5])
def test_tiles_bitwise_identical(acm_mod, tile):
    """The per-node arithmetic does not depend on the tile shape."""
    st = to_f32(inputs.seeded_state((45, 70), seed=2, scale_u=0.03, scale_r=1e-3))
    wu = [[0.0] * 3 for _ in range(6)]
    wu[3] = [0.05, 0.0, 0.0]
    base = acm_mod.make_config(2, 70, 45, nu=0.05, precision="f32", bc=(0, 0, 1, 1, 0, 0), wall_u=wu)
    ref = acm_mod.Solver(base, st)
    ref.run(20)
    r = ref.state()
    cfg = acm_mod.make_config(2, 70, 45, nu=0.05, precision="f32", bc=(0, 0, 1, 1, 0, 0), wall_u=wu, tile=tile)
    s = acm_mod.Solver(cfg, st)
    s.run(20)
    o = s.state()
    for k in r:
        assert np.array_equal(r[k], o[k]), k


BC2D = {
    "periodic": ((0, 0, 0, 0, 0, 0), {}),
    "cavity": ((1, 1, 1, 1, 0, 0), {3: [0.05, 0, 0]}),
    "walls_moving": ((1, 1, 1, 1, 0, 0), {0: [0, -0.02, 0], 1: [0, 0.03, 0], 2: [0.01, 0, 0], 3: [-0.04, 0, 0]}),
    "symmetry": ((2, 2, 2, 2, 0, 0), {}),
    "mixed": ((0, 0, 1, 2, 0, 0), {2: [0.03, 0, 0]}),
    "sym_wall": ((2, 1, 1, 2, 0, 0), {1: [0, 0.02, 0], 2: [0.01, 0, 0]}),
}


@pytest.mark.parametrize("name", list(BC2D))
@pytest.mark.parametrize("shape", [(45, 70), (16, 16), (4, 9)])
@pytest.mark.parametrize("tile", [0, 3])
def test_bc2d_fp64_parity(acm_mod, orc, name, shape, tile):
    faces, walls = BC2D[name]
    wu = [[0.0] * 3 for _ in range(6)]
    for f, v in walls.items():
        wu[f] = v
    ny, nx = shape
    st = inputs.seeded_state(shape, seed=5, scale_u=0.03, scale_r=1e-3)
    cfg = acm_mod.make_config(2, nx, ny, nu=0.04, precision="f64", bc=faces, wall_u=wu, tile=tile,
                              g=(1e-5, -2e-5, 0.0))
    g, o = run_both(acm_mod, orc, cfg, st, 30)
    for k in ("drho", "u", "v"):
        assert rel_l2(g[k], o[k]) <= 1e-12, (k, rel_l2(g[k], o[k]))


def test_body_force_row_profile_parity(acm_mod, orc):
    n = 64
    st = inputs.random_spectrum_field(n, seed=3, u_rms=0.02, kmax=8)
    fx = 1e-5 * np.sin(2 * math.pi * 4 * np.arange(n) / n)
    cfg = acm_mod.make_config(2, n, n, nu=0.02, precision="f64")
    g, o = run_both(acm_mod, orc, cfg, st, 100, force_x=fx)
    for k in ("drho", "u", "v"):
        assert rel_l2(g[k], o[k]) <= 1e-12


# --- 3D ----------------------------------------------------------------------
def test_tgv3d_fp64_parity_64(acm_mod, orc):
    """3D Taylor-Green, FP64 GPU build at 64^3 against the oracle."""
    n, u0 = 64, 0.05
    nu = u0 * (n / (2 * math.pi)) / 1600.0
    cfg = acm_mod.make_config(3, n, n, n, nu=nu, precision="f64")
    g, o = run_both(acm_mod, orc, cfg, inputs.tgv3d(n, u0), 60)
    for k in ("drho", "u", "v", "w"):
        assert rel_l2(g[k], o[k]) <= 1e-12, k


def test_tgv3d_fp32_parity_64(acm_mod, orc):
    n, u0 = 64, 0.05
    nu = u0 * (n / (2 * math.pi)) / 1600.0
    cfg = acm_mod.make_config(3, n, n, n, nu=nu, precision="f32")
    g, o = run_both(acm_mod, orc, cfg, to_f32(inputs.tgv3d(n, u0)), 60)
    assert rel_l2_vec(g, o, ("u", "v", "w")) <= 2e-5
    assert rel_l2(g["drho"], o["drho"]) <= 1e-4


@pytest.fixture(scope="module")
def tgv3d_64_oracle_1000(orc):
    """The FP64 oracle's 1000 steps of the 3D Taylor-Green case at 64^3 from
    the FP32-rounded initial state (shared by the launch shapes below).
    Re = 400 gives the benchmark's lattice viscosity (u0 = 0.05,
    nu = 1.27e-3); at Re = 1600 the 64^3 grid under-resolves the flow and the
    oracle itself blows up between steps 900 and 1000 (max |u| 0.053 ->
    1.7e3), the low tolerance to under-resolution that Sec. 3.3 reports for
    the shear layer on 256^2."""
    n, u0 = 64, 0.05
    nu = u0 * (n / (2 * math.pi)) / 400.0
    st = to_f32(inputs.tgv3d(n, u0))
    return st, nu, orc.run(orc.Params(dim=3, nx=n, ny=n, nz=n, nu=nu), st, 1000)


@pytest.mark.parametrize("tile", [0, 13 | (4 << 8), 13 | (1 << 8), 16 | (2 << 8), 17 | (1 << 8)],
                         ids=["default", "tile13-chunk64", "tile13-chunk16", "rows4-chunk32", "rows6-chunk16"])
def test_tgv3d_fp32_parity_64_1000_steps(acm_mod, tgv3d_64_oracle_1000, tile):
    """The stated FP32 bounds after 1000 steps (u <= 2e-5, drho <= 1e-4
    relative L2) for the 3D Taylor-Green case at 64^3: the default launch
    shape for this grid, the periodic fast path of the column kernel (64 x 8
    tile, two rows per thread, three-plane LDS ring) forced with 64- and
    16-plane z chunks, and the whole-row kernel with 4- and 6-row bands."""
    n = 64
    st, nu, o = tgv3d_64_oracle_1000
    cfg = acm_mod.make_config(3, n, n, n, nu=nu, precision="f32", tile=tile, graph_chunk=100)
    s = acm_mod.Solver(cfg, st)
    s.run(1000)
    g = s.state()
    s.close()
    ev = rel_l2_vec(g, o, ("u", "v", "w"))
    er = rel_l2(g["drho"], o["drho"])
    print(f"tile {tile}: u {ev:.2e} drho {er:.2e}")
    assert ev <= 2e-5
    assert er <= 1e-4


BC3D = {
    "periodic": ((0, 0, 0, 0, 0, 0), {}),
    "cavity": ((1, 1, 1, 1, 1, 1), {5: [0.05, 0, 0]}),
    "mixed": ((2, 2, 0, 0, 1, 1), {4: [0.01, 0.02, 0], 5: [-0.02, 0, 0]}),
    "zsym": ((0, 0, 1, 2, 2, 1), {2: [0, 0, 0.03], 5: [0, 0.01, 0]}),
}


@pytest.mark.parametrize("name", list(BC3D))
@pytest.mark.parametrize("tile", [0, 1, 3 | (1 << 8)])
def test_bc3d_fp64_parity(acm_mod, orc, name, tile):
    faces, walls = BC3D[name]
    wu = [[0.0] * 3 for _ in range(6)]
    for f, v in walls.items():
        wu[f] = v
    shape = (19, 21, 70)
    st = inputs.seeded_state(shape, seed=9, scale_u=0.03, scale_r=1e-3)
    cfg = acm_mod.make_config(3, 70, 21, 19, nu=0.03, precision="f64", bc=faces, wall_u=wu, tile=tile,
                              g=(1e-5, 0.0, -1e-5))
    g, o = run_both(acm_mod, orc, cfg, st, 12)
    for k in ("drho", "u", "v", "w"):
        assert rel_l2(g[k], o[k]) <= 1e-12, (k, rel_l2(g[k], o[k]))


@pytest.mark.parametrize("name", ["cavity", "mixed", "zsym", "periodic"])
def test_tiles3d_bitwise_identical(acm_mod, name):
    """FP32 3D: every launch shape (in-plane tile, rows per thread, z chunk)
    gives the same bits on a ragged grid with walls, symmetry planes and a
    body force."""
    faces, walls = BC3D[name]
    wu = [[0.0] * 3 for _ in range(6)]
    for f, v in walls.items():
        wu[f] = v
    st = to_f32(inputs.seeded_state((37, 45, 70), seed=11, scale_u=0.03, scale_r=1e-3))
    ref = None
    for tile in (3 | (1 << 8), 1, 2, 4, 5, 7, 9, 12, 13, 13 | (1 << 8), 2 | (2 << 8)):
        cfg = acm_mod.make_config(3, 70, 45, 37, nu=0.03, precision="f32", bc=faces, wall_u=wu, tile=tile,
                                  g=(1e-5, 0.0, -1e-5))
        s = acm_mod.Solver(cfg, st)
        s.run(6)
        g = s.state()
        s.close()
        if ref is None:
            ref = g
        else:
            for k in ref:
                assert np.array_equal(g[k], ref[k]), (tile, k)


def test_tgv3d_full_size_one_step_and_invariants(acm_mod, orc):
    """256^3 FP32 in the benchmark's launch configuration: one step compared
    node by node with the oracle, then 200 more steps checked for exact-mass
    and momentum invariants and monotone kinetic-energy decay."""
    n, u0 = 256, 0.05
    nu = u0 * (n / (2 * math.pi)) / 1600.0
    st = to_f32(inputs.tgv3d(n, u0))
    cfg = acm_mod.make_config(3, n, n, n, nu=nu, precision="f32")
    s = acm_mod.Solver(cfg, st)
    d0 = s.diagnostics()
    s.step()
    g = s.state()
    o = orc.step(oparams(orc, cfg), st)
    umax = max(np.abs(o[k]).max() for k in ("u", "v", "w"))
    for k in ("u", "v", "w"):
        err = np.abs(g[k] - o[k]).max() / umax
        assert err < 1e-6, (k, err)
    assert np.abs(g["drho"] - o["drho"]).max() / np.abs(o["drho"]).max() < 1e-6
    del o
    kes = [s.diagnostics()["ke"]]
    for _ in range(4):
        s.run(50)
        d = s.diagnostics(raise_nonfinite=True)
        kes.append(d["ke"])
        assert abs(d["mass"] - d0["mass"]) < 1e-6 * n ** 3 * 1e-3
        for a in ("mom_x", "mom_y", "mom_z"):
            assert abs(d[a]) < 1e-8 * n ** 3
    assert all(kes[i + 1] < kes[i] for i in range(len(kes) - 1))
    s.close()


# --- two-phase -----------------------------------------------------------------
def drop128(u_wall=0.02):
    return inputs.drop_in_shear(128, 128, 16.0, 4.0, u_wall)


def drop_cfg(acm, n, precision, tile=0):
    wu = [[0.0] * 3 for _ in range(6)]
    wu[2] = [-0.02, 0, 0]
    wu[3] = [0.02, 0, 0]
    return acm.make_config(2, n, n, nu=0.1, precision=precision, bc=(0, 0, 1, 1, 0, 0), wall_u=wu,
                           two_phase=True, sigma=0.01, width=4.0, mobility=0.02, tile=tile)


@pytest.mark.parametrize("tile", [0, 1, 3])
def test_twophase_fp64_parity(acm_mod, orc, tile):
    cfg = drop_cfg(acm_mod, 128, "f64", tile)
    g, o = run_both(acm_mod, orc, cfg, drop128(), 300)
    for k in ("drho", "u", "v", "phi"):
        assert rel_l2(g[k], o[k]) <= 1e-12, (k, rel_l2(g[k], o[k]))


def test_twophase_fp32_parity(acm_mod, orc):
    """FP32 two-phase after 1000 steps.  FP32 storage of phi alone moves drho
    by ~3e-4 relative L2 (shown on the CPU by the storage-emulation test), so
    drho is bounded at 1e-3 here; velocity and phi keep 2e-5 and 1e-5."""
    cfg = drop_cfg(acm_mod, 128, "f32")
    g, o = run_both(acm_mod, orc, cfg, to_f32(drop128()), 1000)
    print(f"two-phase fp32: phi {rel_l2(g['phi'], o['phi']):.2e} vel {rel_l2_vec(g, o, ('u', 'v')):.2e} "
          f"drho {rel_l2(g['drho'], o['drho']):.2e}")
    assert rel_l2(g["phi"], o["phi"]) <= 1e-5
    assert rel_l2_vec(g, o, ("u", "v")) <= 2e-5
    assert rel_l2(g["drho"], o["drho"]) <= 1e-3


@pytest.mark.parametrize("faces", [(0, 0, 0, 0, 0, 0), (2, 2, 1, 1, 0, 0), (1, 1, 2, 2, 0, 0)])
def test_twophase_bc_ragged_fp64(acm_mod, orc, faces):
    ny, nx = 37, 53
    st = inputs.seeded_state((ny, nx), seed=4, scale_u=0.02, scale_r=1e-3, two_phase=True)
    wu = [[0.0] * 3 for _ in range(6)]
    if faces[2] == 1:
        wu[2] = [0.01, 0, 0]
    if faces[0] == 1:
        wu[1] = [0, -0.02, 0]
    cfg = acm_mod.make_config(2, nx, ny, nu=0.08, precision="f64", bc=faces, wall_u=wu, two_phase=True,
                              sigma=0.005, width=4.0, mobility=0.05)
    g, o = run_both(acm_mod, orc, cfg, st, 20)
    for k in ("drho", "u", "v", "phi"):
        assert rel_l2(g[k], o[k]) <= 1e-12, (k, rel_l2(g[k], o[k]))


def test_twophase_full_size_one_step(acm_mod, orc):
    """1024^2 drop in shear (FP32, the full two-phase workload): one step node
    by node against the oracle."""
    st = to_f32(inputs.drop_in_shear(1024, 1024, 128.0, 4.0, 0.02))
    cfg = drop_cfg(acm_mod, 1024, "f32")
    s = acm_mod.Solver(cfg, st)
    s.step()
    g = s.state()
    o = orc.step(oparams(orc, cfg), st)
    umax = max(np.abs(o[k]).max() for k in ("u", "v"))
    for k in ("u", "v"):
        assert np.abs(g[k] - o[k]).max() / umax < 1e-6, k
    assert np.abs(g["phi"] - o["phi"]).max() < 1e-6
    assert np.abs(g["drho"] - o["drho"]).max() < 1e-9
    s.close()


# --- wetting walls (2D) and 3D two-phase -------------------------------------------
@pytest.mark.parametrize("tile", [0, 1, 3])
def test_twophase_wetting_2d_fp64(acm_mod, orc, tile):
    """2D drop sitting on a wetting wall (theta = 60 degrees below, 120 above,
    ragged 53 x 37 grid, symmetry planes in x): FP64 against the oracle."""
    nx, ny = 53, 37
    st = inputs.drop_in_shear(nx, ny, 12.0, 4.0, 0.0)
    y = np.arange(ny) + 0.5
    x = np.arange(nx) + 0.5
    r = np.sqrt((x[None, :] - 20.0) ** 2 + (y[:, None] - 2.0) ** 2)
    st["phi"] = np.tanh(2.0 * (12.0 - r) / 4.0)
    wet = (0, 0, math.cos(math.radians(60)), math.cos(math.radians(120)), 0, 0)
    cfg = acm_mod.make_config(2, nx, ny, nu=0.08, precision="f64", bc=(2, 2, 1, 1, 0, 0), two_phase=True,
                              sigma=0.01, width=4.0, mobility=0.05, tile=tile, wet_cos=wet)
    g, o = run_both(acm_mod, orc, cfg, st, 60)
    for k in ("drho", "u", "v", "phi"):
        assert rel_l2(g[k], o[k]) <= 1e-12, (k, rel_l2(g[k], o[k]))


def spreading_cfg(acm, nx, ny, nz, precision, theta_deg=60.0, tile=0, faces=(2, 2, 2, 2, 1, 1)):
    """Drop spreading on a wall (Sec. 3.6): symmetry planes on the sides, no-slip
    walls top and bottom, contact angle theta on the bottom wall (z = 0)."""
    wet = [0.0] * 6
    if faces[4] == 1:
        wet[4] = math.cos(math.radians(theta_deg))
    return acm.make_config(3, nx, ny, nz, nu=0.08, precision=precision, bc=faces, two_phase=True, sigma=0.01,
                           width=3.2, mobility=0.05, tile=tile, wet_cos=wet)


@pytest.mark.parametrize("faces", [(2, 2, 2, 2, 1, 1), (0, 0, 0, 0, 0, 0), (1, 1, 0, 0, 2, 1)])
@pytest.mark.parametrize("tile", [0, 3 | (1 << 8)])
def test_twophase_3d_fp64(acm_mod, orc, faces, tile):
    """3D two-phase step (D3Q19-weighted stencils, wetting on walls) on a
    ragged 21 x 18 x 19 grid: FP64 against the oracle."""
    nx, ny, nz = 21, 18, 19
    st = inputs.drop_on_wall_3d(nx, ny, nz, 8.0, 3.2, center=(0.0, 0.0, 0.0))
    rng = np.random.Generator(np.random.PCG64(17))
    st["u"] = 0.01 * rng.uniform(-1, 1, size=st["u"].shape)
    st["drho"] = 1e-4 * rng.uniform(-1, 1, size=st["u"].shape)
    cfg = spreading_cfg(acm_mod, nx, ny, nz, "f64", tile=tile, faces=faces)
    if faces[0] == 1:
        cfg.wet_cos[0] = math.cos(math.radians(135))
    g, o = run_both(acm_mod, orc, cfg, st, 12)
    for k in ("drho", "u", "v", "w", "phi"):
        assert rel_l2(g[k], o[k]) <= 1e-12, (faces, k, rel_l2(g[k], o[k]))


def test_twophase_3d_fp32(acm_mod, orc):
    """FP32 3D drop spreading (32^3, theta = 60 degrees), 200 steps against
    the FP64 oracle: phi <= 1e-5, velocity <= 1e-4, drho <= 1e-3.  The flow
    is driven only by phi grad mu from rest: FP32 storage of phi alone moves
    the velocity by ~1.4e-5 (CPU storage-emulation test), so the 2e-5 of the
    Taylor-Green case cannot hold here."""
    n = 32
    st = to_f32(inputs.drop_on_wall_3d(n, n, n, 12.0, 3.2, center=(0.0, 0.0, 0.0)))
    cfg = spreading_cfg(acm_mod, n, n, n, "f32")
    g, o = run_both(acm_mod, orc, cfg, st, 200)
    print(f"3D two-phase fp32: phi {rel_l2(g['phi'], o['phi']):.2e} vel {rel_l2_vec(g, o, ('u', 'v', 'w')):.2e} "
          f"drho {rel_l2(g['drho'], o['drho']):.2e}")
    assert rel_l2(g["phi"], o["phi"]) <= 1e-5
    assert rel_l2_vec(g, o, ("u", "v", "w")) <= 1e-4
    assert rel_l2(g["drho"], o["drho"]) <= 1e-3


def jumping_case(acm, NL, precision):
    """The coalescence geometry of Sec. 3.7 at NL nodes per drop radius: the
    quarter domain [0, 3] x [0, 3] x [0, 5] R with symmetry planes at the
    four sides (the plane x = 0 mirrors the drop into its coalescing
    partner), a non-wetting wall (contact angle 180 degrees) at z = 0 and a
    wall at z = 5R; one drop of radius R centred at (R, 0, R).  Lattice
    parameters: capillary-inertial speed 1/40, Oh = 0.119, W = 3, Pe = 2000
    (the Sec. 3.7 values c = 10, Cn = 0.1, Pe = 8000 leave the run unstable
    at this resolution)."""
    U = 1.0 / 40
    sigma = NL * U * U
    nu = 0.119 * U * NL
    M = U * NL * NL / (2000.0 * sigma)
    wet = [0.0] * 6
    wet[4] = -1.0
    cfg = acm.make_config(3, 3 * NL, 3 * NL, 5 * NL, nu=nu, precision=precision, bc=(2, 2, 2, 2, 1, 1),
                          two_phase=True, sigma=sigma, width=3.0, mobility=M, wet_cos=wet)
    st = inputs.drop_on_wall_3d(3 * NL, 3 * NL, 5 * NL, float(NL), 3.0, center=(float(NL), 0.0, float(NL)))
    return cfg, st


def test_twophase_3d_nonwetting_coalescence_fp64(acm_mod, orc):
    """Sec. 3.7 geometry at 10 nodes per radius (30 x 30 x 50), contact angle
    180 degrees, 150 steps: FP64 against the oracle at 1e-12 (the wall value
    of the wetting condition with the mirror value clamped to +-1 on both
    sides)."""
    cfg, st = jumping_case(acm_mod, 10, "f64")
    g, o = run_both(acm_mod, orc, cfg, st, 150)
    for k in ("drho", "u", "v", "w", "phi"):
        assert rel_l2(g[k], o[k]) <= 1e-12, (k, rel_l2(g[k], o[k]))
    assert np.abs(o["w"]).max() > 1e-4  # the drops are moving


def test_twophase_3d_nonwetting_coalescence_fp32(acm_mod, orc):
    cfg, st = jumping_case(acm_mod, 10, "f32")
    st = to_f32(st)
    g, o = run_both(acm_mod, orc, cfg, st, 150)
    assert rel_l2(g["phi"], o["phi"]) <= 1e-5
    assert rel_l2_vec(g, o, ("u", "v", "w")) <= 1e-4
    assert rel_l2(g["drho"], o["drho"]) <= 1e-3


def test_twophase_3d_full_size_one_step(acm_mod, orc):
    """96^3 drop spreading (N_L = 32, Cn = 0.1, the bench workload), FP32:
    one step node by node against the oracle."""
    n = 96
    st = to_f32(inputs.drop_on_wall_3d(n, n, n, 32.0, 3.2, center=(0.0, 0.0, 0.0)))
    cfg = spreading_cfg(acm_mod, n, n, n, "f32")
    s = acm_mod.Solver(cfg, st)
    s.step()
    g = s.state()
    s.close()
    o = orc.step(oparams(orc, cfg), st)
    assert np.abs(g["phi"] - o["phi"]).max() < 1e-6
    umax = max(np.abs(o[k]).max() for k in ("u", "v", "w"))
    for k in ("u", "v", "w"):
        assert np.abs(g[k] - o[k]).max() / umax < 1e-5, k


# --- diagnostics ----------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_diagnostics_match_oracle(acm_mod, orc, dim):
    shape = (20, 24, 28) if dim == 3 else (40, 56)
    st = inputs.seeded_state(shape, seed=8, scale_u=0.03, scale_r=1e-3, two_phase=(dim == 2))
    wu = [[0.0] * 3 for _ in range(6)]
    wu[3] = [0.04, 0, 0]
    faces = (0, 0, 1, 1, 2, 2) if dim == 3 else (0, 0, 1, 1, 0, 0)
    kw = dict(two_phase=True, sigma=0.01, width=4.0, mobility=0.02) if dim == 2 else {}
    cfg = acm_mod.make_config(dim, shape[-1], shape[-2], shape[0] if dim == 3 else 1, nu=0.05,
                              precision="f64", bc=faces, wall_u=wu, dx=0.5, dt=0.25, **kw)
    s = acm_mod.Solver(cfg, st)
    s.run(3)
    prev = None
    d = s.diagnostics()
    cur = s.state()
    w = s.current()[0]
    prev = {k: t.cpu().double().numpy() for k, t in s.sets[1 - w].items()}
    od = orc.diag(oparams(orc, cfg), cur, prev)
    for k in ("mass", "mom_x", "mom_y", "mom_z", "ke", "dumax", "umax", "enstrophy", "energy", "div_rms",
              "div_max", "phi_sum"):
        assert d[k] == pytest.approx(od[k], rel=1e-11, abs=1e-15), k
    assert d["nonfinite"] == 0 and d["step"] == 3


def test_diagnostics_flag_nonfinite(acm_mod):
    st = inputs.seeded_state((16, 16), seed=1)
    st["u"][3, 4] = np.nan
    s = acm_mod.Solver(acm_mod.make_config(2, 16, 16, nu=0.05, precision="f32"), st)
    d = s.diagnostics()
    assert d["nonfinite"] == 1
    with pytest.raises(acm_mod.AcmError):
        s.diagnostics(raise_nonfinite=True)


def test_checkpoint_resume_bitwise(acm_mod):
    """One-step scheme: a state plus its step count is a full checkpoint;
    N steps equal k steps, save, restore into a fresh handle, N-k steps."""
    st = to_f32(tgv64())
    cfg = acm_mod.make_config(2, 64, 64, nu=0.01, precision="f32", graph_chunk=16)
    a = acm_mod.Solver(cfg, st)
    a.run(100)
    full = a.state()
    b = acm_mod.Solver(cfg, st)
    b.run(37)
    ck = b.state()
    c = acm_mod.Solver(cfg, ck)
    c.set_current(0, 37)
    c.run(63)
    out = c.state()
    for k in full:
        assert np.array_equal(full[k], out[k])
