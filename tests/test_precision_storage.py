"""Why the FP32 build stores drho (not rho), and what FP32 storage costs.

These CPU tests emulate FP32 *storage* with the FP64 oracle: every step is
computed in FP64 and the state is then rounded to FP32, exactly what a
kernel with FP32 fields and perfect arithmetic would keep.  They fix the
tolerances the GPU parity tests use."""
import math

import numpy as np

from paper_2012_03525_amd import inputs


def rl2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def f32(x):
    return x.astype(np.float32).astype(np.float64)


def test_drho_storage_meets_bound_rho_storage_does_not(orc):
    """2D Taylor-Green 64^2 (u0 = 0.01, nu = 0.01), 1000 steps.  drho is
    O(Ma^2) ~ 7.5e-5; FP32 storage of rho = 1 + drho keeps it only to the
    ~6e-8 spacing of floats near 1, so rho storage fails the 1e-4 drho
    bound while drho storage passes it with margin (negative control)."""
    p = orc.Params(dim=2, nx=64, ny=64, nu=0.01)
    st0 = {k: f32(v) for k, v in inputs.tgv2d(64, 0.01, noise=1e-6).items()}
    ref = orc.run(p, st0, 1000)
    a = dict(st0)
    b = dict(st0)
    for _ in range(1000):
        a = orc.step(p, a)
        a = {k: f32(v) for k, v in a.items()}
        b = orc.step(p, b)
        rho = (1.0 + b["drho"]).astype(np.float32).astype(np.float64)
        b = {"drho": rho - 1.0, "u": f32(b["u"]), "v": f32(b["v"])}
    assert rl2(a["drho"], ref["drho"]) < 2e-5
    assert rl2(a["u"], ref["u"]) < 2e-6
    assert rl2(b["drho"], ref["drho"]) > 1e-4


def test_phase_field_storage_sets_two_phase_drho_bound(orc):
    """Drop in shear 128^2 (R = 16, W = 4), 1000 steps.  Rounding only phi
    to FP32 after each step moves drho by ~3e-4 (relative L2): the pressure
    balances -phi grad mu, whose bulk value depends on phi - (+-1), which
    FP32 resolves only to ~6e-8.  Rounding only the flow fields costs ~1e-6.
    The GPU two-phase FP32 parity test therefore bounds drho at 1e-3 and
    velocity / phi at 2e-5 / 1e-5."""
    wu = [[0.0] * 3 for _ in range(6)]
    wu[2] = [-0.02, 0, 0]
    wu[3] = [0.02, 0, 0]
    p = orc.Params(dim=2, nx=128, ny=128, nu=0.1, bc=(0, 0, 1, 1, 0, 0), wall_u=wu, two_phase=True,
                   sigma=0.01, width=4.0, mobility=0.02)
    st0 = {k: f32(v) for k, v in inputs.drop_in_shear(128, 128, 16.0, 4.0, 0.02).items()}
    ref = orc.run(p, st0, 1000)
    a = dict(st0)
    b = dict(st0)
    for _ in range(1000):
        a = orc.step(p, a)
        a["phi"] = f32(a["phi"])
        b = orc.step(p, b)
        for k in ("drho", "u", "v"):
            b[k] = f32(b[k])
    e_phi_store = rl2(a["drho"], ref["drho"])
    assert 1e-4 < e_phi_store < 1e-3
    assert rl2(b["drho"], ref["drho"]) < 1e-5
    num = np.sqrt(np.sum((a["u"] - ref["u"]) ** 2 + (a["v"] - ref["v"]) ** 2))
    den = np.sqrt(np.sum(ref["u"] ** 2 + ref["v"] ** 2))
    assert num / den < 2e-5
    assert rl2(a["phi"], ref["phi"]) < 1e-5


def test_phase_field_storage_sets_3d_two_phase_velocity_bound(orc):
    """3D drop spreading on a wetting wall (32^3, R = 12, W = 3.2, theta = 60
    degrees), 200 steps.  The flow starts at rest and is driven only by
    phi grad mu, so rounding only phi to FP32 after each step already moves
    the velocity by ~1.4e-5 (relative L2) and drho by ~2.5e-5, while rounding
    only the flow fields costs ~3e-8.  The GPU FP32 test of this case
    therefore bounds the velocity at 1e-4 (FP32 arithmetic adds about as much
    again) instead of the 2e-5 that holds for the Taylor-Green case."""
    n = 32
    p = orc.Params(dim=3, nx=n, ny=n, nz=n, nu=0.08, bc=(2, 2, 2, 2, 1, 1), two_phase=True, sigma=0.01,
                   width=3.2, mobility=0.05, wet_cos=(0, 0, 0, 0, math.cos(math.radians(60)), 0))
    st0 = {k: f32(v) for k, v in inputs.drop_on_wall_3d(n, n, n, 12.0, 3.2).items()}
    ref = orc.run(p, st0, 200)
    a = dict(st0)
    b = dict(st0)
    for _ in range(200):
        a = orc.step(p, a)
        a["phi"] = f32(a["phi"])
        b = orc.step(p, b)
        for k in ("drho", "u", "v", "w"):
            b[k] = f32(b[k])

    def vel(x, y):
        num = np.sqrt(sum(np.sum((x[k] - y[k]) ** 2) for k in ("u", "v", "w")))
        return num / np.sqrt(sum(np.sum(y[k] ** 2) for k in ("u", "v", "w")))
    assert 5e-6 < vel(a, ref) < 5e-5
    assert vel(b, ref) < 1e-6
    assert rl2(a["phi"], ref["phi"]) < 1e-6


def test_batch_cases_storage_error_fits_the_stated_bounds(orc):
    """The four smallest of the first sixteen cases of the seeded 512-case
    sweep (lid-driven cavities up to Re 1082 and a periodic Taylor-Green
    case, 1000-2500 steps), the cases the GPU batch test compares with the
    oracle.  Rounding the whole state to FP32 after every FP64 step moves
    the velocity by at most ~2e-7 and drho by ~3e-6 (relative L2), a
    hundredth of the stated FP32 bounds (u 2e-5, drho 1e-4), which leaves
    room for the FP32 arithmetic; the GPU batch test uses those bounds."""
    allc = inputs.batch_cases(ncases=16, seed=4)
    pick = sorted(allc, key=lambda c: c.n)[:4]
    worst_v = worst_r = 0.0
    for c in pick:
        wu = [[0.0] * 3 for _ in range(6)]
        bc = (0, 0, 0, 0, 0, 0)
        if c.kind == "cavity":
            bc = (1, 1, 1, 1, 0, 0)
            wu[3] = [0.05, 0, 0]
        p = orc.Params(dim=2, nx=c.n, ny=c.n, nu=c.nu, bc=bc, wall_u=wu)
        st0 = {k: f32(v) for k, v in c.state.items()}
        ref = orc.run(p, st0, c.nsteps)
        a = dict(st0)
        for _ in range(c.nsteps):
            a = {k: f32(v) for k, v in orc.step(p, a).items()}
        num = np.sqrt(np.sum((a["u"] - ref["u"]) ** 2 + (a["v"] - ref["v"]) ** 2))
        worst_v = max(worst_v, num / np.sqrt(np.sum(ref["u"] ** 2 + ref["v"] ** 2)))
        worst_r = max(worst_r, rl2(a["drho"], ref["drho"]))
    assert 1e-8 < worst_v < 2e-5 / 50
    assert 1e-7 < worst_r < 1e-4 / 20
