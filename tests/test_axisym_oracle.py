"""Pins of the axisymmetric oracle step (2D, x axial, y radial, axis on the
-y face): exact discrete fixed points (Hagen-Poiseuille pipe flow, uniform
axial flow, uniform density at rest), exact conservation of sum(r drho), the
approach to the Poiseuille profile from rest, and the parameter checks."""
import numpy as np
import pytest

from paper_2012_03525_amd import inputs

SYM, WALL = 2, 1


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


def pipe(orc, nx, ny, nu, g, **kw):
    return orc.Params(dim=2, nx=nx, ny=ny, nu=nu, g=(g, 0.0, 0.0), bc=(0, 0, SYM, WALL, 0, 0), axisym=True, **kw)


def poiseuille(ny, nu, g):
    """Discrete steady state with the wall halfway above row ny-1 (R = ny):
    u = g (R^2 + 1/4 - r^2) / (4 nu) at r = j + 1/2 (the flux-form radial
    Laplacian of r^2 is exactly 4; the constant 1/4 makes the mirrored wall
    ghost lie on the same parabola)."""
    r = np.arange(ny) + 0.5
    return g * (ny * ny + 0.25 - r * r) / (4.0 * nu)


def test_poiseuille_is_a_fixed_point(orc):
    nx, ny, nu, g = 4, 16, 0.08, 1e-6
    p = pipe(orc, nx, ny, nu, g)
    u = np.tile(poiseuille(ny, nu, g)[:, None], (1, nx))
    st = {"drho": np.zeros((ny, nx)), "u": u, "v": np.zeros((ny, nx))}
    out = orc.step(p, st)
    assert np.max(np.abs(out["u"] - u)) <= 1e-15 * np.max(u)
    assert np.max(np.abs(out["v"])) == 0.0
    assert np.max(np.abs(out["drho"])) == 0.0


def test_pipe_flow_from_rest_reaches_poiseuille(orc):
    """Started from rest, the axially forced pipe flow relaxes to the discrete
    Poiseuille profile (diffusion time R^2/nu = 640 steps; 12,000 steps)."""
    nx, ny, nu, g = 4, 8, 0.1, 1e-6
    p = pipe(orc, nx, ny, nu, g)
    st = {"drho": np.zeros((ny, nx)), "u": np.zeros((ny, nx)), "v": np.zeros((ny, nx))}
    out = orc.run(p, st, 12000)
    ref = poiseuille(ny, nu, g)
    np.testing.assert_allclose(out["u"][:, 0], ref, rtol=1e-6, atol=0)
    assert np.max(np.abs(out["v"])) <= 1e-12 * np.max(ref)


def test_uniform_axial_flow_and_uniform_density_are_fixed_points(orc):
    nx, ny = 6, 10
    p = orc.Params(dim=2, nx=nx, ny=ny, nu=0.05, bc=(0, 0, SYM, SYM, 0, 0), axisym=True)
    st = {"drho": np.full((ny, nx), 3e-3), "u": np.full((ny, nx), 0.04), "v": np.zeros((ny, nx))}
    out = orc.step(p, st)
    for k in st:
        np.testing.assert_allclose(out[k], st[k], rtol=0, atol=1e-17 + 1e-15 * np.abs(st[k]).max())


def test_radial_mass_is_conserved_exactly(orc):
    """sum_j r_j drho_j is invariant (flux form with the axis and wall
    ghosts), for a random state with a moving wall, a body force and 50 steps;
    the unweighted sum is not."""
    nx, ny = 12, 10
    wu = [[0.0] * 3 for _ in range(6)]
    wu[3] = [0.02, 0.0, 0.0]
    p = pipe(orc, nx, ny, 0.05, 2e-6, wall_u=wu)
    st = inputs.seeded_state((ny, nx), seed=41, scale_u=0.03, scale_r=2e-3)
    r = (np.arange(ny) + 0.5)[:, None]
    m0 = float((r * st["drho"]).sum())
    out = orc.run(p, st, 50)
    m1 = float((r * out["drho"]).sum())
    assert abs(m1 - m0) <= 1e-15 * np.abs(r * st["drho"]).sum()
    assert abs(out["drho"].sum() - st["drho"].sum()) > 1e-9


def test_axisym_parameter_checks(orc):
    st = inputs.seeded_state((8, 8), seed=1)
    for kw in (dict(dim=2, nx=8, ny=8, bc=(0, 0, WALL, WALL, 0, 0), axisym=True),     # axis must be a symmetry face
               dict(dim=2, nx=8, ny=8, bc=(0, 0, 0, 0, 0, 0), axisym=True),           # periodic in r
               dict(dim=3, nx=8, ny=8, nz=8, bc=(0, 0, SYM, WALL, 0, 0), axisym=True)):
        with pytest.raises(ValueError):
            orc.step(orc.Params(**kw), dict(st, w=np.zeros((8, 8, 8)), **{k: np.zeros((8, 8, 8)) for k in st}))


def test_radial_vector_laplacian(orc):
    """The viscous term of the radial momentum is nu (L m_r - m_r / r^2): for
    m_r = eps r it vanishes (the flux-form Laplacian of r is exactly 1/r), for
    m_r = eps r^2 it is 3 eps (4 - 1).  Isolated as the difference of two
    steps with different nu and no momentum SAT (continuity does not depend
    on nu), on the rows clear of the outer symmetry face."""
    nx, ny, eps = 4, 12, 1e-4
    r = np.arange(ny) + 0.5
    for power, lap in ((1, 0.0), (2, 3.0)):
        v = np.tile((eps * r ** power)[:, None], (1, nx))
        st = {"drho": np.zeros((ny, nx)), "u": np.zeros((ny, nx)), "v": v}
        outs = [orc.step(orc.Params(dim=2, nx=nx, ny=ny, nu=nu, sat_mom=0.0, bc=(0, 0, SYM, SYM, 0, 0),
                                    axisym=True), st) for nu in (0.02, 0.07)]
        np.testing.assert_array_equal(outs[0]["drho"], outs[1]["drho"])
        rho_n = 1.0 + outs[0]["drho"]
        diff = (outs[1]["v"] - outs[0]["v"]) * rho_n
        np.testing.assert_allclose(diff[:ny - 2], 0.05 * lap * eps, rtol=0, atol=1e-16)  # outputs ~1e-2


def test_axial_momentum_is_conserved_with_a_symmetry_rim(orc):
    """sum_j r_j rho u_z is invariant without body force when the outer radial
    face is a symmetry plane: every axial flux, including the radial flux of
    Pi_zr = rho u_z u_r in face form, telescopes."""
    nx, ny = 10, 8
    p = orc.Params(dim=2, nx=nx, ny=ny, nu=0.04, bc=(0, 0, SYM, SYM, 0, 0), axisym=True)
    st = inputs.seeded_state((ny, nx), seed=42, scale_u=0.04, scale_r=2e-3)
    r = (np.arange(ny) + 0.5)[:, None]

    def mz(s):
        return float((r * (1.0 + s["drho"]) * s["u"]).sum())
    out = orc.run(p, st, 40)
    scale = float((r * np.abs(st["u"])).sum())
    assert abs(mz(out) - mz(st)) <= 1e-15 * scale
    assert abs(float(((1.0 + out["drho"]) * out["u"]).sum()) - float(((1.0 + st["drho"]) * st["u"]).sum())) > 1e-12


def _drop_mu(orc, W, R, nx, ny, axi, sig=0.01):
    p = orc.Params(dim=2, nx=nx, ny=ny, nu=0.1, bc=(0, 0, SYM, SYM, 0, 0), axisym=axi, two_phase=True,
                   sigma=sig, width=W, mobility=0.1)
    return orc.chemical_potential(p, inputs.drop_on_axis(nx, ny, R, W)["phi"])


def test_axisym_chemical_potential_of_a_sphere(orc):
    """For phi = tanh(2 (R - d)/W) centred on the axis, the axisymmetric mu is
    that of a sphere and the planar one that of a circle: their difference is
    the curvature term -kappa psi'(d) / d (psi' = -(2/W)(1 - psi^2)).  Within
    3 % near the interface at W = 8, and second order in dx / W (W = 4 vs 8)."""
    errs = []
    for W, R, nx, ny in ((4.0, 24.0, 96, 48), (8.0, 40.0, 160, 80)):
        kappa = 3 * 0.01 * W / 8
        dmu = _drop_mu(orc, W, R, nx, ny, True) - _drop_mu(orc, W, R, nx, ny, False)
        x = (np.arange(nx) - nx / 2.0)[None, :]
        r = (np.arange(ny) + 0.5)[:, None]
        d = np.sqrt(x * x + r * r)
        psi = np.tanh(2 * (R - d) / W)
        ana = kappa * (2 / W) * (1 - psi * psi) / d
        m = np.abs(d - R) < W
        errs.append(np.abs(dmu[m] - ana[m]).max() / np.abs(ana[m]).max())
    assert errs[1] <= 0.03
    assert errs[0] / errs[1] >= 3.0


def test_axisym_cahn_hilliard_conserves_r_weighted_phi_from_rest(orc):
    """From rest the Cahn-Hilliard update is pure diffusion of mu; summed over
    the axial direction the isotropic cylindrical Laplacian is the radial flux
    form, so sum(r phi) is unchanged by one step (both Heun stages use u^n = 0)
    while the unweighted sum is not."""
    nx, ny, W, R = 48, 32, 4.0, 12.0
    p = orc.Params(dim=2, nx=nx, ny=ny, nu=0.1, bc=(0, 0, SYM, SYM, 0, 0), axisym=True, two_phase=True,
                   sigma=0.01, width=W, mobility=0.1)
    st = inputs.drop_on_axis(nx, ny, R, W)
    rng = np.random.Generator(np.random.PCG64(44))
    st["phi"] = st["phi"] + 0.05 * rng.standard_normal((ny, nx))
    out = orc.step(p, st)
    r = (np.arange(ny) + 0.5)[:, None]
    assert abs(float((r * (out["phi"] - st["phi"])).sum())) <= 1e-14 * float((r * np.abs(st["phi"])).sum())
    assert abs(float((out["phi"] - st["phi"]).sum())) > 1e-3


def test_axisym_diagnostics_are_volume_integrals(orc):
    """Axisymmetric diagnostics weight each node by its cell volume
    2 pi r dx^2: a uniform state drho = c, u = U in a pipe of radius R = ny dx
    and length L = nx dx has mass c pi R^2 L, axial momentum (1 + c) U pi R^2 L,
    kinetic energy U^2 pi R^2 L / 2 and volume-averaged energy U^2 / 2; the
    planar diagnostics of the same arrays are the plain node sums times
    dx^2."""
    nx, ny, dx, c, U = 12, 9, 0.5, 2e-3, 0.04
    st = {"drho": np.full((ny, nx), c), "u": np.full((ny, nx), U), "v": np.zeros((ny, nx))}
    vol = np.pi * (ny * dx) ** 2 * (nx * dx)
    p = orc.Params(dim=2, nx=nx, ny=ny, dx=dx, nu=0.05, bc=(0, 0, SYM, SYM, 0, 0), axisym=True)
    d = orc.diag(p, st)
    assert abs(d["mass"] - c * vol) <= 1e-14 * c * vol
    assert abs(d["mom_x"] - (1 + c) * U * vol) <= 1e-14 * U * vol
    assert abs(d["ke"] - 0.5 * U * U * vol) <= 1e-14 * U * U * vol
    assert abs(d["energy"] - 0.5 * U * U) <= 1e-15
    assert d["div_max"] == 0.0
    pp = orc.Params(dim=2, nx=nx, ny=ny, dx=dx, nu=0.05, bc=(0, 0, SYM, SYM, 0, 0))
    dp = orc.diag(pp, st)
    assert abs(dp["mass"] - c * nx * ny * dx * dx) <= 1e-15


def test_axisym_diagnostic_mass_is_conserved(orc):
    """The volume-integral mass of an axisymmetric run is invariant (it is
    2 pi dx^3 sum((j + 1/2) drho))."""
    nx, ny = 16, 10
    wu = [[0.0] * 3 for _ in range(6)]
    wu[3] = [0.03, 0.0, 0.0]
    p = pipe(orc, nx, ny, 0.05, 2e-6, wall_u=wu)
    st = inputs.seeded_state((ny, nx), seed=46, scale_u=0.03, scale_r=2e-3)
    m0 = orc.diag(p, st)["mass"]
    m1 = orc.diag(p, orc.run(p, st, 40))["mass"]
    assert abs(m1 - m0) <= 1e-14 * abs(m0)
