"""Pins of the oracle's diagnostics (orc_diag) against closed forms.

The quantities are those of the paper: the kinetic energy E_k of Sec. 3.1
(half the sum of |u|^2 times the cell area, not weighted by rho), the
enstrophy and energy of Eq. (3.4) in Sec. 3.3 (area-weighted means over the
domain, vorticity from centred differences), the steady-state quantity
max | |u|^{n+1} - |u|^n | of Sec. 3.2, max |u|, and the rms and maximum of
the centred divergence (Eq. 2.12) that the continuity update (Eq. 2.10)
differences.

On a periodic grid a centred difference maps sin(a x) to
(sin(a dx)/dx) cos(a x) exactly, so products of single Fourier modes have
discrete derivatives, vorticity and divergence in closed form, and sums of
squared modes over whole periods are exact fractions of the node count.
None of these tests re-types the oracle's expressions; each uses fields
chosen so that a wrong normalisation (1/(2S)), a swapped vorticity
component, a wrong divergence stencil or a rho-weighted energy changes the
value.
"""
import math

import numpy as np
import pytest


def _grid2(n, dx):
    x = np.arange(n) * dx
    return np.meshgrid(x, x, indexing="xy")  # arrays [j, i]: X varies along i


def _grid3(n, dx):
    x = np.arange(n) * dx
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z


N2, DX2 = 32, 0.25
KA2, KB2 = 2 * math.pi * 1 / (N2 * DX2), 2 * math.pi * 3 / (N2 * DX2)   # modes 1 and 3


def _field2(A=0.7, B=0.4, c0=2e-3, d=5e-3):
    """u = A cos(a x) sin(b y), v = -B sin(a x) cos(b y),
    drho = c0 + d cos(a x) sin(b y)."""
    X, Y = _grid2(N2, DX2)
    u = A * np.cos(KA2 * X) * np.sin(KB2 * Y)
    v = -B * np.sin(KA2 * X) * np.cos(KB2 * Y)
    r = c0 + d * np.cos(KA2 * X) * np.sin(KB2 * Y)
    return {"drho": r, "u": u, "v": v}


def test_2d_diagnostics_closed_forms(orc):
    """Sec. 3.1 E_k, Eq. (3.4) Omega and E, mass, momentum, max |u| and the
    divergence of a two-mode 2D field with dx = 0.25.  With
    sa = sin(a dx)/dx, sb = sin(b dx)/dx:
      omega = dv/dx - du/dy = -(B sa + A sb) cos(a x) cos(b y),
      div   = du/dx + dv/dy = (B sb - A sa) sin(a x) sin(b y),
    and each squared product of one sine/cosine per axis sums to N/4."""
    A, B, c0, d = 0.7, 0.4, 2e-3, 5e-3
    p = orc.Params(dim=2, nx=N2, ny=N2, dx=DX2, dt=0.1, nu=0.01)
    st = _field2(A, B, c0, d)
    g = orc.diag(p, st)
    N = N2 * N2
    area = DX2 * DX2
    sa, sb = math.sin(KA2 * DX2) / DX2, math.sin(KB2 * DX2) / DX2
    assert g["mass"] == pytest.approx(c0 * N * area, rel=1e-12)
    # (1 + drho) u: only the d-term correlates with u, sum = d A N / 4
    assert g["mom_x"] == pytest.approx(d * A * N / 4 * area, rel=1e-10)
    assert abs(g["mom_y"]) < 1e-15
    assert g["ke"] == pytest.approx(0.5 * (A * A + B * B) * N / 4 * area, rel=1e-12)
    assert g["energy"] == pytest.approx((A * A + B * B) / 8, rel=1e-12)
    assert g["enstrophy"] == pytest.approx((B * sa + A * sb) ** 2 / 8, rel=1e-12)
    assert g["div_rms"] == pytest.approx(abs(B * sb - A * sa) / 2, rel=1e-12)
    # |sin(a x) sin(b y)| reaches 1 on this grid (x = 2, y = 2/3 of a quarter period)
    X, Y = _grid2(N2, DX2)
    smax = np.abs(np.sin(KA2 * X) * np.sin(KB2 * Y)).max()
    assert g["div_max"] == pytest.approx(abs(B * sb - A * sa) * smax, rel=1e-12)
    # |u|^2 = A^2 X Y + B^2 (1-X)(1-Y) with X = cos^2(a x), Y = sin^2(b y): max at a corner
    assert g["umax"] == pytest.approx(max(A, B), rel=1e-12)
    assert g["nonfinite"] == 0.0


def test_2d_taylor_green_enstrophy_is_the_centred_symbol(orc):
    """Eq. (3.1) at t = 0 on [-L, L)^2 (u = -u0 cos kx sin ky, v = u0 sin kx
    cos ky): the centred vorticity is 2 u0 (sin(k dx)/dx) cos kx cos ky, so
    Omega = u0^2 (sin(k dx)/dx)^2 / 2, E = u0^2 / 4 and the divergence
    vanishes; Omega is not the continuum value u0^2 k^2 / 2."""
    n, L, u0 = 40, 1.0, 0.3
    dx = 2 * L / n
    k = math.pi / L
    x = -L + np.arange(n) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    st = {"drho": np.zeros((n, n)), "u": -u0 * np.cos(k * X) * np.sin(k * Y),
          "v": u0 * np.sin(k * X) * np.cos(k * Y)}
    g = orc.diag(orc.Params(dim=2, nx=n, ny=n, dx=dx, dt=0.01, nu=0.01), st)
    s = math.sin(k * dx) / dx
    assert g["enstrophy"] == pytest.approx(u0 * u0 * s * s / 2, rel=1e-12)
    assert g["enstrophy"] != pytest.approx(u0 * u0 * k * k / 2, rel=1e-3)
    assert g["energy"] == pytest.approx(u0 * u0 / 4, rel=1e-12)
    assert g["div_rms"] < 1e-14 and g["div_max"] < 1e-14


N3, DX3 = 16, 0.5
K3 = [2 * math.pi * m / (N3 * DX3) for m in (1, 2, 3)]


def test_3d_diagnostics_closed_forms(orc):
    """3D field u = A sin(ax) cos(by) cos(cz), v = B cos(ax) sin(by) cos(cz),
    w = C cos(ax) cos(by) sin(cz) with three different modes and amplitudes:
      omega_x = (B sc - C sb) cos sin sin,  omega_y = (C sa - A sc) sin cos sin,
      omega_z = (A sb - B sa) sin sin cos,  div = (A sa + B sb + C sc) cos cos cos,
    each squared product summing to N/8.  Swapping any component's order
    (e.g. dz w - dy v) changes Omega."""
    A, B, C = 0.5, -0.3, 0.2
    a, b, c = K3
    X, Y, Z = _grid3(N3, DX3)
    st = {"drho": np.zeros((N3,) * 3),
          "u": A * np.sin(a * X) * np.cos(b * Y) * np.cos(c * Z),
          "v": B * np.cos(a * X) * np.sin(b * Y) * np.cos(c * Z),
          "w": C * np.cos(a * X) * np.cos(b * Y) * np.sin(c * Z)}
    p = orc.Params(dim=3, nx=N3, ny=N3, nz=N3, dx=DX3, dt=0.1, nu=0.01)
    g = orc.diag(p, st)
    sa, sb, sc = (math.sin(k * DX3) / DX3 for k in (a, b, c))
    om2 = (B * sc - C * sb) ** 2 + (C * sa - A * sc) ** 2 + (A * sb - B * sa) ** 2
    N = N3 ** 3
    vol = DX3 ** 3
    assert g["enstrophy"] == pytest.approx(om2 / 16, rel=1e-12)
    assert g["energy"] == pytest.approx((A * A + B * B + C * C) / 16, rel=1e-12)
    assert g["ke"] == pytest.approx(0.5 * (A * A + B * B + C * C) * N / 8 * vol, rel=1e-12)
    dv = abs(A * sa + B * sb + C * sc)
    assert g["div_rms"] == pytest.approx(dv / math.sqrt(8), rel=1e-12)
    assert g["div_max"] == pytest.approx(dv, rel=1e-12)   # cos cos cos = 1 at the origin
    assert g["umax"] == pytest.approx(max(abs(A), abs(B), abs(C)), rel=1e-12)
    # rho = 1: the momentum of each single-mode component sums to zero
    assert max(abs(g["mom_x"]), abs(g["mom_y"]), abs(g["mom_z"])) < 1e-14
    # a swapped order of one vorticity component would give a different value
    wrong = (C * sb - B * sc) ** 2 + (C * sa - A * sc) ** 2 + (A * sb - B * sa) ** 2
    bad = (B * sb - C * sc) ** 2 + (C * sa - A * sc) ** 2 + (A * sb - B * sa) ** 2
    assert wrong == pytest.approx(om2) and abs(bad - om2) > 1e-3 * om2


def test_3d_momentum_is_rho_weighted_and_energy_is_not(orc):
    """Momentum sums rho u (Sec. 2 evolves rho u), E_k and E sum |u|^2 alone
    (Sec. 3.1, Eq. 3.4): a uniform flow U over a density deviation d cos(ax)
    gives mom_x = U N dx^3 (the cosine sums to zero) and E = U^2 / 2, while a
    deviation correlated with u changes only the momentum."""
    n, dx, U, d = 12, 1.0, 0.05, 0.01
    a = 2 * math.pi / n
    X, Y, Z = _grid3(n, dx)
    st = {"drho": d * np.cos(a * X), "u": U + 0.02 * np.cos(a * X), "v": np.zeros((n,) * 3),
          "w": np.zeros((n,) * 3)}
    g = orc.diag(orc.Params(dim=3, nx=n, ny=n, nz=n, dx=dx, nu=0.01), st)
    N = n ** 3
    assert g["mom_x"] == pytest.approx((U + d * 0.02 / 2) * N, rel=1e-12)
    assert g["energy"] == pytest.approx((U * U + 0.02 ** 2 / 2) / 2, rel=1e-12)
    assert g["mass"] == pytest.approx(0.0, abs=1e-14)


def test_steady_state_quantity_on_constructed_pairs(orc):
    """Sec. 3.2's steady-state test quantity max | |u|^{n+1} - |u|^n |:
    (i) prev = s * current gives |1 - s| max |u|; (ii) a pair that differs in
    one node's direction only gives 0 (the speed is unchanged); (iii) one
    node's speed changed by delta gives delta."""
    p = orc.Params(dim=2, nx=N2, ny=N2, dx=DX2, dt=0.1, nu=0.01)
    st = _field2()
    g0 = orc.diag(p, st)
    prev = {k: v * (0.9 if k in ("u", "v") else 1.0) for k, v in st.items()}
    assert orc.diag(p, st, prev)["dumax"] == pytest.approx(0.1 * g0["umax"], rel=1e-12)
    rot = {k: v.copy() for k, v in st.items()}
    rot["u"][5, 7], rot["v"][5, 7] = st["v"][5, 7], st["u"][5, 7]   # same speed, new direction
    assert orc.diag(p, st, rot)["dumax"] == pytest.approx(0.0, abs=1e-16)
    one = {k: v.copy() for k, v in st.items()}
    sp = math.hypot(st["u"][9, 3], st["v"][9, 3])
    scale = (sp + 0.0123) / sp
    one["u"][9, 3] *= scale
    one["v"][9, 3] *= scale
    assert orc.diag(p, st, one)["dumax"] == pytest.approx(0.0123, rel=1e-10)
    # 3D: the w component enters the speed
    X, Y, Z = _grid3(8, 1.0)
    s3 = {"drho": np.zeros((8,) * 3), "u": np.full((8,) * 3, 0.03), "v": np.zeros((8,) * 3),
          "w": np.full((8,) * 3, 0.04)}
    p3 = orc.Params(dim=3, nx=8, ny=8, nz=8, nu=0.01)
    prev3 = dict(s3, w=np.zeros((8,) * 3))
    g3 = orc.diag(p3, s3, prev3)
    assert g3["umax"] == pytest.approx(0.05, rel=1e-12)
    assert g3["dumax"] == pytest.approx(0.02, rel=1e-12)


def test_wall_ghosts_in_the_diagnostics(orc):
    """Between halfway walls moving at -U and +U (reading of the wall
    discretisation) the linear Couette profile u = U (2 y / H - 1) extends
    through the ghost rows unchanged, so the centred vorticity is -2U/H on
    every row, wall rows included: Omega = (2U/H)^2 / 2 and zero divergence.
    A symmetry plane instead mirrors u (zero shear at the plane), which
    halves the difference across the edge rows."""
    nx, ny, dx, U = 8, 20, 0.5, 0.03
    H = ny * dx
    y = (np.arange(ny) + 0.5) * dx
    u = np.broadcast_to((U * (2 * y / H - 1))[:, None], (ny, nx)).copy()
    st = {"drho": np.zeros((ny, nx)), "u": u, "v": np.zeros((ny, nx))}
    wu = [[0.0] * 3 for _ in range(6)]
    wu[2] = [-U, 0, 0]
    wu[3] = [U, 0, 0]
    pw = orc.Params(dim=2, nx=nx, ny=ny, dx=dx, nu=0.01, bc=(0, 0, 1, 1, 0, 0), wall_u=wu)
    g = orc.diag(pw, st)
    assert g["enstrophy"] == pytest.approx((2 * U / H) ** 2 / 2, rel=1e-12)
    assert g["div_max"] < 1e-16
    ps = orc.Params(dim=2, nx=nx, ny=ny, dx=dx, nu=0.01, bc=(0, 0, 2, 2, 0, 0))
    gs = orc.diag(ps, st)
    # interior rows keep -2U/H; each edge row sees half the difference
    w_in, w_edge = 2 * U / H, 0.5 * 2 * U / H
    expect = (w_in ** 2 * (ny - 2) + 2 * w_edge ** 2) / (2 * ny)
    assert gs["enstrophy"] == pytest.approx(expect, rel=1e-12)


def test_nonfinite_flag(orc):
    p = orc.Params(dim=2, nx=8, ny=8, nu=0.01)
    z = np.zeros((8, 8))
    assert orc.diag(p, {"drho": z, "u": z, "v": z})["nonfinite"] == 0.0
    bad = z.copy()
    bad[3, 4] = np.nan
    assert orc.diag(p, {"drho": bad, "u": z, "v": z})["nonfinite"] == 1.0
    inf = z.copy()
    inf[0, 0] = np.inf
    assert orc.diag(p, {"drho": z, "u": z, "v": inf})["nonfinite"] == 1.0
