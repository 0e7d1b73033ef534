"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This module holds initial conditions and workload recipes only: none of the
SMAME update arithmetic lives here.  Every generator returns FP64 numpy
arrays (x fastest: shape (ny, nx) in 2D, (nz, ny, nx) in 3D) in lattice units
(dx = dt = 1, c_s^2 = 1/3 unless stated), and draws its random numbers from
numpy's PCG64 with an explicit seed.

Workloads follow the paper's test problems (Sec. 3): the 2D Taylor-Green
vortex (Eq. 3.1), the doubly periodic shear layer (Eq. 3.3), the capillary
wave (Sec. 3.4) and the lid-driven cavity (Sec. 3.2); plus the 3D textbook
Taylor-Green vortex, a drop in simple shear, a forced periodic flow with a
k^-3 initial spectrum and a batch of uneven cases.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List

import numpy as np

CS2 = 1.0 / 3.0


def lattice_from_paper(N_L: int, c: float, Re: float) -> Dict[str, float]:
    """Map the paper's discretisation (N_L segments per L, c = N_t/N_L,
    Sec. 3 opening) to lattice units: U = 1/c, nu = N_L/(c Re), Ma = sqrt(3)/c."""
    return {"u": 1.0 / c, "nu": N_L / (c * Re), "ma": math.sqrt(3.0) / c}


def _grid2(nx: int, ny: int, x0: float, y0: float, h: float):
    x = x0 + h * np.arange(nx)
    y = y0 + h * np.arange(ny)
    return np.meshgrid(x, y, indexing="xy")


def tgv2d(n: int, u0: float, seed: int = 20201206, noise: float = 0.0, L: float = None,
          cs2: float = CS2) -> Dict[str, np.ndarray]:
    """2D Taylor-Green vortex at t = 0 (Eq. 3.1) on a periodic n x n grid.

    Domain [-L, L)^2 with L = n/2 nodes (dx = 1), x_i = -L + i.  drho is the
    initial pressure deviation divided by c_s^2 (p = rho c_s^2, rho0 = 1).
    `noise` adds seeded U[-noise, noise) to u and v."""
    if L is None:
        L = n / 2.0
    X, Y = _grid2(n, n, -L, -L, 1.0)
    k = math.pi / L
    u = -u0 * np.cos(k * X) * np.sin(k * Y)
    v = u0 * np.sin(k * X) * np.cos(k * Y)
    drho = -0.25 * u0 * u0 * (np.cos(2 * k * X) + np.cos(2 * k * Y)) / cs2
    if noise:
        rng = np.random.Generator(np.random.PCG64(seed))
        u = u + rng.uniform(-noise, noise, size=u.shape)
        v = v + rng.uniform(-noise, noise, size=v.shape)
    return {"drho": np.ascontiguousarray(drho), "u": np.ascontiguousarray(u),
            "v": np.ascontiguousarray(v)}


def tgv2d_exact(n: int, u0: float, nu: float, t: float, L: float = None):
    """Analytic velocity of Eq. (3.1) in lattice units at time t."""
    if L is None:
        L = n / 2.0
    X, Y = _grid2(n, n, -L, -L, 1.0)
    k = math.pi / L
    decay = math.exp(-2.0 * nu * k * k * t)
    return -u0 * np.cos(k * X) * np.sin(k * Y) * decay, u0 * np.sin(k * X) * np.cos(k * Y) * decay


def tgv3d(n: int, u0: float, cs2: float = CS2) -> Dict[str, np.ndarray]:
    """Textbook 3D Taylor-Green vortex on a periodic n^3 box of length 2 pi
    (x_i = 2 pi i / n): u = u0 sin x cos y cos z, v = -u0 cos x sin y cos z,
    w = 0, p - p0 = rho0 u0^2/16 (cos 2x + cos 2y)(cos 2z + 2)."""
    x = 2.0 * math.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    drho = (u0 * u0 / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / cs2
    return {"drho": drho, "u": u, "v": v, "w": w}


def dpsl(n: int, c: float, delta_w: float = 80.0, delta_p: float = 0.05) -> Dict[str, np.ndarray]:
    """Doubly periodic shear layer (Eq. 3.3) on [0,1)^2 with n nodes per side,
    velocities in lattice units (U = 1/c)."""
    h = 1.0 / n
    X, Y = _grid2(n, n, 0.0, 0.0, h)
    u = np.where(Y <= 0.5, np.tanh(delta_w * (Y - 0.25)), np.tanh(delta_w * (0.75 - Y)))
    v = delta_p * np.sin(2.0 * math.pi * (X + 0.25))
    return {"drho": np.zeros_like(u), "u": u / c, "v": v / c}


def couette_profile(ny: int, u_wall: float) -> np.ndarray:
    """Linear profile between halfway walls (nodes at y = j + 1/2, walls at
    y = 0 and y = ny) moving at -u_wall (bottom) and +u_wall (top)."""
    y = np.arange(ny) + 0.5
    return u_wall * (2.0 * y / ny - 1.0)


def drop_in_shear(nx: int, ny: int, radius: float, width: float, u_wall: float) -> Dict[str, np.ndarray]:
    """Circular drop (phi = +1 inside, tanh profile of width W) centred in a
    Couette flow between halfway walls; periodic in x.  Nodes at (i+1/2, j+1/2)."""
    X, Y = _grid2(nx, ny, 0.5, 0.5, 1.0)
    r = np.sqrt((X - nx / 2.0) ** 2 + (Y - ny / 2.0) ** 2)
    phi = np.tanh(2.0 * (radius - r) / width)
    u = np.broadcast_to(couette_profile(ny, u_wall)[:, None], (ny, nx)).copy()
    return {"drho": np.zeros((ny, nx)), "u": u, "v": np.zeros((ny, nx)), "phi": phi}


def capillary_wave(N_L: int, Cn: float, amp: float = 0.01, h_eq: float = 0.5) -> Dict[str, np.ndarray]:
    """Capillary wave of Sec. 3.4 on [0,1]^2: periodic x (x_i = i dx), walls at
    y = 0, 1 with nodes at y_j = (j + 1/2) dx; phi = tanh(2 (y - h(x)) / Cn),
    h(x) = h_eq + A cos(k (x + 0.5)), k = 2 pi."""
    h = 1.0 / N_L
    X, Y = _grid2(N_L, N_L, 0.0, 0.5 * h, h)
    hx = h_eq + amp * np.cos(2.0 * math.pi * (X + 0.5))
    phi = np.tanh(2.0 * (Y - hx) / Cn)
    z = np.zeros_like(phi)
    return {"drho": z.copy(), "u": z.copy(), "v": z.copy(), "phi": phi}


def _stream_velocity_periodic(psi_hat: np.ndarray, n: int):
    k = np.fft.fftfreq(n, d=1.0 / n)
    KY, KX = np.meshgrid(k, k, indexing="ij")
    u = np.real(np.fft.ifft2(1j * KY * psi_hat))
    v = np.real(np.fft.ifft2(-1j * KX * psi_hat))
    return u, v


def random_spectrum_field(n: int, seed: int, u_rms: float, kmax: int = 16,
                          slope: float = -3.0) -> Dict[str, np.ndarray]:
    """Divergence-free periodic velocity on a 2 pi box with energy spectrum
    E(k) ~ k^slope on 1 <= |k| <= kmax and seeded random phases, built from a
    stream function and scaled to the given rms velocity.  drho = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.fft.fftfreq(n, d=1.0 / n)
    KY, KX = np.meshgrid(k, k, indexing="ij")
    kk = np.sqrt(KX ** 2 + KY ** 2)
    band = (kk >= 1.0) & (kk <= kmax)
    amp = np.zeros_like(kk)
    # E(k) ~ k^slope in a shell of circumference 2 pi k: |u_k|^2 ~ k^(slope-1),
    # |psi_k| = |u_k| / k.
    amp[band] = kk[band] ** ((slope - 1.0) / 2.0) / kk[band]
    phase = rng.uniform(0.0, 2.0 * math.pi, size=kk.shape)
    psi_hat = amp * np.exp(1j * phase)
    u, v = _stream_velocity_periodic(psi_hat, n)
    s = u_rms / math.sqrt(np.mean(u * u + v * v))
    return {"drho": np.zeros((n, n)), "u": u * s, "v": v * s}


def low_mode_perturbation(n: int, seed: int, amp: float, walls: bool) -> Dict[str, np.ndarray]:
    """Divergence-free velocity perturbation over modes 1-2 from a seeded
    stream function, scaled to max |u'| = amp.  With walls the modes vanish on
    the boundary (sin basis); otherwise they are periodic."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = (np.arange(n) + 0.5) / n if walls else np.arange(n) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = np.zeros((n, n))
    v = np.zeros((n, n))
    for mx in (1, 2):
        for my in (1, 2):
            a = rng.standard_normal()
            if walls:
                # psi = a sin(mx pi x)^2 sin(my pi y)^2 vanishes with its gradient on the walls
                sx, sy = np.sin(mx * math.pi * X), np.sin(my * math.pi * Y)
                dsx = 2 * sx * np.cos(mx * math.pi * X) * mx * math.pi
                dsy = 2 * sy * np.cos(my * math.pi * Y) * my * math.pi
                u += a * sx * sx * dsy
                v -= a * dsx * sy * sy
            else:
                ph1, ph2 = rng.uniform(0, 2 * math.pi, size=2)
                kx, ky = 2 * math.pi * mx, 2 * math.pi * my
                # psi = a cos(kx x + ph1) cos(ky y + ph2)
                u += -a * ky * np.cos(kx * X + ph1) * np.sin(ky * Y + ph2)
                v -= -a * kx * np.sin(kx * X + ph1) * np.cos(ky * Y + ph2)
    s = amp / max(np.sqrt(u * u + v * v).max(), 1e-300)
    return {"u": u * s, "v": v * s}


@dataclass
class BatchCase:
    index: int
    n: int
    kind: str          # "tgv" (periodic) or "cavity" (four walls, lid on +y)
    re: float
    nu: float
    u_ref: float
    nsteps: int
    state: Dict[str, np.ndarray]


def batch_cases(ncases: int = 512, seed: int = 4, sizes=tuple(range(32, 257, 16)),
                u_ref: float = 0.05, chunk: int = 500, amp: float = 1e-3,
                with_state: bool = True) -> List[BatchCase]:
    """The batched sweep: grid sizes uniform over `sizes`, even index periodic
    Taylor-Green (L = n/2), odd index lid-driven cavity (L = n, lid u_ref),
    Re log-uniform in [100, 5000], seeded low-mode perturbations of amplitude
    `amp`; each case runs chunk * ceil(20 n / chunk) steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.choice(np.asarray(sizes), size=ncases)
    res = np.exp(rng.uniform(math.log(100.0), math.log(5000.0), size=ncases))
    out = []
    for i in range(ncases):
        n = int(ns[i])
        kind = "tgv" if i % 2 == 0 else "cavity"
        L = n / 2.0 if kind == "tgv" else float(n)
        nu = u_ref * L / float(res[i])
        nsteps = chunk * int(math.ceil(20.0 * n / chunk))
        st = None
        if with_state:
            if kind == "tgv":
                st = tgv2d(n, u_ref)
            else:
                z = np.zeros((n, n))
                st = {"drho": z.copy(), "u": z.copy(), "v": z.copy()}
            pert = low_mode_perturbation(n, seed * 100003 + i, amp, walls=(kind == "cavity"))
            st["u"] = st["u"] + pert["u"]
            st["v"] = st["v"] + pert["v"]
        out.append(BatchCase(i, n, kind, float(res[i]), nu, u_ref, nsteps, st))
    return out


def drop_on_wall_3d(nx: int, ny: int, nz: int, radius: float, width: float,
                    center=(0.0, 0.0, 0.0)) -> Dict[str, np.ndarray]:
    """Spherical drop (phi = +1 inside, tanh profile of width W) centred at
    `center` in node coordinates where node (i, j, k) sits at (i + 1/2,
    j + 1/2, k + 1/2); with the centre on the z = 0 wall it is the hemisphere
    of the drop-spreading problem (Sec. 3.6).  Fluid at rest, drho = 0."""
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    phi = np.tanh(2.0 * (radius - r) / width)
    zero = np.zeros_like(phi)
    return {"drho": zero.copy(), "u": zero.copy(), "v": zero.copy(), "w": zero.copy(), "phi": phi}


def seeded_state(shape, seed: int, scale_u: float = 0.02, scale_r: float = 1e-3,
                 two_phase: bool = False) -> Dict[str, np.ndarray]:
    """Smooth-plus-noise random state for parity tests (not a physical flow)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    st = {"drho": scale_r * rng.uniform(-1, 1, size=shape),
          "u": scale_u * rng.uniform(-1, 1, size=shape),
          "v": scale_u * rng.uniform(-1, 1, size=shape)}
    if len(shape) == 3:
        st["w"] = scale_u * rng.uniform(-1, 1, size=shape)
    if two_phase:
        st["phi"] = rng.uniform(-1, 1, size=shape)
    return st


def pipe_state(nx: int, ny: int, seed: int, u_amp: float = 0.04, r_amp: float = 1e-3) -> Dict[str, np.ndarray]:
    """Axisymmetric test state on an axial-periodic pipe (x axial, y radial,
    row j at r = (j + 1/2)/ny of the radius): a seeded axial profile
    u_amp (1 - r^2)(1 + 0.3 sin(2 pi x + p1)), a radial velocity
    0.2 u_amp r (1 - r) sin(2 pi x + p2) (odd at the axis, zero at the wall) and
    a density pulse r_amp sum_m a_m cos(2 pi m x + q_m) cos(pi m r)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = ((np.arange(nx) + 0.5) / nx)[None, :]
    r = ((np.arange(ny) + 0.5) / ny)[:, None]
    p1, p2 = rng.uniform(0, 2 * math.pi, size=2)
    u = u_amp * (1 - r * r) * (1 + 0.3 * np.sin(2 * math.pi * x + p1))
    v = 0.2 * u_amp * r * (1 - r) * np.sin(2 * math.pi * x + p2)
    drho = np.zeros((ny, nx))
    for m in (1, 2):
        a, q = rng.standard_normal(), rng.uniform(0, 2 * math.pi)
        drho = drho + r_amp * a * np.cos(2 * math.pi * m * x + q) * np.cos(math.pi * m * r)
    return {"drho": drho, "u": u, "v": v}


def drop_on_axis(nx: int, ny: int, radius: float, width: float) -> Dict[str, np.ndarray]:
    """A drop (phi = +1 inside) of the given radius centred on the axis at the
    middle of an axial period (x axial, row j at r = j + 1/2), at rest:
    phi = tanh(2 (R - d) / W), d the distance to the centre."""
    x = (np.arange(nx) - nx / 2.0)[None, :]
    r = (np.arange(ny) + 0.5)[:, None]
    d = np.sqrt(x * x + r * r)
    z = np.zeros((ny, nx))
    return {"drho": z.copy(), "u": z.copy(), "v": z.copy(), "phi": np.tanh(2.0 * (radius - d) / width)}
