"""FP64 adjoint of the 2D SMAME step and the unrolled closure loss
(TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg
of the benchmark may use it; the GPU library never loads it).

The step is written once more, here with PyTorch CPU tensors in FP64, from
the continuity update (2.10) and the momentum update (2.11) with the
centred first derivative (2.12), the five-point Laplacian (2.13) and the
body force of Sec. 2 (rho^{n+1} g, g per row for a forcing profile), on a
grid whose four faces are each periodic, a wall or a symmetry plane:

  rho'  = rho - dt G_a(rho u_a) + s_rho 1/2 cs^2 dt^2 L(rho)
  m'_a  = m_a - dt G_b(Pi_ab) + nu dt L(m_a)
          - s_m (nu + 1/2 cs^2 dt) [G_a(rho') - G_a(rho)] + dt rho' g_a
  Pi_ab = rho u_a u_b + cs^2 drho delta_ab,   u'_a = m'_a / rho'

(drho = rho - rho0 is the stored density variable).  The stencils read one
layer of ghost nodes: a periodic face wraps; a wall (halfway between nodes)
gives the ghost the mirror node's drho and the velocity 2 u_wall - u of the
mirror node; a symmetry plane mirrors drho and the tangential velocity and
negates the normal one; the ghosts of rho^{n+1} are filled by the same
scalar rule (the boundary readings of the C oracle).  Its adjoint, the
vector-Jacobian product adj_q = (dS/dq)^T adj_s, is taken from this forward
by torch.autograd, which is the definition of that product; no hand-derived
transposed stencil is involved.

The unrolled closure loss composes k corrected coarse steps,
q_j = S(q_{j-1}) + D f(N S(q_{j-1})), with the five-layer network of
`cnn.py` (written here with torch's conv2d on circularly padded input), and
averages the normalised squared error of q_j against the targets F_j over
the steps, pixels and the channels with D_c > 0.  An optional term
div_weight * mean(div(q_j - S(q_{j-1}))^2), with div the centred divergence
(2.12) of the velocity, penalises the compressive part of each correction.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import Params

F64 = torch.float64


def _t(a) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a, dtype=np.float64), dtype=F64)


def _E(f):  # f[j, i + 1]
    return torch.roll(f, -1, dims=1)


def _W(f):  # f[j, i - 1]
    return torch.roll(f, 1, dims=1)


def _N(f):  # f[j + 1, i]
    return torch.roll(f, -1, dims=0)


def _S(f):  # f[j - 1, i]
    return torch.roll(f, 1, dims=0)


PERIODIC, WALL, SYMMETRY = 0, 1, 2


def _check(p: Params):
    if p.dim != 2 or p.two_phase or getattr(p, "axisym", False):
        raise ValueError("the adjoint oracle covers the planar 2D single-phase step")
    for lo, hi in ((0, 1), (2, 3)):
        if (int(p.bc[lo]) == PERIODIC) != (int(p.bc[hi]) == PERIODIC):
            raise ValueError("a periodic axis has both faces periodic")


def _ghost(p: Params, face: int, m: torch.Tensor, comp: Optional[int]) -> torch.Tensor:
    """Ghost value across `face` (0..3: -x, +x, -y, +y) of the mirror values m:
    a scalar (comp None) is mirrored; velocity component comp is 2 u_w - m at
    a wall, -m for the normal component at a symmetry plane, m otherwise."""
    kind = int(p.bc[face])
    if comp is None or kind == SYMMETRY and comp != face // 2:
        return m
    if kind == WALL:
        return 2.0 * float(p.wall_u[face][comp]) - m
    return -m


def _pad(p: Params, f: torch.Tensor, comp: Optional[int] = None) -> torch.Tensor:
    """f [ny, nx] with one ghost layer on every side (corners unused)."""
    if int(p.bc[0]) == PERIODIC:
        lo, hi = f[:, -1:], f[:, :1]
    else:
        lo, hi = _ghost(p, 0, f[:, :1], comp), _ghost(p, 1, f[:, -1:], comp)
    f = torch.cat([lo, f, hi], dim=1)
    if int(p.bc[2]) == PERIODIC:
        lo, hi = f[-1:, :], f[:1, :]
    else:
        lo, hi = _ghost(p, 2, f[:1, :], comp), _ghost(p, 3, f[-1:, :], comp)
    return torch.cat([lo, f, hi], dim=0)


def step2d(p: Params, r: torch.Tensor, u: torch.Tensor, v: torch.Tensor,
           force_x_row: Optional[torch.Tensor] = None):
    """One step (2.10)-(2.13) with the body force on a planar 2D grid with
    periodic, wall or symmetry faces; differentiable torch FP64 tensors
    [ny, nx] in, (drho', u', v') out."""
    _check(p)
    dx, dt, nu, cs2, rho0 = p.dx, p.dt, p.nu, p.cs * p.cs, p.rho0
    # level-n fields with their ghosts
    rp, up, vp = _pad(p, r), _pad(p, u, 0), _pad(p, v, 1)
    rhop = rho0 + rp
    mxp, myp = rhop * up, rhop * vp
    C = (slice(1, -1), slice(1, -1))
    mx, my = mxp[C], myp[C]

    def E(f):
        return f[1:-1, 2:]

    def W(f):
        return f[1:-1, :-2]

    def N(f):
        return f[2:, 1:-1]

    def S(f):
        return f[:-2, 1:-1]

    def G_x(f):
        return (E(f) - W(f)) / (2.0 * dx)

    def G_y(f):
        return (N(f) - S(f)) / (2.0 * dx)

    def L(f):
        return (E(f) + W(f) + N(f) + S(f) - 4.0 * f[C]) / (dx * dx)

    rn = r - dt * (G_x(mxp) + G_y(myp)) + p.sat_rho * 0.5 * cs2 * dt * dt * L(rp)
    rnp = _pad(p, rn)  # ghosts of rho^{n+1}
    pxx = mxp * up + cs2 * rp
    pxy = mxp * vp
    pyx = myp * up
    pyy = myp * vp + cs2 * rp
    rho_n = rho0 + rn
    kd = nu + 0.5 * cs2 * dt
    gx = p.g[0] + (force_x_row[:, None] if force_x_row is not None else 0.0)
    gy = p.g[1]
    mxn = (mx - dt * (G_x(pxx) + G_y(pxy)) + nu * dt * L(mxp)
           - p.sat_mom * kd * (G_x(rnp) - G_x(rp)) + dt * rho_n * gx)
    myn = (my - dt * (G_x(pyx) + G_y(pyy)) + nu * dt * L(myp)
           - p.sat_mom * kd * (G_y(rnp) - G_y(rp)) + dt * rho_n * gy)
    return rn, mxn / rho_n, myn / rho_n


def step2d_np(p: Params, st: Dict[str, np.ndarray], force_x_row=None) -> Dict[str, np.ndarray]:
    fx = None if force_x_row is None else _t(force_x_row)
    out = step2d(p, _t(st["drho"]), _t(st["u"]), _t(st["v"]), fx)
    return {k: o.numpy() for k, o in zip(("drho", "u", "v"), out)}


def step2d_vjp(p: Params, q: Dict[str, np.ndarray], adj_s: Dict[str, np.ndarray],
               force_x_row=None) -> Dict[str, np.ndarray]:
    """adj_q = (dS/dq)^T adj_s at state q (numpy FP64 dicts drho, u, v)."""
    xs = [_t(q[k]).requires_grad_(True) for k in ("drho", "u", "v")]
    fx = None if force_x_row is None else _t(force_x_row)
    outs = step2d(p, *xs, fx)
    gs = torch.autograd.grad(outs, xs, grad_outputs=[_t(adj_s[k]) for k in ("drho", "u", "v")])
    return {k: g.numpy() for k, g in zip(("drho", "u", "v"), gs)}


# ---------------------------------------------------------------------------
# unrolled closure loss
# ---------------------------------------------------------------------------
def _conv(x: torch.Tensor, w: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """x [C, H, W]; w [9, C_out, C_in] with tap t = (dy + 1) * 3 + (dx + 1);
    circular 3x3 cross-correlation (the convention of `cnn.conv`)."""
    co, ci = w.shape[1], w.shape[2]
    k = w.reshape(3, 3, co, ci).permute(2, 3, 0, 1)  # [C_out, C_in, dy + 1, dx + 1]
    xp = torch.nn.functional.pad(x[None], (1, 1, 1, 1), mode="circular")
    return torch.nn.functional.conv2d(xp, k, b)[0]


def network(params_t, x: torch.Tensor) -> torch.Tensor:
    """f(x) for x [3, H, W]; params_t: list of (w, b) torch tensors."""
    h = x
    for l, (w, b) in enumerate(params_t):
        h = _conv(h, w, b)
        if l < len(params_t) - 1:
            h = torch.relu(h)
    return h


def divergence(p: Params, u: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
    """Centred divergence G_x u + G_y v (2.12) on a periodic grid."""
    return (_E(u) - _W(u) + _N(v) - _S(v)) / (2.0 * p.dx)


def div_penalty(p: Params, a: Dict[str, np.ndarray], b: Dict[str, np.ndarray], weight: float):
    """weight * mean(div(a - b)^2) and its gradients with respect to the
    velocity of a and of b (numpy dicts u, v)."""
    xs = [_t(a[k]).requires_grad_(True) for k in ("u", "v")] + [_t(b[k]).requires_grad_(True) for k in ("u", "v")]
    d = divergence(p, xs[0] - xs[2], xs[1] - xs[3])
    val = weight * (d * d).mean()
    g = torch.autograd.grad(val, xs)
    return (float(val.detach()), {"u": g[0].numpy(), "v": g[1].numpy()},
            {"u": g[2].numpy(), "v": g[3].numpy()})


def unrolled_loss(p: Params, params, in_scale: Sequence[float], out_scale: Sequence[float],
                  q0: Dict[str, np.ndarray], targets: Sequence[Dict[str, np.ndarray]], force_x_row=None,
                  grads: bool = True, div_weight: float = 0.0):
    """Loss (1/k) sum_j [mean_{pixels, c: D_c > 0} ((q_j - F_j)_c / D_c)^2
    + div_weight mean(div(q_j - s_j)^2)] of k corrected steps from q0
    (s_j = S(q_{j-1}), the uncorrected step), with its gradients with respect
    to every layer's (w, b) [numpy, real channels] and to q0.  Returns (loss,
    grads, adj_q0, states) where states are q_1..q_k."""
    fx = None if force_x_row is None else _t(force_x_row)
    pt = [(_t(w).requires_grad_(grads), _t(b).requires_grad_(grads)) for w, b in params]
    q = [_t(q0[k]).requires_grad_(grads) for k in ("drho", "u", "v")]
    q_in = list(q)
    ns = _t(in_scale)
    ds = [float(d) for d in out_scale]
    active = [c for c in range(3) if ds[c] > 0.0]
    k = len(targets)
    loss = torch.zeros((), dtype=F64)
    states = []
    for tgt in targets:
        s = step2d(p, *q, fx)
        x = torch.stack(list(s)) * ns[:, None, None]
        raw = network(pt, x)
        q = [s[c] + ds[c] * raw[c] if ds[c] > 0.0 else s[c] for c in range(3)]
        states.append({kk: t.detach().numpy().copy() for kk, t in zip(("drho", "u", "v"), q)})
        se = sum((((q[c] - _t(tgt[("drho", "u", "v")[c]])) / ds[c]) ** 2).sum() for c in active)
        loss = loss + se / (len(active) * q[0].numel())
        if div_weight:
            d = divergence(p, q[1] - s[1], q[2] - s[2])
            loss = loss + div_weight * (d * d).mean()
    loss = loss / k
    if not grads:
        return float(loss.detach()), None, None, states
    flat = [t for wb in pt for t in wb]
    g = torch.autograd.grad(loss, flat + q_in)
    gp = [[g[2 * l].numpy(), g[2 * l + 1].numpy()] for l in range(len(pt))]
    gq = {kk: t.numpy() for kk, t in zip(("drho", "u", "v"), g[len(flat):])}
    return float(loss.detach()), gp, gq, states
