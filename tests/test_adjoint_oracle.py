"""Pins of the FP64 adjoint oracle (the step's vector-Jacobian product and
the unrolled closure loss) against quantities it does not compute itself:
the C oracle's step, a brute-force finite-difference Jacobian of that step,
mass conservation, the numpy network reference's hand-written backward,
and central differences of the unrolled loss."""
import numpy as np
import pytest

from paper_2012_03525_amd import inputs

KEYS = ("drho", "u", "v")


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="module")
def adj():
    from oracle import adjoint
    return adjoint


def params2d(orc, nx, ny, **kw):
    base = dict(dim=2, nx=nx, ny=ny, nu=0.05, g=(2e-5, -1e-5, 0.0))
    base.update(kw)
    return orc.Params(**base)


def force_row(ny, amp=3e-5):
    return amp * np.sin(2 * np.pi * 2 * np.arange(ny) / ny + 0.3)


@pytest.mark.parametrize("sats", [(1.0, 1.0), (0.0, 1.0), (1.0, 0.0)])
def test_torch_step_equals_c_oracle(orc, adj, sats):
    """The differentiable FP64 step reproduces the C oracle's step (2.10)-(2.13)
    with body force and forcing row on a ragged periodic grid."""
    p = params2d(orc, 13, 10, sat_rho=sats[0], sat_mom=sats[1])
    st = inputs.seeded_state((10, 13), seed=5, scale_u=0.05, scale_r=2e-3)
    fx = force_row(10)
    ref = orc.step(p, st, force_x_row=fx)
    ours = adj.step2d_np(p, st, force_x_row=fx)
    for k in KEYS:
        np.testing.assert_allclose(ours[k], ref[k], rtol=0, atol=1e-15, err_msg=k)


def test_torch_step_physical_units(orc, adj):
    """Same with dx, dt != 1 and an explicit sound speed."""
    p = params2d(orc, 8, 12, dx=0.25, dt=0.05, cs=1.3, nu=0.02)
    st = inputs.seeded_state((12, 8), seed=6, scale_u=0.1, scale_r=1e-2)
    ref = orc.step(p, st)
    ours = adj.step2d_np(p, st)
    for k in KEYS:
        np.testing.assert_allclose(ours[k], ref[k], rtol=0, atol=1e-14, err_msg=k)


def test_vjp_equals_transposed_fd_jacobian(orc, adj):
    """Brute force: the full Jacobian of the C oracle's step on a 5x4 grid by
    central differences (h = 1e-6), transposed, applied to random
    cotangents, equals the oracle's vector-Jacobian product."""
    nx, ny = 5, 4
    p = params2d(orc, nx, ny)
    fx = force_row(ny)
    q = inputs.seeded_state((ny, nx), seed=7, scale_u=0.08, scale_r=5e-3)
    n = nx * ny
    flat = np.concatenate([q[k].ravel() for k in KEYS])

    def S(x):
        st = {k: x[i * n:(i + 1) * n].reshape(ny, nx) for i, k in enumerate(KEYS)}
        o = orc.step(p, st, force_x_row=fx)
        return np.concatenate([o[k].ravel() for k in KEYS])

    h = 1e-6
    J = np.empty((3 * n, 3 * n))
    for c in range(3 * n):
        e = np.zeros(3 * n)
        e[c] = h
        J[:, c] = (S(flat + e) - S(flat - e)) / (2 * h)
    rng = np.random.Generator(np.random.PCG64(8))
    for _ in range(3):
        a = rng.standard_normal(3 * n)
        a_d = {k: a[i * n:(i + 1) * n].reshape(ny, nx) for i, k in enumerate(KEYS)}
        g = adj.step2d_vjp(p, q, a_d, force_x_row=fx)
        ours = np.concatenate([g[k].ravel() for k in KEYS])
        ref = J.T @ a
        assert np.linalg.norm(ours - ref) <= 1e-8 * np.linalg.norm(ref)


def test_vjp_of_total_mass_is_density_indicator(orc, adj):
    """sum(drho') = sum(drho) on a periodic grid (continuity in flux form), so
    the adjoint of the cotangent (1, 0, 0) is (1, 0, 0) at any state."""
    p = params2d(orc, 12, 8)
    q = inputs.seeded_state((8, 12), seed=9, scale_u=0.1, scale_r=1e-2)
    a = {"drho": np.ones((8, 12)), "u": np.zeros((8, 12)), "v": np.zeros((8, 12))}
    g = adj.step2d_vjp(p, q, a, force_x_row=force_row(8))
    np.testing.assert_allclose(g["drho"], 1.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(g["u"], 0.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(g["v"], 0.0, rtol=0, atol=1e-14)


def test_vjp_along_random_direction(orc, adj):
    """<adj_q, d> equals <adj_s, (S(q + h d) - S(q - h d)) / 2h> with S the C
    oracle on a 16x12 grid (h = 1e-5; S is rational in q, so the
    difference quotient is accurate to ~h^2)."""
    nx, ny = 16, 12
    p = params2d(orc, nx, ny, nu=0.03)
    fx = force_row(ny)
    q = inputs.seeded_state((ny, nx), seed=10, scale_u=0.05, scale_r=2e-3)
    rng = np.random.Generator(np.random.PCG64(11))
    d = {k: rng.standard_normal((ny, nx)) for k in KEYS}
    a = {k: rng.standard_normal((ny, nx)) for k in KEYS}
    h = 1e-5
    sp = orc.step(p, {k: q[k] + h * d[k] for k in KEYS}, force_x_row=fx)
    sm = orc.step(p, {k: q[k] - h * d[k] for k in KEYS}, force_x_row=fx)
    lhs = sum(float((a[k] * (sp[k] - sm[k])).sum()) for k in KEYS) / (2 * h)
    g = adj.step2d_vjp(p, q, a, force_x_row=fx)
    rhs = sum(float((g[k] * d[k]).sum()) for k in KEYS)
    assert abs(lhs - rhs) <= 1e-7 * abs(rhs)


def _net_params(seed, last_scale=0.5):
    from oracle import cnn
    return cnn.init_params(seed, last_scale=last_scale)


def test_unrolled_one_step_equals_numpy_backward(orc, adj):
    """k = 1: the unrolled loss and its weight gradients equal the numpy
    network reference (explicit backward) applied to base = S(q0), with the
    residual target (F - base) / D on the velocity channels."""
    from oracle import cnn
    nx, ny = 16, 12
    p = params2d(orc, nx, ny)
    fx = force_row(ny)
    q0 = inputs.seeded_state((ny, nx), seed=12, scale_u=0.05, scale_r=2e-3)
    F = inputs.seeded_state((ny, nx), seed=13, scale_u=0.05, scale_r=2e-3)
    params = _net_params(14)
    N = [300.0, 20.0, 20.0]
    D = [0.0, 2e-3, 3e-3]
    loss, gp, _, _ = adj.unrolled_loss(p, params, N, D, q0, [F], force_x_row=fx)
    s = orc.step(p, q0, force_x_row=fx)
    x0 = np.stack([s[k] * N[c] for c, k in enumerate(KEYS)], axis=-1)
    raw, acts = cnn.forward(params, x0)
    e = np.zeros_like(raw)
    for c in (1, 2):
        e[..., c] = raw[..., c] - (F[KEYS[c]] - s[KEYS[c]]) / D[c]
    n_act = 2 * nx * ny
    ref_loss = float((e * e).sum()) / n_act
    grads = cnn.backward(params, acts, 2.0 * e / n_act)
    assert abs(loss - ref_loss) <= 1e-12 * ref_loss
    for l in range(len(params)):
        for i in range(2):
            np.testing.assert_allclose(gp[l][i], grads[l][i], rtol=1e-9, atol=1e-12 * np.abs(grads[l][i]).max())


def test_unrolled_gradients_match_central_differences(orc, adj):
    """k = 3: directional derivatives of the unrolled loss along random
    directions in each layer's weights and in q0 against central
    differences of the loss itself (h = 1e-7, small enough that no ReLU
    input changes sign between the two evaluations)."""
    nx, ny = 16, 8
    p = params2d(orc, nx, ny)
    fx = force_row(ny)
    q0 = inputs.seeded_state((ny, nx), seed=15, scale_u=0.05, scale_r=2e-3)
    targets = [inputs.seeded_state((ny, nx), seed=16 + j, scale_u=0.05, scale_r=2e-3) for j in range(3)]
    params = _net_params(19)
    N = [300.0, 20.0, 20.0]
    D = [0.0, 2e-3, 3e-3]
    loss, gp, gq, states = adj.unrolled_loss(p, params, N, D, q0, targets, force_x_row=fx)
    assert len(states) == 3
    rng = np.random.Generator(np.random.PCG64(20))
    h = 1e-7
    for l in (0, 2, 4):
        d = rng.standard_normal(params[l][0].shape)
        pp = [[w.copy(), b.copy()] for w, b in params]
        pm = [[w.copy(), b.copy()] for w, b in params]
        pp[l][0] += h * d
        pm[l][0] -= h * d
        fd = (adj.unrolled_loss(p, pp, N, D, q0, targets, fx, grads=False)[0]
              - adj.unrolled_loss(p, pm, N, D, q0, targets, fx, grads=False)[0]) / (2 * h)
        an = float((gp[l][0] * d).sum())
        assert abs(fd - an) <= 1e-6 * abs(an), (l, fd, an)
    dq = {k: rng.standard_normal((ny, nx)) * (2e-3 if k == "drho" else 0.05) for k in KEYS}
    fd = (adj.unrolled_loss(p, params, N, D, {k: q0[k] + h * dq[k] for k in KEYS}, targets, fx, grads=False)[0]
          - adj.unrolled_loss(p, params, N, D, {k: q0[k] - h * dq[k] for k in KEYS}, targets, fx,
                              grads=False)[0]) / (2 * h)
    an = sum(float((gq[k] * dq[k]).sum()) for k in KEYS)
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_div_penalty_closed_form(orc, adj):
    """A single Fourier mode u = A cos(2 pi m x / nx) has centred divergence
    -A sin(2 pi m x / nx) sin(2 pi m / nx) / dx, so mean(div^2) =
    A^2 sin^2(2 pi m / nx) / (2 dx^2); the gradient equals central
    differences of the penalty."""
    nx, ny, m, A = 16, 8, 3, 0.7
    p = params2d(orc, nx, ny)
    x = np.arange(nx)
    a = {"u": np.tile(A * np.cos(2 * np.pi * m * x / nx), (ny, 1)), "v": np.zeros((ny, nx))}
    b = {"u": np.zeros((ny, nx)), "v": np.zeros((ny, nx))}
    val, ga, gb = adj.div_penalty(p, a, b, 2.0)
    assert abs(val - 2.0 * A * A * np.sin(2 * np.pi * m / nx) ** 2 / 2.0) <= 1e-14
    rng = np.random.Generator(np.random.PCG64(30))
    a = {k: rng.standard_normal((ny, nx)) for k in ("u", "v")}
    b = {k: rng.standard_normal((ny, nx)) for k in ("u", "v")}
    val, ga, gb = adj.div_penalty(p, a, b, 0.3)
    d = {k: rng.standard_normal((ny, nx)) for k in ("u", "v")}
    h = 1e-6
    fp = adj.div_penalty(p, {k: a[k] + h * d[k] for k in a}, b, 0.3)[0]
    fm = adj.div_penalty(p, {k: a[k] - h * d[k] for k in a}, b, 0.3)[0]
    an = sum(float((ga[k] * d[k]).sum()) for k in a)
    assert abs((fp - fm) / (2 * h) - an) <= 1e-8 * abs(an)
    for k in ("u", "v"):
        np.testing.assert_allclose(gb[k], -ga[k], rtol=0, atol=1e-15)


def test_unrolled_div_penalty_gradient(orc, adj):
    """k = 2 with the divergence penalty: weight gradients against central
    differences of the loss (h = 1e-7)."""
    nx, ny = 16, 8
    p = params2d(orc, nx, ny)
    fx = force_row(ny)
    q0 = inputs.seeded_state((ny, nx), seed=31, scale_u=0.05, scale_r=2e-3)
    targets = [inputs.seeded_state((ny, nx), seed=32 + j, scale_u=0.05, scale_r=2e-3) for j in range(2)]
    params = _net_params(34)
    N = [300.0, 20.0, 20.0]
    D = [0.0, 2e-3, 3e-3]
    kw = dict(force_x_row=fx, div_weight=5e4)
    l1, _, _, _ = adj.unrolled_loss(p, params, N, D, q0, targets, grads=False, force_x_row=fx)
    loss, gp, _, _ = adj.unrolled_loss(p, params, N, D, q0, targets, **kw)
    assert loss > l1
    rng = np.random.Generator(np.random.PCG64(35))
    h = 1e-7
    for l in (1, 4):
        d = rng.standard_normal(params[l][0].shape)
        pp = [[w.copy(), b.copy()] for w, b in params]
        pm = [[w.copy(), b.copy()] for w, b in params]
        pp[l][0] += h * d
        pm[l][0] -= h * d
        fd = (adj.unrolled_loss(p, pp, N, D, q0, targets, grads=False, **kw)[0]
              - adj.unrolled_loss(p, pm, N, D, q0, targets, grads=False, **kw)[0]) / (2 * h)
        an = float((gp[l][0] * d).sum())
        assert abs(fd - an) <= 1e-6 * abs(an), (l, fd, an)


# boundary sets: (bc of the four faces -x, +x, -y, +y; wall velocities)
WALL_CASES = {
    "channel": ((0, 0, 1, 1), {3: (0.02, 0.0)}),            # periodic x, walls in y, moving lid
    "cavity": ((1, 1, 1, 1), {3: (0.03, 0.0), 0: (0.0, -0.01)}),
    "symmetry": ((2, 1, 2, 2), {1: (0.0, 0.015)}),          # symmetry planes and one moving wall
    "mixed": ((1, 2, 0, 0), {}),                            # wall and symmetry in x, periodic y
}


def wall_params(orc, nx, ny, case, **kw):
    bc, moving = WALL_CASES[case]
    wall_u = [[0.0] * 3 for _ in range(6)]
    for f, (a, b) in moving.items():
        wall_u[f][0], wall_u[f][1] = a, b
    return params2d(orc, nx, ny, bc=tuple(bc) + (0, 0), wall_u=wall_u, **kw)


@pytest.mark.parametrize("case", sorted(WALL_CASES))
def test_torch_step_with_walls_equals_c_oracle(orc, adj, case):
    """With walls (halfway, moving or not) and symmetry planes, the
    differentiable step builds its ghosts itself and reproduces the C
    oracle's step, forcing row included, on a ragged grid."""
    p = wall_params(orc, 13, 10, case)
    st = inputs.seeded_state((10, 13), seed=21, scale_u=0.05, scale_r=2e-3)
    fx = force_row(10)
    ref = orc.step(p, st, force_x_row=fx)
    ours = adj.step2d_np(p, st, force_x_row=fx)
    for k in KEYS:
        np.testing.assert_allclose(ours[k], ref[k], rtol=0, atol=2e-15, err_msg=(case, k))


@pytest.mark.parametrize("case", sorted(WALL_CASES))
def test_vjp_with_walls_equals_transposed_fd_jacobian(orc, adj, case):
    """Brute force on 5x4 grids with walls and symmetry planes: the C
    oracle's Jacobian by central differences, transposed, applied to random
    cotangents, equals the oracle's vector-Jacobian product; the ghost
    rules' transposes (a mirrored scalar, a velocity 2 u_w - u or a negated
    normal component) are inside that Jacobian."""
    nx, ny = 5, 4
    p = wall_params(orc, nx, ny, case)
    fx = force_row(ny)
    q = inputs.seeded_state((ny, nx), seed=22, scale_u=0.08, scale_r=5e-3)
    n = nx * ny
    flat = np.concatenate([q[k].ravel() for k in KEYS])

    def S(x):
        st = {k: x[i * n:(i + 1) * n].reshape(ny, nx) for i, k in enumerate(KEYS)}
        o = orc.step(p, st, force_x_row=fx)
        return np.concatenate([o[k].ravel() for k in KEYS])

    h = 1e-6
    J = np.empty((3 * n, 3 * n))
    for c in range(3 * n):
        e = np.zeros(3 * n)
        e[c] = h
        J[:, c] = (S(flat + e) - S(flat - e)) / (2 * h)
    rng = np.random.Generator(np.random.PCG64(23))
    for _ in range(3):
        a = rng.standard_normal(3 * n)
        a_d = {k: a[i * n:(i + 1) * n].reshape(ny, nx) for i, k in enumerate(KEYS)}
        g = adj.step2d_vjp(p, q, a_d, force_x_row=fx)
        ours = np.concatenate([g[k].ravel() for k in KEYS])
        ref = J.T @ a
        assert np.linalg.norm(ours - ref) <= 1e-8 * np.linalg.norm(ref), case


def test_vjp_with_walls_mass_closed_box(orc, adj):
    """In a closed box with resting walls the continuity update conserves
    sum(drho) exactly (the wall flux of the mirrored momentum cancels), so the
    adjoint of the cotangent (1, 0, 0) is (1, 0, 0) there too; with a
    periodic x axis and walls in y the same holds."""
    for case in ("cavity", "channel"):
        bc, _ = WALL_CASES[case]
        p = params2d(orc, 12, 8, bc=tuple(bc) + (0, 0))
        q = inputs.seeded_state((8, 12), seed=24, scale_u=0.1, scale_r=1e-2)
        a = {"drho": np.ones((8, 12)), "u": np.zeros((8, 12)), "v": np.zeros((8, 12))}
        g = adj.step2d_vjp(p, q, a, force_x_row=force_row(8))
        np.testing.assert_allclose(g["drho"], 1.0, rtol=0, atol=1e-14, err_msg=case)
        np.testing.assert_allclose(g["u"], 0.0, rtol=0, atol=1e-14, err_msg=case)
        np.testing.assert_allclose(g["v"], 0.0, rtol=0, atol=1e-14, err_msg=case)
