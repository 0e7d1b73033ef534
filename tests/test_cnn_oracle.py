"""Pins of the FP64 network reference against finite differences, an
independent convolution routine and closed forms."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def cnn():
    from oracle import cnn
    return cnn


def small_params(cnn, seed=0, channels=(3, 4, 5, 3)):
    return cnn.init_params(seed, channels=channels, last_scale=1.0)


def test_conv_matches_torch_circular(cnn):
    """Cross-check with torch.nn.functional.conv2d (CPU, FP64, circular pad)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.standard_normal((7, 9, 4))
    w = rng.standard_normal((9, 5, 4))
    b = rng.standard_normal(5)
    ours = cnn.conv(x, w, b)
    # torch weight [out, in, kh, kw] with kh index = dy + 1, kw index = dx + 1
    wt = np.zeros((5, 4, 3, 3))
    for t, (dy, dx) in enumerate(cnn.TAPS):
        wt[:, :, dy + 1, dx + 1] = w[t]
    xt = torch.from_numpy(x.transpose(2, 0, 1)[None]).double()
    xp = torch.nn.functional.pad(xt, (1, 1, 1, 1), mode="circular")
    ref = torch.nn.functional.conv2d(xp, torch.from_numpy(wt).double(), torch.from_numpy(b).double())
    np.testing.assert_allclose(ours, ref[0].numpy().transpose(1, 2, 0), rtol=1e-12, atol=1e-12)


def test_conv_delta_kernel_is_shift(cnn):
    """A one-hot tap weight reproduces a circular shift exactly."""
    rng = np.random.Generator(np.random.PCG64(2))
    x = rng.standard_normal((6, 5, 2))
    for t, (dy, dx) in enumerate(cnn.TAPS):
        w = np.zeros((9, 2, 2))
        w[t] = np.eye(2)
        y = cnn.conv(x, w, np.zeros(2))
        np.testing.assert_array_equal(y, np.roll(x, shift=(-dy, -dx), axis=(0, 1)))


def test_gradients_match_central_differences(cnn):
    """d loss / d params and d loss / d input of a tiny net against central
    differences (h = 1e-6): relative error <= 1e-7."""
    rng = np.random.Generator(np.random.PCG64(3))
    params = small_params(cnn, seed=4)
    x0 = rng.standard_normal((5, 6, 3))
    tgt = rng.standard_normal((5, 6, 3))

    def loss_of(ps):
        raw, _ = cnn.forward(ps, x0)
        return cnn.mse_loss_and_grad(raw, tgt)[0]

    raw, acts = cnn.forward(params, x0)
    _, g = cnn.mse_loss_and_grad(raw, tgt)
    grads = cnn.backward(params, acts, g)
    h = 1e-6
    for l in range(len(params)):
        for k in range(2):
            p = params[l][k]
            flat = p.reshape(-1)
            idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
            for i in idx:
                old = flat[i]
                flat[i] = old + h
                lp = loss_of(params)
                flat[i] = old - h
                lm = loss_of(params)
                flat[i] = old
                fd = (lp - lm) / (2 * h)
                an = grads[l][k].reshape(-1)[i]
                assert abs(fd - an) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (l, k, i, fd, an)


def test_adam_first_step_is_lr_times_sign(cnn):
    """Closed form: after one Adam step from zero moments the update is
    -lr * g / (|g| + eps), i.e. about -lr * sign(g)."""
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    cnn.adam_step(p, g, m, v, t=1, lr=0.01)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_box_filter_and_prolongation(cnn):
    """Box filter preserves the mean; bilinear prolongation is exact on
    constants and on fields linear along a period-free direction slice, and
    filtering the prolonged field of a smooth mode changes it by O(k^2)."""
    rng = np.random.Generator(np.random.PCG64(5))
    f = rng.standard_normal((16, 24))
    c = cnn.box_filter(f, 4)
    assert c.shape == (4, 6)
    assert c.mean() == pytest.approx(f.mean(), abs=1e-14)
    np.testing.assert_allclose(cnn.prolong_bilinear(np.full((4, 6), 2.5), 4), 2.5, rtol=0, atol=1e-15)
    n = 64
    y = (np.arange(n // 4) * 4 + 1.5) * 2 * np.pi / n
    cm = np.broadcast_to(np.sin(y)[:, None], (n // 4, n // 4)).copy()
    fine = cnn.prolong_bilinear(cm, 4)
    yf = np.arange(n) * 2 * np.pi / n
    assert np.abs(fine - np.sin(yf)[:, None]).max() < (2 * np.pi * 4 / n) ** 2 / 8 + 1e-12


def test_box_filter_block_assignment_one_hot(cnn):
    """Every fine node (J, I) of a non-square 12 x 20 grid, factor 4, as a
    one-hot field: the filtered field is 1/16 at coarse node (J // 4, I // 4)
    and zero elsewhere (coarse node (K, L) averages fine rows 4K..4K+3 and
    columns 4L..4L+3; a transposed, strided or shifted block assignment fails
    for some node).  A factor-2 filter of the same field puts 1/4 at
    (J // 2, I // 2)."""
    H, W = 12, 20
    for J in range(H):
        for I in range(W):
            f = np.zeros((H, W))
            f[J, I] = 1.0
            for r in (4, 2):
                c = cnn.box_filter(f, r)
                assert c.shape == (H // r, W // r)
                e = np.zeros((H // r, W // r))
                e[J // r, I // r] = 1.0 / (r * r)
                np.testing.assert_array_equal(c, e)


def test_prolongation_places_coarse_nodes_at_block_centres(cnn):
    """Coarse node I sits at fine coordinate r I + (r - 1)/2: prolonging a
    one-hot coarse field gives the tent 1 - |x - x_I| / r around that point
    (product over both axes), periodic, and the fine values of each coarse
    block average back to the tent's cell averages; a linear field in a
    period-free slice is reproduced exactly."""
    Hc, Wc, r = 5, 6, 4
    for K, L in [(0, 0), (2, 3), (4, 5)]:
        c = np.zeros((Hc, Wc))
        c[K, L] = 1.0
        f = cnn.prolong_bilinear(c, r)
        yc, xc = r * K + (r - 1) / 2, r * L + (r - 1) / 2
        def tent(pos, centre, n):
            d = np.abs(pos - centre)
            d = np.minimum(d, n - d)  # periodic distance
            return np.clip(1 - d / r, 0, None)
        ty = tent(np.arange(Hc * r), yc, Hc * r)
        tx = tent(np.arange(Wc * r), xc, Wc * r)
        np.testing.assert_allclose(f, ty[:, None] * tx[None, :], rtol=0, atol=1e-15)
