"""GPU tests of the two-step 3D launch (level n -> n+2 in one z-march, used by
acm_run on fully periodic boxes under tile codes 14 and 15): FP64 against the oracle to 1e-12 on
ragged grids and ragged z chunks, FP32 bit for bit against one-step launches
(tile codes below 14 force one step per launch) on ragged grids, the smallest nz (4) and
the 256^3 benchmark grid, runs through captured graphs of both parities, and
the state one step back that the diagnostics compare with."""
import math

import numpy as np
import pytest

from paper_2012_03525_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("drho", "u", "v", "w")


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import oracle
    from paper_2012_03525_amd import acm
    acm.lib()
    oracle.lib()
    return acm, oracle


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def f32(st):
    return {k: v.astype(np.float32).astype(np.float64) for k, v in st.items()}


def run(acm, cfg, st, nsteps, force_x=None, split=None):
    s = acm.Solver(cfg, st, force_x=force_x)
    for n in (split or [nsteps]):
        s.run(n)
    out = s.state()
    w = s.current()[0]
    other = {k: t.cpu().double().numpy() for k, t in s.sets[1 - w].items()}
    d = s.diagnostics()
    s.close()
    return out, other, d


@pytest.mark.parametrize("shape,tile,nsteps", [((70, 37, 29), 15, 7), ((70, 37, 29), 15 | (1 << 8), 8),
                                               ((33, 20, 5), 15, 5), ((40, 16, 4), 15 | (1 << 8), 6)])
def test_pair_f64_matches_oracle(mods, shape, tile, nsteps):
    """Ragged tiles in x and y, z chunks of 16 over 29 planes, a body force and
    a forcing row, odd and even step counts."""
    acm, oracle = mods
    nx, ny, nz = shape
    st = inputs.seeded_state((nz, ny, nx), seed=nx + ny + nz, scale_u=0.03, scale_r=1e-3)
    fx = 2e-5 * np.sin(2 * np.pi * np.arange(ny) / ny)
    kw = dict(nu=0.03, g=(1e-5, -2e-6, 3e-6))
    cfg = acm.make_config(3, nx, ny, nz, precision="f64", tile=tile, **kw)
    print(f"pair f64 {shape} tile {tile} steps {nsteps}", flush=True)
    got, _, _ = run(acm, cfg, st, nsteps, force_x=fx)
    p = oracle.Params(dim=3, nx=nx, ny=ny, nz=nz, **kw)
    ref = oracle.run(p, st, nsteps, force_x_row=fx)
    for k in KEYS:
        assert rel(got[k], ref[k]) <= 1e-12, k


@pytest.mark.parametrize("shape,pair_tile,chunk", [((100, 52, 40), 14, 0), ((100, 52, 40), 15, 0),
                                                   ((100, 52, 40), 14 | (1 << 8), 6),
                                                   ((64, 24, 4), 14, 4), ((31, 9, 5), 15, 0)])
def test_pair_f32_bitwise_vs_one_step(mods, shape, pair_tile, chunk):
    """Two steps per launch give the bits of one step per launch, for the
    newest state, the state one step back and every diagnostic; graph chunks
    of 6 and 4 steps (3 and 2 launches: both parities of the set flip)."""
    acm, _ = mods
    nx, ny, nz = shape
    st = f32(inputs.seeded_state((nz, ny, nx), seed=7, scale_u=0.03, scale_r=1e-3))
    kw = dict(nu=0.02, g=(2e-6, 0.0, 0.0), precision="f32", graph_chunk=chunk)
    print(f"pair f32 {shape} tile {pair_tile} chunk {chunk}", flush=True)
    a, a_prev, da = run(acm, acm.make_config(3, nx, ny, nz, tile=pair_tile, **kw), st, 23, split=[4, 1, 18])
    b, b_prev, db = run(acm, acm.make_config(3, nx, ny, nz, tile=13, **kw), st, 23, split=[4, 1, 18])
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a_prev[k], b_prev[k]), k
    for k in ("mass", "ke", "dumax", "umax", "enstrophy", "div_rms", "div_max"):
        assert da[k] == db[k], k
    assert da["step"] == db["step"] == 23


def test_pair_full_size_bitwise(mods):
    """The 256^3 Taylor-Green benchmark grid at 64 x 8 with 128-plane
    chunks: 9 steps (4 two-step launches and one one-step launch) equal 9
    one-step launches bit for bit."""
    acm, _ = mods
    n, u0 = 256, 0.05
    nu = u0 * (n / (2 * math.pi)) / 1600.0
    st = f32(inputs.tgv3d(n, u0))
    print("pair f32 256^3", flush=True)
    a, _, _ = run(acm, acm.make_config(3, n, n, n, nu=nu, precision="f32", tile=14), st, 9)
    b, _, _ = run(acm, acm.make_config(3, n, n, n, nu=nu, precision="f32", tile=13), st, 9)
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
