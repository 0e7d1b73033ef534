"""3D fields of 2 GiB and more.  Below 2 GiB per field the z-march addresses
a plane through one descriptor per field plus a scalar byte offset; from
2 GiB on it builds a descriptor per field and plane.  A z-invariant state
must stay z-invariant, and every plane of a 64 x 64 x NZ run must equal,
bit for bit, a 64 x 64 x 4 box run through the small-field path (the per-node
arithmetic is the same; only the addressing differs).  The large fields are
5.2 GB each, so plane byte offsets pass 2^31 and 2^32."""
import numpy as np
import pytest

from paper_2012_03525_amd import inputs

pytestmark = pytest.mark.gpu

NX = NY = 64


@pytest.fixture(scope="module")
def acm_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2012_03525_amd import acm
    acm.lib()
    return acm


@pytest.mark.parametrize("precision,nz_big", [("f32", 320000), ("f64", 160000)])
@pytest.mark.parametrize("walls", [False, True])
def test_wide_field_equals_small_box(acm_mod, precision, nz_big, walls):
    import torch
    dev = torch.device("cuda:0")
    dtype = torch.float32 if precision == "f32" else torch.float64
    faces = (1, 1, 0, 0, 0, 0) if walls else (0, 0, 0, 0, 0, 0)
    wu = [[0.0] * 3 for _ in range(6)]
    if walls:  # x walls moving in the wall plane: the state stays z-invariant
        wu[0] = [0.0, 0.02, 0.01]
        wu[1] = [0.0, -0.01, 0.0]
    plane = inputs.seeded_state((1, NY, NX), seed=31, scale_u=0.03, scale_r=1e-3)
    kw = dict(nu=0.03, precision=precision, bc=faces, wall_u=wu, g=(1e-5, -1e-5, 0.0))

    small = {k: np.repeat(v, 4, axis=0) for k, v in plane.items()}
    if precision == "f32":
        small = {k: v.astype(np.float32).astype(np.float64) for k, v in small.items()}
    s = acm_mod.Solver(acm_mod.make_config(3, NX, NY, 4, **kw), small)
    s.step()
    ref = {k: torch.from_numpy(v[0]).to(dtype) for k, v in s.state().items()}
    s.close()

    names = ("drho", "u", "v", "w")
    nbytes = NX * NY * nz_big * (4 if precision == "f32" else 8)
    assert nbytes > 2 ** 32
    sets = [{k: torch.empty((nz_big, NY, NX), dtype=dtype, device=dev) for k in names} for _ in range(2)]
    for k in names:
        p0 = torch.from_numpy(small[k][0]).to(device=dev, dtype=dtype)
        sets[0][k].copy_(p0.expand(nz_big, NY, NX))
    big = acm_mod.Solver(acm_mod.make_config(3, NX, NY, nz_big, **kw), None, tensors=sets)
    big.step()
    torch.cuda.synchronize()
    which, step = big.current()
    assert step == 1
    out = sets[which]
    zs = sorted({0, 1, 2, nz_big // 2, nz_big - 2, nz_big - 1} |
                {z for z in (2 ** 31 // (nbytes // nz_big) + d for d in (-1, 0, 1)) if z < nz_big} |
                {z for z in (2 ** 32 // (nbytes // nz_big) + d for d in (-1, 0, 1)) if z < nz_big})
    for k in names:
        for z in zs:
            assert torch.equal(out[k][z].cpu(), ref[k]), (k, z)
        assert bool((out[k] == out[k][0:1]).all()), k  # every plane equal
    big.close()
    del sets, out
    torch.cuda.empty_cache()
