"""Batched launch (both modes): every case must be bitwise equal to the same
case run alone through acm_run, divergence must be isolated to its case,
and sampled cases of the 512-case sweep must match the CPU oracle."""
import ctypes
import math

import numpy as np
import pytest

from paper_2012_03525_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def acm_mod():
    import torch
    assert torch.cuda.is_available()
    from paper_2012_03525_amd import acm
    acm.lib()
    return acm


def f32(st):
    return {k: v.astype(np.float32).astype(np.float64) for k, v in st.items()}


def case_cfg(acm, n_x, n_y, kind, nu, precision="f32", allow_unstable=False):
    wu = [[0.0] * 3 for _ in range(6)]
    if kind == "tgv":
        bc = (0, 0, 0, 0, 0, 0)
    elif kind == "cavity":
        bc = (1, 1, 1, 1, 0, 0)
        wu[3] = [0.05, 0, 0]
    elif kind == "channel":
        bc = (0, 0, 1, 2, 0, 0)
        wu[2] = [0.02, 0, 0]
    else:
        bc = (2, 2, 1, 1, 0, 0)
        wu[3] = [-0.03, 0, 0]
    return acm.make_config(2, n_x, n_y, nu=nu, precision=precision, bc=bc, wall_u=wu,
                           allow_unstable=allow_unstable)


SPECS = [  # (nx, ny, kind, tile, nsteps)
    (32, 32, "tgv", -1, 20),
    (48, 48, "cavity", 1, 40),
    (70, 45, "channel", 3, 20),
    (64, 64, "sym", 5, 60),
    (100, 36, "cavity", 4, 40),
    (33, 57, "tgv", 2, 20),
]


def spec_state(nx, ny, seed):
    return f32(inputs.seeded_state((ny, nx), seed=seed, scale_u=0.03, scale_r=1e-3))


@pytest.mark.parametrize("mode,grab,blocks,prec", [(0, 0, 0, "f32"), (1, 0, 0, "f32"), (1, 4, 0, "f32"),
                                                  (1, 3, 0, "f32"), (1, 2, 5, "f32"), (1, 1, 13, "f32"),
                                                  (0, 0, 0, "f64"), (1, 3, 0, "f64")])
def test_batch_bitwise_equals_single_runs(acm_mod, mode, grab, blocks, prec):
    """Every tile shape, walls, symmetry planes and ragged grids.  Mode 1 with
    the default grid (most workgroups get no fixed share and claim at once),
    claims of three or four items (ranges that end inside a case), five
    workgroups (five groups of one, hundreds of items each in fixed shares)
    and thirteen (eight groups of one or two workgroups)."""
    cfgs = [case_cfg(acm_mod, nx, ny, kind, 0.04, precision=prec) for nx, ny, kind, _, _ in SPECS]
    states = [spec_state(nx, ny, 100 + i) for i, (nx, ny, _, _, _) in enumerate(SPECS)]
    b = acm_mod.Batch(cfgs, states, [s[4] for s in SPECS], tiles=[s[3] for s in SPECS], chunk=20, mode=mode,
                      grab=grab, blocks=blocks)
    left = b.run()
    assert left == 0
    for i, (nx, ny, kind, tile, nsteps) in enumerate(SPECS):
        st = b.status(i)
        assert st["state"] == acm_mod.BATCH_FINISHED and st["steps_done"] == nsteps
        assert st["done_ms"] > 0
        got = b.state(i)
        s = acm_mod.Solver(cfgs[i], states[i])
        s.run(nsteps)
        ref = s.state()
        s.close()
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (i, k)
    ms, lups = b.timing()
    assert lups == sum(nx * ny * 20 * math.ceil(n / 20) for nx, ny, _, _, n in SPECS)
    b.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_with_row_forces_bitwise(acm_mod, mode):
    """Cases driven by a per-row body force (force_x, added to g[0] on row j)
    next to an unforced case, both launch modes and every force path (tiles
    with ragged edges, walls and a 128 x 4 tile whose staged region exceeds
    the persistent kernel's register set): bitwise equal to single runs with
    the same force."""
    specs = [(64, 48, "channel", 5), (40, 33, "tgv", 1), (70, 45, "channel", 4), (32, 32, "tgv", 0)]
    cfgs = [case_cfg(acm_mod, nx, ny, kind, 0.04) for nx, ny, kind, _ in specs]
    states = [spec_state(nx, ny, 200 + i) for i, (nx, ny, _, _) in enumerate(specs)]
    forces = []
    for i, (nx, ny, kind, _) in enumerate(specs):
        j = np.arange(ny) + 0.5
        forces.append(None if i == 3 else (2e-6 if kind == "channel" else 1e-6) * np.sin(np.pi * j / ny + i))
    b = acm_mod.Batch(cfgs, states, [40] * len(specs), tiles=[s[3] for s in specs], chunk=20, mode=mode,
                      forces=forces)
    assert b.run() == 0
    for i in range(len(specs)):
        s = acm_mod.Solver(cfgs[i], states[i], force_x=forces[i])
        s.run(40)
        ref = s.state()
        s.close()
        got = b.state(i)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (i, k)
    b.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_tiny_grids_bitwise(acm_mod, mode):
    """Grids smaller than every tile (down to the 4 x 4 minimum), periodic,
    walled and with symmetry planes, one item per case: bitwise equal to
    single runs; a second batch holding one case alone does the same."""
    specs = [(4, 4, "tgv", 0), (5, 4, "cavity", 3), (7, 9, "sym", 4), (6, 5, "channel", 1)]
    cfgs = [case_cfg(acm_mod, nx, ny, kind, 0.04) for nx, ny, kind, _ in specs]
    states = [spec_state(nx, ny, 300 + i) for i, (nx, ny, _, _) in enumerate(specs)]
    for sel in (range(len(specs)), [2]):
        b = acm_mod.Batch([cfgs[i] for i in sel], [states[i] for i in sel], [40] * len(sel),
                          tiles=[specs[i][3] for i in sel], chunk=20, mode=mode)
        assert b.run() == 0
        for k, i in enumerate(sel):
            s = acm_mod.Solver(cfgs[i], states[i])
            s.run(40)
            ref = s.state()
            s.close()
            got = b.state(k)
            for f in ref:
                assert np.array_equal(got[f], ref[f]), (i, f)
        b.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_divergence_is_isolated(acm_mod, mode):
    """A linearly unstable case (nu above the viscous bound, allowed
    explicitly) is retired as diverged; the others finish bitwise equal to
    their single runs."""
    cfgs = [case_cfg(acm_mod, 40, 40, "tgv", 0.04), case_cfg(acm_mod, 40, 40, "tgv", 0.45, allow_unstable=True),
            case_cfg(acm_mod, 48, 32, "cavity", 0.04)]
    states = [spec_state(40, 40, 1), spec_state(40, 40, 2), spec_state(48, 32, 3)]
    b = acm_mod.Batch(cfgs, states, [400, 400, 400], chunk=20, umax_limit=0.3, mode=mode)
    assert b.run() == 0
    assert b.status(1)["state"] == acm_mod.BATCH_DIVERGED
    assert b.status(1)["steps_done"] < 400
    for i in (0, 2):
        assert b.status(i)["state"] == acm_mod.BATCH_FINISHED
        s = acm_mod.Solver(cfgs[i], states[i])
        s.run(400)
        ref = s.state()
        got = b.state(i)
        for k in ref:
            assert np.array_equal(got[k], ref[k])
    b.close()


def test_batch_sampled_sweep_cases_match_oracle(acm_mod, orc):
    """Cases of the seeded 512-case sweep (the four smallest of the first
    sixteen), FP32 batched run of their full step counts against the FP64
    oracle at the stated FP32 bounds, velocity relative L2 <= 2e-5 and drho
    relative L2 <= 1e-4 (FP32 storage alone costs ~2e-7 and ~3e-6 on these
    cases, test_precision_storage.py)."""
    allc = inputs.batch_cases(ncases=16, seed=4)
    pick = sorted(allc, key=lambda c: c.n)[:4]
    cfgs, states = [], []
    for c in pick:
        kind = "tgv" if c.kind == "tgv" else "cavity"
        cfgs.append(case_cfg(acm_mod, c.n, c.n, kind, c.nu))
        states.append(f32(c.state))
    b = acm_mod.Batch(cfgs, states, [c.nsteps for c in pick], chunk=500)
    assert b.run() == 0
    for i, c in enumerate(pick):
        assert b.status(i)["state"] == acm_mod.BATCH_FINISHED
        g = b.state(i)
        wu = [[0.0] * 3 for _ in range(6)]
        bc = (0, 0, 0, 0, 0, 0)
        if c.kind == "cavity":
            bc = (1, 1, 1, 1, 0, 0)
            wu[3] = [0.05, 0, 0]
        o = orc.run(orc.Params(dim=2, nx=c.n, ny=c.n, nu=c.nu, bc=bc, wall_u=wu), states[i], c.nsteps)
        num = np.sqrt(np.sum((g["u"] - o["u"]) ** 2 + (g["v"] - o["v"]) ** 2))
        den = np.sqrt(np.sum(o["u"] ** 2 + o["v"] ** 2))
        er = np.linalg.norm(g["drho"] - o["drho"]) / np.linalg.norm(o["drho"])
        print(f"case n={c.n} {c.kind} Re={c.re:.0f} steps={c.nsteps}: vel relL2 {num / den:.2e} drho {er:.2e}")
        assert num / den <= 2e-5
        assert er <= 1e-4
    b.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_sweep512_first_chunk_sampled_cases_bitwise(acm_mod, mode):
    """The full 512-case sweep (seeded as in the benchmark, autotuned tiles
    for its launch mode), one 500-step chunk: twelve cases spread over the
    sizes and both kinds equal their single runs bit for bit (NaN where a
    case has diverged), and the step accounting covers every node of every
    case."""
    cases = inputs.batch_cases(512, seed=4)
    cfgs, states = [], []
    for c in cases:
        wu = [[0.0] * 3 for _ in range(6)]
        bc = (0, 0, 0, 0, 0, 0)
        if c.kind == "cavity":
            bc = (1, 1, 1, 1, 0, 0)
            wu[3] = [c.u_ref, 0.0, 0.0]
        cfgs.append(acm_mod.make_config(2, c.n, c.n, nu=c.nu, precision="f32", bc=bc, wall_u=wu))
        states.append(c.state)
    b = acm_mod.Batch(cfgs, states, [c.nsteps for c in cases], chunk=500, mode=mode)
    b.run(max_chunks=1)
    ms, lups = b.timing()
    assert lups == 500 * sum(c.n * c.n for c in cases)
    order = sorted(range(len(cases)), key=lambda i: (cases[i].n, i))
    pick = [order[k] for k in np.linspace(0, len(order) - 1, 12).astype(int)]
    assert {cases[i].kind for i in pick} == {"tgv", "cavity"}
    for i in pick:
        assert b.status(i)["steps_done"] == 500
        got = b.state(i)
        s = acm_mod.Solver(cfgs[i], states[i])
        s.run(500)
        ref = s.state()
        s.close()
        for k in ref:
            # cases that diverge within the chunk hold NaN at the same nodes in both
            assert np.array_equal(got[k], ref[k], equal_nan=True), (i, cases[i].n, cases[i].kind, k)
    b.close()


def test_autotune_choice_is_valid_and_result_invariant(acm_mod):
    best, ms = acm_mod.autotune(64, 64, "f32", copies=64, steps=40)
    assert 0 <= best < 6 and all(m > 0 for m in ms)
    assert ms[best] == min(ms)
    t = ctypes.c_int32()
    assert acm_mod.lib().acm_batch_tuned_tile(64, 64, acm_mod.F32, 0, ctypes.byref(t)) == acm_mod.OK
    assert t.value == best
