"""GPU tests of the learned-closure kernels against the FP64 network
reference (oracle.cnn) and of the closure run loop."""
import ctypes
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available()
    from oracle import cnn
    from paper_2012_03525_amd import acm, closure
    acm.lib()
    return torch, acm, closure, cnn


def bf16_round(torch, a):
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).float().double().numpy()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.mark.parametrize("ci,co,mode", [(16, 32, 0), (32, 32, 0), (32, 16, 1), (32, 32, 1), (16, 32, 2), (32, 32, 2)])
def test_conv_modes_match_reference(mods, ci, co, mode):
    torch, acm, closure, cnn = mods
    ny, nx = 16, 64
    rng = np.random.Generator(np.random.PCG64(ci * 100 + co + mode))
    x = bf16_round(torch, rng.standard_normal((ny, nx, ci)))
    w = bf16_round(torch, rng.standard_normal((9, co, ci)) * 0.2)
    b = rng.standard_normal(co).astype(np.float32).astype(np.float64)
    mask = bf16_round(torch, rng.standard_normal((ny, nx, co)))
    dev = "cuda:0"
    xt = torch.from_numpy(x).to(dev, torch.bfloat16)
    wt = torch.from_numpy(w).to(dev, torch.bfloat16)
    bt = torch.from_numpy(b).to(dev, torch.float32)
    mt = torch.from_numpy(mask).to(dev, torch.bfloat16)
    y = torch.zeros((ny, nx, co), dtype=torch.float32 if mode == 1 else torch.bfloat16, device=dev)
    acm.check(acm.lib().acm_cnn_conv(nx, ny, ci, co, mode, ctypes.c_void_p(xt.data_ptr()),
                                     ctypes.c_void_p(wt.data_ptr()), ctypes.c_void_p(bt.data_ptr()),
                                     ctypes.c_void_p(mt.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    got = y.float().double().cpu().numpy()
    if mode == 0:
        ref = np.maximum(cnn.conv(x, w, b), 0.0)
        assert rel(got, ref) < 4e-3
    elif mode == 1:
        ref = cnn.conv(x, w, b)
        assert rel(got, ref) < 1e-5
    else:
        ref = cnn.conv(x, w, np.zeros(co)) * (mask > 0)
        assert rel(got, ref) < 4e-3


def test_network_forward_and_gradients_match_reference(mods):
    """Full network on a 128 x 64 grid with the same (bf16-rounded) weights:
    raw output within 2e-2 and every layer's weight gradient within 5e-2
    relative L2 of the FP64 reference (bf16 activations and gradients)."""
    torch, acm, closure, cnn = mods
    nx, ny = 128, 64
    rng = np.random.Generator(np.random.PCG64(7))
    params = closure.he_init(3, last_scale=1.0)
    params = [[bf16_round(torch, w), b + 0.01 * rng.standard_normal(b.shape)] for w, b in params]
    params = [[w, b.astype(np.float32).astype(np.float64)] for w, b in params]
    net = closure.Network(nx, ny, params=params)
    q = {k: rng.standard_normal((ny, nx)).astype(np.float32) for k in ("drho", "u", "v")}
    tgt = {k: rng.standard_normal((ny, nx)).astype(np.float32) for k in ("drho", "u", "v")}
    dev = "cuda:0"
    qt = {k: torch.from_numpy(v).to(dev) for k, v in q.items()}
    tt = {k: torch.from_numpy(v).to(dev) for k, v in tgt.items()}
    net.forward(qt["drho"], qt["u"], qt["v"])
    loss = net.loss_and_grads(qt, tt)
    torch.cuda.synchronize()
    x0 = np.stack([q["drho"], q["u"], q["v"]], axis=-1).astype(np.float64)
    x0 = bf16_round(torch, x0)
    raw, acts = cnn.forward(params, x0)
    got_raw = net.raw[:, :, :3].double().cpu().numpy()
    assert rel(got_raw, raw) < 2e-2
    resid = np.stack([tgt[k] - q[k] for k in ("drho", "u", "v")], axis=-1).astype(np.float64)
    l_ref, g_ref = cnn.mse_loss_and_grad(raw, resid)
    assert float(loss.item()) == pytest.approx(l_ref, rel=2e-2)
    grads = cnn.backward(params, acts, g_ref)
    for l in range(5):
        ci, co = closure.REAL_CHANNELS[l], closure.REAL_CHANNELS[l + 1]
        gw = net.gw[l][:, :co, :ci].double().cpu().numpy()
        gb = net.gb[l][:co].double().cpu().numpy()
        print(f"layer {l}: dW rel {rel(gw, grads[l][0]):.2e} db rel {rel(gb, grads[l][1]):.2e}")
        assert rel(gw, grads[l][0]) < 5e-2
        assert rel(gb, grads[l][1]) < 5e-2


@pytest.mark.parametrize("nx,ny", [(80, 48), (256, 256)])
def test_fused_correction_matches_reference(mods, nx, ny):
    """One-launch inference q + D f(N q) on several 16x16 tiles (periodic
    wrap across the grid edges): the correction within 2e-2 relative L2 of
    the FP64 reference with the same bf16 weights and bf16-rounded input."""
    torch, acm, closure, cnn = mods
    rng = np.random.Generator(np.random.PCG64(11))
    params = closure.he_init(5, last_scale=1.0)
    params = [[bf16_round(torch, w), (b + 0.01 * rng.standard_normal(b.shape)).astype(np.float32).astype(np.float64)]
              for w, b in params]
    s_in, d_out = [2.0, 0.5, 1.5], [1e-3, 2e-3, 3e-3]
    net = closure.Network(64, 64, params=params, in_scale=s_in, out_scale=d_out)
    net.nx, net.ny = nx, ny
    dev = "cuda:0"
    q = {k: rng.standard_normal((ny, nx)).astype(np.float32) for k in ("drho", "u", "v")}
    qt = {k: torch.from_numpy(v).to(dev) for k, v in q.items()}
    out = {k: torch.full((ny, nx), float("nan"), dtype=torch.float32, device=dev) for k in q}
    net.correct(qt, out)
    torch.cuda.synchronize()
    x0 = np.stack([q["drho"] * np.float32(s_in[0]), q["u"] * np.float32(s_in[1]), q["v"] * np.float32(s_in[2])],
                  axis=-1).astype(np.float64)
    raw, _ = cnn.forward(params, bf16_round(torch, x0))
    for c, k in enumerate(("drho", "u", "v")):
        corr = (out[k].double().cpu().numpy() - q[k].astype(np.float64)) / d_out[c]
        assert np.all(np.isfinite(corr)), k
        assert rel(corr, raw[:, :, c]) < 2e-2, (k, rel(corr, raw[:, :, c]))


def test_fused_correction_matches_layered_path(mods):
    """The fused kernel and the per-layer kernels (acm_cnn_conv chain, then
    acm_cnn_apply) agree to bf16 accuracy on the same weights and state."""
    torch, acm, closure, cnn = mods
    nx, ny = 128, 64
    rng = np.random.Generator(np.random.PCG64(12))
    net = closure.Network(nx, ny, seed=6, in_scale=[1.0, 2.0, 2.0], out_scale=[1e-2, 1e-2, 1e-2])
    dev = "cuda:0"
    q = {k: torch.from_numpy(rng.standard_normal((ny, nx)).astype(np.float32)).to(dev) for k in ("drho", "u", "v")}
    out = {k: torch.empty_like(v) for k, v in q.items()}
    net.correct(q, out)
    lay = {k: v.clone() for k, v in q.items()}
    net.forward(lay["drho"], lay["u"], lay["v"])
    net.apply(lay["drho"], lay["u"], lay["v"])
    torch.cuda.synchronize()
    for k in q:
        a = (out[k] - q[k]).double().cpu().numpy()
        b = (lay[k] - q[k]).double().cpu().numpy()
        assert rel(a, b) < 1e-2, (k, rel(a, b))


def test_excluded_channel_leaves_loss_gradient_and_field_alone(mods):
    """out_scale = 0 for drho: the loss equals the reference MSE over u and
    v only, the drho gradient is zero, and the fused correction copies drho
    bit for bit while still correcting u and v."""
    torch, acm, closure, cnn = mods
    nx, ny = 64, 64
    rng = np.random.Generator(np.random.PCG64(13))
    params = closure.he_init(8, last_scale=1.0)
    params = [[bf16_round(torch, w), b.astype(np.float32).astype(np.float64)] for w, b in params]
    net = closure.Network(nx, ny, params=params, out_scale=[0.0, 0.5, 0.25])
    dev = "cuda:0"
    q = {k: rng.standard_normal((ny, nx)).astype(np.float32) for k in ("drho", "u", "v")}
    tgt = {k: rng.standard_normal((ny, nx)).astype(np.float32) for k in ("drho", "u", "v")}
    qt = {k: torch.from_numpy(v).to(dev) for k, v in q.items()}
    tt = {k: torch.from_numpy(v).to(dev) for k, v in tgt.items()}
    net.forward(qt["drho"], qt["u"], qt["v"])
    loss = net.loss_and_grads(qt, tt)
    out = {k: torch.empty_like(v) for k, v in qt.items()}
    net.correct(qt, out)
    torch.cuda.synchronize()
    raw = net.raw[:, :, :3].double().cpu().numpy()
    resid = np.stack([(tgt[k] - q[k]) / s for k, s in (("u", 0.5), ("v", 0.25))], axis=-1).astype(np.float64)
    l_ref, _ = cnn.mse_loss_and_grad(raw[:, :, 1:], resid)
    assert float(loss.item()) == pytest.approx(l_ref, rel=1e-5)
    assert float(net.gout[:, :, 0].float().abs().max()) == 0.0
    assert torch.equal(out["drho"], qt["drho"])
    assert not torch.equal(out["u"], qt["u"]) and not torch.equal(out["v"], qt["v"])


def test_adam_matches_reference(mods):
    torch, acm, closure, cnn = mods
    rng = np.random.Generator(np.random.PCG64(11))
    n = 1000
    p = rng.standard_normal(n)
    m = np.zeros(n)
    v = np.zeros(n)
    dev = "cuda:0"
    pt, mt, vt = (torch.from_numpy(a.astype(np.float32)).to(dev) for a in (p, m, v))
    p16 = torch.zeros(n, dtype=torch.bfloat16, device=dev)
    pr = p.astype(np.float32).astype(np.float64)
    for t in range(1, 4):
        g = rng.standard_normal(n)
        gt = torch.from_numpy(g.astype(np.float32)).to(dev)
        acm.check(acm.lib().acm_cnn_adam(n, ctypes.c_void_p(pt.data_ptr()), ctypes.c_void_p(gt.data_ptr()),
                                         ctypes.c_void_p(mt.data_ptr()), ctypes.c_void_p(vt.data_ptr()),
                                         ctypes.c_void_p(p16.data_ptr()), 1e-2, 0.9, 0.999, 1e-8, t,
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        cnn.adam_step(pr, g.astype(np.float32).astype(np.float64), m, v, t, 1e-2)
    got = pt.double().cpu().numpy()
    np.testing.assert_allclose(got, pr, rtol=0, atol=1e-6)
    np.testing.assert_allclose(p16.float().cpu().numpy(), got, rtol=8e-3, atol=1e-6)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_filter_and_prolongation_match_reference(mods, precision):
    torch, acm, closure, cnn = mods
    rng = np.random.Generator(np.random.PCG64(13))
    dt = torch.float64 if precision == "f64" else torch.float32
    pr = acm.F64 if precision == "f64" else acm.F32
    fine = {k: rng.standard_normal((64, 96)) for k in ("drho", "u", "v")}
    ft = {k: torch.from_numpy(v).to("cuda:0", dt) for k, v in fine.items()}
    ct = {k: torch.zeros((16, 24), dtype=dt, device="cuda:0") for k in fine}
    bt = {k: torch.zeros((64, 96), dtype=dt, device="cuda:0") for k in fine}
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    acm.check(acm.lib().acm_filter_box(96, 64, 4, pr, ctypes.byref(closure._fields(ft)), ctypes.byref(closure._fields(ct)), s))
    acm.check(acm.lib().acm_prolong_bilinear(24, 16, 4, pr, ctypes.byref(closure._fields(ct)),
                                             ctypes.byref(closure._fields(bt)), s))
    tol = 1e-13 if precision == "f64" else 1e-6
    for k in fine:
        c_ref = cnn.box_filter(fine[k].astype(np.float32).astype(np.float64) if precision == "f32" else fine[k], 4)
        np.testing.assert_allclose(ct[k].double().cpu().numpy(), c_ref, rtol=0, atol=tol)
        p_ref = cnn.prolong_bilinear(ct[k].double().cpu().numpy(), 4)
        np.testing.assert_allclose(bt[k].double().cpu().numpy(), p_ref, rtol=0, atol=tol)


def test_training_overfits_one_pair(mods):
    """Sanity: repeated Adam steps on one (base, target) pair drive the loss
    down by more than an order of magnitude."""
    torch, acm, closure, cnn = mods
    nx = ny = 64
    rng = np.random.Generator(np.random.PCG64(17))
    x = np.linspace(0, 2 * np.pi, nx, endpoint=False)
    X, Y = np.meshgrid(x, x)
    base = {"drho": 1e-3 * np.sin(X + Y), "u": 0.03 * np.sin(Y), "v": 0.02 * np.cos(X)}
    tgt = {k: v + 0.05 * np.abs(v).max() * np.sin(2 * X + 3 * Y + i) for i, (k, v) in enumerate(base.items())}
    dev = "cuda:0"
    bt = {k: torch.from_numpy(v.astype(np.float32)).to(dev) for k, v in base.items()}
    tt = {k: torch.from_numpy(v.astype(np.float32)).to(dev) for k, v in tgt.items()}
    insc = [1.0 / np.sqrt(np.mean(base[k] ** 2)) for k in ("drho", "u", "v")]
    outsc = [np.sqrt(np.mean((tgt[k] - base[k]) ** 2)) for k in ("drho", "u", "v")]
    net = closure.Network(nx, ny, seed=1, in_scale=insc, out_scale=outsc)
    first = float(net.train_step(bt, tt, 2e-3).item())
    for _ in range(300):
        last = net.train_step(bt, tt, 2e-3)
    last = float(last.item())
    assert last < first / 10, (first, last)


@pytest.mark.parametrize("separate_step", [False, True])
def test_closure_handle_equals_manual_sequence(mods, separate_step):
    """The closure handle (graph-captured; the step run inside the correction
    kernel, or as its own launch) is bitwise equal to acm steps followed by
    the fused network correction issued call by call, and with the network
    switched off to plain acm_run."""
    torch, acm, closure, cnn = mods
    from paper_2012_03525_amd import inputs
    spec = closure.FlowSpec(n_fine=256, nu_fine=0.02)
    st = inputs.random_spectrum_field(64, seed=5, u_rms=0.02, kmax=8)
    dev = "cuda:0"
    c0 = {k: torch.from_numpy(v.astype(np.float32)).to(dev) for k, v in st.items()}
    net = closure.Network(64, 64, seed=2, in_scale=[1e3, 30.0, 30.0], out_scale=[1e-6, 1e-5, 1e-5])
    run = closure.ClosureRun(spec, net, c0, chunk=2, separate_step=separate_step)
    run.run(4)
    got = {k: t.clone() for k, t in run.state().items()}
    assert acm.lib().acm_closure_set_network(run.h, 3) == acm.EINVAL
    run.close()
    s = acm.Solver(spec.coarse_config(), {k: v.astype(np.float32).astype(np.float64) for k, v in st.items()},
                   force_x=spec.coarse_force())
    tmp = {k: torch.empty((64, 64), dtype=torch.float32, device=dev) for k in ("drho", "u", "v")}
    for _ in range(4):
        s.step()
        q = s.tensors()
        net.correct(q, tmp)
        for k in q:
            q[k].copy_(tmp[k])
    torch.cuda.synchronize()
    for k in got:
        assert torch.equal(got[k], s.tensors()[k]), k
    s.close()
    plain = closure.ClosureRun(spec, None, c0, chunk=2)
    plain.run(6)
    ref = acm.Solver(spec.coarse_config(), {k: v.astype(np.float32).astype(np.float64) for k, v in st.items()},
                     force_x=spec.coarse_force())
    ref.run(6)
    torch.cuda.synchronize()
    for k in ("drho", "u", "v"):
        assert torch.equal(plain.state()[k], ref.tensors()[k])
    plain.close()
    ref.close()


def test_gate_trip_falls_back_to_fine_grid(mods):
    """A trip forced from the host hands the state to the fine grid: after
    the trip the run equals prolonging that state and stepping the fine grid."""
    torch, acm, closure, cnn = mods
    spec = closure.FlowSpec(n_fine=256, nu_fine=0.02, u_rms=0.02, kmax=8)
    net = closure.Network(64, 64, seed=4, in_scale=[1e3, 30.0, 30.0], out_scale=[1e-6, 1e-5, 1e-5])
    st = spec.initial_state(9)
    fine = acm.Solver(spec.fine_config(), st, force_x=spec.fine_force())
    dev = "cuda:0"
    c0 = {k: torch.zeros((64, 64), dtype=torch.float32, device=dev) for k in ("drho", "u", "v")}
    stream = ctypes.c_void_p(fine.stream.cuda_stream)
    closure.filter_to(fine.tensors(), c0, spec, stream)
    states, gate, _ = closure.gated_run(spec, net, c0, coarse_steps=40, gate_every=10, force_trip_at=20)
    assert gate.tripped and gate.at_step == 20 and gate.reason == "forced"
    # manual: closure 20 steps, prolong, 20 coarse-step equivalents of fine steps
    run = closure.ClosureRun(spec, net, c0, chunk=10)
    run.run(20)
    f2 = acm.Solver(spec.fine_config(), {k: np.zeros((256, 256)) for k in ("drho", "u", "v")},
                    force_x=spec.fine_force())
    closure.prolong_to(run.state(), f2.sets[0], spec, stream)
    torch.cuda.synchronize()
    assert all(torch.equal(states[1][k], run.state()[k]) for k in ("drho", "u", "v"))
    f2.run(20 * spec.ratio)
    ck = {k: torch.zeros((64, 64), dtype=torch.float32, device=dev) for k in ("drho", "u", "v")}
    closure.filter_to(f2.tensors(), ck, spec, stream)
    torch.cuda.synchronize()
    for k in ck:
        assert torch.equal(states[3][k], ck[k]), k
    run.close()
    f2.close()
    fine.close()


def test_trained_network_gains_over_plain_coarse(mods):
    """Gain test: the network trained by the library's own kernels (fine
    256^2 -> coarse 64^2, 24 training seeds) cuts the relative L2 velocity
    error against the filtered fine run on held-out seeds well below that of
    the plain coarse run over 2000 coarse steps, without tripping the gate;
    the preset's second stage trains through the solver step with the
    divergence penalty, as the full preset does."""
    torch, acm, closure, cnn = mods
    from paper_2012_03525_amd import closure_experiment
    summary, _ = closure_experiment.run_experiment("small", log=lambda m: None, eval_seeds=(1000, 1002))
    for r in summary["per_seed"]:
        print(f"seed {r['seed']}: plain {r['err_plain_end']:.4f} closure {r['err_cnn_end']:.4f}")
        assert not r["gate"]["tripped"], r["gate"]["reason"]
        assert r["err_cnn_end"] < 0.6 * r["err_plain_end"]
        assert r["err_cnn_max"] < 0.02
    assert summary["epoch_loss"][-1] < 0.2 * summary["epoch_loss"][0]
    # the stage trained through the solver (divergence penalty) ran
    assert summary["unroll"] == 1 and len(summary["unroll_epoch_loss"]) == 2
    assert summary["unroll_epoch_loss"][-1] <= summary["unroll_epoch_loss"][0]
