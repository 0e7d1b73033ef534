"""Learned closure for a 4x-coarser SMAME grid (not part of the paper's
method): q <- S_c(q) + D f(N S_c(q)), with f the 5-layer CNN of the HIP
library (bf16 matrix-core convolutions), trained on pairs of box-filtered
fine-grid states this solver generates, and a fine-grid fallback when a
divergence / energy gate trips.

Every numerical step runs in libacm (acm_cnn_*, acm_closure_*, acm_filter_box,
acm_prolong_bilinear, acm_step/acm_run); this module allocates buffers with
PyTorch and sequences the calls.
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import acm, inputs

LAYERS = 5
CONV_RELU, CONV_RAW, CONV_MASK = 0, 1, 2
REAL_CHANNELS = (3, 32, 32, 32, 32, 3)


def _f3(v) -> ctypes.Array:
    return (ctypes.c_float * 3)(*[float(x) for x in v])


def _vp(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None else None)


def _fields(d: Dict[str, "object"]) -> acm.Fields:
    return acm.Fields(d["drho"].data_ptr(), d["u"].data_ptr(), d["v"].data_ptr(), None, None)


def layer_shape(l: int) -> Tuple[int, int]:
    ci, co = ctypes.c_int32(), ctypes.c_int32()
    acm.check(acm.lib().acm_cnn_layer_shape(l, ctypes.byref(ci), ctypes.byref(co)))
    return ci.value, co.value


def he_init(seed: int, last_scale: float = 0.1):
    """Seeded He-normal weights [9, C_out, C_in] (real channels), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for l in range(LAYERS):
        ci, co = REAL_CHANNELS[l], REAL_CHANNELS[l + 1]
        w = rng.standard_normal((9, co, ci)) * math.sqrt(2.0 / (9 * ci))
        if l == LAYERS - 1:
            w *= last_scale
        out.append([w, np.zeros(co)])
    return out


class Network:
    """Parameters, optimizer state and work buffers of the closure network
    for one nx x ny grid (nx % 64 == 0, ny % 8 == 0)."""

    def __init__(self, nx: int, ny: int, params=None, seed: int = 0, device: str = "cuda:0",
                 in_scale=(1.0, 1.0, 1.0), out_scale=(1.0, 1.0, 1.0)):
        import torch
        self.torch = torch
        self.nx, self.ny = nx, ny
        self.dev = torch.device(device)
        self.in_scale = list(in_scale)
        self.out_scale = list(out_scale)
        self.shapes = [layer_shape(l) for l in range(LAYERS)]
        f32, b16 = torch.float32, torch.bfloat16
        self.w32 = [torch.zeros((9, co, ci), dtype=f32, device=self.dev) for ci, co in self.shapes]
        self.b32 = [torch.zeros(co, dtype=f32, device=self.dev) for ci, co in self.shapes]
        self.w16 = [torch.zeros((9, co, ci), dtype=b16, device=self.dev) for ci, co in self.shapes]
        self.wt16 = [torch.zeros((9, ci, co), dtype=b16, device=self.dev) for ci, co in self.shapes]
        self.gw = [torch.zeros_like(w) for w in self.w32]
        self.gb = [torch.zeros_like(b) for b in self.b32]
        self.mw = [torch.zeros_like(w) for w in self.w32]
        self.vw = [torch.zeros_like(w) for w in self.w32]
        self.mb = [torch.zeros_like(b) for b in self.b32]
        self.vb = [torch.zeros_like(b) for b in self.b32]
        self.acts = [torch.zeros((ny, nx, ci), dtype=b16, device=self.dev) for ci, _ in self.shapes]
        self.raw = torch.zeros((ny, nx, 16), dtype=f32, device=self.dev)
        self.gout = torch.zeros((ny, nx, 16), dtype=b16, device=self.dev)
        self.gacts = [torch.zeros((ny, nx, co), dtype=b16, device=self.dev) for _, co in self.shapes]
        ws = max(acm.lib().acm_cnn_wgrad_workspace(nx, ny, ci, co) for ci, co in self.shapes)
        self.wg_ws = torch.zeros(ws // 4 + 1, dtype=f32, device=self.dev)
        self.loss_ws = torch.zeros(acm.lib().acm_cnn_loss_workspace(nx, ny) // 8 + 1, dtype=torch.float64,
                                   device=self.dev)
        self.loss_buf = torch.zeros(1, dtype=torch.float64, device=self.dev)
        self.t = 0
        self.load(params if params is not None else he_init(seed))

    @property
    def stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.dev).cuda_stream)

    def load(self, params):
        """Set weights from real-channel numpy arrays (zero padding elsewhere)."""
        torch = self.torch
        for l, (w, b) in enumerate(params):
            ci, co = REAL_CHANNELS[l], REAL_CHANNELS[l + 1]
            self.w32[l].zero_()
            self.b32[l].zero_()
            self.w32[l][:, :co, :ci] = torch.from_numpy(np.asarray(w, dtype=np.float32)).to(self.dev)
            self.b32[l][:co] = torch.from_numpy(np.asarray(b, dtype=np.float32)).to(self.dev)
        self.refresh_bf16()

    def export(self):
        out = []
        for l in range(LAYERS):
            ci, co = REAL_CHANNELS[l], REAL_CHANNELS[l + 1]
            out.append([self.w32[l][:, :co, :ci].double().cpu().numpy(), self.b32[l][:co].double().cpu().numpy()])
        return out

    def refresh_bf16(self):
        L = acm.lib()
        for l, (ci, co) in enumerate(self.shapes):
            acm.check(L.acm_cnn_to_bf16(self.w32[l].numel(), _vp(self.w32[l]), _vp(self.w16[l]), self.stream))
        self.refresh_transposed()

    def refresh_transposed(self):
        L = acm.lib()
        for l, (ci, co) in enumerate(self.shapes):
            acm.check(L.acm_cnn_transpose(ci, co, _vp(self.w16[l]), _vp(self.wt16[l]), self.stream))

    # -- forward / backward ---------------------------------------------------
    def forward(self, drho, u, v):
        """raw = f(N q) for the state tensors (ny, nx) fp32."""
        L = acm.lib()
        acm.check(L.acm_cnn_pack(self.nx, self.ny, _vp(drho), _vp(u), _vp(v), _f3(self.in_scale),
                                 _vp(self.acts[0]), self.stream))
        for l, (ci, co) in enumerate(self.shapes):
            last = l == LAYERS - 1
            y = self.raw if last else self.acts[l + 1]
            acm.check(L.acm_cnn_conv(self.nx, self.ny, ci, co, CONV_RAW if last else CONV_RELU, _vp(self.acts[l]),
                                     _vp(self.w16[l]), _vp(self.b32[l]), None, _vp(y), self.stream))

    def correct(self, src: Dict[str, "object"], dst: Dict[str, "object"]):
        """dst = src + D f(N src) in one fused launch (nx, ny multiples of 16)."""
        ws16 = (ctypes.c_void_p * LAYERS)(*[self.w16[l].data_ptr() for l in range(LAYERS)])
        bs = (ctypes.c_void_p * LAYERS)(*[self.b32[l].data_ptr() for l in range(LAYERS)])
        fi, fo = _fields(src), _fields(dst)
        acm.check(acm.lib().acm_cnn_correct(self.nx, self.ny, ctypes.byref(fi), ctypes.byref(fo), ws16, bs,
                                            _f3(self.in_scale), _f3(self.out_scale), self.stream))

    def apply(self, drho, u, v):
        acm.check(acm.lib().acm_cnn_apply(self.nx, self.ny, _vp(self.raw), _f3(self.out_scale), _vp(drho), _vp(u),
                                          _vp(v), self.stream))

    def loss_and_grads(self, base: Dict[str, "object"], target: Dict[str, "object"]):
        """Loss of the last forward against target and gradients of all
        parameters (into gw, gb).  Returns the device loss tensor."""
        L = acm.lib()
        b = (ctypes.c_void_p * 3)(*[base[k].data_ptr() for k in ("drho", "u", "v")])
        t = (ctypes.c_void_p * 3)(*[target[k].data_ptr() for k in ("drho", "u", "v")])
        acm.check(L.acm_cnn_loss(self.nx, self.ny, _vp(self.raw), b, t, _f3(self.out_scale), _vp(self.gout),
                                 _vp(self.loss_ws), _vp(self.loss_buf), self.stream))
        g = self.gout
        for l in range(LAYERS - 1, -1, -1):
            ci, co = self.shapes[l]
            acm.check(L.acm_cnn_wgrad(self.nx, self.ny, ci, co, _vp(self.acts[l]), _vp(g), _vp(self.wg_ws),
                                      _vp(self.gw[l]), _vp(self.gb[l]), self.stream))
            if l > 0:
                gx = self.gacts[l - 1]  # gradient w.r.t. the pre-activation producing acts[l]
                acm.check(L.acm_cnn_conv(self.nx, self.ny, co, ci, CONV_MASK, _vp(g), _vp(self.wt16[l]), None,
                                         _vp(self.acts[l]), _vp(gx), self.stream))
                g = gx
        return self.loss_buf

    def adam(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        L = acm.lib()
        self.t += 1
        for l in range(LAYERS):
            acm.check(L.acm_cnn_adam(self.w32[l].numel(), _vp(self.w32[l]), _vp(self.gw[l]), _vp(self.mw[l]),
                                     _vp(self.vw[l]), _vp(self.w16[l]), lr, b1, b2, eps, self.t, self.stream))
            acm.check(L.acm_cnn_adam(self.b32[l].numel(), _vp(self.b32[l]), _vp(self.gb[l]), _vp(self.mb[l]),
                                     _vp(self.vb[l]), None, lr, b1, b2, eps, self.t, self.stream))
        self.refresh_transposed()

    def train_step(self, base, target, lr: float):
        self.forward(base["drho"], base["u"], base["v"])
        loss = self.loss_and_grads(base, target)
        self.adam(lr)
        return loss


# ---------------------------------------------------------------------------
# forced periodic flow: fine / coarse configurations
# ---------------------------------------------------------------------------
@dataclass
class FlowSpec:
    """2 pi periodic box with Kolmogorov forcing g_x = F sin(k_f y).  Lattice
    units of the fine grid; the coarse grid uses the acoustic scaling
    dx_c = r dx_f, dt_c = r dt_f (same Mach number): nu_c = nu_f / r and
    g_c = r g_f in coarse lattice units."""
    n_fine: int = 1024
    ratio: int = 4
    nu_fine: float = 0.02
    k_force: int = 4
    amp_laminar: float = 0.03   # F / (nu k^2) in fine lattice units
    u_rms: float = 0.03
    kmax: int = 16

    @property
    def n_coarse(self):
        return self.n_fine // self.ratio

    def force_amplitude(self):
        k = 2 * math.pi * self.k_force / self.n_fine
        return self.amp_laminar * self.nu_fine * k * k

    # 2D tile variant 5 (32 x 16) is the fastest step kernel shape on the
    # 1024^2 fine grid (8.2 us vs 9.1 us for the default), so the fine
    # reference runs at its best; on the 256^2 coarse grid the default 64 x 4
    # (twice as many workgroups) is faster (3.4 us vs 4.1 us)
    FINE_TILE, COARSE_TILE = 5, 0

    def fine_config(self, tile: int = FINE_TILE):
        return acm.make_config(2, self.n_fine, self.n_fine, nu=self.nu_fine, precision="f32", tile=tile,
                               graph_chunk=100)

    def coarse_config(self, tile: int = COARSE_TILE):
        return acm.make_config(2, self.n_coarse, self.n_coarse, nu=self.nu_fine / self.ratio, precision="f32",
                               tile=tile, graph_chunk=100)

    def fine_force(self):
        y = 2 * math.pi * np.arange(self.n_fine) / self.n_fine
        return self.force_amplitude() * np.sin(self.k_force * y)

    def coarse_force(self):
        r = self.ratio
        y = 2 * math.pi * (r * np.arange(self.n_coarse) + 0.5 * (r - 1)) / self.n_fine
        return r * self.force_amplitude() * np.sin(self.k_force * y)

    def initial_state(self, seed: int):
        return inputs.random_spectrum_field(self.n_fine, seed, self.u_rms, kmax=self.kmax)


def filter_to(fine: Dict[str, "object"], coarse: Dict[str, "object"], spec: FlowSpec, stream):
    acm.check(acm.lib().acm_filter_box(spec.n_fine, spec.n_fine, spec.ratio, acm.F32, ctypes.byref(_fields(fine)),
                                       ctypes.byref(_fields(coarse)), stream))


def prolong_to(coarse: Dict[str, "object"], fine: Dict[str, "object"], spec: FlowSpec, stream):
    acm.check(acm.lib().acm_prolong_bilinear(spec.n_coarse, spec.n_coarse, spec.ratio, acm.F32,
                                             ctypes.byref(_fields(coarse)), ctypes.byref(_fields(fine)), stream))


def rel_l2_velocity(a: Dict[str, "object"], b: Dict[str, "object"]) -> float:
    """Relative L2 velocity error ||a - b|| / ||b|| (device tensors, FP64 sum)."""
    num = ((a["u"] - b["u"]).double() ** 2 + (a["v"] - b["v"]).double() ** 2).sum()
    den = (b["u"].double() ** 2 + b["v"].double() ** 2).sum()
    return float((num / den).sqrt())


def generate_pairs(spec: FlowSpec, seeds: Sequence[int], warmup: int, pairs_per_seed: int, stride: int):
    """Training pairs from fine runs: for each snapshot time t, base =
    S_c(F(fine_t)) (one coarse step of the filtered state) and target =
    F(fine_{t + r steps}).  Returns a list of (base, target) dicts of
    device tensors."""
    import torch
    dev = torch.device("cuda:0")
    shape_c = (spec.n_coarse, spec.n_coarse)
    ff = spec.fine_force()
    cf = spec.coarse_force()
    out = []
    for seed in seeds:
        fine = acm.Solver(spec.fine_config(), spec.initial_state(seed), force_x=ff)
        coarse = acm.Solver(spec.coarse_config(), {k: np.zeros(shape_c) for k in ("drho", "u", "v")}, force_x=cf)
        fine.run(warmup)
        for p in range(pairs_per_seed):
            snap = {k: torch.empty(shape_c, dtype=torch.float32, device=dev) for k in ("drho", "u", "v")}
            filter_to(fine.tensors(), snap, spec, ctypes.c_void_p(fine.stream.cuda_stream))
            fine.run(spec.ratio)
            target = {k: torch.empty(shape_c, dtype=torch.float32, device=dev) for k in ("drho", "u", "v")}
            filter_to(fine.tensors(), target, spec, ctypes.c_void_p(fine.stream.cuda_stream))
            w, s = coarse.current()
            for k in snap:
                coarse.sets[w][k].copy_(snap[k])
            coarse.step()
            base = {k: coarse.tensors()[k].clone() for k in ("drho", "u", "v")}
            out.append((base, target))
            fine.run(stride - spec.ratio)
        fine.close()
        coarse.close()
    torch.cuda.synchronize()
    return out


def channel_scales(pairs, correct_density: bool = False, eps: float = 1e-12):
    """N = 1 / rms of each base channel; D = rms of each target residual.
    Unless correct_density, D = 0 for drho: the density is left to the
    scheme (a learned density correction feeds the acoustic mode, whose
    divergence then grows until the gate trips) and the channel is left out
    of the loss."""
    n_in = np.zeros(3)
    n_out = np.zeros(3)
    for base, tgt in pairs:
        for c, k in enumerate(("drho", "u", "v")):
            n_in[c] += float((base[k].double() ** 2).mean())
            n_out[c] += float(((tgt[k] - base[k]).double() ** 2).mean())
    n_in = np.sqrt(n_in / len(pairs))
    n_out = np.maximum(np.sqrt(n_out / len(pairs)), eps)
    if not correct_density:
        n_out[0] = 0.0
    return (1.0 / np.maximum(n_in, eps)).tolist(), n_out.tolist()


def train(net: Network, pairs, epochs: int, lr: float, seed: int = 0, lr_decay: float = 1.0, log=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    losses = []
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        tot = 0.0
        for i in order:
            base, tgt = pairs[i]
            loss = net.train_step(base, tgt, lr)
            tot += float(loss.item()) if log is not None else 0.0
        losses.append(tot / len(pairs))
        if log is not None:
            log(f"epoch {ep}: mean loss {losses[-1]:.4e} lr {lr:.2e}")
        lr *= lr_decay
    return losses


def generate_windows(spec: FlowSpec, seeds: Sequence[int], warmup: int, windows_per_seed: int, stride: int,
                     k: int):
    """Trajectory windows for training through the solver: for each snapshot
    time t, the box-filtered fine states F(fine_t), F(fine_{t + r}), ...,
    F(fine_{t + k r}) one coarse step apart.  Returns a list of lists of
    k + 1 state dicts (device tensors)."""
    import torch
    if stride < k * spec.ratio:
        raise ValueError(f"stride {stride} is shorter than a window of {k} coarse steps ({k * spec.ratio} fine steps)")
    dev = torch.device("cuda:0")
    shape_c = (spec.n_coarse, spec.n_coarse)
    out = []
    for seed in seeds:
        fine = acm.Solver(spec.fine_config(), spec.initial_state(seed), force_x=spec.fine_force())
        stream = ctypes.c_void_p(fine.stream.cuda_stream)
        fine.run(warmup)
        for _ in range(windows_per_seed):
            win = []
            for j in range(k + 1):
                if j:
                    fine.run(spec.ratio)
                f = {kk: torch.empty(shape_c, dtype=torch.float32, device=dev) for kk in ("drho", "u", "v")}
                filter_to(fine.tensors(), f, spec, stream)
                win.append(f)
            out.append(win)
            fine.run(stride - k * spec.ratio)
        fine.close()
    torch.cuda.synchronize()
    return out


def pairs_from_windows(spec: FlowSpec, windows):
    """One-step training pairs (S_c(F_0), F_1) of each window."""
    import torch
    shape_c = (spec.n_coarse, spec.n_coarse)
    coarse = acm.Solver(spec.coarse_config(), {k: np.zeros(shape_c) for k in ("drho", "u", "v")},
                        force_x=spec.coarse_force())
    out = []
    for win in windows:
        for k in win[0]:
            coarse.sets[0][k].copy_(win[0][k])
        coarse.set_current(0, 0)
        coarse.step()
        out.append(({k: coarse.sets[1][k].clone() for k in ("drho", "u", "v")}, win[1]))
    coarse.close()
    torch.cuda.synchronize()
    return out


class Unroll:
    """Training through k corrected coarse steps (solver in the loop):
    q_j = s_j + D f(N s_j), s_j = S(q_{j-1}), loss (1/k) sum_j [mean((q_j -
    F_j)/D)^2 over the corrected channels + div_beta mean((div(q_j - s_j) /
    D_vel)^2)], the last term penalising the compressive part of each
    correction (centred divergence, grid units; D_vel the mean output scale
    of the velocity channels, so div_beta is dimensionless).  The backward
    pass runs, for j = k .. 1, the state loss of step j, the network
    backward (weight gradients summed over the steps, and the gradient with
    respect to the network input) and the adjoint of the SMAME step, all in
    libacm; the network activations of each step are recomputed from the
    stored uncorrected state."""

    def __init__(self, spec: FlowSpec, net: Network, k: int, div_beta: float = 0.0):
        import torch
        self.torch = torch
        self.spec, self.net, self.k = spec, net, k
        d_vel = 0.5 * (net.out_scale[1] + net.out_scale[2])
        self.div_weight = float(div_beta) / (d_vel * d_vel) if div_beta else 0.0
        dev = net.dev
        shape = (spec.n_coarse, spec.n_coarse)
        assert (net.ny, net.nx) == shape

        def state():
            return {kk: torch.zeros(shape, dtype=torch.float32, device=dev) for kk in ("drho", "u", "v")}
        self.q = [state() for _ in range(k + 1)]   # q_0 .. q_k
        self.s = [None] + [state() for _ in range(k)]   # s_1 .. s_k (uncorrected)
        self.lam = [state(), state()]
        self.gin = torch.zeros((shape[0], shape[1], 16), dtype=torch.float32, device=dev)
        self.zero16 = torch.zeros(16, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.loss_dummy = torch.zeros(1, dtype=torch.float64, device=dev)
        self.solver = acm.Solver(spec.coarse_config(), None, tensors=[state(), state()],
                                 force_x=spec.coarse_force())

    def close(self):
        self.solver.close()

    def _step(self, src, dst):
        for kk in src:
            self.solver.sets[0][kk].copy_(src[kk])
        self.solver.set_current(0, 0)
        self.solver.step()
        for kk in dst:
            dst[kk].copy_(self.solver.sets[1][kk])

    def forward(self, q0):
        net = self.net
        for kk in q0:
            self.q[0][kk].copy_(q0[kk])
        for j in range(1, self.k + 1):
            self._step(self.q[j - 1], self.s[j])
            net.forward(self.s[j]["drho"], self.s[j]["u"], self.s[j]["v"])
            for kk in self.s[j]:
                self.q[j][kk].copy_(self.s[j][kk])
            net.apply(self.q[j]["drho"], self.q[j]["u"], self.q[j]["v"])

    def loss_and_grads(self, q0, targets, adj_q0: bool = False):
        """Loss of the window and its gradients in net.gw / net.gb (and, with
        adj_q0, dL/dq_0 in self.adj_q0).  Returns the device loss tensor."""
        L = acm.lib()
        net, k = self.net, self.k
        assert len(targets) == k
        nx, ny = net.nx, net.ny
        self.forward(q0)
        self.loss.zero_()
        lam, lam_next = self.lam
        for kk in lam:
            lam[kk].zero_()
        first = True
        for j in range(k, 0, -1):
            qj = (ctypes.c_void_p * 3)(*[self.q[j][kk].data_ptr() for kk in ("drho", "u", "v")])
            tj = (ctypes.c_void_p * 3)(*[targets[j - 1][kk].data_ptr() for kk in ("drho", "u", "v")])
            aj = (ctypes.c_void_p * 3)(*[lam[kk].data_ptr() for kk in ("drho", "u", "v")])
            acm.check(L.acm_cnn_state_loss(nx, ny, qj, tj, _f3(net.out_scale), 1.0 / k, aj, _vp(net.loss_ws),
                                           _vp(self.loss), net.stream))
            sj = self.s[j]
            if self.div_weight:
                qv = (ctypes.c_void_p * 2)(self.q[j]["u"].data_ptr(), self.q[j]["v"].data_ptr())
                sv = (ctypes.c_void_p * 2)(sj["u"].data_ptr(), sj["v"].data_ptr())
                av = (ctypes.c_void_p * 2)(lam["u"].data_ptr(), lam["v"].data_ptr())
                acm.check(L.acm_cnn_div_penalty(nx, ny, qv, sv, self.div_weight / k, av, None, _vp(net.loss_ws),
                                                _vp(self.loss), net.stream))
            # lam = dL/dq_j; the correction adds D raw, so dL/draw = D lam
            net.forward(sj["drho"], sj["u"], sj["v"])
            acm.check(L.acm_cnn_pack(nx, ny, _vp(lam["drho"]), _vp(lam["u"]), _vp(lam["v"]), _f3(net.out_scale),
                                     _vp(net.gout), net.stream))
            g = net.gout
            wg = L.acm_cnn_wgrad if first else L.acm_cnn_wgrad_add
            for l in range(LAYERS - 1, -1, -1):
                ci, co = net.shapes[l]
                acm.check(wg(nx, ny, ci, co, _vp(net.acts[l]), _vp(g), _vp(net.wg_ws), _vp(net.gw[l]),
                             _vp(net.gb[l]), net.stream))
                if l > 0:
                    gx = net.gacts[l - 1]
                    acm.check(L.acm_cnn_conv(nx, ny, co, ci, CONV_MASK, _vp(g), _vp(net.wt16[l]), None,
                                             _vp(net.acts[l]), _vp(gx), net.stream))
                    g = gx
            first = False
            # gradient with respect to the network input, then through N
            ci0, co0 = net.shapes[0]
            acm.check(L.acm_cnn_conv(nx, ny, co0, ci0, CONV_RAW, _vp(g), _vp(net.wt16[0]), _vp(self.zero16), None,
                                     _vp(self.gin), net.stream))
            acm.check(L.acm_cnn_apply(nx, ny, _vp(self.gin), _f3(net.in_scale), _vp(lam["drho"]), _vp(lam["u"]),
                                      _vp(lam["v"]), net.stream))
            if self.div_weight:  # the penalty's own dependence on s_j (div(s - q) = -div(q - s))
                acm.check(L.acm_cnn_div_penalty(nx, ny, sv, qv, self.div_weight / k, av, None, _vp(net.loss_ws),
                                                _vp(self.loss_dummy), net.stream))
            # lam = dL/ds_j; through the step to dL/dq_{j-1}
            if j > 1 or adj_q0:
                self.solver.adjoint(self.q[j - 1], sj, lam, lam_next)
                lam, lam_next = lam_next, lam
        self.adj_q0 = lam if adj_q0 else None
        return self.loss

    def train_step(self, q0, targets, lr: float):
        loss = self.loss_and_grads(q0, targets)
        self.net.adam(lr)
        return loss


def train_unrolled(net: Network, spec: FlowSpec, windows, k: int, epochs: int, lr: float, seed: int = 0,
                   lr_decay: float = 1.0, div_beta: float = 0.0, log=None):
    """Adam epochs of training through k steps over every window (the first
    k + 1 states of each are used)."""
    un = Unroll(spec, net, k, div_beta)
    rng = np.random.Generator(np.random.PCG64(seed))
    losses = []
    try:
        for ep in range(epochs):
            order = rng.permutation(len(windows))
            tot = 0.0
            for i in order:
                win = windows[i]
                loss = un.train_step(win[0], win[1:k + 1], lr)
                tot += float(loss.item()) if log is not None else 0.0
            losses.append(tot / len(windows))
            if log is not None:
                log(f"unrolled epoch {ep} (k = {k}): mean loss {losses[-1]:.4e} lr {lr:.2e}")
            lr *= lr_decay
    finally:
        un.close()
    return losses


@dataclass
class GateResult:
    tripped: bool
    at_step: int
    reason: str
    history: Optional[List[Tuple[int, float, float]]] = None  # (coarse step, E_k, divergence ratio) per gate


class ClosureRun:
    """Coarse run of the closure handle (network on or off) on its own pair
    of state buffers, with a monitor handle on the same buffers for the
    gate diagnostics."""

    def __init__(self, spec: FlowSpec, net: Optional[Network], state_coarse: Dict[str, "object"], chunk: int = 100,
                 separate_step: bool = False):
        import torch
        self.torch = torch
        self.spec = spec
        dev = torch.device("cuda:0")
        shape = (spec.n_coarse, spec.n_coarse)
        cfg = spec.coarse_config()
        self.cf = torch.from_numpy(spec.coarse_force()).to(device=dev, dtype=torch.float32)
        self.sets = [{k: torch.empty(shape, dtype=torch.float32, device=dev) for k in ("drho", "u", "v")}
                     for _ in range(2)]
        for k in self.sets[0]:
            self.sets[0][k].copy_(state_coarse[k])
        self.ws = torch.zeros(acm.lib().acm_closure_workspace(*shape) // 4 + 1, dtype=torch.float32, device=dev)
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        self.fa, self.fb = _fields(self.sets[0]), _fields(self.sets[1])
        self.net = net if net is not None else Network(spec.n_coarse, spec.n_coarse)
        ws16 = (ctypes.c_void_p * LAYERS)(*[self.net.w16[l].data_ptr() for l in range(LAYERS)])
        bs = (ctypes.c_void_p * LAYERS)(*[self.net.b32[l].data_ptr() for l in range(LAYERS)])
        h = ctypes.c_void_p()
        acm.check(acm.lib().acm_closure_init(ctypes.byref(cfg), ctypes.byref(self.fa), ctypes.byref(self.fb),
                                             _vp(self.cf), ws16, bs, _f3(self.net.in_scale),
                                             _f3(self.net.out_scale), _vp(self.ws), chunk, stream, ctypes.byref(h)))
        self.h = h
        if net is None:
            acm.check(acm.lib().acm_closure_set_network(self.h, 0))
        elif separate_step:  # step kernel, then correction kernel (same results)
            acm.check(acm.lib().acm_closure_set_network(self.h, 2))
        self.mon = acm.Solver(cfg, None, tensors=self.sets, force_x=spec.coarse_force())

    def current(self):
        w, s = ctypes.c_int32(), ctypes.c_int64()
        acm.check(acm.lib().acm_closure_current(self.h, ctypes.byref(w), ctypes.byref(s)))
        return w.value, s.value

    def state(self):
        return self.sets[self.current()[0]]

    def run(self, n: int):
        acm.check(acm.lib().acm_closure_run(self.h, int(n)))

    def diagnostics(self):
        w, s = self.current()
        self.mon.set_current(w, s)
        return self.mon.diagnostics()

    def close(self):
        if getattr(self, "h", None):
            acm.lib().acm_closure_destroy(self.h)
            self.h = None
        if getattr(self, "mon", None):
            self.mon.close()
            self.mon = None


def divergence_ratio(d: dict) -> float:
    """rms divergence over rms vorticity: O(Ma^2) for the weakly
    compressible scheme, O(1) when a correction injects compression."""
    return d["div_rms"] / max(math.sqrt(2.0 * d["enstrophy"]), 1e-300)


def gated_run(spec: FlowSpec, net: Optional[Network], c0, coarse_steps: int, gate_every: int = 100,
              energy_tol: float = 0.05, div_tol: float = 0.05, force_trip_at: Optional[int] = None,
              keep_states: bool = True):
    """Closure (or plain coarse, net=None) run with the gate every
    `gate_every` coarse steps.  The gate trips on a non-finite value, on a
    relative kinetic-energy change above energy_tol between two gates, or on
    a divergence ratio above div_tol; the state is then prolonged to the
    fine grid and plain fine steps finish the horizon.  Returns the filtered
    state at every gate, the gate outcome and the wall time."""
    import torch
    dev = torch.device("cuda:0")
    shape_c = (spec.n_coarse, spec.n_coarse)
    run = ClosureRun(spec, net, c0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    gate = GateResult(False, -1, "", [])
    states = []
    fine = None
    e_prev = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(coarse_steps // gate_every):
        step_no = (g + 1) * gate_every
        if fine is None:
            run.run(gate_every)
            d = run.diagnostics()
            reason = ""
            if d["nonfinite"]:
                reason = "non-finite"
            elif e_prev is not None and abs(d["ke"] / e_prev - 1.0) > energy_tol:
                reason = "energy drift"
            elif divergence_ratio(d) > div_tol:
                reason = "divergence"
            elif force_trip_at is not None and step_no >= force_trip_at:
                reason = "forced"
            e_prev = d["ke"]
            gate.history.append((step_no, float(d["ke"]), float(divergence_ratio(d))))
            cur = run.state()
            if reason:
                gate.tripped, gate.at_step, gate.reason = True, step_no, reason
                fine = acm.Solver(spec.fine_config(), None,
                                  tensors=[{k: torch.empty((spec.n_fine, spec.n_fine), dtype=torch.float32,
                                                           device=dev) for k in ("drho", "u", "v")}
                                           for _ in range(2)], force_x=spec.fine_force())
                prolong_to(cur, fine.sets[0], spec, stream)
        else:
            fine.run(gate_every * spec.ratio)
            cur = {k: torch.empty(shape_c, dtype=torch.float32, device=dev) for k in ("drho", "u", "v")}
            filter_to(fine.tensors(), cur, spec, stream)
        if keep_states:
            states.append({k: t.clone() for k, t in cur.items()})
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    run.close()
    if fine is not None:
        fine.close()
    return states, gate, wall


def evaluate_seed(spec: FlowSpec, net: Network, seed: int, warmup: int, coarse_steps: int, gate_every: int = 100,
                  energy_tol: float = 0.05, div_tol: float = 0.05, force_trip_at: Optional[int] = None):
    """Fine reference, plain coarse run and closure run from the same
    filtered state: velocity errors against the filtered fine reference at
    every gate, the gate outcome and the time-to-solution of the closure
    (gates included) and of the plain fine run."""
    import torch
    dev = torch.device("cuda:0")
    shape_c = (spec.n_coarse, spec.n_coarse)
    ff = spec.fine_force()
    fine = acm.Solver(spec.fine_config(), spec.initial_state(seed), force_x=ff)
    fine.run(warmup)
    stream = ctypes.c_void_p(fine.stream.cuda_stream)
    c0 = {k: torch.empty(shape_c, dtype=torch.float32, device=dev) for k in ("drho", "u", "v")}
    filter_to(fine.tensors(), c0, spec, stream)
    start = [{k: t.clone() for k, t in fine.tensors().items()},
             {k: torch.empty_like(t) for k, t in fine.tensors().items()}]
    ref = []
    for g in range(coarse_steps // gate_every):
        fine.run(gate_every * spec.ratio)
        ck = {k: torch.empty(shape_c, dtype=torch.float32, device=dev) for k in ("drho", "u", "v")}
        filter_to(fine.tensors(), ck, spec, stream)
        ref.append(ck)
    fine.close()
    timed = acm.Solver(spec.fine_config(), None, tensors=start, force_x=ff)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed.run(coarse_steps * spec.ratio)
    torch.cuda.synchronize()
    t_fine = time.perf_counter() - t0
    timed.close()
    plain_states, gate_plain, t_plain = gated_run(spec, None, c0, coarse_steps, gate_every, energy_tol=1e9,
                                                  div_tol=1e9)
    cnn_states, gate, t_closure = gated_run(spec, net, c0, coarse_steps, gate_every, energy_tol, div_tol,
                                            force_trip_at)
    err_plain = [rel_l2_velocity(a, b) for a, b in zip(plain_states, ref)]
    err_cnn = [rel_l2_velocity(a, b) for a, b in zip(cnn_states, ref)]
    return {"seed": seed, "err_cnn_end": err_cnn[-1], "err_cnn_max": max(err_cnn),
            "err_plain_end": err_plain[-1], "err_plain_max": max(err_plain), "gate": gate.__dict__, "gate_plain": gate_plain.__dict__,
            "t_fine_s": t_fine, "t_closure_s": t_closure, "t_plain_coarse_s": t_plain,
            "err_cnn": err_cnn, "err_plain": err_plain}
