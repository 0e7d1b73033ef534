"""ctypes binding of libacm.so (include/acm.h): argument marshalling only.

Every step of the solver runs in the HIP library; PyTorch provides device
memory (tensor.data_ptr()) and the stream (torch.cuda.current_stream()).
Importing this module fails loudly if libacm.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libacm.so")

OK, EINVAL, EUNSTABLE, EHIP, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5
PERIODIC, WALL, SYMMETRY = 0, 1, 2
F64, F32 = 0, 1


class AcmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"acm status {status}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("nu", ctypes.c_double), ("cs", ctypes.c_double),
        ("rho0", ctypes.c_double), ("sat_rho", ctypes.c_double), ("sat_mom", ctypes.c_double),
        ("g", ctypes.c_double * 3), ("bc", ctypes.c_int32 * 6), ("wall_u", (ctypes.c_double * 3) * 6),
        ("two_phase", ctypes.c_int32), ("sigma", ctypes.c_double), ("width", ctypes.c_double),
        ("mobility", ctypes.c_double), ("precision", ctypes.c_int32), ("allow_unstable", ctypes.c_int32),
        ("graph_chunk", ctypes.c_int32), ("tile", ctypes.c_int32), ("wet_cos", ctypes.c_double * 6),
        ("axisym", ctypes.c_int32),
    ]


class Fields(ctypes.Structure):
    _fields_ = [("drho", ctypes.c_void_p), ("u", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("phi", ctypes.c_void_p)]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("mom", ctypes.c_double * 3), ("ke", ctypes.c_double),
        ("dumax", ctypes.c_double), ("umax", ctypes.c_double), ("enstrophy", ctypes.c_double),
        ("energy", ctypes.c_double), ("div_rms", ctypes.c_double), ("div_max", ctypes.c_double),
        ("phi_sum", ctypes.c_double), ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int32),
        ("which", ctypes.c_int32),
    ]


class BatchCase(ctypes.Structure):
    _fields_ = [("cfg", Config), ("a", Fields), ("b", Fields), ("force_x", ctypes.c_void_p),
                ("nsteps", ctypes.c_int64), ("tile", ctypes.c_int32)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("blocks", ctypes.c_int32), ("grab", ctypes.c_int32),
                ("umax_limit", ctypes.c_double), ("mode", ctypes.c_int32)]


class BatchCaseStatus(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int64), ("state", ctypes.c_int32), ("which", ctypes.c_int32),
                ("done_ms", ctypes.c_double), ("umax", ctypes.c_double)]


_lib: Optional[ctypes.CDLL] = None

# exported symbols and their ctypes signatures (also checked by the CPU tests)
SIGNATURES = {
    "acm_stability": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]),
    "acm_scratch_bytes": (ctypes.c_size_t, [ctypes.POINTER(Config)]),
    "acm_init": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(Fields), ctypes.POINTER(Fields),
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_void_p)]),
    "acm_step": (ctypes.c_int, [ctypes.c_void_p]),
    "acm_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "acm_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Diag)]),
    "acm_current": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int64)]),
    "acm_set_current": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64]),
    "acm_step_adjoint": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(Fields)] * 4),
    "acm_destroy": (None, [ctypes.c_void_p]),
    "acm_last_error": (ctypes.c_char_p, []),
    "acm_version": (ctypes.c_char_p, []),
    "acm_stream_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "acm_batch_scratch_bytes": (ctypes.c_size_t, [ctypes.POINTER(BatchCase), ctypes.c_int32,
                                                  ctypes.POINTER(BatchOpts)]),
    "acm_batch_init": (ctypes.c_int, [ctypes.POINTER(BatchCase), ctypes.c_int32, ctypes.POINTER(BatchOpts),
                                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "acm_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "acm_batch_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(BatchCaseStatus)]),
    "acm_batch_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "acm_batch_destroy": (None, [ctypes.c_void_p]),
    "acm_batch_autotune_scratch_bytes": (ctypes.c_size_t, [ctypes.c_int32] * 4),
    "acm_batch_autotune": (ctypes.c_int, [ctypes.c_int32] * 6 + [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                                                 ctypes.POINTER(ctypes.c_double),
                                                                 ctypes.POINTER(ctypes.c_int32)]),
    "acm_batch_tuned_tile": (ctypes.c_int, [ctypes.c_int32] * 4 + [ctypes.POINTER(ctypes.c_int32)]),
    "acm_batch_set_tuned_tile": (ctypes.c_int, [ctypes.c_int32] * 5),
    "acm_cnn_layer_shape": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32)]),
    "acm_cnn_conv": (ctypes.c_int, [ctypes.c_int32] * 5 + [ctypes.c_void_p] * 6),
    "acm_cnn_transpose": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "acm_cnn_wgrad_workspace": (ctypes.c_size_t, [ctypes.c_int32] * 4),
    "acm_cnn_wgrad": (ctypes.c_int, [ctypes.c_int32] * 4 + [ctypes.c_void_p] * 6),
    "acm_cnn_wgrad_add": (ctypes.c_int, [ctypes.c_int32] * 4 + [ctypes.c_void_p] * 6),
    "acm_cnn_pack": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32] + [ctypes.c_void_p] * 3 +
                     [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]),
    "acm_cnn_apply": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]
                      + [ctypes.c_void_p] * 4),
    "acm_cnn_loss_workspace": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "acm_cnn_loss": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                    ctypes.POINTER(ctypes.c_float)] + [ctypes.c_void_p] * 4),
    "acm_cnn_loss_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "acm_cnn_state_loss": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_float),
                                          ctypes.c_float, ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "acm_cnn_div_penalty": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.c_float,
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "acm_cnn_adam": (ctypes.c_int, [ctypes.c_int64] + [ctypes.c_void_p] * 5 + [ctypes.c_float] * 4 +
                     [ctypes.c_int64, ctypes.c_void_p]),
    "acm_cnn_to_bf16": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "acm_filter_box": (ctypes.c_int, [ctypes.c_int32] * 4 + [ctypes.POINTER(Fields), ctypes.POINTER(Fields),
                                                             ctypes.c_void_p]),
    "acm_prolong_bilinear": (ctypes.c_int, [ctypes.c_int32] * 4 + [ctypes.POINTER(Fields), ctypes.POINTER(Fields),
                                                                   ctypes.c_void_p]),
    "acm_cnn_correct": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Fields), ctypes.POINTER(Fields),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                       ctypes.c_void_p]),
    "acm_closure_workspace": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "acm_closure_init": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(Fields), ctypes.POINTER(Fields),
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "acm_closure_set_network": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "acm_closure_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "acm_closure_current": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int64)]),
    "acm_closure_destroy": (None, [ctypes.c_void_p]),
}


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2012_03525_amd.build`")
        # torch first: its HIP runtime then satisfies the library's libamdhip64
        # dependency, so the process holds one runtime and torch's device
        # pointers and streams are valid in the library's calls
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> int:
    if status != OK:
        raise AcmError(status, lib().acm_last_error().decode())
    return status


def make_config(dim: int, nx: int, ny: int, nz: int = 1, *, dx: float = 1.0, dt: float = 1.0,
                nu: float = 0.0, cs: float = 0.0, rho0: float = 1.0, sat_rho: float = 1.0,
                sat_mom: float = 1.0, g: Sequence[float] = (0.0, 0.0, 0.0),
                bc: Sequence[int] = (0, 0, 0, 0, 0, 0), wall_u=None, two_phase: bool = False,
                sigma: float = 0.0, width: float = 4.0, mobility: float = 0.0, precision: str = "f32",
                allow_unstable: bool = False, graph_chunk: int = 0, tile: int = 0,
                wet_cos: Optional[Sequence[float]] = None, axisym: bool = False) -> Config:
    c = Config()
    c.dim, c.nx, c.ny, c.nz = dim, nx, ny, (nz if dim == 3 else 1)
    c.dx, c.dt, c.nu, c.cs, c.rho0 = dx, dt, nu, cs, rho0
    c.sat_rho, c.sat_mom = sat_rho, sat_mom
    for a in range(3):
        c.g[a] = float(g[a])
    for f in range(6):
        c.bc[f] = int(bc[f])
        for a in range(3):
            c.wall_u[f][a] = float(wall_u[f][a]) if wall_u is not None else 0.0
    c.two_phase = 1 if two_phase else 0
    c.sigma, c.width, c.mobility = sigma, width, mobility
    c.precision = {"f64": F64, "f32": F32}[precision]
    c.allow_unstable = 1 if allow_unstable else 0
    c.graph_chunk = graph_chunk
    c.tile = tile
    for f in range(6):
        c.wet_cos[f] = float(wet_cos[f]) if wet_cos is not None else 0.0
    c.axisym = 1 if axisym else 0
    return c


def stability(cfg: Config):
    amp, che = ctypes.c_double(), ctypes.c_double()
    check(lib().acm_stability(ctypes.byref(cfg), ctypes.byref(amp), ctypes.byref(che)))
    return amp.value, che.value


def scratch_bytes(cfg: Config) -> int:
    """Device scratch bytes acm_init needs for cfg."""
    n = lib().acm_scratch_bytes(ctypes.byref(cfg))
    if n == 0:
        raise AcmError(EINVAL, lib().acm_last_error().decode())
    return int(n)


def scratch_tensor(nbytes: int, device):
    """A device byte buffer of at least nbytes, 256-byte aligned (torch's
    caching allocator hands out 512-byte aligned blocks; checked here)."""
    import torch
    t = torch.empty(max(1, nbytes), dtype=torch.uint8, device=device)
    if t.data_ptr() % 256:
        raise AcmError(EINVAL, "torch returned a scratch block that is not 256-byte aligned")
    return t


def stream_copy(dst, src, nbytes: int, stream=None):
    """Device copy through the library's plain copy kernel (torch tensors)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    check(lib().acm_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                ctypes.c_size_t(nbytes), ctypes.c_void_p(s.cuda_stream)))


def _names(cfg: Config):
    names = ["drho", "u", "v"]
    if cfg.dim == 3:
        names.append("w")
    if cfg.two_phase:
        names.append("phi")
    return names


class Solver:
    """Owns two device state sets (torch tensors) and a libacm handle."""

    def __init__(self, cfg: Config, state: Dict[str, np.ndarray], device: str = "cuda:0",
                 force_x: Optional[np.ndarray] = None, tensors=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.dtype = torch.float64 if cfg.precision == F64 else torch.float32
        self.shape = (cfg.nz, cfg.ny, cfg.nx) if cfg.dim == 3 else (cfg.ny, cfg.nx)
        self.names = _names(cfg)
        if tensors is not None:
            self.sets = tensors
        else:
            self.sets = [{k: torch.empty(self.shape, dtype=self.dtype, device=self.device) for k in self.names}
                         for _ in range(2)]
            for k in self.names:
                a = np.ascontiguousarray(np.asarray(state[k], dtype=np.float64).reshape(self.shape))
                self.sets[0][k].copy_(torch.from_numpy(a).to(self.dtype))
        self.force = None
        if force_x is not None:
            self.force = torch.from_numpy(np.ascontiguousarray(force_x, dtype=np.float64)).to(
                device=self.device, dtype=self.dtype)
        self._f = [self._fields(s) for s in self.sets]
        self.stream = torch.cuda.current_stream(self.device)
        nbytes = scratch_bytes(cfg)
        self.scratch = scratch_tensor(nbytes, self.device)
        h = ctypes.c_void_p()
        check(lib().acm_init(ctypes.byref(cfg), ctypes.byref(self._f[0]), ctypes.byref(self._f[1]),
                             ctypes.c_void_p(self.force.data_ptr() if self.force is not None else None),
                             ctypes.c_void_p(self.scratch.data_ptr()), ctypes.c_size_t(nbytes),
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def _fields(self, s):
        f = Fields()
        for k in self.names:
            setattr(f, k, s[k].data_ptr())
        return f

    def step(self):
        check(lib().acm_step(self.h))

    def run(self, nsteps: int):
        check(lib().acm_run(self.h, int(nsteps)))

    def adjoint(self, q: Dict[str, "object"], s: Dict[str, "object"], adj_s: Dict[str, "object"],
                adj_q: Dict[str, "object"]):
        """adj_q = (dS/dq)^T adj_s for s = S(q) (device tensor dicts drho, u,
        v of this grid and precision; 2D periodic single-phase).  Async."""
        f = [self._fields(d) for d in (q, s, adj_s, adj_q)]
        check(lib().acm_step_adjoint(self.h, *[ctypes.byref(x) for x in f]))

    def current(self):
        w, s = ctypes.c_int32(), ctypes.c_int64()
        check(lib().acm_current(self.h, ctypes.byref(w), ctypes.byref(s)))
        return w.value, s.value

    def set_current(self, which: int, step: int):
        check(lib().acm_set_current(self.h, int(which), int(step)))

    def diagnostics(self, raise_nonfinite: bool = False) -> dict:
        d = Diag()
        st = lib().acm_diagnostics(self.h, ctypes.byref(d))
        if st not in (OK, ENONFINITE) or (st == ENONFINITE and raise_nonfinite):
            check(st)
        return {"mass": d.mass, "mom_x": d.mom[0], "mom_y": d.mom[1], "mom_z": d.mom[2], "ke": d.ke,
                "dumax": d.dumax, "umax": d.umax, "enstrophy": d.enstrophy, "energy": d.energy,
                "div_rms": d.div_rms, "div_max": d.div_max, "phi_sum": d.phi_sum, "step": d.step,
                "nonfinite": d.nonfinite, "which": d.which}

    def tensors(self) -> Dict[str, "object"]:
        """Device tensors of the newest state (no copy)."""
        return self.sets[self.current()[0]]

    def state(self) -> Dict[str, np.ndarray]:
        """Newest state copied to host as FP64 numpy arrays (synchronises)."""
        self.torch.cuda.synchronize(self.device)
        return {k: t.detach().to("cpu", dtype=self.torch.float64).numpy() for k, t in self.tensors().items()}

    def close(self):
        if getattr(self, "h", None):
            lib().acm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


BATCH_RUNNING, BATCH_FINISHED, BATCH_DIVERGED = 0, 1, 2


class Batch:
    """Independent 2D single-phase cases advanced together by the batched
    kernel (mode 0: one workgroup per item; 1: persistent work queue).  All
    states live in one arena tensor (6 fields per case: set a then set b),
    sliced into per-case views.  `forces`, if given, holds per case None or
    the ny values of a row force added to g[0] (kept on the device for the
    life of the batch)."""

    def __init__(self, cfgs, states, nsteps, tiles=None, chunk: int = 500, device: str = "cuda:0",
                 umax_limit: float = 0.3, grab: int = 0, blocks: int = 0, mode: int = 0, forces=None):
        import torch
        self.torch = torch
        n = len(cfgs)
        prec = cfgs[0].precision
        self.dtype = torch.float64 if prec == F64 else torch.float32
        sizes = [c.nx * c.ny for c in cfgs]
        self.offsets = np.concatenate([[0], np.cumsum([6 * z for z in sizes])]).astype(np.int64)
        self.arena = torch.empty(int(self.offsets[-1]), dtype=self.dtype, device=device)
        self.views = []
        self.forces = []  # device copies of the per-row forces, kept alive with the batch
        arr = (BatchCase * n)()
        for i, (c, st) in enumerate(zip(cfgs, states)):
            o, z = int(self.offsets[i]), sizes[i]
            v = [self.arena[o + f * z:o + (f + 1) * z].view(c.ny, c.nx) for f in range(6)]
            for f, k in enumerate(("drho", "u", "v")):
                v[f].copy_(torch.from_numpy(np.ascontiguousarray(st[k], dtype=np.float64)).to(self.dtype))
            self.views.append(v)
            bc = arr[i]
            bc.cfg = c
            bc.a = Fields(v[0].data_ptr(), v[1].data_ptr(), v[2].data_ptr(), None, None)
            bc.b = Fields(v[3].data_ptr(), v[4].data_ptr(), v[5].data_ptr(), None, None)
            bc.force_x = None
            if forces is not None and forces[i] is not None:
                f = torch.from_numpy(np.ascontiguousarray(forces[i], dtype=np.float64)).to(device, self.dtype)
                self.forces.append(f)
                bc.force_x = f.data_ptr()
            bc.nsteps = int(nsteps[i])
            bc.tile = -1 if tiles is None else int(tiles[i])
        self._cases = arr
        opts = BatchOpts(chunk, blocks, grab, umax_limit, mode)
        self.stream = torch.cuda.current_stream()
        untuned = {(c.nx, c.ny) for i, c in enumerate(cfgs) if tiles is None or int(tiles[i]) < 0}
        if untuned:
            ensure_tuned(sorted(untuned), prec, mode)
        nbytes = lib().acm_batch_scratch_bytes(arr, n, ctypes.byref(opts))
        if nbytes == 0:
            raise AcmError(EINVAL, lib().acm_last_error().decode())
        self.scratch = scratch_tensor(nbytes, device)
        h = ctypes.c_void_p()
        check(lib().acm_batch_init(arr, n, ctypes.byref(opts), ctypes.c_void_p(self.scratch.data_ptr()),
                                   ctypes.c_size_t(nbytes), ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h)))
        self.h = h
        self.n = n

    def run(self, max_chunks: int = -1) -> int:
        left = ctypes.c_int32()
        check(lib().acm_batch_run(self.h, int(max_chunks), ctypes.byref(left)))
        return left.value

    def status(self, i: int) -> dict:
        st = BatchCaseStatus()
        check(lib().acm_batch_status(self.h, int(i), ctypes.byref(st)))
        return {"steps_done": st.steps_done, "state": st.state, "which": st.which, "done_ms": st.done_ms,
                "umax": st.umax}

    def timing(self):
        ms, lups = ctypes.c_double(), ctypes.c_int64()
        check(lib().acm_batch_timing(self.h, ctypes.byref(ms), ctypes.byref(lups)))
        return ms.value, lups.value

    def state(self, i: int) -> Dict[str, np.ndarray]:
        self.torch.cuda.synchronize()
        w = self.status(i)["which"]
        v = self.views[i][3 * w:3 * w + 3]
        return {k: t.detach().to("cpu", dtype=self.torch.float64).numpy() for k, t in zip(("drho", "u", "v"), v)}

    def close(self):
        if getattr(self, "h", None):
            lib().acm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(nx: int, ny: Optional[int] = None, precision: str = "f32", copies: int = 0, steps: int = 100,
             mode: int = 0):
    """Time every 2D tile variant on copies of a periodic nx x ny case through
    the batched kernel; the library records the fastest for (nx, ny,
    precision, mode).  Returns (best_tile, ms_per_step_per_tile)."""
    import torch
    ny = nx if ny is None else ny
    prec = {"f64": F64, "f32": F32}[precision] if isinstance(precision, str) else int(precision)
    if copies <= 0:
        copies = min(1024, max(1, (1 << 22) // (nx * ny)))
    nbytes = lib().acm_batch_autotune_scratch_bytes(nx, ny, prec, copies)
    if nbytes == 0:
        raise AcmError(EINVAL, lib().acm_last_error().decode())
    scratch = scratch_tensor(nbytes, torch.device("cuda", torch.cuda.current_device()))
    ms = (ctypes.c_double * 6)()
    best = ctypes.c_int32()
    check(lib().acm_batch_autotune(int(nx), int(ny), prec, int(mode), int(copies), int(steps),
                                   ctypes.c_void_p(scratch.data_ptr()), ctypes.c_size_t(nbytes),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ms,
                                   ctypes.byref(best)))
    del scratch
    return best.value, list(ms)


def _tune_cache_path() -> str:
    base = os.environ.get("ACM_TUNE_CACHE")
    if base:
        return base
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2012_03525_amd", "batch_tiles.json")


def _gpu_arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def ensure_tuned(shapes, precision: int, mode: int = 0, steps: int = 20):
    """Make sure the library holds a tuned tile for every (nx, ny) in shapes:
    take it from the on-disk cache (keyed by GPU architecture, grid shape,
    precision and launch mode) when present, else run the autotuner and add
    its choice to the cache.  The tile changes only speed, never results."""
    import json
    path = _tune_cache_path()
    try:
        with open(path) as f:
            disk = json.load(f)
    except (OSError, ValueError):
        disk = {}
    arch = _gpu_arch()
    changed = False
    for nx, ny in shapes:
        t = ctypes.c_int32()
        if lib().acm_batch_tuned_tile(nx, ny, precision, mode, ctypes.byref(t)) == OK:
            continue
        key = f"{arch}/{nx}x{ny}/{'f64' if precision == F64 else 'f32'}/mode{mode}"
        if key in disk and 0 <= int(disk[key]) < 6:
            check(lib().acm_batch_set_tuned_tile(nx, ny, precision, mode, int(disk[key])))
            continue
        best, _ = autotune(nx, ny, precision, steps=steps, mode=mode)
        disk[key] = best
        changed = True
    if changed:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + f".{os.getpid()}.tmp"
            with open(tmp, "w") as f:
                json.dump(disk, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass  # the in-process choice still holds
