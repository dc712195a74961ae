"""Thin ctypes binding of libd2q37 (C ABI in include/lb.h).

Argument marshalling only: every step of the lattice update runs in the HIP
kernels of the library. PyTorch provides the device memory (the two
population buffers and the scratch area) and the stream. There is no CPU
fallback: if the library or a GPU is missing, calls raise.
"""
from __future__ import annotations

import ctypes
import functools
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# D2Q37_LIB selects another build of the same library (e.g. one compiled
# with different -D options); the default is the in-tree build.
LIB_PATH = os.environ.get("D2Q37_LIB") or os.path.join(HERE, "libd2q37.so")

LB_OK, LB_EINVAL, LB_EDEVICE, LB_EUNSUPPORTED, LB_ENONFINITE = 0, -1, -2, -3, -4
PRECISIONS = {"f64": 0, "f32s": 1, "f16s": 2}
LAYOUTS = {"soa": 0, "aos": 1, "csoa": 2, "caosoa": 3}
ELEM_BYTES = {"f64": 8, "f32s": 4, "f16s": 2}
Q = 37


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class LBNonFinite(LBError):
    def __init__(self, code: int, msg: str, totals):
        super().__init__(code, msg)
        self.totals = totals


class Config(ctypes.Structure):
    _fields_ = [
        ("lx", ctypes.c_int32),
        ("ly", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("compensated", ctypes.c_int32),
        ("audit", ctypes.c_int32),
        ("buf", ctypes.c_void_p * 2),
        ("scratch", ctypes.c_void_p),
        ("scratch_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("gx", ctypes.c_double),
        ("gy", ctypes.c_double),
        ("walls", ctypes.c_int32),
        ("t_bottom", ctypes.c_double),
        ("t_top", ctypes.c_double),
    ]


_VP, _I32, _I64, _SZ, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double

_SIGNATURES = {
    "lb_buffer_bytes": (_SZ, [_I32, _I32, _I32, _I32]),
    "lb_scratch_bytes": (_SZ, [_I32, _I32]),
    "lb_init": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(Config), _VP, _VP, _VP, _VP]),
    "lb_propagate": (ctypes.c_int, [_VP]),
    "lb_collide": (ctypes.c_int, [_VP]),
    "lb_step": (ctypes.c_int, [_VP, _I32]),
    "lb_moments": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "lb_get_populations": (ctypes.c_int, [_VP, _VP]),
    "lb_set_populations": (ctypes.c_int, [_VP, _VP]),
    "lb_audit": (ctypes.c_int, [_VP, ctypes.POINTER(_D)]),
    "lb_audit_static": (ctypes.c_int, [_VP, ctypes.POINTER(_D)]),
    "lb_current_buffer": (ctypes.c_int, [_VP]),
    "lb_steps_done": (_I64, [_VP]),
    "lb_destroy": (None, [_VP]),
    "lb_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lb_last_error": (ctypes.c_char_p, [_VP]),
    "lb_model_constants": (ctypes.c_int, [ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_I32)]),
    "lb_copy": (ctypes.c_int, [_VP, _VP, _SZ, _VP]),
    "lb_mlp_param_count": (_SZ, []),
    "lb_mlp_workspace_bytes": (_SZ, [_I32]),
    "lb_mlp_create": (ctypes.c_int, [ctypes.POINTER(_VP), _VP, _SZ, _I32, _VP]),
    "lb_mlp_destroy": (None, [_VP]),
    "lb_mlp_last_error": (ctypes.c_char_p, [_VP]),
    "lb_mlp_init": (ctypes.c_int, [_VP, ctypes.c_uint64]),
    "lb_mlp_set_params": (ctypes.c_int, [_VP, _VP]),
    "lb_mlp_get_params": (ctypes.c_int, [_VP, _VP]),
    "lb_mlp_set_normalization": (ctypes.c_int, [_VP, _VP]),
    "lb_mlp_get_normalization": (ctypes.c_int, [_VP, _VP]),
    "lb_mlp_fit_normalization": (ctypes.c_int, [_VP, _VP, _VP, _I64, _D]),
    "lb_mlp_gradient": (ctypes.c_int, [_VP, _VP, _VP, _I32, _D, _VP, ctypes.POINTER(_D)]),
    "lb_mlp_train": (ctypes.c_int, [_VP, _VP, _VP, _I64, _D, _I32, _I32, ctypes.c_float, ctypes.c_uint64, _I64,
                                    _VP]),
    "lb_mlp_equilibrium": (ctypes.c_int, [_VP, _VP, _I64, ctypes.c_float, _VP, _VP, _VP]),
    "lb_pairgen": (ctypes.c_int, [_VP, _VP, _I64, ctypes.c_uint64, _D, _VP]),
    "lb_mlp_set_precision": (ctypes.c_int, [_VP, _I32]),
    "lb_mlp_get_precision": (ctypes.c_int, [_VP]),
    "lb_mlp_gelu16": (ctypes.c_int, [_VP, _VP, _I64, _VP]),
    "lb_set_surrogate": (ctypes.c_int, [_VP, _VP, _D]),
    "lb_surrogate_counts": (ctypes.c_int, [_VP, _VP]),
}


@functools.lru_cache(maxsize=None)
def lib() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_1804_01918_amd.build` "
            "(or __graft_entry__.build()) first")
    so = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(so, name)
        fn.restype = res
        fn.argtypes = args
    return so


def _check(rc: int, ctx=None, what: str = ""):
    if rc == LB_OK:
        return
    msg = lib().lb_last_error(ctx).decode(errors="replace")
    raise LBError(rc, f"{what}: {msg}" if what else msg)


def buffer_bytes(lx: int, ly: int, precision: str = "f64", layout: str = "soa") -> int:
    return lib().lb_buffer_bytes(lx, ly, PRECISIONS[precision], LAYOUTS[layout])


def scratch_bytes(lx: int, ly: int) -> int:
    return lib().lb_scratch_bytes(lx, ly)


def model_constants():
    """(r, w[37], c[37, 2]) as compiled into the library."""
    r = ctypes.c_double()
    w = np.zeros(Q)
    c = np.zeros((Q, 2), dtype=np.int32)
    _check(lib().lb_model_constants(ctypes.byref(r), w.ctypes.data_as(ctypes.POINTER(_D)),
                                    c.ctypes.data_as(ctypes.POINTER(_I32))))
    return r.value, w, c


# ---- the C-ABI calls under their own names (marshalling only) -----------------
# ctx is the lb_ctx handle (ctypes.c_void_p); device arrays are torch CUDA
# tensors (or raw device addresses as int). Errors raise LBError.

def _ptr(a) -> int:
    return a if isinstance(a, int) else a.data_ptr()


def lb_buffer_bytes(lx: int, ly: int, precision: str = "f64", layout: str = "soa") -> int:
    return lib().lb_buffer_bytes(lx, ly, PRECISIONS[precision], LAYOUTS[layout])


def lb_scratch_bytes(lx: int, ly: int) -> int:
    return lib().lb_scratch_bytes(lx, ly)


def lb_init(cfg: Config, rho, ux, uy, T) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(lib().lb_init(ctypes.byref(ctx), ctypes.byref(cfg), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T)), None,
           "lb_init")
    return ctx


def lb_propagate(ctx):
    _check(lib().lb_propagate(ctx), ctx, "lb_propagate")


def lb_collide(ctx):
    _check(lib().lb_collide(ctx), ctx, "lb_collide")


def lb_step(ctx, nsteps: int = 1):
    _check(lib().lb_step(ctx, int(nsteps)), ctx, "lb_step")


def lb_moments(ctx, rho, ux, uy, T):
    _check(lib().lb_moments(ctx, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T)), ctx, "lb_moments")


def lb_audit(ctx) -> np.ndarray:
    out = (ctypes.c_double * 4)()
    rc = lib().lb_audit(ctx, out)
    vals = np.array(list(out))
    if rc == LB_ENONFINITE:
        raise LBNonFinite(rc, lib().lb_last_error(ctx).decode(), vals)
    _check(rc, ctx, "lb_audit")
    return vals


def lb_audit_static(ctx) -> np.ndarray:
    out = (ctypes.c_double * 4)()
    rc = lib().lb_audit_static(ctx, out)
    vals = np.array(list(out))
    if rc == LB_ENONFINITE:
        raise LBNonFinite(rc, lib().lb_last_error(ctx).decode(), vals)
    _check(rc, ctx, "lb_audit_static")
    return vals


def lb_destroy(ctx):
    if ctx is not None and ctx.value:
        lib().lb_destroy(ctx)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libd2q37 needs a ROCm GPU; torch.cuda.is_available() is False")
    return torch


def gelu16(x, stream=None):
    """The binary16 GELU of the inference form on a device int16/uint16
    tensor of binary16 bit patterns; returns the result patterns (int16)."""
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    x = x.contiguous()
    y = torch.empty_like(x)
    _check(lib().lb_mlp_gelu16(x.data_ptr(), y.data_ptr(), x.numel(), s.cuda_stream), None, "lb_mlp_gelu16")
    return y


def device_copy(dst, src, stream=None):
    """Streaming copy kernel of the library (bandwidth reference)."""
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    nbytes = src.numel() * src.element_size()
    _check(lib().lb_copy(dst.data_ptr(), src.data_ptr(), nbytes, s.cuda_stream), None, "lb_copy")


NPARAM = 26149


def pairgen(n: int, seed: int, tau: float, device: str = "cuda"):
    """n training pairs (pre, post) of shifted FP32 populations, (n, 37) each,
    drawn on the GPU."""
    torch = _torch()
    pre = torch.empty((n, Q), dtype=torch.float32, device=device)
    post = torch.empty_like(pre)
    _check(lib().lb_pairgen(pre.data_ptr(), post.data_ptr(), n, seed, tau, torch.cuda.current_stream().cuda_stream),
           None, "lb_pairgen")
    return pre, post


def _pairs_arg(t, name: str):
    """A device FP32 (n, 37) tensor in row-major order (copied if needed)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != Q:
        raise ValueError(f"{name} must be float32 of shape (n, {Q}), got {t.dtype} {tuple(t.shape)}")
    return t.contiguous()


def _mcheck(rc, m, what):
    if rc != LB_OK:
        raise LBError(rc, f"{what}: {lib().lb_mlp_last_error(m).decode(errors='replace')}")


class Mlp:
    """The learned-collide network (37-128-128-37, GELU) in a PyTorch-owned
    device workspace; every computation runs in libd2q37's kernels."""

    def __init__(self, max_batch: int = 8192, device: str = "cuda"):
        torch = _torch()
        self.max_batch = int(max_batch)
        nbytes = lib().lb_mlp_workspace_bytes(self.max_batch)
        if nbytes == 0:
            raise LBError(LB_EINVAL, f"invalid max_batch {max_batch}")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream()
        self._m = ctypes.c_void_p()
        _mcheck(lib().lb_mlp_create(ctypes.byref(self._m), self.ws.data_ptr(), nbytes, self.max_batch,
                                    self.stream.cuda_stream), None, "lb_mlp_create")

    @property
    def handle(self):
        if self._m is None or not self._m.value:
            raise RuntimeError("network is closed")
        return self._m

    def init(self, seed: int):
        _mcheck(lib().lb_mlp_init(self.handle, seed), self.handle, "lb_mlp_init")

    MLP_PRECISIONS = {"f16": 0, "fp8": 1}

    def set_precision(self, precision: str):
        """Inference precision: "f16" (hidden activations and the last two
        layers in binary16, the default), or "fp8" (the hidden layer in e4m3)."""
        _mcheck(lib().lb_mlp_set_precision(self.handle, self.MLP_PRECISIONS[precision]), self.handle,
                "lb_mlp_set_precision")

    def get_precision(self) -> str:
        code = lib().lb_mlp_get_precision(self.handle)
        return {v: k for k, v in self.MLP_PRECISIONS.items()}[code]

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == NPARAM
        _mcheck(lib().lb_mlp_set_params(self.handle, a.ctypes.data), self.handle, "lb_mlp_set_params")

    def get_params(self) -> np.ndarray:
        a = np.empty(NPARAM, dtype=np.float32)
        _mcheck(lib().lb_mlp_get_params(self.handle, a.ctypes.data), self.handle, "lb_mlp_get_params")
        return a

    def set_normalization(self, norm):
        a = np.ascontiguousarray(norm, dtype=np.float32).reshape(4, Q)
        _mcheck(lib().lb_mlp_set_normalization(self.handle, a.ctypes.data), self.handle, "lb_mlp_set_normalization")

    def get_normalization(self) -> np.ndarray:
        a = np.empty((4, Q), dtype=np.float32)
        _mcheck(lib().lb_mlp_get_normalization(self.handle, a.ctypes.data), self.handle, "lb_mlp_get_normalization")
        return a

    def fit_normalization(self, pre, post, tau: float):
        pre, post = _pairs_arg(pre, "pre"), _pairs_arg(post, "post")
        _mcheck(lib().lb_mlp_fit_normalization(self.handle, pre.data_ptr(), post.data_ptr(), pre.shape[0], tau),
                self.handle, "lb_mlp_fit_normalization")

    def gradient(self, pre, post, tau: float):
        pre, post = _pairs_arg(pre, "pre"), _pairs_arg(post, "post")
        g = np.empty(NPARAM, dtype=np.float32)
        loss = ctypes.c_double()
        _mcheck(lib().lb_mlp_gradient(self.handle, pre.data_ptr(), post.data_ptr(), pre.shape[0], tau,
                                      g.ctypes.data, ctypes.byref(loss)), self.handle, "lb_mlp_gradient")
        return g, loss.value

    def train(self, pre, post, tau: float, batch: int, epochs: int, lr: float, seed: int, max_steps: int = 0):
        pre, post = _pairs_arg(pre, "pre"), _pairs_arg(post, "post")
        losses = np.zeros(epochs)
        _mcheck(lib().lb_mlp_train(self.handle, pre.data_ptr(), post.data_ptr(), pre.shape[0], tau, batch, epochs,
                                   lr, seed, max_steps, losses.ctypes.data), self.handle, "lb_mlp_train")
        return losses

    def equilibrium(self, pre, threshold: float):
        torch = _torch()
        pre = _pairs_arg(pre, "pre")
        n = pre.shape[0]
        geq = torch.empty_like(pre)
        res = torch.empty(n, dtype=torch.float32, device=pre.device)
        fb = torch.empty(n, dtype=torch.int32, device=pre.device)
        _mcheck(lib().lb_mlp_equilibrium(self.handle, pre.data_ptr(), n, threshold, geq.data_ptr(), res.data_ptr(),
                                         fb.data_ptr()), self.handle, "lb_mlp_equilibrium")
        return geq, res, fb

    def close(self):
        if self._m is not None and self._m.value:
            lib().lb_mlp_destroy(self._m)
        self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lattice:
    """One D2Q37 lattice on the GPU: two population buffers and scratch owned
    by PyTorch, kernels from libd2q37, launched on the current stream."""

    def __init__(self, lx: int, ly: int, tau: float, fields, precision: str = "f64",
                 layout: str = "soa", compensated: bool | None = None, audit: bool = False,
                 device: str = "cuda", force=(0.0, 0.0), walls: bool = False, t_bottom: float = 1.0,
                 t_top: float = 1.0):
        """compensated=None picks the default of the precision: compensated
        FP32 moment sums for f32s; plain sums for f16s, whose 11-bit storage
        rounding is far above the FP32 summation error. force: body force
        (acceleration per step, thermal units); walls: diffuse walls at rest
        below row 0 (t_bottom) and above row ly - 1 (t_top)."""
        torch = _torch()
        if compensated is None:
            compensated = precision == "f32s"
        self.lx, self.ly, self.tau = int(lx), int(ly), float(tau)
        self.precision, self.layout = precision, layout
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        nbytes = lib().lb_buffer_bytes(self.lx, self.ly, PRECISIONS[precision], LAYOUTS[layout])
        if nbytes == 0:
            raise LBError(LB_EUNSUPPORTED if self.lx >= 1 and self.ly >= 1 else LB_EINVAL,
                          f"invalid lattice {lx}x{ly} for precision={precision} layout={layout}")
        sbytes = lib().lb_scratch_bytes(self.lx, self.ly)
        self.bufs = [torch.empty(nbytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self.scratch = torch.empty(sbytes, dtype=torch.uint8, device=self.device)
        self.cfg = Config()
        self.cfg.lx, self.cfg.ly, self.cfg.tau = self.lx, self.ly, self.tau
        self.cfg.precision, self.cfg.layout = PRECISIONS[precision], LAYOUTS[layout]
        self.cfg.compensated, self.cfg.audit = int(bool(compensated)), int(bool(audit))
        self.cfg.buf[0], self.cfg.buf[1] = self.bufs[0].data_ptr(), self.bufs[1].data_ptr()
        self.cfg.scratch, self.cfg.scratch_bytes = self.scratch.data_ptr(), sbytes
        self.cfg.stream = self.stream.cuda_stream
        self.force = (float(force[0]), float(force[1]))
        self.cfg.gx, self.cfg.gy = self.force
        self.cfg.walls = int(bool(walls))
        self.cfg.t_bottom, self.cfg.t_top = float(t_bottom), float(t_top)
        fl = [self._field(a) for a in fields]
        self._ctx = None
        self._ctx = lb_init(self.cfg, *fl)
        self._fields_keepalive = fl

    def _field(self, a):
        torch = _torch()
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        t = a.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(t.shape) != (self.lx, self.ly):
            raise ValueError(f"field shape {tuple(t.shape)} != {(self.lx, self.ly)}")
        return t

    @property
    def ctx(self):
        if self._ctx is None or not self._ctx.value:
            raise RuntimeError("lattice is closed")
        return self._ctx

    # -- the method ---------------------------------------------------------
    def propagate(self):
        lb_propagate(self.ctx)

    def collide(self):
        lb_collide(self.ctx)

    def step(self, nsteps: int = 1):
        lb_step(self.ctx, nsteps)

    # -- readouts -----------------------------------------------------------
    def moments(self):
        torch = _torch()
        out = [torch.empty((self.lx, self.ly), dtype=torch.float64, device=self.device) for _ in range(4)]
        lb_moments(self.ctx, *out)
        return tuple(out)

    def get_populations(self):
        torch = _torch()
        f = torch.empty((Q, self.lx, self.ly), dtype=torch.float64, device=self.device)
        _check(lib().lb_get_populations(self.ctx, f.data_ptr()), self.ctx, "lb_get_populations")
        return f

    def set_populations(self, f):
        torch = _torch()
        if isinstance(f, np.ndarray):
            f = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float64))
        t = f.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(t.shape) != (Q, self.lx, self.ly):
            raise ValueError(f"populations shape {tuple(t.shape)} != {(Q, self.lx, self.ly)}")
        _check(lib().lb_set_populations(self.ctx, t.data_ptr()), self.ctx, "lb_set_populations")
        self.stream.synchronize()

    def audit(self) -> np.ndarray:
        return lb_audit(self.ctx)

    def set_surrogate(self, mlp, threshold: float = 1e-3):
        """Collide with the network (FP32-shifted lattices); None restores the
        plain collide."""
        self._mlp = mlp
        _check(lib().lb_set_surrogate(self.ctx, mlp.handle if mlp is not None else None, threshold), self.ctx,
               "lb_set_surrogate")

    def surrogate_counts(self):
        out = (ctypes.c_int64 * 2)()
        _check(lib().lb_surrogate_counts(self.ctx, out), self.ctx, "lb_surrogate_counts")
        return int(out[0]), int(out[1])

    def current_buffer(self) -> int:
        return lib().lb_current_buffer(self.ctx)

    def steps_done(self) -> int:
        return lib().lb_steps_done(self.ctx)

    def raw_state(self):
        """Raw bytes of the current buffer (bit-exact checkpoint)."""
        return self.bufs[self.current_buffer()].clone()

    def load_raw_state(self, raw):
        self.bufs[self.current_buffer()].copy_(raw)

    def close(self):
        lb_destroy(self._ctx)
        self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
