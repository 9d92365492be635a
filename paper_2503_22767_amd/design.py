"""Thin binding of the design front end (include/mpm_mag_design.h): argument
marshalling only; the filter, projection and magnetization run in the HIP
library, and there is no CPU fallback.

    fe = MpmMagDesign(x0, radius, region=None, n_regions=None, precision=4)
    density, br = DesignFn.apply(fe, phi, br_mag, zeta, beta, br_max, delta)

`density` and `br` are the `density` and `br` inputs of MpmMag.rollout, so
DesignFn composed with MpmMagFn gives gradients with respect to the design
variables of Sec. 3.1 (phi, per-region magnitude and orientation).

    b_prog = HarmonicFn.apply(b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta)

is the harmonic stimulus (Sec. 3.1.2) as a field program of one row per step,
for instances made with n_segments = n_steps and seg_steps = 1.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import torch

from .mpm_mag import OK, MpmMagError, _ptr, lib as _mpm_lib

_bound = False


class HarmonicDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_inst", C.c_int), ("n_steps", C.c_int), ("dt", C.c_double),
                ("b_max", C.c_double), ("f_min", C.c_double), ("f_max", C.c_double), ("delta", C.c_double)]


def lib():
    global _bound
    L = _mpm_lib()
    if not _bound:
        vp, i64 = C.c_void_p, C.c_int64
        d = C.c_double
        L.mpm_mag_design_create.argtypes = [C.c_int, i64, vp, d, vp, C.c_int, C.c_int, vp, C.POINTER(vp)]
        L.mpm_mag_design_create.restype = C.c_int
        L.mpm_mag_design_forward.argtypes = [vp, vp, vp, d, vp, vp, d, d, C.c_int, vp, vp]
        L.mpm_mag_design_forward.restype = C.c_int
        L.mpm_mag_design_backward.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, vp]
        L.mpm_mag_design_backward.restype = C.c_int
        L.mpm_mag_design_nnz.argtypes = [vp]
        L.mpm_mag_design_nnz.restype = i64
        L.mpm_mag_design_last_error.argtypes = [vp]
        L.mpm_mag_design_last_error.restype = C.c_char_p
        L.mpm_mag_design_destroy.argtypes = [vp]
        L.mpm_mag_design_destroy.restype = None
        hp = C.POINTER(HarmonicDesc)
        L.mpm_mag_harmonic_program.argtypes = [hp, C.c_int, vp, vp, vp, vp, vp]
        L.mpm_mag_harmonic_program.restype = C.c_int
        L.mpm_mag_harmonic_backward.argtypes = [hp, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp]
        L.mpm_mag_harmonic_backward.restype = C.c_int
        _bound = True
    return L


class MpmMagDesign:
    """Neighbour matrix of one particle set (built on the device from x0) and
    the region map; forward and backward of the design front end."""

    def __init__(self, x0, radius: float, region=None, n_regions: Optional[int] = None, precision: int = 4,
                 device: str = "cuda"):
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("MpmMagDesign runs on a HIP device only")
        self.precision = int(precision)
        self.dtype = torch.float32 if precision == 4 else torch.float64
        x0 = torch.as_tensor(x0, device=self.device).to(self.dtype).contiguous()
        if x0.dim() != 2 or x0.shape[1] not in (2, 3):
            raise ValueError("x0 must be [N][2] or [N][3]")
        self.N, self.dim = int(x0.shape[0]), int(x0.shape[1])
        if region is not None:
            region = torch.as_tensor(region, device=self.device).to(torch.int32).contiguous()
            if tuple(region.shape) != (self.N,):
                raise ValueError("region must be [N]")
            if n_regions is None:
                n_regions = int(region.max().item()) + 1
            self.n_m = int(n_regions)
        else:
            self.n_m = self.N
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib().mpm_mag_design_create(self.dim, self.N, _ptr(x0), float(radius), _ptr(region),
                                             int(n_regions or 0), self.precision, self._stream(), C.byref(h))
        if st != OK:
            raise MpmMagError(st, "mpm_mag_design_create", lib().mpm_mag_design_last_error(None).decode())
        self._h = h

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, st, where):
        if st != OK:
            raise MpmMagError(st, where, lib().mpm_mag_design_last_error(self._h).decode())

    def _arg(self, t, shape, name):
        t = torch.as_tensor(t, device=self.device).to(self.dtype).contiguous()
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    @property
    def nnz(self) -> int:
        return int(lib().mpm_mag_design_nnz(self._h))

    def forward(self, phi, br_mag, zeta, beta: float, br_max: float = 1.0, delta: float = 1e-6, copies: int = 1):
        """density [copies * N], br [copies * N][dim]: one copy per task sharing the design."""
        phi = self._arg(phi, (self.N,), "phi")
        br_mag = self._arg(br_mag, (self.n_m,), "br_mag")
        zeta = self._arg(zeta, (self.n_m, self.dim), "zeta")
        density = torch.empty(copies * self.N, dtype=self.dtype, device=self.device)
        br = torch.empty((copies * self.N, self.dim), dtype=self.dtype, device=self.device)
        with torch.cuda.device(self.device):
            st = lib().mpm_mag_design_forward(self._h, self._stream(), _ptr(phi), float(beta), _ptr(br_mag),
                                              _ptr(zeta), float(br_max), float(delta), int(copies), _ptr(density),
                                              _ptr(br))
        self._check(st, "mpm_mag_design_forward")
        return density, br

    def backward(self, g_density, g_br, want=(True, True, True), copies: int = 1):
        """Gradients of (phi, br_mag, zeta), the copies' gradients summed."""
        g_density = self._arg(g_density, (copies * self.N,), "g_density")
        g_br = self._arg(g_br, (copies * self.N, self.dim), "g_br")
        g_phi = torch.empty(self.N, dtype=self.dtype, device=self.device) if want[0] else None
        g_mag = torch.empty(self.n_m, dtype=self.dtype, device=self.device) if want[1] else None
        g_zeta = torch.empty((self.n_m, self.dim), dtype=self.dtype, device=self.device) if want[2] else None
        with torch.cuda.device(self.device):
            st = lib().mpm_mag_design_backward(self._h, self._stream(), int(copies), _ptr(g_density), _ptr(g_br),
                                               _ptr(g_phi), _ptr(g_mag), _ptr(g_zeta))
        self._check(st, "mpm_mag_design_backward")
        return g_phi, g_mag, g_zeta

    def close(self):
        if getattr(self, "_h", None):
            lib().mpm_mag_design_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DesignFn(torch.autograd.Function):
    """density, br = DesignFn.apply(fe, phi, br_mag, zeta, beta, br_max, delta, copies).

    The backward runs the transpose on the device at the forward's point; it
    relies on the handle's last forward call being this one (as MpmMagFn
    relies on the last recorded rollout)."""

    @staticmethod
    def forward(ctx, fe: MpmMagDesign, phi, br_mag, zeta, beta, br_max=1.0, delta=1e-6, copies=1):
        density, br = fe.forward(phi, br_mag, zeta, beta, br_max, delta, copies)
        ctx.fe = fe
        ctx.copies = copies
        return density, br

    @staticmethod
    def backward(ctx, g_density, g_br):
        need = ctx.needs_input_grad
        fe, c = ctx.fe, ctx.copies
        if g_density is None:
            g_density = torch.zeros(c * fe.N, dtype=fe.dtype, device=fe.device)
        if g_br is None:
            g_br = torch.zeros((c * fe.N, fe.dim), dtype=fe.dtype, device=fe.device)
        g_phi, g_mag, g_zeta = fe.backward(g_density, g_br, want=(need[1], need[2], need[3]), copies=c)
        return None, g_phi, g_mag, g_zeta, None, None, None, None


def _harmonic_args(b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta):
    eta = torch.as_tensor(eta)
    dev = eta.device if eta.is_cuda else torch.device("cuda")
    dtype = eta.dtype if eta.dtype in (torch.float32, torch.float64) else torch.float32
    conv = lambda t: torch.as_tensor(t, device=dev).to(dtype).contiguous()
    b_a, f, eta = conv(b_a), conv(f), conv(eta)
    n_inst, dim = eta.shape
    if tuple(b_a.shape) != (n_inst,) or tuple(f.shape) != (n_inst,):
        raise ValueError("b_a and f must be [n_inst], eta [n_inst][dim]")
    d = HarmonicDesc(int(dim), int(n_inst), int(n_steps), float(dt), float(b_max), float(f_min), float(f_max),
                     float(delta))
    prec = 4 if dtype == torch.float32 else 8
    return d, prec, dev, dtype, b_a, f, eta


def harmonic_program(b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta=1e-6):
    """Field program [n_inst * n_steps][dim] of the harmonic stimulus (Eqs. 29-30)."""
    d, prec, dev, dtype, b_a, f, eta = _harmonic_args(b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta)
    out = torch.empty((d.n_inst * d.n_steps, d.dim), dtype=dtype, device=dev)
    with torch.cuda.device(dev):
        st = lib().mpm_mag_harmonic_program(C.byref(d), prec, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream),
                                            _ptr(b_a), _ptr(f), _ptr(eta), _ptr(out))
    if st != OK:
        raise MpmMagError(st, "mpm_mag_harmonic_program")
    return out


def harmonic_backward(b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta, g_b_prog, want=(True, True, True)):
    """Gradients of (b_a, f, eta) from the program gradient g_b_prog."""
    d, prec, dev, dtype, b_a, f, eta = _harmonic_args(b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta)
    g = torch.as_tensor(g_b_prog, device=dev).to(dtype).contiguous()
    if tuple(g.shape) != (d.n_inst * d.n_steps, d.dim):
        raise ValueError("g_b_prog must be [n_inst * n_steps][dim]")
    gb = torch.empty(d.n_inst, dtype=dtype, device=dev) if want[0] else None
    gf = torch.empty(d.n_inst, dtype=dtype, device=dev) if want[1] else None
    ge = torch.empty((d.n_inst, d.dim), dtype=dtype, device=dev) if want[2] else None
    with torch.cuda.device(dev):
        st = lib().mpm_mag_harmonic_backward(C.byref(d), prec, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream),
                                             _ptr(b_a), _ptr(f), _ptr(eta), _ptr(g), _ptr(gb), _ptr(gf), _ptr(ge))
    if st != OK:
        raise MpmMagError(st, "mpm_mag_harmonic_backward")
    return gb, gf, ge


class HarmonicFn(torch.autograd.Function):
    """b_prog = HarmonicFn.apply(b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta)."""

    @staticmethod
    def forward(ctx, b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta=1e-6):
        ctx.args = (n_steps, dt, b_max, f_min, f_max, delta)
        ctx.save_for_backward(b_a, f, eta)
        return harmonic_program(b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta)

    @staticmethod
    def backward(ctx, g):
        b_a, f, eta = ctx.saved_tensors
        need = ctx.needs_input_grad
        gb, gf, ge = harmonic_backward(b_a, f, eta, *ctx.args, g, want=(need[0], need[1], need[2]))
        return gb, gf, ge, None, None, None, None, None, None
