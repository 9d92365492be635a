"""Python binding of the C ABI in include/mpm_mag.h (ctypes; argument marshalling only).

Every step of the rollout and of its adjoint runs in the HIP kernels of
libmpm_mag.so; PyTorch provides device memory and the stream. Importing this
module on a machine without the built library raises immediately: there is no
CPU fallback.

  sim = MpmMag(params_list, n_particles, precision=4)     # mpm_mag_create
  loss, x_final = sim.rollout(x0, density, br, b_prog, target, mask, record=True)
  g_density, g_br, g_b_prog = sim.backward(dloss)          # mpm_mag_backward
  sim.close()                                              # mpm_mag_destroy

MpmMagFn wraps the pair as a torch.autograd.Function so that
loss.backward() yields d(loss)/d(density, br, b_prog).
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; MPM_MAG_LIB may name another build of the same library
LIB_PATH = os.environ.get("MPM_MAG_LIB") or os.path.join(HERE, "libmpm_mag.so")

OK, EINVAL, ENOMEM, EHIP, EDOMAIN, EINVERT, ENONFINITE, ESTATE = range(8)


MAX_OBSTACLES = 4
OBSTACLE_HALFSPACE, OBSTACLE_SPHERE, OBSTACLE_BOX = 1, 2, 3


class ObstacleDesc(C.Structure):
    """Mirror of mpm_mag_obstacle."""
    _fields_ = [("kind", C.c_int), ("attached", C.c_int), ("a", C.c_double * 3), ("b", C.c_double * 3),
                ("mu", C.c_double), ("vel", C.c_double * 3)]


class InstanceDesc(C.Structure):
    """Mirror of mpm_mag_instance_desc."""
    _fields_ = [
        ("dim", C.c_int), ("n_grid", C.c_int), ("dt", C.c_double), ("n_steps", C.c_int),
        ("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double), ("mu0", C.c_double),
        ("simp_eps", C.c_double), ("simp_q", C.c_double), ("damping", C.c_double),
        ("gravity", C.c_double * 3), ("wall_cells", C.c_int), ("clamp_xmax", C.c_double),
        ("floor_on", C.c_int), ("floor_y", C.c_double), ("floor_mu", C.c_double),
        ("particle_volume", C.c_double), ("n_segments", C.c_int), ("seg_steps", C.c_int),
        ("periodic", C.c_int), ("loss_kind", C.c_int), ("loss_dir", C.c_double * 3),
        ("ckpt_every", C.c_int), ("n_obstacles", C.c_int), ("obstacles", ObstacleDesc * MAX_OBSTACLES),
        ("ckpt_budget_bytes", C.c_int64), ("mass_eps", C.c_double),
    ]


def _vec3(v):
    return (C.c_double * 3)(*([float(x) for x in list(v)] + [0.0] * 3)[:3])


def desc_from_params(p: dict) -> InstanceDesc:
    """p["obstacles"] (optional): a list of dicts with kind, a, b, mu (default 0),
    vel (default 0) and attached (default 0)."""
    d = InstanceDesc()
    obst = list(p.get("obstacles", []))
    if len(obst) > MAX_OBSTACLES:
        raise ValueError(f"at most {MAX_OBSTACLES} obstacles")
    d.n_obstacles = len(obst)
    for j, o in enumerate(obst):
        d.obstacles[j] = ObstacleDesc(int(o["kind"]), int(o.get("attached", 0)), _vec3(o["a"]), _vec3(o["b"]),
                                      float(o.get("mu", 0.0)), _vec3(o.get("vel", [0.0, 0.0, 0.0])))
    for name, _ in InstanceDesc._fields_:
        if name not in p or name in ("n_obstacles", "obstacles"):
            continue
        val = p[name]
        if name in ("gravity", "loss_dir"):
            vals = [float(v) for v in list(val)] + [0.0] * 3
            setattr(d, name, (C.c_double * 3)(*vals[:3]))
        else:
            setattr(d, name, val)
    return d


class MpmMagError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {_strerror(status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


_lib = None


def lib():
    """Load libmpm_mag.so (built in-tree by paper_2503_22767_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the MPM path has no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i64 = C.c_void_p, C.c_int64
    L.mpm_mag_create.argtypes = [C.POINTER(InstanceDesc), C.c_int, C.POINTER(i64), C.c_int, C.POINTER(vp)]
    L.mpm_mag_create.restype = C.c_int
    L.mpm_mag_rollout.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]
    L.mpm_mag_rollout.restype = C.c_int
    L.mpm_mag_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.mpm_mag_backward.restype = C.c_int
    L.mpm_mag_destroy.argtypes = [vp]
    L.mpm_mag_destroy.restype = None
    L.mpm_mag_strerror.argtypes = [C.c_int]
    L.mpm_mag_strerror.restype = C.c_char_p
    L.mpm_mag_last_error.argtypes = [vp]
    L.mpm_mag_last_error.restype = C.c_char_p
    L.mpm_mag_set_option.argtypes = [vp, C.c_char_p, i64]
    L.mpm_mag_set_option.restype = C.c_int
    L.mpm_mag_num_kernels.argtypes = []
    L.mpm_mag_num_kernels.restype = C.c_int
    L.mpm_mag_kernel_name.argtypes = [C.c_int]
    L.mpm_mag_kernel_name.restype = C.c_char_p
    L.mpm_mag_kernel_stats.argtypes = [vp, C.c_int, C.POINTER(i64), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.mpm_mag_kernel_stats.restype = C.c_int
    L.mpm_mag_kernel_flops.argtypes = [vp, C.c_int, C.POINTER(C.c_double)]
    L.mpm_mag_kernel_flops.restype = C.c_int
    L.mpm_mag_device_bytes.argtypes = [vp]
    L.mpm_mag_device_bytes.restype = i64
    L.mpm_mag_rollout_noalloc.argtypes = [C.POINTER(InstanceDesc), C.c_int, C.POINTER(i64), C.c_int, vp, vp, vp, vp,
                                          vp, vp, vp, vp, vp]
    L.mpm_mag_rollout_noalloc.restype = C.c_int
    L.mpm_mag_noalloc_scratch_bytes.argtypes = []
    L.mpm_mag_noalloc_scratch_bytes.restype = i64
    L.mpm_mag_set_branch_trace.argtypes = [vp, vp, i64]
    L.mpm_mag_set_branch_trace.restype = C.c_int
    L.mpm_mag_trace_nodes.argtypes = [vp]
    L.mpm_mag_trace_nodes.restype = i64
    L.mpm_mag_scatter_stats.argtypes = [vp, C.POINTER(i64), C.c_int]
    L.mpm_mag_scatter_stats.restype = C.c_int
    _lib = L
    return L


def _strerror(status: int) -> str:
    try:
        return lib().mpm_mag_strerror(status).decode()
    except Exception:  # library missing while formatting another error
        return f"status {status}"


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class MpmMag:
    """One handle of the library: a batch of design instances advanced together."""

    def __init__(self, params: Sequence[dict], n_particles: Sequence[int], precision: int = 4,
                 device: str = "cuda"):
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("MpmMag runs on a HIP device only")
        self.params = [dict(p) for p in params]
        self.n_particles = [int(n) for n in n_particles]
        self.n_inst = len(self.params)
        self.dim = int(self.params[0]["dim"])
        self.precision = int(precision)
        self.dtype = torch.float32 if precision == 4 else torch.float64
        self.N = sum(self.n_particles)
        self.S_tot = sum(int(p["n_segments"]) for p in self.params)
        descs = (InstanceDesc * self.n_inst)(*[desc_from_params(p) for p in self.params])
        counts = (C.c_int64 * self.n_inst)(*self.n_particles)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib().mpm_mag_create(descs, self.n_inst, counts, self.precision, C.byref(h))
        if st != OK:
            raise MpmMagError(st, "mpm_mag_create", lib().mpm_mag_last_error(None).decode())
        self._h = h
        # MPM_MAG_KERNEL_TIMING=1: time every launch with events and print the
        # per-kernel table to stderr when the handle is closed
        self._print_timing = os.environ.get("MPM_MAG_KERNEL_TIMING", "0") not in ("", "0")
        if self._print_timing:
            self.set_option("kernel_timing", 1)

    # -- helpers --------------------------------------------------------------
    def _check(self, st: int, where: str):
        if st != OK:
            raise MpmMagError(st, where, lib().mpm_mag_last_error(self._h).decode())

    def _arg(self, t, shape, dtype=None, name="") -> Optional[torch.Tensor]:
        if t is None:
            return None
        dtype = dtype or self.dtype
        t = torch.as_tensor(t, device=self.device).to(dtype).contiguous()
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # -- ABI ------------------------------------------------------------------
    def rollout(self, x0, density, br, b_prog, target=None, mask=None, record: bool = False,
                want_x: bool = True):
        d, N = self.dim, self.N
        x0 = self._arg(x0, (N, d), name="x0")
        density = self._arg(density, (N,), name="density")
        br = self._arg(br, (N, d), name="br")
        b_prog = self._arg(b_prog, (self.S_tot, d), name="b_prog")
        target = self._arg(target, (N, d), name="target")
        mask = self._arg(mask, (N,), dtype=torch.uint8, name="mask")
        loss = torch.empty(self.n_inst, dtype=self.dtype, device=self.device)
        x_final = torch.empty((N, d), dtype=self.dtype, device=self.device) if want_x else None
        with torch.cuda.device(self.device):
            st = lib().mpm_mag_rollout(self._h, self._stream(), _ptr(x0), _ptr(density), _ptr(br), _ptr(b_prog),
                                       _ptr(target), _ptr(mask), _ptr(x_final), _ptr(loss), int(bool(record)))
        self._check(st, "mpm_mag_rollout")
        return loss, x_final

    def backward(self, dloss, want=(True, True, True), dx_final=None):
        """Gradients (density, br, b_prog) of sum_k dloss[k] loss_k plus, when
        dx_final [N, dim] is given, of sum_p dx_final_p . x_p(T)."""
        dloss = self._arg(dloss, (self.n_inst,), name="dloss")
        dx_final = self._arg(dx_final, (self.N, self.dim), name="dx_final")
        gd = torch.empty(self.N, dtype=self.dtype, device=self.device) if want[0] else None
        gb = torch.empty((self.N, self.dim), dtype=self.dtype, device=self.device) if want[1] else None
        gp = torch.empty((self.S_tot, self.dim), dtype=self.dtype, device=self.device) if want[2] else None
        with torch.cuda.device(self.device):
            st = lib().mpm_mag_backward(self._h, self._stream(), _ptr(dloss), _ptr(dx_final), _ptr(gd), _ptr(gb),
                                        _ptr(gp))
        self._check(st, "mpm_mag_backward")
        return gd, gb, gp

    def set_option(self, key: str, value: int):
        self._check(lib().mpm_mag_set_option(self._h, key.encode(), int(value)), f"mpm_mag_set_option({key})")

    def kernel_stats(self, reset: bool = False) -> dict:
        L = lib()
        out = {}
        for k in range(L.mpm_mag_num_kernels()):
            n, ms, b, f = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
            self._check(L.mpm_mag_kernel_stats(self._h, k, C.byref(n), C.byref(ms), C.byref(b)), "kernel_stats")
            self._check(L.mpm_mag_kernel_flops(self._h, k, C.byref(f)), "kernel_flops")
            out[L.mpm_mag_kernel_name(k).decode()] = dict(launches=n.value, ms=ms.value, bytes=b.value, flops=f.value)
        if reset:
            L.mpm_mag_kernel_stats(self._h, -1, None, None, None)
        return out

    def device_bytes(self) -> int:
        return int(lib().mpm_mag_device_bytes(self._h))

    def trace_nodes(self) -> int:
        return int(lib().mpm_mag_trace_nodes(self._h))

    def scatter_stats(self) -> dict:
        """Scatter fallback counts of the last rollout or backward."""
        out = (C.c_int64 * 3)()
        self._check(lib().mpm_mag_scatter_stats(self._h, out, 3), "mpm_mag_scatter_stats")
        return {"wave_boxes": int(out[0]), "atomic_waves": int(out[1]), "list_overflows": int(out[2])}

    def set_branch_trace(self, trace: Optional[torch.Tensor]):
        """Record the grid update's per-node branch decisions of the following
        rollouts' forward steps into `trace` (a device int16/uint16 tensor with
        n_steps * trace_nodes() elements), or stop with None."""
        if trace is not None:
            if trace.device.type != "cuda" or trace.element_size() != 2 or not trace.is_contiguous():
                raise ValueError("branch trace: a contiguous 16-bit device tensor")
            self._trace = trace
            n = trace.numel()
        else:
            self._trace = None
            n = 0
        self._check(lib().mpm_mag_set_branch_trace(self._h, _ptr(trace), int(n)), "mpm_mag_set_branch_trace")

    def print_kernel_stats(self, file=None):
        """Per-kernel launches, time and rates since the last reset."""
        file = file or sys.stderr
        print(f"{'kernel':14s} {'launches':>9s} {'total ms':>10s} {'avg us':>9s} {'GB/s':>8s} {'TFLOP/s':>8s}", file=file)
        for k, v in self.kernel_stats().items():
            if not v["launches"]:
                continue
            avg = v["ms"] / v["launches"] * 1e3
            gbs = v["bytes"] / v["launches"] / (avg * 1e3) if avg > 0 and v["bytes"] else 0.0
            tfl = v["flops"] / v["launches"] / (avg * 1e6) if avg > 0 and v["flops"] else 0.0
            print(f"{k:14s} {v['launches']:9d} {v['ms']:10.3f} {avg:9.2f} {gbs:8.1f} {tfl:8.2f}", file=file)

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_print_timing", False):
                torch.cuda.synchronize(self.device)
                self.print_kernel_stats()
            lib().mpm_mag_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rollout_noalloc(params, n_particles, precision, x0, density, br, b_prog, target=None, mask=None,
                    device="cuda"):
    """Plain rollout through mpm_mag_rollout_noalloc (no device allocation in
    the library: its buffers come from a static per-GPU scratch array). Inputs
    are device tensors of the precision's dtype as for MpmMag.rollout; returns
    (loss[n_inst], x_final[N, dim]), allocated here by the caller's side."""
    L = lib()
    n_inst = len(params)
    descs = (InstanceDesc * n_inst)(*[desc_from_params(p) for p in params])
    counts = (C.c_int64 * n_inst)(*[int(n) for n in n_particles])
    dtype = torch.float32 if precision == 4 else torch.float64
    N, d = int(sum(n_particles)), int(params[0]["dim"])
    loss = torch.empty(n_inst, dtype=dtype, device=device)
    x_final = torch.empty((N, d), dtype=dtype, device=device)
    with torch.cuda.device(device):
        st = L.mpm_mag_rollout_noalloc(descs, n_inst, counts, int(precision),
                                       C.c_void_p(torch.cuda.current_stream(device).cuda_stream), _ptr(x0),
                                       _ptr(density), _ptr(br), _ptr(b_prog), _ptr(target), _ptr(mask),
                                       _ptr(x_final), _ptr(loss))
    if st != OK:
        raise MpmMagError(st, "mpm_mag_rollout_noalloc", L.mpm_mag_last_error(None).decode())
    return loss, x_final


class MpmMagFn(torch.autograd.Function):
    """loss[n_inst], x_final = MpmMagFn.apply(sim, x0, density, br, b_prog, target, mask).

    Backward returns the gradient with respect to density, br and b_prog,
    computed by mpm_mag_backward over the recorded rollout, of the losses and of
    any function of the final positions the caller builds on x_final (its
    gradient goes in as mpm_mag_backward's dx_final seed)."""

    @staticmethod
    def forward(ctx, sim: MpmMag, x0, density, br, b_prog, target=None, mask=None):
        loss, x_final = sim.rollout(x0, density, br, b_prog, target, mask, record=True)
        ctx.sim = sim
        ctx.set_materialize_grads(False)   # an unused output's gradient arrives as None
        return loss, x_final

    @staticmethod
    def backward(ctx, dloss, dx_final):
        sim = ctx.sim
        need = ctx.needs_input_grad
        if dloss is None:
            dloss = torch.zeros(sim.n_inst, dtype=sim.dtype, device=sim.device)
        gd, gb, gp = sim.backward(dloss, want=(need[2], need[3], need[4]), dx_final=dx_final)
        return None, None, gd, gb, gp, None, None


def instance_tensors(instances, device="cuda", dtype=torch.float32):
    """Concatenate the arrays of several workload instances into device tensors."""
    cat = lambda xs: torch.cat([torch.as_tensor(x) for x in xs]).to(device=device, dtype=dtype).contiguous()
    x0 = cat([i.x0 for i in instances])
    density = cat([i.density for i in instances])
    br = cat([i.br for i in instances])
    b_prog = cat([i.b_prog for i in instances])
    if any(i.target is not None for i in instances):
        target = cat([i.target if i.target is not None else i.x0 for i in instances])
    else:
        target = None
    if any(i.mask is not None for i in instances):
        mask = torch.cat([torch.as_tensor(i.mask if i.mask is not None else [1] * i.n, dtype=torch.uint8)
                          for i in instances]).to(device).contiguous()
    else:
        mask = None
    return x0, density, br, b_prog, target, mask
