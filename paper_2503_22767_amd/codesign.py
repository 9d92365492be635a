"""Co-design loop (Sec. 3.2): structure, material and stimulus optimized
together with Adam over the device path.

One iteration, every arithmetic step in the HIP library:
  design front end (filter, projection, magnetization; one copy of the shared
  design per task, Eq. 35) -> harmonic stimulus of every task (Eqs. 29-30) ->
  recorded rollout and losses -> adjoint -> transposes of the stimulus and the
  front end (the tasks' design gradients summed) -> Adam with the variables
  mapped back into their bounds (Eqs. 34c-d, 35c-d).
The host keeps the loss history for the convergence rule (the mean of the last
10 losses against the 10 before, relative change below 1e-3) and raises the
projection sharpness beta every 10 iterations up to 128 (its schedule; the
starting value and the factor are parameters).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import design as PD
from .mpm_mag import OK, MpmMag, MpmMagError, _ptr


def _lib():
    L = PD.lib()
    if not getattr(L, "_adam_bound", False):
        vp = C.c_void_p
        d = C.c_double
        L.mpm_mag_adam_step.argtypes = [C.c_int, vp, C.c_int64, vp, vp, vp, vp, C.c_int, d, d, d, d, d, d]
        L.mpm_mag_adam_step.restype = C.c_int
        L._adam_bound = True
    return L


def adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
              lo: float, hi: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """In-place Adam update of a contiguous device tensor (and its moments) with
    the bound map; all four tensors share dtype and size."""
    for t in (param, grad, m, v):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != param.dtype or t.numel() != param.numel():
            raise ValueError("adam_step: contiguous device tensors of one dtype and size")
    prec = 4 if param.dtype == torch.float32 else 8
    st = _lib().mpm_mag_adam_step(prec, C.c_void_p(torch.cuda.current_stream(param.device).cuda_stream),
                                  param.numel(), _ptr(param), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                                  float(beta1), float(beta2), float(eps), float(lo), float(hi))
    if st != OK:
        raise MpmMagError(st, "mpm_mag_adam_step")


def converged(history: Sequence[float], window: int = 10, tol: float = 1e-3) -> bool:
    """The paper's rule: relative absolute change between the mean of the last
    `window` objective values and the mean of the `window` before, below tol."""
    if len(history) < 2 * window:
        return False
    last = float(np.mean(history[-window:]))
    prev = float(np.mean(history[-2 * window:-window]))
    return abs(last - prev) <= tol * max(abs(prev), 1e-300)


def beta_at(iteration: int, beta0: float = 1.0, factor: float = 2.0, every: int = 10, beta_max: float = 128.0):
    """Projection sharpness at a 0-based iteration: beta0, multiplied by factor
    every `every` iterations, capped at beta_max."""
    return min(beta_max, beta0 * factor ** (iteration // every))


@dataclass
class Bounds:
    phi: tuple = (0.0, 1.0)
    br_mag: tuple = (0.0, 1.0)
    zeta: tuple = (-1.0, 1.0)
    b_a: tuple = (0.0, 1.0)
    f: tuple = (0.0, 1.0)
    eta: tuple = (-1.0, 1.0)


@dataclass
class CoDesignConfig:
    radius: float                    # filter radius R
    b_max: float                     # B_max of Eq. 29
    f_min: float
    f_max: float
    br_max: float = 1.0              # Br_max of Eq. 26
    delta: float = 1e-6              # delta of Eqs. 27 and 30
    lr: float = 0.01
    beta0: float = 1.0
    beta_factor: float = 2.0
    beta_every: int = 10
    beta_max: float = 128.0
    bounds: Bounds = field(default_factory=Bounds)


class CoDesign:
    """Tasks l = 0..L-1 share one particle set x0 and design (phi, region
    magnitudes and orientations); each has its own instance parameters (loss,
    contact, ...) and harmonic stimulus. Every task's parameters must have
    n_segments = n_steps and seg_steps = 1 (one program row per step)."""

    def __init__(self, task_params: Sequence[dict], x0, cfg: CoDesignConfig, region=None,
                 n_regions: Optional[int] = None, targets=None, masks=None, precision: int = 4, seed: int = 0,
                 init=None):
        self.cfg = cfg
        self.L = len(task_params)
        p0 = task_params[0]
        self.T, self.dim, self.dt = int(p0["n_steps"]), int(p0["dim"]), float(p0["dt"])
        for p in task_params:
            if int(p["n_segments"]) != self.T or int(p.get("seg_steps", 1)) != 1 or p.get("periodic", 0):
                raise ValueError("co-design tasks need one field segment per step (n_segments = n_steps, "
                                 "seg_steps = 1, not periodic)")
            if float(p["dt"]) != self.dt or int(p["dim"]) != self.dim:
                raise ValueError("tasks must share dt and dim")
        self.dtype = torch.float32 if precision == 4 else torch.float64
        x0 = np.asarray(x0, dtype=np.float64)
        self.N = len(x0)
        self.fe = PD.MpmMagDesign(x0, cfg.radius, region=region, n_regions=n_regions, precision=precision)
        self.sim = MpmMag(list(task_params), [self.N] * self.L, precision=precision)
        dev = self.fe.device
        cu = lambda a: torch.as_tensor(np.asarray(a), device=dev).to(self.dtype).contiguous()
        self.x0 = cu(np.tile(x0, (self.L, 1)))
        self.target = None if targets is None else cu(np.concatenate(targets))
        self.mask = None if masks is None else torch.as_tensor(np.concatenate(masks), dtype=torch.uint8,
                                                               device=dev).contiguous()
        rng = np.random.default_rng(seed)
        n_m, d, L = self.fe.n_m, self.dim, self.L
        init = dict(init or {})
        self.var = {
            "phi": cu(init.get("phi", np.full(self.N, 0.5))),
            "br_mag": cu(init.get("br_mag", np.full(n_m, 0.5))),
            "zeta": cu(init.get("zeta", rng.uniform(-1, 1, (n_m, d)))),
            "b_a": cu(init.get("b_a", np.full(L, 0.5))),
            "f": cu(init.get("f", np.full(L, 0.5))),
            "eta": cu(init.get("eta", rng.uniform(-1, 1, (L, d)))),
        }
        self.m = {k: torch.zeros_like(t) for k, t in self.var.items()}
        self.v = {k: torch.zeros_like(t) for k, t in self.var.items()}
        self.dloss = torch.ones(L, dtype=self.dtype, device=dev)
        self.history: List[float] = []
        self.betas: List[float] = []     # the sharpness each history entry was taken at
        self.iteration = 0

    @property
    def beta(self) -> float:
        c = self.cfg
        return beta_at(self.iteration, c.beta0, c.beta_factor, c.beta_every, c.beta_max)

    def _harm(self):
        c = self.cfg
        return (self.T, self.dt, c.b_max, c.f_min, c.f_max, c.delta)

    def evaluate(self, record: bool = True):
        """Losses [L] of the current design (and, with record, the state for gradients)."""
        c, v = self.cfg, self.var
        density, br = self.fe.forward(v["phi"], v["br_mag"], v["zeta"], self.beta, c.br_max, c.delta, copies=self.L)
        b_prog = PD.harmonic_program(v["b_a"], v["f"], v["eta"], *self._harm())
        loss, _ = self.sim.rollout(self.x0, density, br, b_prog, self.target, self.mask, record=record, want_x=False)
        return loss

    def gradients(self):
        """Gradients of the summed loss (Eq. 35) with respect to every design variable."""
        g_d, g_b, g_p = self.sim.backward(self.dloss)
        g_phi, g_mag, g_zeta = self.fe.backward(g_d, g_b, copies=self.L)
        v = self.var
        g_ba, g_f, g_eta = PD.harmonic_backward(v["b_a"], v["f"], v["eta"], *self._harm(), g_p)
        return {"phi": g_phi, "br_mag": g_mag, "zeta": g_zeta, "b_a": g_ba, "f": g_f, "eta": g_eta}

    def step(self) -> float:
        """One co-design iteration; returns the summed loss of the design it started from."""
        loss = self.evaluate(record=True)
        grads = self.gradients()
        b = self.cfg.bounds
        t = self.iteration + 1
        for k, g in grads.items():
            lo, hi = getattr(b, k)
            adam_step(self.var[k], g, self.m[k], self.v[k], t, self.cfg.lr, lo, hi)
        total = float(loss.double().sum())
        self.history.append(total)
        self.betas.append(self.beta)
        self.iteration += 1
        return total

    def converged(self, at_final_beta: bool = False) -> bool:
        """The paper's convergence rule over the loss history; with
        at_final_beta, over the iterations taken at the capped sharpness only
        (the loss moves each time beta rises)."""
        if not at_final_beta:
            return converged(self.history)
        k = next((i for i, b in enumerate(self.betas) if b >= self.cfg.beta_max), None)
        return k is not None and converged(self.history[k:])

    def close(self):
        self.fe.close()
        self.sim.close()
