"""Seeded synthetic workloads for the magneto-elastic MPM rollout.

This module only builds inputs: particle lattices, design densities, remanent
magnetization vectors, piecewise-constant field programs, loss targets and the
per-instance parameter records. It holds none of the simulation's arithmetic,
so both the FP64 oracle (tests) and the HIP library consume exactly the same
arrays.

Geometry follows the paper's particle representation (Sec. 2.2: particles are
distributed uniformly inside the material body, each carrying volume and mass;
Eq. 33 for the mass). Design variables are the projected density (Sec. 3.1,
Eq. 25 output) and the reference remanence vector (Eq. 26 output); the field
program is a piecewise-constant stand-in for the harmonic stimulus of Eq. 29.

Workloads (the paper prints no particle counts, grids or targets, so these are
synthetic stand-ins with its case-study shapes):
  cantilever2d  2D cantilever, 64^2 grid, 1,280 particles, FP64, 500 steps,
                final-shape loss
  walker2d      2D three-leg walker on a frictional floor, 256^2 grid, 30,593
                particles, 2,000 steps, centre-of-mass displacement loss
  plate3d       3D clamped plate, 64^3 grid, 16,384 particles, 1,000 steps,
                surface-shape loss
  batch2d       64 independent 2D beams/walkers, 1k..30k particles each, 1,000 steps
  quadruped3d   3D quadruped, 128^3 grid, 1,146,344 particles, three field
                programs sharing one design (Eq. 35), 4,000 steps each
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Loss kinds (interface values shared by every consumer of these records).
LOSS_FINAL_MSE = 0   # mean squared distance of final positions to a target (Eq. 38)
LOSS_COM_DISP = 1    # minus the centre-of-mass displacement along e (Eq. 40)
LOSS_TRAJ_VEL = 2    # minus the time-integrated mass-averaged velocity along e (Eq. 39)
LOSS_TIP_DISP = 3    # minus the mean displacement of a particle subset along e (Eqs. 36-37)


def default_params(dim: int, n_grid: int, dt: float, n_steps: int, spacing: float) -> dict:
    """Per-instance scalar parameters with the nondimensional defaults."""
    return dict(
        dim=dim, n_grid=n_grid, dt=dt, n_steps=n_steps,
        E=1.0, nu=0.3, rho=1.0, mu0=1.0, simp_eps=1e-3, simp_q=3.0, damping=0.0,
        gravity=[0.0, 0.0, 0.0], wall_cells=3, clamp_xmax=-1.0,
        floor_on=0, floor_y=0.0, floor_mu=0.0,
        particle_volume=spacing ** dim,
        n_segments=1, seg_steps=0, periodic=0,
        loss_kind=LOSS_FINAL_MSE, loss_dir=[1.0, 0.0, 0.0],
        ckpt_every=0,
    )


@dataclasses.dataclass
class Instance:
    params: dict
    x0: np.ndarray                  # (N, d) float64
    density: np.ndarray             # (N,)
    br: np.ndarray                  # (N, d) reference remanence
    b_prog: np.ndarray              # (S, d) applied field per segment
    target: Optional[np.ndarray]    # (N, d) or None
    mask: Optional[np.ndarray]      # (N,) uint8 or None
    group: int = 0                  # instances with equal group share density and br

    @property
    def n(self) -> int:
        return int(self.x0.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    instances: List[Instance]
    precision: int                  # 4 = FP32, 8 = FP64
    description: str = ""

    @property
    def n_particles(self) -> int:
        return sum(i.n for i in self.instances)

    @property
    def n_steps(self) -> int:
        return self.instances[0].params["n_steps"]

    def particle_steps(self) -> int:
        return sum(i.n * i.params["n_steps"] for i in self.instances)


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def box_particles(corner, lengths, spacing) -> np.ndarray:
    """Lattice points (k + 1/2) * spacing inside an axis-aligned box, x fastest.

    The count per axis is round(length / spacing)."""
    d = len(corner)
    counts = [int(math.floor(lengths[k] / spacing + 0.5)) for k in range(d)]
    axes = [corner[k] + (np.arange(counts[k]) + 0.5) * spacing for k in range(d)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    pts = np.stack([g.ravel() for g in grids[::-1]], axis=1)
    return pts.astype(np.float64)


def _unit_vectors(rng, n: int, dim: int) -> np.ndarray:
    if dim == 2:
        th = rng.uniform(0.0, 2.0 * np.pi, size=n)
        return np.stack([np.cos(th), np.sin(th)], axis=1)
    v = rng.standard_normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _rotation_target(x0: np.ndarray, centre, alpha: float) -> np.ndarray:
    c, s = math.cos(alpha), math.sin(alpha)
    d = x0 - np.asarray(centre)[None, :]
    out = x0.copy()
    out[:, 0] = centre[0] + c * d[:, 0] - s * d[:, 1]
    out[:, 1] = centre[1] + s * d[:, 0] + c * d[:, 1]
    return out


# ----------------------------------------------------------------------------
# individual robots
# ----------------------------------------------------------------------------

def beam_instance(rng, *, dim: int, n_grid: int, s: int, length: float, height: float,
                  dt: float, n_steps: int, n_segments: int, width: float = None,
                  loss: str = "rotation") -> Instance:
    """Cantilever beam/plate clamped at its left end, centred on the y (and z) = 0.5
    node line, loaded only by the field (no gravity)."""
    dx = 1.0 / n_grid
    h = dx / s
    x_left = 4 * dx
    if dim == 2:
        corner = [x_left, 0.5 - height / 2]
        lengths = [length, height]
    else:
        w = height if width is None else width
        corner = [x_left, 0.5 - height / 2, 0.5 - w / 2]
        lengths = [length, height, w]
    x0 = box_particles(corner, lengths, h)
    n = x0.shape[0]
    p = default_params(dim, n_grid, dt, n_steps, h)
    p["clamp_xmax"] = x_left + dx
    p["n_segments"] = n_segments
    p["seg_steps"] = (n_steps + n_segments - 1) // n_segments
    density = rng.uniform(0.3, 1.0, size=n)
    br = _unit_vectors(rng, n, dim)
    b_prog = rng.uniform(-0.5, 0.5, size=(n_segments, dim))
    if loss == "rotation":
        alpha = rng.uniform(-0.05, 0.05)
        target = _rotation_target(x0, [x_left + dx, 0.5], alpha)
        mask = None
        p["loss_kind"] = LOSS_FINAL_MSE
    else:  # surface bend
        a = rng.uniform(-0.5, 0.5)
        lo = np.min(x0, axis=0) - 0.5 * h
        hi = np.max(x0, axis=0) + 0.5 * h
        near = np.zeros(n, dtype=bool)
        for k in range(1, dim):
            near |= (x0[:, k] - lo[k] < h) | (hi[k] - x0[:, k] < h)
        mask = near.astype(np.uint8)
        target = x0.copy()
        target[:, 1] += a * (x0[:, 0] - x_left) ** 2
        p["loss_kind"] = LOSS_FINAL_MSE
    return Instance(p, x0, density, br, b_prog, target, mask)


def walker2d_particles(n_grid: int, s: int, scale: float = 1.0, x_left: float = 0.1,
                       floor_y: float = 0.05) -> np.ndarray:
    """Rectangle body 0.4 x 0.1 on three 0.05 x 0.08 legs (left, centre, right),
    leg bottoms on the floor line; all lengths multiplied by `scale`."""
    h = (1.0 / n_grid) / s
    bw, bh, lw, lh = 0.4 * scale, 0.1 * scale, 0.05 * scale, 0.08 * scale
    parts = [box_particles([x_left, floor_y + lh], [bw, bh], h)]
    for lx in (x_left, x_left + 0.5 * (bw - lw), x_left + bw - lw):
        parts.append(box_particles([lx, floor_y], [lw, lh], h))
    return np.concatenate(parts, axis=0)


def walker_instance(rng, *, n_grid: int, s: int, dt: float, n_steps: int, n_segments: int,
                    seg_steps: int = 25, scale: float = 1.0) -> Instance:
    dx = 1.0 / n_grid
    h = dx / s
    x0 = walker2d_particles(n_grid, s, scale)
    n = x0.shape[0]
    p = default_params(2, n_grid, dt, n_steps, h)
    p.update(gravity=[0.0, -1.0, 0.0], floor_on=1, floor_y=0.05, floor_mu=0.5,
             n_segments=n_segments, seg_steps=seg_steps, periodic=1,
             loss_kind=LOSS_COM_DISP, loss_dir=[1.0, 0.0, 0.0])
    density = rng.uniform(0.3, 1.0, size=n)
    br = _unit_vectors(rng, n, 2)
    b_prog = rng.uniform(-0.5, 0.5, size=(n_segments, 2))
    return Instance(p, x0, density, br, b_prog, None, None)


def quadruped_particles(n_grid: int, s: int, floor_y: float = 0.05) -> np.ndarray:
    """Block body 0.6 (x) x 0.15 (y, height) x 0.2 (z) on four 0.08^3 corner legs."""
    h = (1.0 / n_grid) / s
    leg = 0.08
    body = box_particles([0.1, floor_y + leg, 0.4], [0.6, 0.15, 0.2], h)
    parts = [body]
    for lx in (0.1, 0.7 - leg):
        for lz in (0.4, 0.6 - leg):
            parts.append(box_particles([lx, floor_y, lz], [leg, leg, leg], h))
    return np.concatenate(parts, axis=0)


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def make_cantilever2d(seed: int = 1, n_steps: int = 500) -> Workload:
    rng = np.random.default_rng(seed)
    inst = beam_instance(rng, dim=2, n_grid=64, s=2, length=0.625, height=0.125,
                         dt=1e-4, n_steps=500, n_segments=5)
    inst.params["n_steps"] = n_steps
    inst.params["ckpt_every"] = 1
    return Workload("cantilever2d", [inst], 8,
                    "2D plane-strain cantilever, 64^2 grid, 1,280 particles, FP64")


def make_walker2d(seed: int = 2, n_steps: int = 2000) -> Workload:
    rng = np.random.default_rng(seed)
    inst = walker_instance(rng, n_grid=256, s=3, dt=5e-5, n_steps=2000, n_segments=20)
    inst.params["n_steps"] = n_steps
    inst.params["ckpt_every"] = 100
    return Workload("walker2d", [inst], 4,
                    "2D three-leg walker, 256^2 grid, 30,593 particles, floor mu=0.5")


def make_plate3d(seed: int = 3, n_steps: int = 1000, n_grid: int = 64) -> Workload:
    rng = np.random.default_rng(seed)
    inst = beam_instance(rng, dim=3, n_grid=n_grid, s=2, length=0.5, height=0.125,
                         dt=1e-4, n_steps=1000, n_segments=10, loss="bend")
    inst.params["n_steps"] = n_steps
    inst.params["ckpt_every"] = 100
    return Workload("plate3d", [inst], 4,
                    f"3D clamped plate, {n_grid}^3 grid, {inst.n} particles")


def make_batch2d(seed: int = 4, n_steps: int = 1000, n_instances: int = 64) -> Workload:
    rng = np.random.default_rng(seed)
    counts = np.round(np.exp(rng.uniform(math.log(1e3), math.log(3e4), size=n_instances)))
    insts = []
    for k in range(n_instances):
        nk = int(counts[k])
        n_grid = 128 if nk < 8000 else 256
        s_prog = int(rng.integers(5, 21))
        if k % 2 == 0:
            # beam of aspect 5:1 at 2 particles per cell and axis
            ny = max(2, int(round(math.sqrt(nk / 5.0))))
            h = (1.0 / n_grid) / 2
            inst = beam_instance(rng, dim=2, n_grid=n_grid, s=2, length=5 * ny * h,
                                 height=ny * h, dt=1e-4, n_steps=n_steps, n_segments=s_prog)
        else:
            scale = math.sqrt(nk / 30593.0) * 256.0 / n_grid
            inst = walker_instance(rng, n_grid=n_grid, s=3, dt=5e-5, n_steps=n_steps,
                                   n_segments=s_prog, scale=scale)
        inst.params["n_steps"] = n_steps
        inst.params["ckpt_every"] = 100
        insts.append(inst)
    return Workload("batch2d", insts, 4, f"{n_instances} batched 2D beams/walkers")


def make_quadruped3d(seed: int = 5, n_steps: int = 4000, n_grid: int = 128, s: int = 3) -> Workload:
    rng = np.random.default_rng(seed)
    dx = 1.0 / n_grid
    h = dx / s
    x0 = quadruped_particles(n_grid, s)
    n = x0.shape[0]
    density = rng.uniform(0.3, 1.0, size=n)
    br = _unit_vectors(rng, n, 3)
    progs = [rng.uniform(-0.5, 0.5, size=(40, 3)) for _ in range(3)]
    a = rng.uniform(-0.5, 0.5)
    top = x0[:, 1].max()
    mask = (top - x0[:, 1] < h).astype(np.uint8)
    target = x0.copy()
    target[:, 1] += a * (x0[:, 0] - 0.4) ** 2
    insts = []
    for task in range(3):
        p = default_params(3, n_grid, 5e-5, n_steps, h)
        p.update(gravity=[0.0, -1.0, 0.0], floor_on=1, floor_y=0.05, floor_mu=0.5,
                 n_segments=40, ckpt_every=0)
        if task < 2:
            p.update(seg_steps=25, periodic=1, loss_kind=LOSS_COM_DISP,
                     loss_dir=[1.0, 0.0, 0.0] if task == 0 else [0.0, 0.0, 1.0])
            insts.append(Instance(p, x0, density, br, progs[task], None, None, group=0))
        else:
            p.update(seg_steps=100, periodic=0, loss_kind=LOSS_FINAL_MSE)
            insts.append(Instance(p, x0, density, br, progs[task], target, mask, group=0))
    return Workload("quadruped3d", insts, 4,
                    f"3D quadruped, {n_grid}^3 grid, {n} particles x 3 field programs")


def make_tiny(seed: int = 0, dim: int = 2, n_grid: int = 16, s: int = 2, n_steps: int = 10,
              size=(0.25, 0.125, 0.125), corner=None, dt: float = 2e-3,
              loss_kind: int = LOSS_FINAL_MSE, floor: bool = False, clamp: bool = False,
              gravity: float = 0.0, n_segments: int = 3, periodic: int = 0,
              seg_steps: int = 0, b_scale: float = 0.5, damping: float = 0.0,
              E: float = 1.0) -> Instance:
    """A small block for finite-difference and parity tests."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n_grid
    h = dx / s
    if corner is None:
        corner = [6 * dx + 0.3 * h, 6 * dx + 0.7 * h, 6 * dx + 0.45 * h][:dim]
    x0 = box_particles(corner, list(size[:dim]), h)
    n = x0.shape[0]
    p = default_params(dim, n_grid, dt, n_steps, h)
    p["E"] = E
    p["damping"] = damping
    p["n_segments"] = n_segments
    p["periodic"] = periodic
    p["seg_steps"] = seg_steps if seg_steps else (n_steps + n_segments - 1) // n_segments
    p["loss_kind"] = loss_kind
    p["loss_dir"] = [0.8, 0.6, 0.0] if dim == 2 else [0.48, 0.6, 0.64]
    if gravity:
        p["gravity"] = [0.0, -gravity, 0.0]
    if floor:
        p["floor_on"] = 1
        p["floor_y"] = corner[1] + 0.25 * dx
        p["floor_mu"] = 0.5
    if clamp:
        p["clamp_xmax"] = corner[0] + 0.5 * dx
    density = rng.uniform(0.3, 1.0, size=n)
    br = _unit_vectors(rng, n, dim)
    b_prog = rng.uniform(-b_scale, b_scale, size=(n_segments, dim))
    target = x0 + rng.uniform(-0.01, 0.01, size=x0.shape)
    mask = (rng.uniform(size=n) < 0.7).astype(np.uint8)
    mask[0] = 1
    return Instance(p, x0, density, br, b_prog, target, mask)


WORKLOADS = {"cantilever2d": make_cantilever2d, "walker2d": make_walker2d, "plate3d": make_plate3d, "batch2d": make_batch2d, "quadruped3d": make_quadruped3d}


def make(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)
