"""Physics pins of the oracle rollout against closed forms.

Cantilever (Sec. 2.1, Eq. 5 and the torque remark under Eq. 9): for a uniform
remanence Br e_x the magnetic potential integrates to a dead end load
(Br / mu0) B_a per unit height on the free end, so a damped small-deflection run
must settle at the Timoshenko beam deflection
  delta = F L^3 / (3 E' I) + F L / (kappa G h),  F = Br B_a h / mu0,
with plane-strain E' = E / (1 - nu^2), I = h^3 / 12, kappa = 5/6. The clamp
(nodes with x_i <= x_left + dx) fixes the beam about one cell into the body,
so the free length is L - dx. The deflection must lift the tip toward the
field, be linear in B_a and follow sin(angle between B and Br).

Sliding block (Eq. 18): Coulomb friction on floor nodes decelerates a block at
mu g, so it stops after v0^2 / (2 mu g); with mu = 0 the tangential momentum is
untouched.
"""
import math

import numpy as np
import pytest

import oracle as orc
from paper_2503_22767_amd import workloads as W


def _cantilever(Ba, theta, n_steps, dt=4e-3, c=0.7):
    inst = W.make_cantilever2d().instances[0]
    p = dict(inst.params)
    p.update(dt=dt, n_steps=n_steps, damping=c, n_segments=1, seg_steps=0)
    br = np.zeros_like(inst.br); br[:, 0] = 1.0
    prog = np.array([[Ba * math.cos(theta), Ba * math.sin(theta)]])
    r = orc.rollout(p, inst.x0, np.ones(inst.n), br, prog)
    tip = inst.x0[:, 0] > inst.x0[:, 0].max() - 1e-9
    return float(np.mean(r["x"][tip, 1] - inst.x0[tip, 1]))


def test_cantilever_sign_linearity_sin_law():
    d1 = _cantilever(1e-4, math.pi / 2, 1500)
    assert d1 > 0.0                                            # lifts toward +B
    assert _cantilever(-1e-4, math.pi / 2, 1500) == pytest.approx(-d1, rel=1e-9)
    assert _cantilever(2e-4, math.pi / 2, 1500) == pytest.approx(2 * d1, rel=1e-3)
    assert _cantilever(1e-4, math.pi / 6, 1500) == pytest.approx(0.5 * d1, rel=1e-2)
    assert abs(_cantilever(1e-4, 0.0, 1500)) < 1e-3 * abs(d1)  # parallel: no bending


def test_cantilever_settles_at_beam_theory_deflection():
    E, nu, Br, Ba, mu0 = 1.0, 0.3, 1.0, 1e-4, 1.0
    L, h, dx = 0.625, 0.125, 1.0 / 64
    Ep = E / (1 - nu * nu)
    G = E / (2 * (1 + nu))
    I = h ** 3 / 12
    F = Br * Ba * h / mu0
    Leff = L - dx
    delta = F * Leff ** 3 / (3 * Ep * I) + F * Leff / (5.0 / 6.0 * G * h)
    got = _cantilever(Ba, math.pi / 2, 6000)
    assert got == pytest.approx(delta, rel=0.05)


def _block(mu, v0x=0.3, n_steps=1500):
    n_grid = 64
    h = (1.0 / n_grid) / 2
    floor_y = 0.25
    x0 = W.box_particles([0.2, floor_y], [0.125, 0.0625], h)
    n = len(x0)
    p = W.default_params(2, n_grid, 1e-3, n_steps, h)
    p.update(gravity=[0.0, -1.0, 0.0], floor_on=1, floor_y=floor_y, floor_mu=mu, E=20.0)
    v0 = np.zeros_like(x0); v0[:, 0] = v0x
    r = orc.rollout(p, x0, np.ones(n), np.zeros((n, 2)), np.zeros((1, 2)), v0=v0, traj=True)
    return r, x0


@pytest.mark.parametrize("mu", [0.5, 0.25])
def test_sliding_block_stopping_distance(mu):
    r, x0 = _block(mu)
    com = r["traj"][:, :, 0].mean(axis=1)
    dist = com[-1] - com[0]
    assert dist == pytest.approx(0.3 ** 2 / (2 * mu * 1.0), rel=0.05)
    assert abs(np.mean(r["v"][:, 0])) < 0.01 * 0.3


def test_frictionless_floor_keeps_tangential_momentum():
    r, x0 = _block(0.0, n_steps=300)
    assert np.mean(r["v"][:, 0]) == pytest.approx(0.3, rel=1e-12)


def test_simp_interpolation_scales_the_response():
    """Eqs. 31 and 33: with eps = 1/2 and phi = (sqrt(5) - 1) / 2 the elastic scaling
    eps + (1 - eps) phi^3 equals phi, the same factor as the mass, so the motion is
    that of a full-density beam whose magnetic load is scaled by s_m / phi = phi^2."""
    phi_g = (math.sqrt(5.0) - 1.0) / 2.0
    inst = W.make_cantilever2d().instances[0]
    outs = []
    for phi, eps in ((1.0, 0.5), (phi_g, 0.5)):
        p = dict(inst.params)
        p.update(dt=4e-3, n_steps=1200, damping=0.7, n_segments=1, seg_steps=0, simp_eps=eps)
        br = np.zeros_like(inst.br); br[:, 0] = 1.0
        r = orc.rollout(p, inst.x0, np.full(inst.n, phi), br, np.array([[0.0, 1e-4]]))
        outs.append(r["x"][:, :2] - inst.x0)
    ratio = np.sum(outs[1] * outs[0]) / np.sum(outs[0] * outs[0])
    assert ratio == pytest.approx(phi_g ** 2, rel=1e-4)


@pytest.mark.parametrize("dim", [2, 3])
def test_deformation_gradient_follows_particle_motion(dim):
    """Eq. 22 against Eq. 21: particles on an affine image x = F X + c of a lattice,
    moved by an affine grid velocity v = v0 + L x, land on the affine image under
    the returned F' (fit by least squares over the particles)."""
    rng = np.random.default_rng(70 + dim)
    n_grid = 32
    p = W.default_params(dim, n_grid, 1e-2, 1, 1.0 / 64)
    X = W.box_particles([0.0] * dim, [0.1] * dim, 1.0 / 64) - 0.05
    n = len(X)
    F = np.eye(3); F[:dim, :dim] += 0.2 * rng.standard_normal((dim, dim))
    c = np.zeros(3); c[:dim] = 0.5
    x = np.zeros((n, 3)); x[:, :dim] = X @ F[:dim, :dim].T + c[:dim]
    Lm = np.zeros((3, 3)); Lm[:dim, :dim] = 0.5 * rng.standard_normal((dim, dim))
    v0 = np.zeros(3); v0[:dim] = 0.1 * rng.standard_normal(dim)
    G = orc.num_nodes(p)
    idx = np.arange(G)
    xi = np.zeros((G, 3))
    xi[:, 0] = (idx % n_grid) / n_grid
    xi[:, 1] = ((idx // n_grid) % n_grid) / n_grid
    if dim == 3:
        xi[:, 2] = (idx // (n_grid * n_grid)) / n_grid
    vg = v0[None, :] + xi @ Lm.T
    x1, v1, C1, F1 = orc.g2p(p, x, np.tile(F, (n, 1, 1)), vg)
    A = np.hstack([X, np.ones((n, 1))])
    fit, *_ = np.linalg.lstsq(A, x1[:, :dim], rcond=None)
    F_fit = fit[:dim].T
    assert np.max(np.abs(F1[:, :dim, :dim] - F_fit[None])) < 1e-12
    assert np.max(np.abs(C1[:, :dim, :dim] - Lm[None, :dim, :dim])) < 1e-11   # affine field reproduced


def test_domain_walls_stop_a_block():
    """Walls (b cells, separating, frictionless): a block thrown at the left wall
    never leaves the domain and its leftward momentum is removed."""
    n_grid = 32
    h = (1.0 / n_grid) / 2
    x0 = W.box_particles([0.2, 0.4], [0.125, 0.125], h)
    n = len(x0)
    p = W.default_params(2, n_grid, 1e-3, 600, h)
    p["E"] = 5.0
    v0 = np.zeros_like(x0); v0[:, 0] = -0.5
    r = orc.rollout(p, x0, np.ones(n), np.zeros((n, 2)), np.zeros((1, 2)), v0=v0, traj=True)
    b = p["wall_cells"]
    assert np.min(r["traj"][:, :, 0]) > (b - 1) / n_grid
    assert np.mean(r["v"][:, 0]) > -0.05
