"""Pins of the mass floor for void particles.

Eq. 33 gives a particle the mass phi rho V; as the Heaviside projection
sharpens (Eq. 25 up to beta = 128), void particles tend to zero mass while
their stiffness stays at the SIMP floor eps of Eq. 31, and nodes fed mostly by
void particles get velocities p/m far beyond the body's: the explicit step
goes unstable. The reading taken floors the mass interpolation like Eq. 31
floors the stiffness: m = (eps_m + (1 - eps_m) phi) rho V (eps_m = 0 is Eq. 33).
Pinned by:
  - a reparametrization identity: with no stress (E = 0, no field) the mass is
    the only place the density enters, so a rollout with floor eps_m and
    density phi equals one without the floor and density
    eps_m + (1 - eps_m) phi, and their density gradients differ by the factor
    (1 - eps_m); the case (a block falling onto a frictional floor, its
    velocities averaged through the grid by mass, a mass-weighted loss)
    exercises every place the mass enters;
  - central differences of the whole rollout with the floor and full physics;
  - its purpose: a floor block whose right half is void (phi = 1e-6) breaks
    down within 400 steps without it (the oracle reports the failure), and
    runs with eps_m = 1e-3.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2503_22767_amd import workloads as W


def _falling_block(dim, kind):
    inst = W.make_tiny(seed=40 + dim, dim=dim, n_steps=30, loss_kind=kind, floor=True, gravity=2.0,
                       size=(0.3, 0.15, 0.15), n_grid=16, n_segments=3)
    p = inst.params
    p["E"] = 0.0
    p["floor_y"] = inst.x0[:, 1].min() - 0.2 / 16
    p["floor_mu"] = 0.4
    rng = np.random.default_rng(dim)
    dens = rng.uniform(0.0, 1.0, inst.n)
    prog = np.zeros_like(inst.b_prog)
    return inst, dens, prog


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", [W.LOSS_COM_DISP, W.LOSS_TRAJ_VEL])
def test_mass_floor_is_a_reparametrization_of_the_density(dim, kind):
    inst, dens, prog = _falling_block(dim, kind)
    eps = 0.2
    pf = dict(inst.params, mass_eps=eps)
    p0 = dict(inst.params, mass_eps=0.0)
    dens2 = eps + (1.0 - eps) * dens
    # the velocity given to the block makes the friction matter
    a = orc.rollout(pf, inst.x0, dens, inst.br, prog)
    b = orc.rollout(p0, inst.x0, dens2, inst.br, prog)
    assert np.max(np.abs(a["x"] - b["x"])) < 1e-14
    assert abs(a["loss"] - b["loss"]) <= 1e-12 * abs(b["loss"])
    ga = orc.backward(pf, inst.x0, dens, inst.br, prog, ckpt_every=7)
    gb = orc.backward(p0, inst.x0, dens2, inst.br, prog, ckpt_every=7)
    ref = (1.0 - eps) * gb["g_density"]
    assert np.linalg.norm(ref) > 0
    assert np.linalg.norm(ga["g_density"] - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_floor_gradient_matches_central_fd(dim):
    inst = W.make_tiny(seed=50 + dim, dim=dim, n_steps=14, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0,
                       size=(0.3, 0.15, 0.15), n_grid=16, n_segments=3)
    p = dict(inst.params, mass_eps=1e-2)
    rng = np.random.default_rng(dim)
    dens = np.where(rng.uniform(size=inst.n) < 0.5, 1e-3, 1.0)
    g = orc.backward(p, inst.x0, dens, inst.br, inst.b_prog, ckpt_every=4)
    u = rng.standard_normal(inst.n) * 1e-3
    h = 1e-2          # density steps of ~1e-5: smaller ones lose the loss difference to rounding
    lp = orc.rollout(p, inst.x0, dens + h * u, inst.br, inst.b_prog)["loss"]
    lm = orc.rollout(p, inst.x0, dens - h * u, inst.br, inst.b_prog)["loss"]
    fd = (lp - lm) / (2 * h)
    adj = float(g["g_density"] @ u)
    assert abs(fd - adj) <= 1e-6 * abs(adj), (fd, adj)


def _half_void_block(mass_eps):
    inst = W.make_tiny(seed=3, dim=2, n_steps=400, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0,
                       size=(0.3, 0.15, 0.2), n_grid=32, n_segments=4, dt=1e-3, b_scale=0.5)
    dens = np.where(inst.x0[:, 0] > np.median(inst.x0[:, 0]), 1e-6, 1.0)
    return dict(inst.params, mass_eps=mass_eps), inst, dens


def test_void_particles_break_the_step_without_the_floor_and_not_with_it():
    p, inst, dens = _half_void_block(0.0)
    with pytest.raises(orc.OracleError):
        orc.rollout(p, inst.x0, dens, inst.br, inst.b_prog)
    p, inst, dens = _half_void_block(1e-3)
    r = orc.rollout(p, inst.x0, dens, inst.br, inst.b_prog)
    assert np.all(np.isfinite(r["x"]))
