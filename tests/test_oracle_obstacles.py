"""Pins of the oracle's obstacles: the solid boundaries of Eq. 18 beyond the
floor (half-space, sphere, axis-aligned box; static or translating with v_b;
sliding, no-slip or attached).

- A half-space obstacle through the floor line with the floor's friction is the
  floor: the same grid velocities bit for bit, the same transpose to rounding.
- Per-branch vector-Jacobian dot tests of the grid update with obstacles.
- An attached obstacle moving with v_b carries the particles inside it exactly.
- A block falling onto a sphere rests on it instead of sinking in.
- Central finite differences of a whole rollout with a sliding sphere and a
  moving half-space.
"""
import math

import numpy as np
import pytest

import oracle as orc
from paper_2503_22767_amd import workloads as W

from test_oracle_adjoint import _mask_dim, _state


def _grid_params(dim, n_grid=16):
    p = W.default_params(dim, n_grid, 2e-3, 1, 1.0 / 32)
    p["damping"] = 0.3
    p["gravity"] = [0.1, -1.0, 0.05][:dim] + [0.0] * (3 - dim)
    return p


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mu", [0.4, math.inf])
def test_halfspace_at_the_floor_line_is_the_floor(dim, mu):
    rng = np.random.default_rng(70 + dim)
    n_grid = 16
    dx = 1.0 / n_grid
    y = 0.5 + 1.2 * dx
    pf = _grid_params(dim, n_grid)
    pf.update(floor_on=1, floor_y=y, floor_mu=mu)
    po = _grid_params(dim, n_grid)
    po["obstacles"] = [dict(kind=orc.OBST_HALFSPACE, a=[0.3, y, 0.7], b=[0.0, 1.0, 0.0], mu=mu)]
    x, v, Cm, F, phi, br = _state(rng, dim, 12, n_grid, floor=True)
    m, mom = orc.p2g(pf, x, v, Cm, F, phi, br, np.zeros(3))
    vf, vo = orc.grid(pf, m, mom), orc.grid(po, m, mom)
    assert np.array_equal(vf, vo)
    on = (m > 0) & ((np.arange(len(m)) // n_grid) % n_grid * dx <= y)
    assert np.any(on & np.any(vf != orc.grid(_grid_params(dim, n_grid), m, mom), axis=1))
    vbar = _mask_dim(rng.standard_normal((len(m), 3)), dim)
    (pbf, mbf), (pbo, mbo) = orc.grid_adj(pf, m, mom, vbar), orc.grid_adj(po, m, mom, vbar)
    assert np.allclose(pbo, pbf, rtol=1e-13, atol=1e-15) and np.allclose(mbo, mbf, rtol=1e-13, atol=1e-15)


OBSTACLE_CASES = {
    # a tilted half-space, sliding
    "halfspace_tilted": dict(kind=orc.OBST_HALFSPACE, a=[0.5, 0.5, 0.5], b=[0.6, 0.8, 0.0], mu=0.4),
    "sphere_slide": dict(kind=orc.OBST_SPHERE, a=[0.5, 0.45, 0.5], b=[0.13, 0, 0], mu=0.3),
    "box_noslip": dict(kind=orc.OBST_BOX, a=[0.52, 0.48, 0.5], b=[0.12, 0.1, 0.1], mu=math.inf),
    "sphere_moving": dict(kind=orc.OBST_SPHERE, a=[0.5, 0.45, 0.5], b=[0.13, 0, 0], mu=0.2, vel=[0.2, -0.1, 0.05]),
    "box_attached_moving": dict(kind=orc.OBST_BOX, a=[0.45, 0.5, 0.5], b=[0.08, 0.3, 0.3], attached=1,
                                vel=[0.3, 0.1, -0.2]),
}


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("case", sorted(OBSTACLE_CASES))
def test_vjp_grid_with_obstacles(dim, case):
    rng = np.random.default_rng(80 + dim)
    n_grid = 16
    p = _grid_params(dim, n_grid)
    p["obstacles"] = [OBSTACLE_CASES[case]]
    step = 3
    x, v, Cm, F, phi, br = _state(rng, dim, 12, n_grid)
    m, mom = orc.p2g(p, x, v, Cm, F, phi, br, np.zeros(3))
    G = orc.num_nodes(p)
    vbar = _mask_dim(rng.standard_normal((G, 3)), dim)
    pbar, mbar = orc.grid_adj(p, m, mom, vbar, step=step)
    active = m > 0
    dm = rng.standard_normal(G) * m * 1e-1 * active
    dp = _mask_dim(rng.standard_normal((G, 3)), dim) * m[:, None] * active[:, None]
    h = 1e-7
    vp = orc.grid(p, m + h * dm, mom + h * dp, step=step)
    vm = orc.grid(p, m - h * dm, mom - h * dp, step=step)
    lhs = np.sum(vbar * (vp - vm)) / (2 * h)
    rhs = np.sum(pbar * dp) + np.sum(mbar * dm)
    assert rhs == pytest.approx(lhs, rel=1e-6, abs=1e-12)
    # the obstacle changed some active nodes
    free = _grid_params(dim, n_grid)
    changed = active & np.any(orc.grid(p, m, mom, step=step) != orc.grid(free, m, mom), axis=1)
    assert changed.sum() >= 2
    if OBSTACLE_CASES[case].get("attached"):
        vb = np.array(OBSTACLE_CASES[case]["vel"][:dim])
        assert np.allclose(orc.grid(p, m, mom, step=step)[changed][:, :dim], vb, atol=0)


def _block(dim, n_steps, gravity, size, seed=90):
    inst = W.make_tiny(seed=seed, dim=dim, n_steps=n_steps, loss_kind=W.LOSS_COM_DISP, floor=False,
                       gravity=gravity, size=size, n_grid=32)
    return inst


@pytest.mark.parametrize("dim", [2, 3])
def test_attached_moving_box_carries_its_particles(dim):
    inst = _block(dim, 12, 0.0, (0.2, 0.15, 0.15))
    p = dict(inst.params)
    dt, T = p["dt"], p["n_steps"]
    lo, hi = inst.x0.min(0), inst.x0.max(0)
    c = (lo + hi) / 2
    vb = np.array([0.5, 0.25, -0.2])[:dim]
    p["obstacles"] = [dict(kind=orc.OBST_BOX, a=list(c) + [0.0] * (3 - dim), b=list((hi - lo) / 2 + 0.2) + [0.0] * (3 - dim),
                           attached=1, vel=list(vb) + [0.0] * (3 - dim))]
    r = orc.rollout(p, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask)
    disp = r["x"][:, :dim] - inst.x0
    assert np.allclose(disp, vb * T * dt, rtol=0, atol=1e-12)


@pytest.mark.parametrize("mu", [0.5, math.inf])
def test_block_falling_on_a_sphere_rests_on_it(mu):
    inst = _block(2, 300, 1.0, (0.15, 0.06, 0.06), seed=91)
    p = dict(inst.params)
    dx = 1.0 / p["n_grid"]
    lo, hi = inst.x0.min(0), inst.x0.max(0)
    c = np.array([(lo[0] + hi[0]) / 2, lo[1] - 0.12])
    R = 0.1   # the sphere's top 0.02 below the block
    p["obstacles"] = [dict(kind=orc.OBST_SPHERE, a=[c[0], c[1], 0.0], b=[R, 0, 0], mu=mu)]
    r = orc.rollout(p, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask)
    d = np.linalg.norm(r["x"][:, :2] - c, axis=1)
    free = orc.rollout(inst.params, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask)
    # without it the block falls through the sphere's place (to the wall band
    # of the domain); with it, no particle gets deeper than 1.5 cells, and the
    # block does reach the surface
    assert np.linalg.norm(free["x"][:, :2] - c, axis=1).min() < R - 1.5 * dx
    assert d.min() >= R - 1.5 * dx
    assert d.min() <= R + 2 * dx


def test_gradient_with_obstacles_matches_central_fd():
    inst = W.make_tiny(seed=92, dim=2, n_steps=20, loss_kind=W.LOSS_COM_DISP, floor=False, gravity=1.0,
                       size=(0.25, 0.125, 0.125))
    p = dict(inst.params)
    lo, hi = inst.x0.min(0), inst.x0.max(0)
    dx = 1.0 / p["n_grid"]
    p["obstacles"] = [
        dict(kind=orc.OBST_SPHERE, a=[(lo[0] + hi[0]) / 2, lo[1] - 0.2 + 0.5 * dx, 0], b=[0.2, 0, 0], mu=0.3),
        dict(kind=orc.OBST_HALFSPACE, a=[hi[0] + 0.5 * dx, 0, 0], b=[-1.0, 0.1, 0], mu=0.2, vel=[-0.05, 0, 0]),
    ]
    g = orc.backward(p, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask, ckpt_every=4)
    rng = np.random.default_rng(93)

    def L(which, delta):
        kw = dict(phi=inst.density, br=inst.br, bp=inst.b_prog)
        kw[which] = kw[which] + delta
        return orc.rollout(p, inst.x0, kw["phi"], kw["br"], kw["bp"], inst.target, inst.mask)["loss"]

    for which, gname in (("phi", "g_density"), ("br", "g_br"), ("bp", "g_b_prog")):
        base = {"phi": inst.density, "br": inst.br, "bp": inst.b_prog}[which]
        u = rng.standard_normal(base.shape)
        h = 1e-5
        fd = (L(which, h * u) - L(which, -h * u)) / (2 * h)
        an = float(np.sum(g[gname] * u))
        assert an == pytest.approx(fd, rel=2e-5, abs=1e-12), (which, an, fd)
