"""Pins of the oracle's hand-derived adjoint.

- Central finite differences of the oracle's own forward loss on tiny inputs
  (the forward is pinned by the step and constitutive tests), for density,
  remanence and field program, every loss kind, with and without floor contact
  and clamp.
- Per-phase vector-Jacobian dot tests <ybar, J xdot> = <J^T ybar, xdot> for P2G,
  the grid update (each boundary branch) and G2P, with J xdot by central FD.
- The trajectory loss of Eq. 39 telescopes (Eq. 21) into the centre-of-mass
  loss of Eq. 40: equal values and gradients.
- Checkpoint spacing does not change the gradient.
"""
import math

import numpy as np
import pytest

import oracle as orc
from paper_2503_22767_amd import workloads as W


def _fd_dir(inst, which, u, h):
    def L(delta):
        kw = dict(phi=inst.density, br=inst.br, bp=inst.b_prog)
        kw[which] = kw[which] + delta
        return orc.rollout(inst.params, inst.x0, kw["phi"], kw["br"], kw["bp"], inst.target, inst.mask)["loss"]
    return (L(h * u) - L(-h * u)) / (2 * h)


CASES = [
    # dim, loss kind, floor, clamp
    (2, W.LOSS_FINAL_MSE, False, False),
    (2, W.LOSS_FINAL_MSE, True, True),
    (2, W.LOSS_TIP_DISP, False, True),
    (2, W.LOSS_COM_DISP, True, False),
    (2, W.LOSS_TRAJ_VEL, True, False),
    (3, W.LOSS_FINAL_MSE, False, True),
    (3, W.LOSS_TIP_DISP, True, False),
    (3, W.LOSS_TRAJ_VEL, True, True),
]


@pytest.mark.parametrize("dim,kind,floor,clamp", CASES)
def test_gradient_matches_central_fd(dim, kind, floor, clamp):
    size = (0.25, 0.125, 0.125) if dim == 2 else (0.125, 0.125, 0.125)
    inst = W.make_tiny(seed=2 + dim, dim=dim, n_steps=15, loss_kind=kind, floor=floor, clamp=clamp,
                       gravity=1.0 if floor else 0.0, size=size)
    g = orc.backward(inst.params, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask,
                     ckpt_every=4)
    rng = np.random.default_rng(100 + dim)
    for which, gname in (("phi", "g_density"), ("br", "g_br"), ("bp", "g_b_prog")):
        base = {"phi": inst.density, "br": inst.br, "bp": inst.b_prog}[which]
        u = rng.standard_normal(base.shape)
        fd = _fd_dir(inst, which, u, 1e-5)
        an = float(np.sum(g[gname] * u))
        assert an == pytest.approx(fd, rel=2e-5, abs=1e-12), (which, an, fd)


def test_gradient_elementwise_field_segments():
    """Every field-program entry by central FD (2D walker-like block on a floor)."""
    inst = W.make_tiny(seed=9, dim=2, n_steps=18, loss_kind=W.LOSS_TRAJ_VEL, floor=True, gravity=1.0,
                       n_segments=3, periodic=1, seg_steps=4)
    g = orc.backward(inst.params, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask,
                     ckpt_every=5)
    for idx in np.ndindex(inst.b_prog.shape):
        u = np.zeros_like(inst.b_prog); u[idx] = 1.0
        fd = _fd_dir(inst, "bp", u, 1e-5)
        assert g["g_b_prog"][idx] == pytest.approx(fd, rel=2e-5, abs=1e-13)


def test_trajectory_loss_equals_com_loss():
    base = W.make_tiny(seed=4, dim=2, n_steps=20, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0)
    res = {}
    for kind in (W.LOSS_COM_DISP, W.LOSS_TRAJ_VEL):
        p = dict(base.params); p["loss_kind"] = kind
        res[kind] = orc.backward(p, base.x0, base.density, base.br, base.b_prog, ckpt_every=6)
    a, b = res[W.LOSS_COM_DISP], res[W.LOSS_TRAJ_VEL]
    assert a["loss"] == pytest.approx(b["loss"], rel=1e-9)
    for k in ("g_density", "g_br", "g_b_prog"):
        assert np.linalg.norm(a[k] - b[k]) <= 1e-8 * np.linalg.norm(a[k])


def test_checkpoint_spacing_does_not_change_gradient():
    inst = W.make_tiny(seed=6, dim=2, n_steps=23, loss_kind=W.LOSS_FINAL_MSE, floor=True, gravity=1.0)
    outs = [orc.backward(inst.params, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask,
                         ckpt_every=k) for k in (1, 5, 23, 100)]
    for o in outs[1:]:
        for k in ("g_density", "g_br", "g_b_prog"):
            assert np.array_equal(o[k], outs[0][k])
        assert o["loss"] == outs[0]["loss"]


# ----------------------------------------------------------------------------
# per-phase VJP dot tests
# ----------------------------------------------------------------------------

def _state(rng, dim, n, n_grid, floor=False):
    dx = 1.0 / n_grid
    x = np.zeros((n, 3)); v = np.zeros((n, 3)); Cm = np.zeros((n, 3, 3)); F = np.tile(np.eye(3), (n, 1, 1))
    x[:, :dim] = 0.5 + rng.uniform(-3 * dx, 3 * dx, size=(n, dim))
    if floor:
        x[:, 1] = 0.5 + rng.uniform(0.3 * dx, 3 * dx, size=n)
    v[:, :dim] = 0.3 * rng.standard_normal((n, dim))
    if floor:
        v[:, 1] = -np.abs(v[:, 1]) - 0.05
    Cm[:, :dim, :dim] = 2.0 * rng.standard_normal((n, dim, dim))
    F[:, :dim, :dim] += 0.1 * rng.standard_normal((n, dim, dim))
    phi = rng.uniform(0.3, 1.0, n)
    br = np.zeros((n, 3)); br[:, :dim] = rng.standard_normal((n, dim))
    return x, v, Cm, F, phi, br


def _mask_dim(a, dim):
    a = np.array(a, dtype=float)
    if dim == 2:
        if a.ndim >= 2 and a.shape[-1] == 3 and a.shape[-2] == 3:
            a[..., 2, :] = 0.0; a[..., :, 2] = 0.0
        elif a.shape[-1] == 3:
            a[..., 2] = 0.0
    return a


@pytest.mark.parametrize("dim", [2, 3])
def test_vjp_p2g(dim):
    rng = np.random.default_rng(40 + dim)
    n_grid = 16
    p = W.default_params(dim, n_grid, 2e-3, 1, 1.0 / 32)
    x, v, Cm, F, phi, br = _state(rng, dim, 12, n_grid)
    B = np.zeros(3); B[:dim] = rng.uniform(-0.5, 0.5, dim)
    G = orc.num_nodes(p)
    mbar = rng.standard_normal(G); pbar = _mask_dim(rng.standard_normal((G, 3)), dim)
    adj = orc.p2g_adj(p, x, v, Cm, F, phi, br, B, pbar, mbar)
    dirs = dict(x=_mask_dim(rng.standard_normal(x.shape), dim) * 1e-3,
                v=_mask_dim(rng.standard_normal(v.shape), dim),
                C=_mask_dim(rng.standard_normal(Cm.shape), dim),
                F=_mask_dim(rng.standard_normal(F.shape), dim),
                phi=rng.standard_normal(phi.shape),
                br=_mask_dim(rng.standard_normal(br.shape), dim),
                B=_mask_dim(rng.standard_normal(3), dim))
    for key, d in dirs.items():
        h = 1e-6
        def out(sgn):
            args = dict(x=x, v=v, C=Cm, F=F, phi=phi, br=br, B=B)
            args[key] = args[key] + sgn * h * d
            return orc.p2g(p, args["x"], args["v"], args["C"], args["F"], args["phi"], args["br"], args["B"])
        (mp, pp), (mm, pm) = out(1), out(-1)
        lhs = (np.sum(mbar * (mp - mm)) + np.sum(pbar * (pp - pm))) / (2 * h)
        rhs = np.sum(adj[key] * d)
        assert rhs == pytest.approx(lhs, rel=1e-7, abs=1e-12), key


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("bc", ["none", "floor_slide", "floor_noslip", "clamp_walls"])
def test_vjp_grid(dim, bc):
    rng = np.random.default_rng(50 + dim)
    n_grid = 16
    dx = 1.0 / n_grid
    p = W.default_params(dim, n_grid, 2e-3, 1, 1.0 / 32)
    p["damping"] = 0.3
    p["gravity"] = [0.1, -1.0, 0.05][:dim] + [0.0] * (3 - dim)
    floor = bc.startswith("floor")
    if floor:
        p.update(floor_on=1, floor_y=0.5 + 1.2 * dx, floor_mu=0.4 if bc == "floor_slide" else math.inf)
    if bc == "clamp_walls":
        p["clamp_xmax"] = 0.5 - 0.5 * dx
        p["wall_cells"] = 8    # put the particle block inside the wall band
    x, v, Cm, F, phi, br = _state(rng, dim, 12, n_grid, floor=floor)
    B = np.zeros(3)
    m, mom = orc.p2g(p, x, v, Cm, F, phi, br, B)
    G = orc.num_nodes(p)
    vbar = _mask_dim(rng.standard_normal((G, 3)), dim)
    pbar, mbar = orc.grid_adj(p, m, mom, vbar)
    active = m > 0
    dm = rng.standard_normal(G) * m * 1e-1 * active
    dp = _mask_dim(rng.standard_normal((G, 3)), dim) * m[:, None] * active[:, None]
    h = 1e-7
    vp = orc.grid(p, m + h * dm, mom + h * dp)
    vm = orc.grid(p, m - h * dm, mom - h * dp)
    lhs = np.sum(vbar * (vp - vm)) / (2 * h)
    rhs = np.sum(pbar * dp) + np.sum(mbar * dm)
    assert rhs == pytest.approx(lhs, rel=1e-6, abs=1e-12)
    vout = orc.grid(p, m, mom)
    on_floor = active & ((np.arange(G) // n_grid) % n_grid * dx <= p["floor_y"]) if floor else None
    if bc == "floor_slide":   # some floor nodes slide: normal velocity removed, tangential kept
        assert np.any(on_floor & (vout[:, 1] == 0.0) & (np.abs(vout[:, 0]) > 0.0))
    if bc == "floor_noslip":
        assert np.any(on_floor & np.all(vout == 0.0, axis=1))
    if bc == "clamp_walls":
        ijk0 = np.arange(G) % n_grid
        clamped = active & (ijk0 * dx <= p["clamp_xmax"])
        assert clamped.any()
        assert np.all(pbar[clamped] == 0.0) and np.all(mbar[clamped] == 0.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_vjp_g2p(dim):
    rng = np.random.default_rng(60 + dim)
    n_grid = 16
    p = W.default_params(dim, n_grid, 2e-3, 1, 1.0 / 32)
    x, v, Cm, F, phi, br = _state(rng, dim, 12, n_grid)
    G = orc.num_nodes(p)
    vg = _mask_dim(0.3 * rng.standard_normal((G, 3)), dim)
    n = len(phi)
    xb1 = _mask_dim(rng.standard_normal((n, 3)), dim); vb1 = _mask_dim(rng.standard_normal((n, 3)), dim)
    Cb1 = _mask_dim(rng.standard_normal((n, 3, 3)), dim); Fb1 = _mask_dim(rng.standard_normal((n, 3, 3)), dim)
    vbar, xb0, Fb0 = orc.g2p_adj(p, x, F, vg, xb1, vb1, Cb1, Fb1)
    dirs = dict(x=(_mask_dim(rng.standard_normal(x.shape), dim) * 1e-3, xb0),
                F=(_mask_dim(rng.standard_normal(F.shape), dim), Fb0),
                vg=(_mask_dim(rng.standard_normal(vg.shape), dim), vbar))
    for key, (d, adj) in dirs.items():
        h = 1e-6
        def out(sgn):
            a = dict(x=x, F=F, vg=vg)
            a[key] = a[key] + sgn * h * d
            return orc.g2p(p, a["x"], a["F"], a["vg"])
        op, om = out(1), out(-1)
        lhs = sum(np.sum(b * (u - w)) for b, u, w in zip((xb1, vb1, Cb1, Fb1), op, om)) / (2 * h)
        rhs = np.sum(adj * d)
        assert rhs == pytest.approx(lhs, rel=1e-7, abs=1e-12), key
