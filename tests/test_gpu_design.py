"""Parity of the design front end (HIP, through the C ABI) with its FP64 oracle:
density filter, Heaviside projection, magnetization with region sharing, and
the transpose of their Jacobian (Sec. 3.1, Eqs. 23-28).

Bars: FP64 within 1e-12 (values, absolute; gradients, norm-wise relative),
only summation order differing; FP32 within 1e-5 (values, absolute, on
quantities of order one) and 1e-5 (gradients, norm-wise relative). The
neighbour count is an integer: exact in FP64; in FP32 it may differ only by
pairs whose FP64 distance lies within 1e-5 of the radius (none in these cases).
"""
import numpy as np
import pytest
import torch

from oracle import design as OD
from paper_2503_22767_amd import design as PD
from paper_2503_22767_amd import mpm_mag as M
from paper_2503_22767_amd import workloads as W

from gpu_util import log, rel_norm

pytestmark = pytest.mark.gpu


def _cloud(dim, n_side, h, seed, jitter=0.3):
    rng = np.random.default_rng(seed)
    axes = [np.arange(n_side[k]) * h for k in range(dim)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, dim)
    x = g + jitter * h * rng.uniform(-1, 1, g.shape)
    return x[rng.permutation(len(x))] + 0.3   # caller order not spatial


def _pairs_within(x0, R):
    d = np.sqrt(((x0[:, None, :] - x0[None, :, :]) ** 2).sum(-1))
    return int((d < R).sum()), int((np.abs(d - R) < 1e-5 * R).sum())


def _case(dim, n_m, seed, n_side=None, h=0.01, Rh=1.7):
    rng = np.random.default_rng(seed)
    n_side = n_side or ((37, 29) if dim == 2 else (13, 11, 9))
    x0 = _cloud(dim, n_side, h, seed)
    n = len(x0)
    region = None if n_m is None else rng.integers(0, n_m, n).astype(np.int32)
    nm = n if n_m is None else n_m
    return dict(x0=x0, R=Rh * h, region=region, n_m=n_m, phi=rng.uniform(0, 1, n), mag=rng.uniform(0.2, 1, nm),
                zeta=rng.uniform(-1, 1, (nm, dim)), beta=8.0, br_max=1.2, delta=1e-3,
                gd=rng.standard_normal(n), gb=rng.standard_normal((n, dim)))


def _oracle(c):
    reg = np.arange(len(c["x0"])) if c["region"] is None else c["region"]
    _, pb, br = OD.front_end(c["x0"], c["phi"], c["R"], c["beta"], reg, c["mag"], c["zeta"], c["br_max"], c["delta"])
    g = OD.front_end_backward(c["x0"], c["phi"], c["R"], c["beta"], reg, c["mag"], c["zeta"], c["br_max"],
                              c["delta"], c["gd"], c["gb"])
    return pb, br, g


def _device(c, precision, **kw):
    fe = PD.MpmMagDesign(c["x0"], c["R"], region=c["region"], n_regions=c["n_m"], precision=precision)
    try:
        dens, br = fe.forward(c["phi"], c["mag"], c["zeta"], c["beta"], c["br_max"], c["delta"])
        g = fe.backward(c["gd"], c["gb"])
        torch.cuda.synchronize()
        out = (dens.double().cpu().numpy(), br.double().cpu().numpy(),
               tuple(t.double().cpu().numpy() for t in g), fe.nnz)
    finally:
        fe.close()
    return out


CASES = [(2, None, 1), (2, 7, 2), (3, None, 3), (3, 5, 4), (3, 1, 5)]


@pytest.mark.parametrize("dim,n_m,seed", CASES, ids=[f"d{c[0]}-regions{c[1]}" for c in CASES])
@pytest.mark.parametrize("precision", [8, 4])
def test_front_end_matches_oracle(dim, n_m, seed, precision):
    c = _case(dim, n_m, seed)
    pb, br, (g_phi, g_mag, g_zeta) = _oracle(c)
    dens, dbr, (d_phi, d_mag, d_zeta), nnz = _device(c, precision)
    pairs, near = _pairs_within(c["x0"], c["R"])
    assert near == 0
    assert nnz == pairs
    vt, gt = (1e-12, 1e-12) if precision == 8 else (1e-5, 1e-5)
    errs = dict(density=np.abs(dens - pb).max(), br=np.abs(dbr - br).max(), g_phi=rel_norm(d_phi, g_phi),
                g_mag=rel_norm(d_mag, g_mag), g_zeta=rel_norm(d_zeta, g_zeta))
    log(f"front end d{dim} regions={n_m} fp{32 if precision == 4 else 64}", len(c["x0"]), nnz, errs)
    assert errs["density"] <= vt and errs["br"] <= vt
    assert errs["g_phi"] <= gt and errs["g_mag"] <= gt and errs["g_zeta"] <= gt


def test_radius_below_the_spacing_is_the_identity():
    c = _case(3, None, 7, h=0.01, Rh=0.3)
    dens, _, (g_phi, _, _), nnz = _device(c, 8)
    assert nnz == len(c["x0"])
    assert np.allclose(dens, OD.heaviside(c["phi"], c["beta"]), rtol=0, atol=1e-14)
    assert np.allclose(g_phi, c["gd"] * OD.heaviside_derivative(c["phi"], c["beta"]), rtol=1e-13, atol=1e-15)


def test_single_particle_and_coincident_particles():
    one = _case(2, None, 8, n_side=(1, 1))
    dens, br, g, nnz = _device(one, 8)
    pb, obr, og = _oracle(one)
    assert nnz == 1 and np.allclose(dens, pb, atol=1e-14) and np.allclose(br, obr, atol=1e-14)
    # fifty particles at one point: every pair at distance 0 (weight 1), the filter is the mean
    c = _case(3, 3, 9, n_side=(5, 5, 2))
    c["x0"] = np.tile(c["x0"][:1], (len(c["x0"]), 1))
    dens, br, (d_phi, d_mag, d_zeta), nnz = _device(c, 8)
    assert nnz == 50 * 50
    assert np.allclose(dens, OD.heaviside(np.full(50, c["phi"].mean()), c["beta"]), atol=1e-13)
    pb, obr, (g_phi, g_mag, g_zeta) = _oracle(c)
    assert rel_norm(d_phi, g_phi) < 1e-12 and rel_norm(d_zeta, g_zeta) < 1e-12


def test_empty_region_gets_zero_gradient():
    c = _case(2, 6, 10)
    c["region"][c["region"] == 4] = 5   # region 4 has no particles
    _, _, (_, d_mag, d_zeta), _ = _device(c, 8)
    _, _, (_, g_mag, g_zeta) = _oracle(c)
    assert d_mag[4] == 0 and np.all(d_zeta[4] == 0)
    assert rel_norm(d_mag, g_mag) < 1e-12 and rel_norm(d_zeta, g_zeta) < 1e-12


@pytest.mark.parametrize("precision", [8, 4])
def test_chunked_region_sums_with_an_empty_region(precision):
    """Few large regions (mean above 2048 members) take the chunked, atomic-free
    region sums: 40,000 particles in 5 regions of 3 to 19 chunks each, region 2
    empty. Region gradients need only the per-particle gradient, so the oracle
    side is cheap."""
    rng = np.random.default_rng(14)
    n = 40000
    x0 = rng.uniform(0.2, 0.8, (n, 2))
    region = rng.choice([0, 1, 3, 4], size=n, p=[0.1, 0.2, 0.3, 0.4]).astype(np.int32)
    mag, zeta = rng.uniform(0.2, 1, 5), rng.uniform(-1, 1, (5, 2))
    gb = rng.standard_normal((n, 2))
    fe = PD.MpmMagDesign(x0, 0.004, region=region, n_regions=5, precision=precision)
    try:
        fe.forward(rng.uniform(0, 1, n), mag, zeta, 8.0, 1.3, 1e-4)
        _, d_mag, d_zeta = fe.backward(np.zeros(n), gb, want=(False, True, True))
        torch.cuda.synchronize()
        d_mag, d_zeta = d_mag.double().cpu().numpy(), d_zeta.double().cpu().numpy()
    finally:
        fe.close()
    g_mag, g_zeta = OD.magnetization_transpose(region, mag, zeta, 1.3, 1e-4, gb)
    tol = 1e-12 if precision == 8 else 1e-5
    assert d_mag[2] == 0 and np.all(d_zeta[2] == 0)
    assert rel_norm(d_mag, g_mag) <= tol and rel_norm(d_zeta, g_zeta) <= tol


def test_errors_are_reported():
    c = _case(2, 4, 11)
    bad = c["region"].copy()
    bad[3] = 4
    with pytest.raises(M.MpmMagError, match="invalid argument|EINVAL|region"):
        PD.MpmMagDesign(c["x0"], c["R"], region=bad, n_regions=4, precision=8)
    x = c["x0"].copy()
    x[5, 1] = np.nan
    with pytest.raises(M.MpmMagError, match="non-finite"):
        PD.MpmMagDesign(x, c["R"], precision=8)
    fe = PD.MpmMagDesign(c["x0"], c["R"], region=c["region"], n_regions=4, precision=8)
    try:
        with pytest.raises(M.MpmMagError, match="forward"):
            fe.backward(c["gd"], c["gb"])
    finally:
        fe.close()


def test_quadruped_particle_set_full_size():
    """The quadruped's 1,146,344 particles, R = 1.5 spacings, 8 regions by x
    slab, FP32 and FP64: sampled rows of the forward against the oracle's rows,
    region gradients against the oracle (they need only the per-particle
    gradient), and the filter's gradient against a central difference of the
    device forward along a random direction (FP64)."""
    inst = W.make_quadruped3d(n_steps=1).instances[0]
    x0 = inst.x0
    h = 1.0 / (128 * 3)
    R = 1.5 * h
    n = len(x0)
    rng = np.random.default_rng(21)
    region = np.clip(((x0[:, 0] - x0[:, 0].min()) / np.ptp(x0[:, 0]) * 8).astype(np.int32), 0, 7)
    phi = rng.uniform(0, 1, n)
    mag, zeta = rng.uniform(0.2, 1, 8), rng.uniform(-1, 1, (8, 3))
    gd, gb = rng.standard_normal(n), rng.standard_normal((n, 3))
    rows = rng.choice(n, 64, replace=False)
    ref_br = OD.magnetization(region, mag, zeta, 1.0, 1e-6)
    ref_gm, ref_gz = OD.magnetization_transpose(region, mag, zeta, 1.0, 1e-6, gb)
    for precision, vt, gt in ((4, 1e-5, 1e-5), (8, 1e-12, 1e-12)):
        # the oracle takes the positions the device gets: rounded to FP32 they
        # move a neighbour distance by ~2e-8 of 2.6e-3, and its weight by ~5e-6
        xr = x0.astype(np.float32).astype(np.float64) if precision == 4 else x0
        ref_rows = OD.heaviside(OD.density_filter(xr, phi, R, rows=rows), 8.0)
        fe = PD.MpmMagDesign(x0, R, region=region, n_regions=8, precision=precision)
        try:
            dens, br = fe.forward(phi, mag, zeta, 8.0, 1.0, 1e-6)
            g_phi, g_mag, g_zeta = fe.backward(gd, gb)
            torch.cuda.synchronize()
            dens_h = dens.double().cpu().numpy()
            e_rows = np.abs(dens_h[rows] - ref_rows).max()
            e_br = np.abs(br.double().cpu().numpy() - ref_br).max()
            e_gm = rel_norm(g_mag.double().cpu().numpy(), ref_gm)
            e_gz = rel_norm(g_zeta.double().cpu().numpy(), ref_gz)
            log(f"quadruped front end fp{32 if precision == 4 else 64}: nnz {fe.nnz} ({fe.nnz / n:.1f} per row)",
                dict(rows=e_rows, br=e_br, g_mag=e_gm, g_zeta=e_gz))
            assert e_rows <= vt and e_br <= vt and e_gm <= gt and e_gz <= gt
            if precision == 8:
                d = torch.as_tensor(rng.standard_normal(n), dtype=torch.float64, device="cuda")
                p = torch.as_tensor(phi, dtype=torch.float64, device="cuda")
                g = torch.as_tensor(gd, dtype=torch.float64, device="cuda")
                e = 1e-5
                lp = float(fe.forward(p + e * d, mag, zeta, 8.0, 1.0, 1e-6)[0] @ g)
                lm = float(fe.forward(p - e * d, mag, zeta, 8.0, 1.0, 1e-6)[0] @ g)
                adj = float(g_phi @ d)
                fd = (lp - lm) / (2 * e)
                log("quadruped filter FD", fd, adj)
                assert abs(fd - adj) <= 1e-7 * abs(adj)
        finally:
            fe.close()


def test_chain_through_the_rollout_matches_the_oracle_chain():
    """design variables -> front end -> rollout -> loss, differentiated by torch
    autograd through DesignFn and MpmMagFn, against the oracle's front end,
    rollout adjoint and front-end transpose (FP64)."""
    import oracle as orc
    inst = W.make_tiny(seed=12, dim=2, n_steps=16, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0,
                       size=(0.4, 0.2, 0.2), n_grid=16, n_segments=4)
    rng = np.random.default_rng(13)
    n = inst.n
    region = (np.arange(n) % 3).astype(np.int32)
    phi, mag, zeta = rng.uniform(0.3, 1, n), rng.uniform(0.3, 1, 3), rng.uniform(-1, 1, (3, 2))
    R = 1.6 * inst.params["particle_volume"] ** 0.5
    beta, bmax, delta = 4.0, 1.0, 1e-4
    # oracle chain
    _, pb, br = OD.front_end(inst.x0, phi, R, beta, region, mag, zeta, bmax, delta)
    ref = orc.backward(inst.params, inst.x0, pb, br, inst.b_prog, inst.target, inst.mask, ckpt_every=4)
    og_phi, og_mag, og_zeta = OD.front_end_backward(inst.x0, phi, R, beta, region, mag, zeta, bmax, delta,
                                                    ref["g_density"], ref["g_br"])
    # device chain
    sim = M.MpmMag([inst.params], [n], precision=8)
    fe = PD.MpmMagDesign(inst.x0, R, region=region, n_regions=3, precision=8)
    try:
        x0, _, _, b_prog, target, mask = M.instance_tensors([inst], dtype=torch.float64)
        tp = torch.tensor(phi, dtype=torch.float64, device="cuda", requires_grad=True)
        tm = torch.tensor(mag, dtype=torch.float64, device="cuda", requires_grad=True)
        tz = torch.tensor(zeta, dtype=torch.float64, device="cuda", requires_grad=True)
        dens, tbr = PD.DesignFn.apply(fe, tp, tm, tz, beta, bmax, delta)
        loss, _ = M.MpmMagFn.apply(sim, x0, dens, tbr, b_prog, target, mask)
        loss.sum().backward()
        torch.cuda.synchronize()
        errs = dict(loss=abs(loss.item() - ref["loss"]), g_phi=rel_norm(tp.grad.cpu().numpy(), og_phi),
                    g_mag=rel_norm(tm.grad.cpu().numpy(), og_mag), g_zeta=rel_norm(tz.grad.cpu().numpy(), og_zeta))
        log("design chain fp64", errs)
        assert errs["loss"] <= 1e-9 * max(1.0, abs(ref["loss"]))
        assert errs["g_phi"] <= 1e-9 and errs["g_mag"] <= 1e-9 and errs["g_zeta"] <= 1e-9
    finally:
        fe.close()
        sim.close()


# ---------------------------------------------------------------- harmonic stimulus (Eqs. 29-30)

@pytest.mark.parametrize("dim,n_inst", [(2, 1), (3, 3)])
@pytest.mark.parametrize("precision", [8, 4])
def test_harmonic_program_matches_oracle(dim, n_inst, precision):
    rng = np.random.default_rng(40 + dim)
    T, dt, bmax, fmin, fmax, delta = 4000, 5e-5, 0.8, 2.0, 60.0, 1e-4
    b_a, f, eta = rng.uniform(0.1, 1, n_inst), rng.uniform(0, 1, n_inst), rng.uniform(-1, 1, (n_inst, dim))
    g = rng.standard_normal((n_inst * T, dim))
    dt_ = torch.float32 if precision == 4 else torch.float64
    cu = lambda a: torch.as_tensor(a, dtype=dt_, device="cuda")
    prog = PD.harmonic_program(cu(b_a), cu(f), cu(eta), T, dt, bmax, fmin, fmax, delta)
    gb, gf, ge = PD.harmonic_backward(cu(b_a), cu(f), cu(eta), T, dt, bmax, fmin, fmax, delta, cu(g))
    torch.cuda.synchronize()
    # the oracle takes the inputs the device got
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64) if precision == 4 else a
    ref = OD.harmonic_program(r(b_a), r(f), r(eta), T, dt, bmax, fmin, fmax, delta)
    rgb, rgf, rge = OD.harmonic_program_transpose(r(b_a), r(f), r(eta), T, dt, bmax, fmin, fmax, delta, r(g))
    vt, gt = (1e-13, 1e-12) if precision == 8 else (1e-6, 1e-6)
    assert np.abs(prog.double().cpu().numpy() - ref).max() <= vt
    assert rel_norm(gb.double().cpu().numpy(), rgb) <= gt
    assert rel_norm(gf.double().cpu().numpy(), rgf) <= gt
    assert rel_norm(ge.double().cpu().numpy(), rge) <= gt


def test_harmonic_errors_are_reported():
    e = torch.ones(1, 2, dtype=torch.float64, device="cuda")
    o = torch.ones(1, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MpmMagError, match="invalid argument"):
        PD.harmonic_program(o, o, e, 10, -1.0, 1.0, 0.0, 1.0, 0.0)   # dt <= 0
    with pytest.raises(M.MpmMagError, match="invalid argument"):
        PD.harmonic_program(o, o, e, 0, 1e-3, 1.0, 0.0, 1.0, 0.0)    # no steps


def test_harmonic_chain_through_the_rollout_matches_the_oracle_chain():
    """(B_a, f, eta) -> one-row-per-step program -> rollout -> loss, by torch
    autograd through HarmonicFn and MpmMagFn, against the oracle's program, its
    rollout adjoint and the program transpose (FP64)."""
    import oracle as orc
    T = 24
    inst = W.make_tiny(seed=15, dim=3, n_steps=T, loss_kind=W.LOSS_TRAJ_VEL, floor=True, gravity=1.0,
                       size=(0.3, 0.2, 0.25), n_grid=16, n_segments=T)
    p = dict(inst.params)
    assert p["n_segments"] == T and p["seg_steps"] == 1 and not p["periodic"]
    dt = p["dt"]
    fmin, fmax = 0.5 / (T * dt), 3.0 / (T * dt)   # half a period to three over the rollout
    b_a, f, eta = np.array([0.7]), np.array([0.4]), np.array([[0.3, -0.8, 0.5]])
    args = (T, dt, 0.5, fmin, fmax, 1e-4)
    prog = OD.harmonic_program(b_a, f, eta, *args)
    ref = orc.backward(p, inst.x0, inst.density, inst.br, prog, inst.target, inst.mask, ckpt_every=5)
    rgb, rgf, rge = OD.harmonic_program_transpose(b_a, f, eta, *args, ref["g_b_prog"])
    sim = M.MpmMag([p], [inst.n], precision=8)
    try:
        x0, density, br, _, target, mask = M.instance_tensors([inst], dtype=torch.float64)
        tb = torch.tensor(b_a, dtype=torch.float64, device="cuda", requires_grad=True)
        tf = torch.tensor(f, dtype=torch.float64, device="cuda", requires_grad=True)
        te = torch.tensor(eta, dtype=torch.float64, device="cuda", requires_grad=True)
        bp = PD.HarmonicFn.apply(tb, tf, te, *args)
        loss, _ = M.MpmMagFn.apply(sim, x0, density, br, bp, target, mask)
        loss.sum().backward()
        torch.cuda.synchronize()
        errs = dict(loss=abs(loss.item() - ref["loss"]), g_b_a=rel_norm(tb.grad.cpu().numpy(), rgb),
                    g_f=rel_norm(tf.grad.cpu().numpy(), rgf), g_eta=rel_norm(te.grad.cpu().numpy(), rge))
        log("harmonic chain fp64", errs)
        assert errs["loss"] <= 1e-9 * max(1.0, abs(ref["loss"]))
        assert errs["g_b_a"] <= 1e-9 and errs["g_f"] <= 1e-9 and errs["g_eta"] <= 1e-9
    finally:
        sim.close()
