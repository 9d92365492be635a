"""The co-design loop on the device (Sec. 3.2): the Adam update with the bound
map against its oracle, the front end's design copies (one per task, Eq. 35),
and whole iterations: the first one's gradients against the oracle's chain over
every task, then bounds, the beta schedule and a falling loss."""
import numpy as np
import pytest
import torch

import oracle as orc
from oracle import design as OD
from paper_2503_22767_amd import codesign as CD
from paper_2503_22767_amd import design as PD
from paper_2503_22767_amd import workloads as W

from gpu_util import log, rel_norm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [8, 4])
def test_adam_step_matches_oracle(precision):
    rng = np.random.default_rng(50)
    n = 100003
    dt = torch.float32 if precision == 4 else torch.float64
    p = rng.uniform(0, 1, n)
    cu = lambda a: torch.as_tensor(a, dtype=dt, device="cuda").contiguous()
    tp, tm, tv = cu(p), torch.zeros(n, dtype=dt, device="cuda"), torch.zeros(n, dtype=dt, device="cuda")
    rp, rm, rv = p.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 1, n)
        g32 = g.astype(np.float32).astype(np.float64) if precision == 4 else g
        CD.adam_step(tp, cu(g), tm, tv, t, 0.05, 0.0, 1.0)
        rp, rm, rv = OD.adam_step(rp, g32, rm, rv, t, 0.05, 0.9, 0.999, 1e-8, 0.0, 1.0)
    torch.cuda.synchronize()
    tol = 1e-13 if precision == 8 else 2e-6
    assert np.abs(tp.double().cpu().numpy() - rp).max() <= tol
    assert rel_norm(tm.double().cpu().numpy(), rm) <= tol and rel_norm(tv.double().cpu().numpy(), rv) <= tol
    assert (tp.double().cpu().numpy().min() >= 0.0) and (tp.double().cpu().numpy().max() <= 1.0)


def test_front_end_copies_sum_the_tasks_gradients():
    rng = np.random.default_rng(51)
    x0 = rng.uniform(0.3, 0.5, (900, 3))
    region = rng.integers(0, 4, 900).astype(np.int32)
    phi, mag, zeta = rng.uniform(0, 1, 900), rng.uniform(0.2, 1, 4), rng.uniform(-1, 1, (4, 3))
    c = 3
    gd, gb = rng.standard_normal((c, 900)), rng.standard_normal((c, 900, 3))
    fe = PD.MpmMagDesign(x0, 0.03, region=region, n_regions=4, precision=8)
    try:
        dens, br = fe.forward(phi, mag, zeta, 6.0, 1.1, 1e-4, copies=c)
        g_phi, g_mag, g_zeta = fe.backward(gd.reshape(-1), gb.reshape(-1, 3), copies=c)
        torch.cuda.synchronize()
        dens, br = dens.cpu().numpy().reshape(c, 900), br.cpu().numpy().reshape(c, 900, 3)
    finally:
        fe.close()
    _, pb, obr = OD.front_end(x0, phi, 0.03, 6.0, region, mag, zeta, 1.1, 1e-4)
    for k in range(c):
        assert np.abs(dens[k] - pb).max() <= 1e-13 and np.abs(br[k] - obr).max() <= 1e-13
    r_phi, r_mag, r_zeta = OD.front_end_backward(x0, phi, 0.03, 6.0, region, mag, zeta, 1.1, 1e-4, gd.sum(0),
                                                 gb.sum(0))
    assert rel_norm(g_phi.cpu().numpy(), r_phi) <= 1e-12
    assert rel_norm(g_mag.cpu().numpy(), r_mag) <= 1e-12 and rel_norm(g_zeta.cpu().numpy(), r_zeta) <= 1e-12


def _tasks(T=30):
    """Two tasks on one 2D body: walk along +x (centre-of-mass loss, floor and
    gravity) and reach a bent shape (final-shape loss)."""
    base = W.make_tiny(seed=52, dim=2, n_steps=T, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0,
                       size=(0.4, 0.2, 0.2), n_grid=16, n_segments=T)
    bend = W.make_tiny(seed=52, dim=2, n_steps=T, loss_kind=W.LOSS_FINAL_MSE, floor=True, gravity=1.0,
                       size=(0.4, 0.2, 0.2), n_grid=16, n_segments=T)
    assert np.array_equal(base.x0, bend.x0)
    return [base, bend]


def _cfg(inst):
    T, dt = inst.params["n_steps"], inst.params["dt"]
    h = inst.params["particle_volume"] ** 0.5
    return CD.CoDesignConfig(radius=1.6 * h, b_max=0.6, f_min=0.5 / (T * dt), f_max=3.0 / (T * dt), br_max=1.0,
                             delta=1e-4, lr=0.02)


def test_first_iteration_gradients_match_the_oracle_chain():
    tasks = _tasks()
    x0 = tasks[0].x0
    n = len(x0)
    region = (np.arange(n) % 4).astype(np.int32)
    cfg = _cfg(tasks[0])
    targets = [t.target if t.target is not None else t.x0 for t in tasks]
    masks = [t.mask if t.mask is not None else np.ones(n, np.uint8) for t in tasks]
    cd = CD.CoDesign([t.params for t in tasks], x0, cfg, region=region, n_regions=4, targets=targets, masks=masks,
                     precision=8, seed=3, init=dict(phi=np.random.default_rng(4).uniform(0.3, 1.0, n)))
    try:
        v = {k: t.cpu().numpy().copy() for k, t in cd.var.items()}
        beta = cd.beta
        loss = cd.evaluate(record=True)
        g = {k: t.cpu().numpy() for k, t in cd.gradients().items()}
        torch.cuda.synchronize()
    finally:
        cd.close()
    # oracle chain: front end, each task's rollout adjoint, the transposes
    _, pb, br = OD.front_end(x0, v["phi"], cfg.radius, beta, region, v["br_mag"], v["zeta"], cfg.br_max, cfg.delta)
    T, dt = tasks[0].params["n_steps"], tasks[0].params["dt"]
    harm = (T, dt, cfg.b_max, cfg.f_min, cfg.f_max, cfg.delta)
    prog = OD.harmonic_program(v["b_a"], v["f"], v["eta"], *harm).reshape(2, T, 2)
    gd, gb, gp, losses = np.zeros(n), np.zeros((n, 2)), np.zeros((2 * T, 2)), []
    for l, t in enumerate(tasks):
        r = orc.backward(t.params, x0, pb, br, prog[l], targets[l], masks[l], ckpt_every=6)
        gd += r["g_density"]
        gb += r["g_br"]
        gp[l * T:(l + 1) * T] = r["g_b_prog"]
        losses.append(r["loss"])
    r_phi, r_mag, r_zeta = OD.front_end_backward(x0, v["phi"], cfg.radius, beta, region, v["br_mag"], v["zeta"],
                                                 cfg.br_max, cfg.delta, gd, gb)
    r_ba, r_f, r_eta = OD.harmonic_program_transpose(v["b_a"], v["f"], v["eta"], *harm, gp)
    errs = dict(loss=np.abs(loss.cpu().numpy() - losses).max(), phi=rel_norm(g["phi"], r_phi),
                br_mag=rel_norm(g["br_mag"], r_mag), zeta=rel_norm(g["zeta"], r_zeta), b_a=rel_norm(g["b_a"], r_ba),
                f=rel_norm(g["f"], r_f), eta=rel_norm(g["eta"], r_eta))
    log("co-design first iteration vs oracle chain", errs)
    assert errs["loss"] <= 1e-9 * max(1.0, np.abs(losses).max())
    assert all(errs[k] <= 1e-9 for k in ("phi", "br_mag", "zeta", "b_a", "f", "eta"))


def test_iterations_keep_bounds_follow_the_schedule_and_lower_the_loss():
    tasks = _tasks()
    x0 = tasks[0].x0
    n = len(x0)
    cfg = _cfg(tasks[0])
    targets = [t.target if t.target is not None else t.x0 for t in tasks]
    masks = [t.mask if t.mask is not None else np.ones(n, np.uint8) for t in tasks]
    cd = CD.CoDesign([t.params for t in tasks], x0, cfg, region=(np.arange(n) % 4).astype(np.int32), n_regions=4,
                     targets=targets, masks=masks, precision=4, seed=5)
    try:
        betas = []
        for _ in range(14):
            betas.append(cd.beta)
            cd.step()
            b = cfg.bounds
            for k, t in cd.var.items():
                lo, hi = getattr(b, k)
                a = t.double().cpu().numpy()
                assert a.min() >= lo and a.max() <= hi, k
        hist = list(cd.history)
    finally:
        cd.close()
    log("co-design loss history", [f"{h:.5g}" for h in hist])
    assert betas[:10] == [1.0] * 10 and betas[10:] == [2.0] * 4
    assert min(hist[1:]) < hist[0]
    assert all(np.isfinite(hist))
