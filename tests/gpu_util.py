"""Helpers shared by the GPU tests: run a workload instance list through the
C ABI and through the FP64 oracle on the same seeded arrays, and compare with
the parity metrics (positions: max abs error; gradients: norm-wise relative)."""
import sys

import numpy as np
import torch

import oracle as orc
from paper_2503_22767_amd import mpm_mag as M


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(instances, precision, record=True, backward=True, options=None, dloss=None):
    dtype = torch.float32 if precision == 4 else torch.float64
    sim = M.MpmMag([i.params for i in instances], [i.n for i in instances], precision=precision)
    try:
        for k, v in (options or {}).items():
            sim.set_option(k, v)
        x0, density, br, b_prog, target, mask = M.instance_tensors(instances, dtype=dtype)
        loss, x = sim.rollout(x0, density, br, b_prog, target, mask, record=record)
        out = dict(loss=loss.double().cpu().numpy(), x=x.double().cpu().numpy())
        if backward:
            dl = torch.ones(len(instances), dtype=dtype, device="cuda") if dloss is None else \
                torch.as_tensor(dloss, dtype=dtype, device="cuda")
            gd, gb, gp = sim.backward(dl)
            out.update(g_density=gd.double().cpu().numpy(), g_br=gb.double().cpu().numpy(),
                       g_b_prog=gp.double().cpu().numpy())
        torch.cuda.synchronize()
        return out
    finally:
        sim.close()


def oracle_run(instances, backward=True, ckpt_every=None):
    xs, losses, gds, gbs, gps = [], [], [], [], []
    for inst in instances:
        p = inst.params
        r = orc.rollout(p, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask)
        xs.append(r["x"][:, :p["dim"]])
        losses.append(r["loss"])
        if backward:
            g = orc.backward(p, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask,
                             ckpt_every=ckpt_every or max(1, int(np.sqrt(max(1, p["n_steps"])))))
            gds.append(g["g_density"]); gbs.append(g["g_br"]); gps.append(g["g_b_prog"])
    out = dict(x=np.concatenate(xs), loss=np.array(losses))
    if backward:
        out.update(g_density=np.concatenate(gds), g_br=np.concatenate(gbs), g_b_prog=np.concatenate(gps))
    return out


def rel_norm(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / den if den > 0 else np.linalg.norm(a - b)


def compare(gpu, ref, pos_tol, grad_tol, loss_tol=None, label=""):
    errs = dict(x=float(np.max(np.abs(gpu["x"] - ref["x"]))))
    if loss_tol is not None:
        errs["loss"] = float(np.max(np.abs(gpu["loss"] - ref["loss"]) / np.maximum(1e-30, np.abs(ref["loss"]))))
    for k in ("g_density", "g_br", "g_b_prog"):
        if k in gpu and k in ref:
            errs[k] = float(rel_norm(gpu[k], ref[k]))
    log(label, {k: f"{v:.3e}" for k, v in errs.items()})
    assert errs["x"] <= pos_tol, (label, errs)
    if loss_tol is not None:
        assert errs["loss"] <= loss_tol, (label, errs)
    for k in ("g_density", "g_br", "g_b_prog"):
        if k in errs:
            assert errs[k] <= grad_tol, (label, k, errs)
    return errs
