"""Obstacles on the device (solid boundaries of Eq. 18 beyond the floor:
half-space, sphere, box; static or moving with v_b; sliding, no-slip or
attached) against the FP64 oracle on the same seeded inputs, forward and
gradient, FP64 (1e-10 / 1e-9) and FP32 (1e-4 / 1e-3)."""
import math

import numpy as np
import pytest

from paper_2503_22767_amd import mpm_mag as M
from paper_2503_22767_amd import workloads as W

from gpu_util import compare, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu

HS, SP, BX = M.OBSTACLE_HALFSPACE, M.OBSTACLE_SPHERE, M.OBSTACLE_BOX


def _inst(dim, case, seed):
    size = (0.3, 0.15, 0.15) if dim == 2 else (0.2, 0.15, 0.15)
    inst = W.make_tiny(seed=seed, dim=dim, n_steps=24, loss_kind=W.LOSS_COM_DISP, floor=case == "floor_and_two",
                       gravity=1.0, size=size, n_grid=16, n_segments=4)
    p = dict(inst.params)
    lo, hi = inst.x0.min(0), inst.x0.max(0)
    mid = (lo + hi) / 2
    dx = 1.0 / p["n_grid"]
    z = lambda v: list(v) + [0.0] * (3 - len(v))
    below = z([mid[0], lo[1] - 0.25 + 0.6 * dx] + ([mid[2]] if dim == 3 else []))
    cases = {
        "sphere_slide": [dict(kind=SP, a=below, b=[0.25, 0, 0], mu=0.4)],
        "halfspace_tilted_moving": [dict(kind=HS, a=z([hi[0] + 0.3 * dx, mid[1]] + ([mid[2]] if dim == 3 else [])),
                                         b=[-1.0, 0.3, 0.2], mu=0.2, vel=[-0.3, 0.05, 0.0])],
        "box_noslip": [dict(kind=BX, a=z([mid[0], lo[1] - 0.1 + 0.4 * dx] + ([mid[2]] if dim == 3 else [])),
                            b=[0.3, 0.1, 0.3], mu=math.inf)],
        "box_attached_moving": [dict(kind=BX, a=z([lo[0] + dx] + list(mid[1:dim])), b=[1.5 * dx, 0.2, 0.2],
                                     attached=1, vel=[0.2, 0.3, -0.1])],
        "floor_and_two": [dict(kind=SP, a=z([lo[0], mid[1]] + ([mid[2]] if dim == 3 else [])), b=[2 * dx, 0, 0],
                               mu=0.3, vel=[0.4, 0.0, 0.0]),
                          dict(kind=HS, a=z([hi[0] - dx, 0.0, 0.0]), b=[-1.0, 0.0, 0.0], mu=math.inf)],
    }
    # the most an instance takes: one of each kind plus a second box, in this order
    cases["four"] = cases["sphere_slide"] + cases["halfspace_tilted_moving"] + cases["box_attached_moving"] + \
        cases["box_noslip"]
    p["obstacles"] = cases[case]
    return W.Instance(p, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask)


CASES = ["sphere_slide", "halfspace_tilted_moving", "box_noslip", "box_attached_moving", "floor_and_two", "four"]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("case", CASES)
def test_obstacles_match_oracle(dim, case):
    inst = _inst(dim, case, seed=60 + dim)
    ref = oracle_run([inst])
    free = oracle_run([W.Instance({k: v for k, v in inst.params.items() if k != "obstacles"}, inst.x0,
                                  inst.density, inst.br, inst.b_prog, inst.target, inst.mask)], backward=False)
    moved = np.abs(ref["x"] - free["x"]).max()
    log(f"obstacle {case} d{dim}: N {inst.n}, largest position change the obstacles make {moved:.3e}")
    assert moved > 1e-6   # the obstacles act in this case
    got = gpu_run([inst], precision=8)
    compare(got, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label=f"{case} d{dim} fp64")
    got = gpu_run([inst], precision=4)
    compare(got, ref, pos_tol=1e-4, grad_tol=1e-3, label=f"{case} d{dim} fp32")


def test_batched_instances_with_different_obstacles():
    insts = [_inst(2, c, seed=70 + k) for k, c in enumerate(CASES)]
    ref = oracle_run(insts)
    got = gpu_run(insts, precision=8, options={"streams": 2})
    compare(got, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label="batched obstacles fp64")


@pytest.mark.parametrize("bad", ["kind", "normal", "radius", "count"])
def test_bad_obstacles_are_refused(bad):
    inst = _inst(2, "sphere_slide", seed=80)
    p = dict(inst.params)
    o = dict(p["obstacles"][0])
    if bad == "kind":
        o["kind"] = 7
    elif bad == "normal":
        o.update(kind=HS, b=[0.0, 0.0, 0.0])
    elif bad == "radius":
        o["b"] = [0.0, 0, 0]
    p["obstacles"] = [o] * (5 if bad == "count" else 1)
    if bad == "count":
        with pytest.raises(ValueError):
            M.MpmMag([p], [inst.n], precision=8)
        return
    with pytest.raises(M.MpmMagError, match="invalid argument|obstacle"):
        M.MpmMag([p], [inst.n], precision=8)
