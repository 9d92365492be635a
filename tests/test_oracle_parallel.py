"""The oracle's parallel loops against its serial order.

With one thread the oracle's loops run in particle order; with several, each
thread scatters its block of particles into a private grid and the grids are
summed in thread order. The two differ only in the order of additions, so
rollouts and gradients agree to round-off, and a run with a given thread count
repeats bit for bit. The cases cover 2D and 3D, floor contact, a clamp,
obstacles and every loss kind, and one error path (a stencil leaving the grid
is reported with the same status as in the serial order).
"""
import numpy as np
import pytest

import oracle as orc
from paper_2503_22767_amd import workloads as W


@pytest.fixture
def threads():
    yield
    orc.set_threads(0)


def _case(dim, kind, seed):
    inst = W.make_tiny(seed=seed, dim=dim, n_steps=12, loss_kind=kind, floor=True, gravity=1.0,
                       clamp=(kind == W.LOSS_FINAL_MSE), n_grid=16 if dim == 3 else 24,
                       size=(0.3, 0.15, 0.15))
    if kind == W.LOSS_TIP_DISP:
        inst.params["obstacles"] = [dict(kind=orc.OBST_SPHERE, a=[0.3, 0.2, 0.3], b=[0.08, 0, 0], mu=0.3,
                                         vel=[0.1, 0.0, 0.0])]
    return inst


def _run(inst):
    r = orc.rollout(inst.params, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask)
    g = orc.backward(inst.params, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask,
                     ckpt_every=4)
    return r, g


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", [W.LOSS_FINAL_MSE, W.LOSS_COM_DISP, W.LOSS_TRAJ_VEL, W.LOSS_TIP_DISP])
def test_threads_agree_with_serial_order(threads, dim, kind):
    inst = _case(dim, kind, 40 + 4 * dim + kind)
    orc.set_threads(1)
    assert orc.get_threads() == 1
    r1, g1 = _run(inst)
    orc.set_threads(4)
    assert orc.get_threads() == 4
    r4, g4 = _run(inst)
    r4b, g4b = _run(inst)
    assert np.max(np.abs(r4["x"] - r1["x"])) < 1e-14
    assert abs(r4["loss"] - r1["loss"]) <= 1e-12 * abs(r1["loss"])
    for k in ("g_density", "g_br", "g_b_prog"):
        ref = g1[k]
        assert np.linalg.norm(g4[k] - ref) <= 1e-11 * np.linalg.norm(ref), k
        assert np.array_equal(g4[k], g4b[k]), k           # a thread count repeats exactly
    assert np.array_equal(r4["x"], r4b["x"])


def test_error_status_does_not_depend_on_threads(threads):
    inst = W.make_tiny(seed=3, dim=2, n_steps=5, n_grid=16)
    x0 = inst.x0.copy()
    x0[len(x0) // 2, 0] = 0.999          # a stencil beyond the grid, in the middle of the list
    x0[len(x0) - 1, 1] = np.nan          # and a later non-finite particle
    codes = []
    for t in (1, 3):
        orc.set_threads(t)
        with pytest.raises(orc.OracleError) as e:
            orc.rollout(inst.params, x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask)
        codes.append(e.value.code)
    assert codes == [orc.EDOMAIN, orc.EDOMAIN]
