"""Graph replay and instance batching on the device.

* Graph replay: the step loop of a rollout and the reverse sweep of backward,
  captured once into HIP graphs, give the eager launches' results on every
  replay (several replays with other device work and synchronizations between
  them), and a changed checkpoint plan rebuilds the graphs.
* Batching: many instances of uneven size advanced together in one launch per
  phase give the results of separate handles, and sampled instances of the
  batch match the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from paper_2503_22767_amd import mpm_mag as M
from paper_2503_22767_amd import workloads as W

from gpu_util import compare, gpu_run, log, oracle_run, rel_norm

pytestmark = pytest.mark.gpu


def _run(sim, tens, dtype, n_inst):
    loss, x = sim.rollout(*tens, record=True)
    gd, gb, gp = sim.backward(torch.ones(n_inst, dtype=dtype, device="cuda"))
    torch.cuda.synchronize()
    return dict(loss=loss.double().cpu().numpy(), x=x.double().cpu().numpy(),
                g_density=gd.double().cpu().numpy(), g_br=gb.double().cpu().numpy(),
                g_b_prog=gp.double().cpu().numpy())


def _max_rel(a, b):
    errs = {}
    for k in a:
        den = max(1e-300, float(np.max(np.abs(b[k]))))
        errs[k] = float(np.max(np.abs(a[k] - b[k]))) / den
    return errs


@pytest.mark.parametrize("precision,tol", [(8, 1e-12), (4, 1e-5)], ids=["fp64", "fp32"])
def test_graph_replay_matches_direct_launches(precision, tol):
    insts = [W.make_tiny(seed=7, dim=2, n_steps=36, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0,
                         size=(0.4, 0.2, 0.2), n_grid=16, n_segments=4),
             W.make_tiny(seed=8, dim=2, n_steps=36, loss_kind=W.LOSS_FINAL_MSE, clamp=True,
                         size=(0.3, 0.15, 0.2), n_grid=16, n_segments=3)]
    dtype = torch.float32 if precision == 4 else torch.float64
    sim = M.MpmMag([i.params for i in insts], [i.n for i in insts], precision=precision)
    try:
        tens = M.instance_tensors(insts, dtype=dtype)
        ref = _run(sim, tens, dtype, len(insts))
        sim.set_option("graph", 1)
        scratch = torch.randn(1 << 16, device="cuda", dtype=dtype)
        for rep in range(3):
            got = _run(sim, tens, dtype, len(insts))
            errs = _max_rel(got, ref)
            log("graph replay", rep, {k: f"{v:.2e}" for k, v in errs.items()})
            assert all(v <= tol for v in errs.values()), (rep, errs)
            # other device work between replays
            scratch.mul_(1.0001).add_(0.5)
            torch.cuda.synchronize()
        # a new checkpoint plan changes the buffers: the graphs must be rebuilt
        sim.set_option("ckpt_every", 5)
        got = _run(sim, tens, dtype, len(insts))
        errs = _max_rel(got, ref)
        log("graph after new plan", {k: f"{v:.2e}" for k, v in errs.items()})
        assert all(v <= tol for v in errs.values()), errs
        # and back to direct launches
        sim.set_option("graph", 0)
        got = _run(sim, tens, dtype, len(insts))
        assert all(v <= tol for v in _max_rel(got, ref).values())
    finally:
        sim.close()
    # the graph path against the oracle too
    got = gpu_run(insts, precision=precision, options={"graph": 1})
    ref_o = oracle_run(insts)
    if precision == 8:
        compare(got, ref_o, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label="graph fp64")
    else:
        compare(got, ref_o, pos_tol=1e-4, grad_tol=1e-3, label="graph fp32")


def test_graph_replay_walker_first_steps():
    """The 2D walker at full size, 120 steps, replayed twice from graphs."""
    wl = W.make_walker2d(n_steps=120)
    inst = wl.instances[0]
    dtype = torch.float32
    sim = M.MpmMag([inst.params], [inst.n], precision=4)
    try:
        sim.set_option("ckpt_every", 12)
        tens = M.instance_tensors([inst], dtype=dtype)
        ref = _run(sim, tens, dtype, 1)
        sim.set_option("graph", 1)
        for rep in range(2):
            got = _run(sim, tens, dtype, 1)
            errs = _max_rel(got, ref)
            log("walker graph replay", rep, {k: f"{v:.2e}" for k, v in errs.items()})
            assert all(v <= 1e-5 for v in errs.values()), errs
    finally:
        sim.close()


def _batch(n_instances, n_steps):
    return W.make_batch2d(n_steps=n_steps, n_instances=n_instances)


def test_batched_instances_match_separate_handles():
    """All 64 instances of the batched workload (1k..30k particles each, own
    grid size, program and loss) in one handle vs one handle per instance.

    Same arithmetic, but not the same rounding: the batch orders particles on
    the Hilbert curve of its largest grid, so chunks (and their fixed-point
    scales) differ from a lone instance's, and both are FP32 results that must
    each meet the parity bar against the FP64 oracle. Bars: positions 1e-5
    absolute, loss 1e-6 absolute (the centre-of-mass losses are ~1e-6 after 40
    steps), gradients the parity bar 1e-3 norm-wise (a mix-up of instances,
    programs or offsets shows as O(1))."""
    wl = _batch(64, 40)
    got = gpu_run(wl.instances, precision=4)
    offs = np.cumsum([0] + [i.n for i in wl.instances])
    soffs = np.cumsum([0] + [i.params["n_segments"] for i in wl.instances])
    worst = {}
    for k, inst in enumerate(wl.instances):
        one = gpu_run([inst], precision=4)
        sl = slice(offs[k], offs[k + 1])
        sp = slice(soffs[k], soffs[k + 1])
        errs = dict(x=float(np.max(np.abs(got["x"][sl] - one["x"]))),
                    loss=float(abs(got["loss"][k] - one["loss"][0])),
                    g_density=rel_norm(got["g_density"][sl], one["g_density"]),
                    g_br=rel_norm(got["g_br"][sl], one["g_br"]),
                    g_b_prog=rel_norm(got["g_b_prog"][sp], one["g_b_prog"]))
        for name, e in errs.items():
            worst[name] = max(worst.get(name, 0.0), float(e))
    log("batched vs separate (worst over instances)", {k: f"{v:.2e}" for k, v in worst.items()})
    bars = dict(x=1e-5, loss=1e-6, g_density=1e-3, g_br=1e-3, g_b_prog=1e-3)
    for name, e in worst.items():
        assert e <= bars[name], (name, e)


def test_batched_instances_match_oracle():
    """Instances sampled from the 64-instance batch (a beam, a walker, the
    largest) against the FP64 oracle, run inside the full batch."""
    wl = _batch(64, 40)
    got = gpu_run(wl.instances, precision=4)
    sizes = [i.n for i in wl.instances]
    pick = sorted({0, 1, int(np.argmax(sizes))})
    offs = np.cumsum([0] + sizes)
    soffs = np.cumsum([0] + [i.params["n_segments"] for i in wl.instances])
    for k in pick:
        inst = wl.instances[k]
        ref = oracle_run([inst])
        sl = slice(offs[k], offs[k + 1])
        sp = slice(soffs[k], soffs[k + 1])
        sub = dict(x=got["x"][sl], loss=got["loss"][k:k + 1], g_density=got["g_density"][sl],
                   g_br=got["g_br"][sl], g_b_prog=got["g_b_prog"][sp])
        compare(sub, ref, pos_tol=1e-4, grad_tol=1e-3, label=f"batch instance {k} (N={inst.n})")


@pytest.mark.parametrize("streams", [2, 3])
def test_instance_groups_on_streams_match_one_stream(streams):
    """Instances advanced in groups on separate streams give the one-stream
    results (FP64, only summation order may differ) and the oracle's."""
    insts = [W.make_tiny(seed=30, dim=2, n_steps=18, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0,
                         size=(0.3, 0.2, 0.25), n_grid=16, n_segments=3)]
    insts += [W.make_tiny(seed=40 + k, dim=2, n_steps=18, loss_kind=W.LOSS_FINAL_MSE, clamp=True,
                          size=(0.3 + 0.05 * k, 0.15, 0.2), n_grid=16 + 8 * k, n_segments=2) for k in range(2)]
    one = gpu_run(insts, precision=8, options={"streams": 1})
    many = gpu_run(insts, precision=8, options={"streams": streams})
    errs = _max_rel(many, one)
    log("streams", streams, {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(v <= 1e-12 for v in errs.values()), errs
    ref = oracle_run(insts)
    compare(many, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label=f"streams={streams} fp64")
    # and with graph replay of the grouped launches
    g = gpu_run(insts, precision=4, options={"streams": streams, "graph": 1})
    compare(g, ref, pos_tol=1e-4, grad_tol=1e-3, label=f"streams={streams} graph fp32")


def test_most_instance_groups_match_one_stream():
    """Eight instance groups, the most the library runs (more streams than the
    device's hardware queues), over ten instances of different grids, losses
    and boundaries: the one-stream results in FP64, and the oracle's, also under
    graph replay."""
    kinds = [W.LOSS_COM_DISP, W.LOSS_FINAL_MSE, W.LOSS_TIP_DISP, W.LOSS_TRAJ_VEL]
    insts = [W.make_tiny(seed=90 + k, dim=2, n_steps=14, loss_kind=kinds[k % 4], floor=k % 2 == 0,
                         gravity=1.0, clamp=k % 3 == 1, size=(0.25 + 0.02 * k, 0.15, 0.2),
                         n_grid=16 + 8 * (k % 3), n_segments=2 + k % 3) for k in range(10)]
    one = gpu_run(insts, precision=8, options={"streams": 1})
    many = gpu_run(insts, precision=8, options={"streams": 8})
    errs = _max_rel(many, one)
    log("streams 8", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(v <= 1e-12 for v in errs.values()), errs
    ref = oracle_run(insts)
    compare(many, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label="streams=8 fp64")
    g = gpu_run(insts, precision=4, options={"streams": 8, "graph": 1})
    compare(g, ref, pos_tol=1e-4, grad_tol=1e-3, label="streams=8 graph fp32")


def test_lane_order_leaves_fp32_results_unchanged():
    """The lane order of the particle kernels only changes which lane works on
    which particle: in FP32 the grid sums are exact integers, so positions and
    per-particle gradients are bit-identical with and without it, and the
    block-summed loss and program gradient agree to FP64 rounding. The 3D
    block falls under gravity for 60 steps, so particles change cells and the
    order is not the identity."""
    inst = W.make_tiny(seed=21, dim=3, n_steps=60, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=4.0,
                       size=(0.3, 0.2, 0.25), n_grid=16, n_segments=4)
    on = gpu_run([inst], precision=4, options={"lane_sort": 1, "ckpt_every": 7})
    off = gpu_run([inst], precision=4, options={"lane_sort": 0, "ckpt_every": 7})
    for k in ("x", "g_density", "g_br"):
        assert np.array_equal(on[k], off[k]), (k, float(np.max(np.abs(on[k] - off[k]))))
    errs = _max_rel(dict(loss=on["loss"], g_b_prog=on["g_b_prog"]), dict(loss=off["loss"], g_b_prog=off["g_b_prog"]))
    log("lane order on/off", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(v <= 1e-6 for v in errs.values()), errs
    ref = oracle_run([inst])
    compare(on, ref, pos_tol=1e-4, grad_tol=1e-3, label="lane order fp32")
