"""The grid store: the recorded forward keeps every step's active grid blocks,
so the reverse sweep rebuilds a stored segment's grids from it and runs only
the G2P to regain the segment's states; segments beyond the store are
recomputed in full. Every mix gives the oracle's results."""
import pytest
import torch

from paper_2503_22767_amd import mpm_mag as M
from paper_2503_22767_amd import workloads as W

from gpu_util import compare, log, oracle_run

pytestmark = pytest.mark.gpu


def _run_twice(insts, precision, options):
    """Two recorded rollouts and backward passes on one handle; the first sizes
    the store from an estimate, the second from the first one's counts."""
    dtype = torch.float32 if precision == 4 else torch.float64
    sim = M.MpmMag([i.params for i in insts], [i.n for i in insts], precision=precision)
    outs = []
    try:
        for k, v in options.items():
            sim.set_option(k, v)
        x0, density, br, b_prog, target, mask = M.instance_tensors(insts, dtype=dtype)
        for _ in range(2):
            sim.kernel_stats(reset=True)
            loss, x = sim.rollout(x0, density, br, b_prog, target, mask, record=True)
            gd, gb, gp = sim.backward(torch.ones(len(insts), dtype=dtype, device="cuda"))
            torch.cuda.synchronize()
            st = sim.kernel_stats()
            outs.append((dict(loss=loss.double().cpu().numpy(), x=x.double().cpu().numpy(),
                              g_density=gd.double().cpu().numpy(), g_br=gb.double().cpu().numpy(),
                              g_b_prog=gp.double().cpu().numpy()),
                         st["grid_restore"]["launches"], st["p2g"]["launches"] + st["g2p_p2g"]["launches"]))
    finally:
        sim.close()
    return outs


@pytest.mark.parametrize("graph", [0, 1])
def test_whole_store_matches_oracle_fp64(graph):
    """Everything stored from the second rollout on: the reverse sweep restores
    every step's grid (one restore per step) and runs no P2G."""
    inst = W.make_tiny(seed=5, dim=3, n_steps=24, loss_kind=W.LOSS_TRAJ_VEL, floor=True, gravity=1.0,
                       size=(0.3, 0.2, 0.25), n_grid=16, n_segments=4)
    ref = oracle_run([inst])
    for k, (got, restores, p2g) in enumerate(_run_twice([inst], 8, {"graph": graph, "ckpt_every": 5})):
        log("whole store", f"graph={graph} pass {k}: restores {restores}, forward P2G launches {p2g}")
        compare(got, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label=f"store pass {k} fp64")
        if k == 1:
            assert restores == 24
            # the recorded forward's P2G launches only (24 steps, the first unfused)
            assert p2g == 24


@pytest.mark.parametrize("graph", [0, 1])
def test_partial_store_matches_oracle_fp32(graph):
    """A 5 MiB store (639 FP32 block slots; the walker's steps touch 20 to 39
    coarse blocks) holds the first of its ten 16-step segments only:
    that one is restored, the other nine are recomputed."""
    wl = W.make_walker2d(n_steps=160)
    inst = wl.instances[0]
    ref = oracle_run([inst], ckpt_every=16)
    for k, (got, restores, p2g) in enumerate(_run_twice([inst], 4, {"graph": graph, "ckpt_every": 16,
                                                                      "grid_store": 5})):
        log("partial store", f"graph={graph} pass {k}: restores {restores}, P2G launches {p2g}")
        compare(got, ref, pos_tol=1e-4, grad_tol=1e-3, label=f"walker2d[:160] partial store pass {k}")
        assert 0 < restores < 160 and restores % 16 == 0
        assert p2g == 160 + (160 - restores)


def test_store_off_recomputes_every_segment():
    inst = W.make_tiny(seed=6, dim=2, n_steps=20, loss_kind=W.LOSS_FINAL_MSE, floor=False, clamp=True,
                       size=(0.4, 0.2, 0.2), n_grid=16, n_segments=4)
    ref = oracle_run([inst])
    for k, (got, restores, p2g) in enumerate(_run_twice([inst], 8, {"grid_store": 0})):
        compare(got, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label=f"store off pass {k}")
        assert restores == 0 and p2g == 40


def test_batched_chains_share_the_store_fp32():
    """Three instances of different sizes (one 256-particle chunk each, so one
    per stream) on three streams: each stream has its own part of the store;
    both passes match the oracle per instance."""
    insts = [W.make_tiny(seed=30 + k, dim=2, n_steps=30, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0,
                         size=(0.25 + 0.05 * k, 0.15, 0.2), n_grid=32, n_segments=5) for k in range(3)]
    assert all(i.n <= 256 for i in insts)
    ref = oracle_run(insts)
    for k, (got, restores, _) in enumerate(_run_twice(insts, 4, {"streams": 3})):
        compare(got, ref, pos_tol=1e-4, grad_tol=1e-3, label=f"batched store pass {k}")
        if k == 1:
            assert restores == 3 * 30
