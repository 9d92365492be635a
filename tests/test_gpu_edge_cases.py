"""Degenerate inputs and error paths of the device library, through the C ABI.

* A rollout of zero steps (loss of the initial state; the gradient is the
  loss's direct dependence on the design), and a single particle, against the
  FP64 oracle.
* A particle whose stencil lies partly outside the grid: the stencils are
  clamped so every access stays in bounds, and the call reports EDOMAIN.
* A non-finite design value: the call reports a non-finite (or derived domain /
  inversion) error instead of returning numbers.
* backward after a plain (record=0) rollout reports ESTATE.
"""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_2503_22767_amd import mpm_mag as M
from paper_2503_22767_amd import workloads as W

from gpu_util import compare, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu


def _block(dim, steps, kind=W.LOSS_COM_DISP, floor=True, seed=3):
    size = (0.4, 0.2, 0.2) if dim == 2 else (0.3, 0.2, 0.25)
    return W.make_tiny(seed=seed, dim=dim, n_steps=steps, loss_kind=kind, floor=floor, gravity=1.0 if floor else 0.0,
                       size=size, n_grid=16, n_segments=2)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", [W.LOSS_COM_DISP, W.LOSS_FINAL_MSE], ids=["com", "mse"])
def test_zero_steps_matches_oracle(dim, kind):
    inst = _block(dim, 0, kind=kind, floor=kind == W.LOSS_COM_DISP)
    ref = oracle_run([inst])
    got = gpu_run([inst], precision=8)
    # the gradients vanish or nearly so at T = 0 (the centre-of-mass loss is
    # zero whatever the design): compare absolutely
    errs = {k: float(np.max(np.abs(got[k] - ref[k]))) for k in ("x", "loss", "g_density", "g_br", "g_b_prog")}
    log("T=0", dim, kind, {k: f"{v:.2e}" for k, v in errs.items()})
    assert errs["x"] <= 1e-14 and errs["loss"] <= 1e-12, errs
    for k in ("g_density", "g_br", "g_b_prog"):
        assert errs[k] <= 1e-10 * max(1.0, float(np.max(np.abs(ref[k])))), (k, errs)


@pytest.mark.parametrize("dim", [2, 3])
def test_single_particle_matches_oracle(dim):
    inst = _block(dim, 12)
    one = W.Instance(dict(inst.params), inst.x0[:1], inst.density[:1], inst.br[:1], inst.b_prog,
                     inst.target[:1] if inst.target is not None else None, None)
    ref = oracle_run([one])
    got = gpu_run([one], precision=8)
    compare(got, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label=f"N=1 d{dim}")
    got = gpu_run([one], precision=4)
    compare(got, ref, pos_tol=1e-4, grad_tol=1e-3, label=f"N=1 d{dim} fp32")


def _status_of(fn):
    try:
        fn()
    except M.MpmMagError as e:
        return e.status
    return M.OK


def test_grid_threads_and_parts_options_are_validated():
    inst = _block(3, 4, floor=False)
    sim = M.MpmMag([inst.params], [len(inst.x0)], precision=4)
    try:
        for bad in (128, 300, 1088, -1):
            assert _status_of(lambda: sim.set_option("grid_threads", bad)) == M.EINVAL, bad
        for good in (0, 256, 384, 512, 1024):
            sim.set_option("grid_threads", good)
        for bad in (3, 5, 16, -1):
            assert _status_of(lambda: sim.set_option("grid_parts", bad)) == M.EINVAL, bad
        for good in (0, 1, 2, 4, 8):
            sim.set_option("grid_parts", good)
    finally:
        sim.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_particle_outside_the_grid_reports_edomain(dim):
    inst = _block(dim, 4, floor=False)
    x0 = inst.x0.copy()
    x0[0, 0] = 0.004   # base cell -1 at 16 nodes per axis: the stencil leaves the grid
    bad = W.Instance(dict(inst.params), x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask)
    for prec in (8, 4):
        st = _status_of(lambda: gpu_run([bad], precision=prec, backward=False))
        log("outside grid", dim, prec, st)
        assert st == M.EDOMAIN, st


@pytest.mark.parametrize("what", ["density", "br", "b_prog", "x0"])
def test_nonfinite_input_reports_enonfinite(what):
    """The rollout checks its inputs as it takes them: a NaN design value,
    remanence, field value or position is ENONFINITE, in both precisions."""
    inst = _block(3, 4, floor=False)
    arrs = dict(x0=inst.x0.copy(), density=inst.density.copy(), br=inst.br.copy(), b_prog=inst.b_prog.copy())
    a = arrs[what]
    a.reshape(-1)[min(5, a.size - 1)] = np.nan
    bad = W.Instance(dict(inst.params), arrs["x0"], arrs["density"], arrs["br"], arrs["b_prog"], inst.target,
                     inst.mask)
    for prec in (8, 4):
        st = _status_of(lambda: gpu_run([bad], precision=prec, backward=False))
        log("nan", what, prec, st)
        assert st == M.ENONFINITE, st


@pytest.mark.parametrize("dim", [2, 3])
def test_inverted_deformation_reports_einvert(dim):
    """A field three orders of magnitude beyond the workloads' drives the
    magnetic stress of Eq. 7 so hard that det F drops below zero within two
    steps: EINVERT, as the oracle reports for the same input."""
    inst = W.make_tiny(seed=7, dim=dim, n_steps=2, n_grid=32, size=(0.2, 0.15, 0.15), corner=[0.4, 0.4, 0.4][:dim],
                       n_segments=1)
    prog = np.zeros((1, dim))
    prog[0, 0] = 3e3
    bad = W.Instance(dict(inst.params), inst.x0, inst.density, inst.br, prog, inst.target, inst.mask)
    with pytest.raises(orc.OracleError) as e:
        orc.rollout(bad.params, bad.x0, bad.density, bad.br, bad.b_prog, bad.target, bad.mask)
    assert e.value.code == orc.EINVERT
    for prec in (8, 4):
        st = _status_of(lambda: gpu_run([bad], precision=prec, backward=False))
        log("huge field", dim, prec, st)
        assert st == M.EINVERT, st


def test_backward_needs_a_recorded_rollout():
    inst = _block(2, 4)
    sim = M.MpmMag([inst.params], [inst.n], precision=8)
    try:
        tens = M.instance_tensors([inst], dtype=torch.float64)
        sim.rollout(*tens, record=False)
        st = _status_of(lambda: sim.backward(torch.ones(1, dtype=torch.float64, device="cuda")))
        assert st == M.ESTATE, st
        # a recorded rollout then makes it work, and the handle stays usable
        sim.rollout(*tens, record=True)
        g = sim.backward(torch.ones(1, dtype=torch.float64, device="cuda"))
        assert all(torch.isfinite(x).all() for x in g)
    finally:
        sim.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_scatter_fallback_counts(dim):
    """The scatter's fallback counters: none on a compact block with the
    default staging box; per-wave boxes when the block box is capped below the
    block's stencils; every live wave on global atomics without LDS staging.
    The results of the three settings agree with each other to rounding."""
    # a block whose stencil box exceeds the smallest box cap (64 nodes)
    size, n_grid = ((0.4, 0.3), 32) if dim == 2 else ((0.3, 0.2, 0.25), 16)
    inst = W.make_tiny(seed=3, dim=dim, n_steps=6, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0, size=size,
                       n_grid=n_grid, n_segments=2)
    tens = M.instance_tensors([inst], dtype=torch.float64)
    xs, counts = {}, {}
    for name, opts in (("default", {}), ("box_cap", {"box_cap": 64}), ("no_lds", {"p2g_lds": 0})):
        sim = M.MpmMag([inst.params], [inst.n], precision=8)
        try:
            for k, v in opts.items():
                sim.set_option(k, v)
            _, x = sim.rollout(*tens, record=True)
            counts[name] = sim.scatter_stats()
            xs[name] = x.cpu().numpy()
            sim.backward(torch.ones(1, dtype=torch.float64, device="cuda"))
            counts[name + " backward"] = sim.scatter_stats()
        finally:
            sim.close()
    log("scatter fallbacks", dim, counts)
    waves = -(-inst.n // 64)   # live waves of one scatter launch
    assert counts["default"] == {"wave_boxes": 0, "atomic_waves": 0, "list_overflows": 0}
    assert counts["box_cap"]["wave_boxes"] > 0 and counts["box_cap"]["atomic_waves"] == 0
    assert counts["box_cap backward"]["wave_boxes"] > 0
    # one forward scatter per step: T steps of the rollout, all waves on atomics
    assert counts["no_lds"]["atomic_waves"] == inst.params["n_steps"] * waves, counts["no_lds"]
    assert counts["no_lds"]["wave_boxes"] == 0
    for name in ("box_cap", "no_lds"):
        assert np.max(np.abs(xs[name] - xs["default"])) <= 1e-12


def _two_blobs(dim, n_steps=16, seed=9):
    """One chunk (128 particles) made of two small blobs in opposite corners
    of the grid (16 nodes per axis in 3D, 64 in 2D): its box of stencil base
    cells (14^3, 62^2) exceeds the lane sort's table, its staging box exceeds
    the block box, and its waves span both blobs, so the per-wave boxes and
    the global-atomic fallback of the scatter are taken."""
    rng = np.random.default_rng(seed)
    n_grid = 16 if dim == 3 else 64
    dx = 1.0 / n_grid
    h = dx / 2
    side = 2 * dx if dim == 3 else 4 * dx
    lo = [0.55 * dx] * dim                              # base cell 0
    hi = [(n_grid - 2.45) * dx - side + dx] * dim       # base cells up to n - 3
    x0 = np.concatenate([W.box_particles(lo, [side] * dim, h), W.box_particles(hi, [side] * dim, h)])
    n = x0.shape[0]
    p = W.default_params(dim, n_grid, 1e-3, n_steps, h)
    p["n_segments"] = 2
    p["seg_steps"] = (n_steps + 1) // 2
    p["loss_kind"] = W.LOSS_FINAL_MSE
    density = rng.uniform(0.3, 1.0, size=n)
    br = W._unit_vectors(rng, n, dim)
    b_prog = rng.uniform(-0.3, 0.3, size=(2, dim))
    target = x0 + rng.uniform(-0.01, 0.01, size=x0.shape)
    return W.Instance(p, x0, density, br, b_prog, target, None)


@pytest.mark.parametrize("dim", [2, 3])
def test_chunk_spanning_distant_blobs_matches_oracle(dim):
    inst = _two_blobs(dim)
    log("two blobs", dim, "particles", inst.n)
    assert inst.n <= 256
    ref = oracle_run([inst])
    got = gpu_run([inst], precision=8)
    compare(got, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label=f"two blobs d{dim} fp64")
    got = gpu_run([inst], precision=4)
    compare(got, ref, pos_tol=1e-4, grad_tol=1e-3, label=f"two blobs d{dim} fp32")


def test_kernel_timing_env_var_prints_the_table(monkeypatch, capfd):
    """MPM_MAG_KERNEL_TIMING=1 times every launch and prints the per-kernel
    table when the handle closes."""
    import torch
    from paper_2503_22767_amd import mpm_mag as M
    monkeypatch.setenv("MPM_MAG_KERNEL_TIMING", "1")
    inst = W.make_tiny(seed=3, dim=2, n_steps=6, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0,
                       size=(0.4, 0.2, 0.2), n_grid=16)
    sim = M.MpmMag([inst.params], [inst.n], precision=8)
    x0, density, br, b_prog, target, mask = M.instance_tensors([inst], dtype=torch.float64)
    sim.rollout(x0, density, br, b_prog, target, mask, record=True)
    sim.backward(torch.ones(1, dtype=torch.float64, device="cuda"))
    sim.close()
    err = capfd.readouterr().err
    rows = {line.split()[0]: line.split() for line in err.splitlines() if line.strip()}
    assert "kernel" in rows and "grid_update" in rows and "p2g_g2p_adj" in rows
    # 6 forward steps; the reverse sweep restores the stored grids instead: two
    # segments of 3 steps, each restored for its recompute (3) and before the
    # transpose of its first step (the ring holds the last two)
    assert int(rows["grid_update"][1]) == 6 and float(rows["grid_update"][3]) > 0.0
    assert int(rows["grid_restore"][1]) == 2 * (3 + 1)


def _crowded_coarse_block(n_steps=4, seed=12):
    """75,625 particles (25 per cell and axis) inside one 16 x 16 coarse block of
    a 32-node 2D grid: 296 chunk boxes register with that block, more than its
    list of 256 holds, so the last ones add their staged values to the dense
    fallback accumulator, in the forward scatter and in the transposed one."""
    rng = np.random.default_rng(seed)
    n_grid = 32
    dx = 1.0 / n_grid
    h = dx / 25
    x0 = W.box_particles([18.2 * dx, 18.2 * dx], [11 * dx, 11 * dx], h)
    n = x0.shape[0]
    p = W.default_params(2, n_grid, 1e-3, n_steps, h)
    p["loss_kind"] = W.LOSS_FINAL_MSE
    density = rng.uniform(0.3, 1.0, size=n)
    br = W._unit_vectors(rng, n, 2)
    b_prog = rng.uniform(-0.3, 0.3, size=(1, 2))
    target = x0 + rng.uniform(-0.01, 0.01, size=x0.shape)
    return W.Instance(p, x0, density, br, b_prog, target, None)


def test_coarse_block_list_overflow_matches_oracle():
    inst = _crowded_coarse_block()
    base = np.floor(inst.x0 / (1.0 / 32) - 0.5).astype(int)
    # every stencil (base .. base + 2) lies in coarse block (1, 1): nodes 16 .. 31
    assert base.min() >= 16 and base.max() + 2 <= 31
    n_chunks = (inst.n + 255) // 256
    log("crowded coarse block", inst.n, "particles", n_chunks, "chunk boxes")
    assert n_chunks > 256
    ref = oracle_run([inst])
    got = gpu_run([inst], precision=8)
    compare(got, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label="crowded block fp64")
    got = gpu_run([inst], precision=4)
    compare(got, ref, pos_tol=1e-4, grad_tol=1e-3, label="crowded block fp32")


def _grid_limit_instance(dim, n_grid, cells, far, steps, seed=11):
    """A block of cells[k] cells per axis (2 particles per cell and axis) three
    cells from the grid's low faces, or eight cells from its high faces, in a
    grid of n_grid nodes per axis with walls one cell thick. The same seed gives
    the same design, program and target offsets in both places."""
    dx = 1.0 / n_grid
    h = dx / 2
    lo = n_grid - 8 - cells[0] if far else 3
    corner = [lo * dx + 0.3 * h, lo * dx + 0.7 * h, lo * dx + 0.45 * h][:dim]
    inst = W.make_tiny(seed=seed, dim=dim, n_grid=n_grid, n_steps=steps, size=[c * dx for c in cells][:dim],
                       corner=corner, dt=1e-4 if n_grid > 64 else 1e-3, loss_kind=W.LOSS_FINAL_MSE, n_segments=2)
    inst.params["wall_cells"] = 1
    return inst


@pytest.mark.parametrize("dim", [2, 3])
def test_smallest_grid_matches_oracle(dim):
    """n_grid = 8, the smallest grid the library accepts (one coarse block in 3D)."""
    inst = _grid_limit_instance(dim, 8, (2, 2, 2), False, 30)
    ref = oracle_run([inst])
    compare(gpu_run([inst], precision=8), ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label=f"n_grid 8 d{dim}")
    compare(gpu_run([inst], precision=4), ref, pos_tol=1e-4, grad_tol=1e-3, label=f"n_grid 8 d{dim} fp32")


@pytest.mark.parametrize("far", [False, True], ids=["low_faces", "high_faces"])
def test_largest_grid_2d_matches_oracle(far):
    """n_grid = 1024, the largest grid, with the block near the low or the high
    faces (node indices up to about 2^20)."""
    inst = _grid_limit_instance(2, 1024, (12, 6), far, 30)
    ref = oracle_run([inst])
    compare(gpu_run([inst], precision=8), ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9,
            label=f"n_grid 1024 d2 far={far}")
    compare(gpu_run([inst], precision=4), ref, pos_tol=1e-4, grad_tol=1e-3, label=f"n_grid 1024 d2 far={far} fp32")


def test_largest_grid_3d_is_translation_invariant():
    """n_grid = 1024 in 3D: 2^30 nodes, about 140 GB of device grids in FP32 for
    a recorded rollout and its adjoint. The oracle cannot hold such a grid, so
    this checks a property instead: the same block moved by whole cells from
    the low faces to the high ones (node indices near 2^30, value offsets past
    2^32) moves, loses and differentiates the same. The two runs order and
    chunk their particles differently along the Hilbert curve, so they agree to
    rounding, not bit for bit."""
    near = _grid_limit_instance(3, 1024, (8, 6, 6), False, 20)
    far = _grid_limit_instance(3, 1024, (8, 6, 6), True, 20)
    shift = far.x0 - near.x0
    assert np.allclose(shift, shift[0]) and np.allclose(far.target - far.x0, near.target - near.x0, atol=1e-12)
    a = gpu_run([near], precision=4)
    log("n_grid 1024 d3: low faces done")
    b = gpu_run([far], precision=4)
    du_a, du_b = a["x"] - near.x0, b["x"] - far.x0
    scale = float(np.max(np.abs(du_a)))
    ex = float(np.max(np.abs(du_a - du_b)))
    errs = {k: float(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(a[k])) for k in ("g_density", "g_br", "g_b_prog")}
    el = float(abs(a["loss"][0] - b["loss"][0]) / abs(a["loss"][0]))
    log("n_grid 1024 d3 translation: max displacement", f"{scale:.3e}", "difference", f"{ex:.2e}", "loss", f"{el:.2e}",
        {k: f"{v:.2e}" for k, v in errs.items()})
    # x_final comes back as FP32 positions near 1.0 on the far side, whose ulp
    # (6e-8) quantizes the displacement taken from them: allow 4 such ulps
    assert scale > 0 and ex <= 1e-3 * scale + 4 * 2.0 ** -24, (ex, scale)
    assert el <= 1e-4, el
    for k, v in errs.items():
        assert v <= 1e-3, (k, errs)


def test_most_instances_per_handle_match_oracle():
    """4096 instances in one handle, the most it accepts (each a 2D block of 16
    particles with its own design and program, on its own 8^2 grid), advanced
    as instance groups on streams; an evenly spread sample of them, the first
    and the last included, against the oracle in FP64."""
    n_inst = 4096
    insts = [_grid_limit_instance(2, 8, (2, 2), False, 10, seed=1000 + k) for k in range(n_inst)]
    got = gpu_run(insts, precision=8)
    pick = sorted(set(range(0, n_inst, 97)) | {1, n_inst - 1})
    ref = oracle_run([insts[k] for k in pick])
    p_off = np.concatenate([[0], np.cumsum([i.n for i in insts])])
    s_off = np.concatenate([[0], np.cumsum([i.params["n_segments"] for i in insts])])
    part = np.concatenate([np.arange(p_off[k], p_off[k + 1]) for k in pick])
    segs = np.concatenate([np.arange(s_off[k], s_off[k + 1]) for k in pick])
    sub = dict(x=got["x"][part], loss=got["loss"][pick], g_density=got["g_density"][part], g_br=got["g_br"][part],
               g_b_prog=got["g_b_prog"][segs])
    compare(sub, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label=f"{n_inst} instances, {len(pick)} sampled")
