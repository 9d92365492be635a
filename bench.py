"""Throughput of the magneto-elastic MPM rollout + adjoint on one MI355X.

One bench step = one pass of the whole hot path over the workload: cell sort,
the recorded forward rollout (P2G, grid operation with contact, G2P, step
checkpoints), the losses, and the reverse sweep (segment recompute and the
transposed G2P, grid and P2G kernels) down to d(loss)/d(density, remanence,
field program). Inputs are resident in HBM before the timed region.

Prints one JSON line. Besides the contract fields it carries the plain-forward
rate, the adjoint/forward cost ratio, the dominant kernel's roofline fraction
(algorithmic FLOPs or bytes per launch over the average launch time measured
with HIP events on the library's stream), the device memory the handle holds,
and the FP64 CPU oracle timed on a bounded sample of the same workload (on all
host cores, and on one), whose gradient is also compared with the device's on
that sample. The recorded rollout runs within a checkpoint budget (64 GB by
default): checkpoints, segment stash, grid ring and grid stores together; the
rate of the same handle without a bound is reported beside it.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2503_22767_amd import mpm_mag as M  # noqa: E402
from paper_2503_22767_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s fwd+adjoint vs plain fwd; grad rel err vs FP64 oracle"

# particle-steps the oracle samples cover, per workload: (instances, steps) on
# all host cores (also the gradient check: for the quadruped one whole
# checkpoint segment of task 0), and (instances, steps) on one core
CPU_SAMPLE = {"cantilever2d": (1, 500), "walker2d": (1, 400), "plate3d": (1, 300), "batch2d": (4, 200),
              "quadruped3d": (1, 64)}
CPU_SAMPLE_1CORE = {"cantilever2d": (1, 500), "walker2d": (1, 100), "plate3d": (1, 60), "batch2d": (2, 60),
                    "quadruped3d": (1, 6)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_sim(wl, options=None):
    sim = M.MpmMag([i.params for i in wl.instances], [i.n for i in wl.instances], precision=wl.precision)
    for k, v in (options or {}).items():
        sim.set_option(k, v)
    dtype = torch.float32 if wl.precision == 4 else torch.float64
    tens = M.instance_tensors(wl.instances, dtype=dtype)
    return sim, tens, dtype


def shared_design(wl):
    """Instances of one group share density and remanence (Eq. 35); in the flat
    ABI their arrays are repeated, which the caller's chain rule sums."""
    return len({i.group for i in wl.instances}) < len(wl.instances)


def run_step(sim, tens, dloss, record=True, backward=True):
    x0, density, br, b_prog, target, mask = tens
    loss, _ = sim.rollout(x0, density, br, b_prog, target, mask, record=record, want_x=False)
    if backward:
        sim.backward(dloss)
    return loss


def timed(fn, n):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / n


# Peaks of one MI355X. HBM3E 8 TB/s. Vector ALU: 256 CUs x 4 SIMDs x 16 lanes
# x 2 FLOP (FMA) x 2.4 GHz = 78.6 TFLOP/s for unpacked FP32 and for FP64; the
# 157.3 TFLOP/s FP32 figure counts packed two-wide FP32 instructions, which this
# build does not emit.
ALU_PEAK_TFLOPS = {4: 78.6, 8: 78.6}
ALU_PEAK_PACKED_TFLOPS = {4: 157.3, 8: 78.6}

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE, then
# WRITE_SIZE, on the quadruped workload, scaled by what the counters read for a
# device-to-device copy of 1 GiB (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0). Valid
# only for that workload and for the kernel code they were taken on (hash of
# csrc/device.hpp and csrc/kernels.hpp, comments left out); other workloads
# report null.
TRAFFIC = {
    "quadruped3d": {
        # (530089.6 KiB fetched x 2.0 + 257609.8 KiB written) x 1024, mean of 5 launches
        "p2g_g2p_adj": 1349415974,
        # (142473.6 x 2.0 + 221035.4) x 1024, mean of 21 launches (plain and recorded steps)
        "g2p_p2g": 518126120,
    },
}
TRAFFIC_SRC_HASH = "74cbf943f8aa8c1f"


def code_text(src):
    """C++ source without its comments and with whitespace collapsed, so that
    an edit of a comment does not count as a change of the code."""
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def csrc_hash():
    """Hash of the device kernels' code (the particle and grid kernels and
    their device helpers, comments left out; host-side launch code is not part
    of it)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2503_22767_amd", "csrc")
    for f in ("device.hpp", "kernels.hpp"):
        h.update(f.encode())
        h.update(code_text(open(os.path.join(d, f)).read()).encode())
    return h.hexdigest()[:16]


def roofline(sim, tens, dloss, precision, streams=0, workload=""):
    """One extra instrumented pass with per-launch HIP events on the library's
    stream. The dominant kernel (largest total time) is placed on the roofline
    by its arithmetic intensity against the ridge of the ALU and HBM peaks."""
    # one stream, so that launches do not overlap and each launch's time is
    # its own (the timed passes may run instance groups on several streams)
    sim.set_option("streams", 1)
    sim.set_option("kernel_timing", 1)
    sim.kernel_stats(reset=True)
    run_step(sim, tens, dloss)
    torch.cuda.synchronize()
    stats = sim.kernel_stats(reset=True)
    sim.set_option("kernel_timing", 0)
    sim.set_option("streams", streams)
    timed_k = {k: v for k, v in stats.items() if v["launches"] and (v["bytes"] > 0 or v["flops"] > 0)}
    dom = max(timed_k, key=lambda k: timed_k[k]["ms"])
    s = timed_k[dom]
    avg_s = s["ms"] / s["launches"] * 1e-3
    bpl = s["bytes"] / s["launches"]
    fpl = s["flops"] / s["launches"]
    alu_peak = ALU_PEAK_TFLOPS[precision]
    ridge = alu_peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    intensity = fpl / bpl if bpl > 0 else float("inf")
    gbs = bpl / avg_s / 1e9
    tflops = fpl / avg_s / 1e12
    traffic = None
    if dom in TRAFFIC.get(workload, {}) and TRAFFIC_SRC_HASH == csrc_hash():
        traffic = TRAFFIC[workload][dom]
    if intensity > ridge:
        rl = dict(bound="alu", achieved=round(tflops, 2), peak=alu_peak, unit="TFLOP/s",
                  frac=round(tflops / alu_peak, 4), traffic=traffic,
                  peak_packed_fp32=ALU_PEAK_PACKED_TFLOPS[precision],
                  frac_vs_packed=round(tflops / ALU_PEAK_PACKED_TFLOPS[precision], 4))
    else:
        rl = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                  frac=round(gbs / HBM_PEAK_GBS, 4), traffic=traffic)
    rl.update(kernel=dom, avg_launch_us=round(avg_s * 1e6, 2), timed_on_one_stream=True, flops_per_launch=fpl,
              bytes_per_launch=int(bpl),
              intensity_flop_per_byte=round(intensity, 2), ridge_flop_per_byte=round(ridge, 2),
              hbm_gbs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
    per_kernel = {}
    for k, v in stats.items():
        if not v["launches"]:
            continue
        t = v["ms"] / v["launches"] * 1e-3
        if t <= 0.0:   # counted but not timed (the checkpoint copies are runtime copies)
            per_kernel[k] = dict(launches=v["launches"], avg_us=None, total_ms=None, gbs=None, tflops=None)
            continue
        per_kernel[k] = dict(launches=v["launches"], avg_us=t * 1e6, total_ms=v["ms"],
                             gbs=(v["bytes"] / v["launches"]) / t / 1e9 if v["bytes"] else None,
                             tflops=(v["flops"] / v["launches"]) / t / 1e12 if v["flops"] else None)
    return rl, per_kernel


def separate(wl, opts, reps=2):
    """Forward + adjoint of every instance through a handle of its own, run
    one after another; returns seconds per pass over all instances."""
    runs = []
    for inst in wl.instances:
        one = W.Workload(wl.name, [inst], wl.precision)
        sim, tens, dtype = make_sim(one, opts)
        runs.append((sim, tens, torch.ones(1, dtype=dtype, device="cuda")))
    for sim, tens, dl in runs:
        run_step(sim, tens, dl)
    t = timed(lambda: [run_step(sim, tens, dl) for sim, tens, dl in runs], reps)
    for sim, _, _ in runs:
        sim.close()
    return t


def _oracle_sample(wl_name, wl, sample, threads):
    """FP64 oracle forward + checkpointed adjoint on the first instances and
    steps of the workload, on `threads` host threads (0: all)."""
    import oracle as orc
    n_inst, steps = sample
    insts = []
    for inst in wl.instances[:n_inst]:
        p = dict(inst.params)
        p["n_steps"] = steps
        insts.append(W.Instance(p, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask, inst.group))
    ps = sum(i.n * steps for i in insts)
    orc.set_threads(threads)
    cores = orc.get_threads()
    try:
        t0 = time.perf_counter()
        grads = []
        for inst in insts:
            g = orc.backward(inst.params, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask,
                             ckpt_every=max(1, int(math.isqrt(steps))))
            grads.append(g)
        dt = time.perf_counter() - t0
    finally:
        orc.set_threads(0)
    rec = dict(value=round(ps / dt, 1), unit="particle-steps/s fwd+adjoint", cores=cores, kind="oracle",
               sample=f"{wl_name}: first {n_inst} instance(s), first {steps} steps, {ps} particle-steps, "
                      f"FP64 forward + checkpointed adjoint, {dt:.1f} s on {cores} thread(s)")
    return rec, insts, grads


def cpu_baseline(wl_name, wl):
    """The FP64 oracle on all host cores (the baseline record; its sample also
    serves the gradient check) and on one core (reported beside it)."""
    rec, insts, grads = _oracle_sample(wl_name, wl, CPU_SAMPLE[wl_name], 0)
    one, _, _ = _oracle_sample(wl_name, wl, CPU_SAMPLE_1CORE[wl_name], 1)
    rec["one_core"] = dict(value=one["value"], cores=1, sample=one["sample"])
    rec["host_cpus"] = os.cpu_count()
    return rec, insts, grads


def grad_error(wl, insts, oracle_grads):
    """Device gradient on the oracle's sample vs the oracle (norm-wise
    relative): against the oracle deciding its own branches of the grid
    operation, and against the oracle replaying the device's (the decisions
    the FP32 run takes differently near ties are counted)."""
    import oracle as orc
    sub = W.Workload(wl.name, insts, wl.precision)
    sim, tens, dtype = make_sim(sub)
    T = insts[0].params["n_steps"]
    trace = torch.zeros(T * sim.trace_nodes(), dtype=torch.int16, device="cuda")
    sim.set_branch_trace(trace)
    dl = torch.ones(len(insts), dtype=dtype, device="cuda")
    sim.rollout(*tens, record=True, want_x=False)
    gd, gb, gp = sim.backward(dl)
    torch.cuda.synchronize()
    full = trace.cpu().numpy().view(np.uint16).reshape(T, -1)
    sim.set_branch_trace(None)
    sim.close()
    got = dict(g_density=gd.double().cpu().numpy().ravel(), g_br=gb.double().cpu().numpy().ravel(),
               g_b_prog=gp.double().cpu().numpy().ravel())
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(1e-300, np.linalg.norm(b)))
    ref = {k: np.concatenate([g[k].ravel() for g in oracle_grads]) for k in got}
    out = dict(own_branches={k: rel(got[k], ref[k]) for k in got})
    # the oracle on the device's branches, and the oracle's own decisions
    reps, flips, off = [], 0, 0
    for inst in insts:
        n = inst.params["n_grid"] ** inst.params["dim"]
        tab = np.ascontiguousarray(full[:, off:off + n])
        off += n
        with orc.branch_trace(inst.params, record=True) as own:
            orc.rollout(inst.params, inst.x0, inst.density, inst.br, inst.b_prog, inst.target, inst.mask)
        flips += int(np.count_nonzero(own != tab))
        with orc.branch_trace(inst.params, replay=tab):
            reps.append(orc.backward(inst.params, inst.x0, inst.density, inst.br, inst.b_prog, inst.target,
                                     inst.mask, ckpt_every=max(1, int(math.isqrt(T)))))
    rref = {k: np.concatenate([g[k].ravel() for g in reps]) for k in got}
    out["device_branches"] = {k: rel(got[k], rref[k]) for k in got}
    out["branch_decisions_differing"] = flips
    return out


def front_end(wl, reps=20):
    """The design front end on the particle set of the workload's first
    instance: filter radius 1.5 particle spacings, 8 regions by x slab, the
    handle's precision. Times the neighbour-matrix build once, then forward and
    backward calls with events on the stream they run on, and places each on
    the HBM roofline by its algorithmic bytes (the harmonic stimulus of every
    instance over the rollout, a few hundred KB, is timed too; launch latency
    bounds it):
      forward:  matrix (4 B column + weight per entry), row offsets, 1/s, phi,
                region ids, phit, density and br written: nnz (4 + r) + N (8 + 4r + d r)
      backward: u = g H'/s (read g, phit, 1/s; write u), the matrix again with u
                and g_phi, and the region sums (sorted ids and members, g_br):
                nnz (4 + r) + N (12 + 6r + d r)."""
    from paper_2503_22767_amd import design as PD
    inst = wl.instances[0]
    d, r = inst.params["dim"], (4 if wl.precision == 4 else 8)
    h = inst.params["particle_volume"] ** (1.0 / d)
    x0 = torch.as_tensor(inst.x0, device="cuda")
    n = len(inst.x0)
    xs = x0[:, 0]
    region = ((xs - xs.min()) / (xs.max() - xs.min()) * 8).clamp(0, 7).to(torch.int32)
    gen = torch.Generator(device="cpu").manual_seed(7)
    dt = torch.float32 if wl.precision == 4 else torch.float64
    rnd = lambda *shape: torch.rand(*shape, generator=gen, dtype=torch.float64).to(device="cuda", dtype=dt)
    phi, mag, zeta = rnd(n), rnd(8), rnd(8, d) * 2 - 1
    gd, gb = rnd(n) - 0.5, rnd(n, d) - 0.5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fe = PD.MpmMagDesign(x0, 1.5 * h, region=region, n_regions=8, precision=wl.precision)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    try:
        def ev_time(fn):
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) * 1e3 / reps   # us per call
        f_us = ev_time(lambda: fe.forward(phi, mag, zeta, 8.0, 1.0, 1e-6))
        b_us = ev_time(lambda: fe.backward(gd, gb))
        nnz = fe.nnz
        # harmonic stimulus of every instance over the rollout (one program row per step)
        ni, T = len(wl.instances), wl.n_steps
        hb, hf, he = rnd(ni), rnd(ni), rnd(ni, d) * 2 - 1
        hg = rnd(ni * T, d) - 0.5
        dt_s = inst.params["dt"]
        hargs = (T, dt_s, 0.5, 1.0, 50.0, 1e-6)
        hp_us = ev_time(lambda: PD.harmonic_program(hb, hf, he, *hargs))
        hb_us = ev_time(lambda: PD.harmonic_backward(hb, hf, he, *hargs, hg))
    finally:
        fe.close()
    fb = nnz * (4 + r) + n * (8 + 4 * r + d * r)
    bb = nnz * (4 + r) + n * (12 + 6 * r + d * r)
    out = dict(particles=n, nnz=nnz, radius_spacings=1.5, regions=8, build_ms=round(build_ms, 2),
               forward_us=round(f_us, 2), backward_us=round(b_us, 2), bytes_forward=fb, bytes_backward=bb,
               bound="hbm", peak_gbs=HBM_PEAK_GBS,
               forward_gbs=round(fb / f_us / 1e3, 1), backward_gbs=round(bb / b_us / 1e3, 1),
               harmonic=dict(instances=ni, steps=T, program_us=round(hp_us, 2), backward_us=round(hb_us, 2),
                             bound="latency"))
    out["forward_frac"] = round(out["forward_gbs"] / HBM_PEAK_GBS, 4)
    out["backward_frac"] = round(out["backward_gbs"] / HBM_PEAK_GBS, 4)
    return out


def obstacles(wl):
    """A plain forward of the workload, one stream, kernel timing on, with two
    obstacles added to every instance (a sphere whose top is one cell below
    the front of the body and a tilted half-space moving towards it) and
    without: the grid update's time per launch, and the forward's."""
    import dataclasses
    out = {}
    for label in ("without", "with"):
        insts = []
        for i in wl.instances:
            p = dict(i.params)
            if label == "with":
                lo, hi = i.x0.min(0), i.x0.max(0)
                d = p["dim"]
                z = lambda v: list(v) + [0.0] * (3 - len(v))
                mid = (lo + hi) / 2
                p["obstacles"] = [
                    dict(kind=M.OBSTACLE_SPHERE, a=z([hi[0] - 0.05, lo[1] - 0.1 - 1.0 / p["n_grid"]] + list(mid[2:d])),
                         b=[0.1, 0, 0], mu=0.5),
                    dict(kind=M.OBSTACLE_HALFSPACE, a=z([hi[0] + 0.1, 0.0] + [0.0] * (d - 2)),
                         b=z([-1.0, 0.3] + [0.0] * (d - 2)), mu=0.3, vel=z([-0.2] + [0.0] * (d - 1)))]
            insts.append(dataclasses.replace(i, params=p))
        w2 = dataclasses.replace(wl, instances=insts)
        sim, tens, dtype = make_sim(w2, {"streams": 1, "kernel_timing": 1})
        try:
            dloss = torch.ones(len(insts), dtype=dtype, device="cuda")
            sim.kernel_stats(reset=True)
            t = timed(lambda: run_step(sim, tens, dloss, record=False, backward=False), 1)
            st = sim.kernel_stats()["grid_update"]
        finally:
            sim.close()
        out[label] = dict(grid_update_us=round(st["ms"] / st["launches"] * 1e3, 2), fwd_ms=round(t * 1e3, 1))
    out["obstacles_per_instance"] = 2
    return out


def codesign(wl, iters=2):
    """Co-design iterations (Sec. 3.2) over the workload's tasks sharing one
    design: every task driven by its own harmonic stimulus (one program row per
    step), 8 regions by x slab, filter radius 1.5 spacings. One warm-up
    iteration (it sizes the checkpoints and the grid store), then `iters` timed
    ones, host clock around each (an iteration ends by reading its losses)."""
    from paper_2503_22767_amd import codesign as CD
    insts = wl.instances
    x0 = insts[0].x0
    if not all(np.array_equal(i.x0, x0) for i in insts):
        return None
    params = []
    for i in insts:
        p = dict(i.params)
        p.update(n_segments=wl.n_steps, seg_steps=1, periodic=0)
        params.append(p)
    n, d = len(x0), insts[0].params["dim"]
    h = insts[0].params["particle_volume"] ** (1.0 / d)
    T, dt = wl.n_steps, insts[0].params["dt"]
    region = np.clip(((x0[:, 0] - x0[:, 0].min()) / np.ptp(x0[:, 0]) * 8).astype(np.int32), 0, 7)
    cfg = CD.CoDesignConfig(radius=1.5 * h, b_max=0.5, f_min=2.0 / (T * dt), f_max=20.0 / (T * dt), lr=0.01)
    cd = CD.CoDesign(params, x0, cfg, region=region, n_regions=8,
                     targets=[i.target if i.target is not None else i.x0 for i in insts],
                     masks=[i.mask if i.mask is not None else np.ones(n, np.uint8) for i in insts],
                     precision=wl.precision, seed=3)
    try:
        cd.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            cd.step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / iters
        hist = [float(f"{v:.6g}") for v in cd.history]
    finally:
        cd.close()
    return dict(tasks=len(insts), particles_per_task=n, steps=T, regions=8, timed_iterations=iters,
                ms_per_iteration=round(ms, 1), loss_history=hist)


def codesign_to_convergence(wl, max_iters, topology=False, mass_eps=1e-3):
    """The workload's tasks co-designed until the paper's convergence rule
    holds (or max_iters): magnetization magnitudes and orientations of 8
    regions and each task's harmonic stimulus, from a solid design (density 1).
    Without topology the density stays at 1, as in the paper's 3D cases (Sec.
    4.3); with it the per-particle topology is optimized too, under the beta
    continuation, with void particles' mass floored at mass_eps, and the rule
    is taken over the iterations at the capped sharpness. Host clock around
    the iterations."""
    from paper_2503_22767_amd import codesign as CD
    insts = wl.instances
    x0 = insts[0].x0
    if not all(np.array_equal(i.x0, x0) for i in insts):
        return None
    params = []
    for i in insts:
        p = dict(i.params)
        p.update(n_segments=wl.n_steps, seg_steps=1, periodic=0)
        if topology:
            p.update(mass_eps=mass_eps)
        params.append(p)
    n, d = len(x0), insts[0].params["dim"]
    h = insts[0].params["particle_volume"] ** (1.0 / d)
    T, dt = wl.n_steps, insts[0].params["dt"]
    region = np.clip(((x0[:, 0] - x0[:, 0].min()) / np.ptp(x0[:, 0]) * 8).astype(np.int32), 0, 7)
    cfg = CD.CoDesignConfig(radius=1.5 * h, b_max=0.5, f_min=2.0 / (T * dt), f_max=20.0 / (T * dt), lr=0.01,
                            bounds=CD.Bounds() if topology else CD.Bounds(phi=(1.0, 1.0)))
    cd = CD.CoDesign(params, x0, cfg, region=region, n_regions=8,
                     targets=[i.target if i.target is not None else i.x0 for i in insts],
                     masks=[i.mask if i.mask is not None else np.ones(n, np.uint8) for i in insts],
                     precision=wl.precision, seed=3, init={"phi": np.ones(n)})
    err = None
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while cd.iteration < max_iters and not cd.converged(at_final_beta=topology):
            try:
                cd.step()
            except M.MpmMagError as e:
                err = f"iteration {cd.iteration}: {e}"
                break
            if cd.iteration % 10 == 0:
                log(f"[bench] co-design to convergence, iteration {cd.iteration}, beta {cd.beta:g}, "
                    f"loss {cd.history[-1]:.6g}, "
                    f"{(time.perf_counter() - t0) / cd.iteration:.2f} s per iteration")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        conv = cd.converged(at_final_beta=topology)
    finally:
        cd.close()
    hist = cd.history
    return dict(tasks=len(insts), particles_per_task=n, steps=T, regions=8,
                topology=f"optimized from solid, mass floor {mass_eps}" if topology else "held solid",
                iterations=len(hist), converged=conv, s_per_iteration=round(el / max(1, len(hist)), 3),
                loss_first=hist[0] if hist else None, loss_last=hist[-1] if hist else None, error=err,
                loss_every_10=[float(f"{v:.5g}") for v in hist[::10]])


def long_horizon(n_steps=100000):
    """The 2D walker (30,593 particles, FP32) over the paper's horizon of its 2D
    crawlers and walkers, 10^5 steps (Sec. 4.2): one recorded rollout and its
    adjoint (host clock), with the scatter fallbacks over the whole rollout.
    Particles are sorted into chunks once per rollout, so this shows whether
    the chunks' boxes stay compact as the body moves."""
    inst = W.make_walker2d(n_steps=n_steps).instances[0]
    sim = M.MpmMag([inst.params], [inst.n], precision=4)
    try:
        x0, density, br, b_prog, target, mask = M.instance_tensors([inst], dtype=torch.float32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss, x = sim.rollout(x0, density, br, b_prog, target, mask, record=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fwd = sim.scatter_stats()
        gd, gb, gp = sim.backward(torch.ones(1, device="cuda"))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        bwd = sim.scatter_stats()
        finite = bool(torch.isfinite(gd).all() and torch.isfinite(gb).all() and torch.isfinite(gp).all())
        shift = (x.double().mean(0).cpu().numpy() - inst.x0.mean(0)) * inst.params["n_grid"]
    finally:
        sim.close()
    ps = inst.n * n_steps
    return dict(workload="walker2d", particles=inst.n, steps=n_steps, forward_s=round(t1 - t0, 3),
                adjoint_s=round(t2 - t1, 3), fwdadj_value=round(ps / (t2 - t0), 1), unit="particle-steps/s",
                centre_shift_cells=[round(float(v), 2) for v in shift], scatter_fallbacks_forward=fwd,
                scatter_fallbacks_backward=bwd, gradients_finite=finite)


def walker_codesign(max_iters=1000, mass_eps=1e-3, lr=0.01):
    """The co-design loop on the 2D walker (30,593 particles, 2,000 steps,
    floor contact, a harmonic stimulus, 8 magnetization regions by x slab,
    per-particle topology) with void particles' mass floored at mass_eps: beta
    doubles every 10 iterations from 1 to 128, and the loop runs until the
    paper's convergence rule holds over the iterations at beta = 128 (or
    max_iters). Host clock around the iterations; one iteration is front end,
    stimulus, recorded rollout, adjoint, transposes and Adam."""
    from paper_2503_22767_amd import codesign as CD
    inst = W.make_walker2d().instances[0]
    p = dict(inst.params)
    T, dt = p["n_steps"], p["dt"]
    p.update(n_segments=T, seg_steps=1, periodic=0, mass_eps=mass_eps)
    x0 = inst.x0
    h = p["particle_volume"] ** 0.5
    region = np.clip(((x0[:, 0] - x0[:, 0].min()) / np.ptp(x0[:, 0]) * 8).astype(np.int32), 0, 7)
    cfg = CD.CoDesignConfig(radius=1.5 * h, b_max=0.15, f_min=2.0 / (T * dt), f_max=20.0 / (T * dt), br_max=0.5,
                            lr=lr)
    cd = CD.CoDesign([p], x0, cfg, region=region, n_regions=8, precision=4, seed=3)
    out = dict(particles=len(x0), steps=T, regions=8, mass_eps=mass_eps, lr=cfg.lr, b_max=cfg.b_max,
               br_max=cfg.br_max)
    err = None
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while cd.iteration < max_iters:
            try:
                cd.step()
            except M.MpmMagError as e:
                err = f"iteration {cd.iteration} (beta {cd.beta:g}): {e}"
                break
            if cd.converged(at_final_beta=True):
                break
            if cd.iteration % 100 == 0:
                log(f"[bench] walker co-design iteration {cd.iteration}, beta {cd.beta:g}, loss {cd.history[-1]:.4g}, "
                    f"{(time.perf_counter() - t0) / cd.iteration * 1e3:.1f} ms per iteration")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        cd.close()
    hist = cd.history
    out.update(iterations=len(hist), converged=cd.converged(at_final_beta=True), final_beta=cd.betas[-1] if hist else None,
               ms_per_iteration=round(el * 1e3 / max(1, len(hist)), 1), loss_first=hist[0] if hist else None,
               loss_last=hist[-1] if hist else None, error=err,
               loss_every_10=[float(f"{v:.4g}") for v in hist[::10]])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="quadruped3d", choices=sorted(W.WORKLOADS))
    ap.add_argument("--n-steps", type=int, default=0, help="override the rollout length (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--option", action="append", default=[], help="library option key=value")
    ap.add_argument("--autotune", action="store_true",
                    help="pick launch options with the autotuner (cached) before timing")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-sized device buffer (reference kernel for HBM byte counters)")
    ap.add_argument("--no-front-end", action="store_true", help="skip the design front-end leg")
    ap.add_argument("--no-obstacles", action="store_true", help="skip the obstacle leg")
    ap.add_argument("--codesign", type=int, default=2, metavar="K",
                    help="timed co-design iterations after one warm-up (0 skips the leg)")
    ap.add_argument("--front-end-only", action="store_true", help="run only the design front-end leg")
    ap.add_argument("--compare-separate", action="store_true",
                    help="also time one handle per instance (default for the batched workload)")
    ap.add_argument("--budget-gb", type=float, default=64.0,
                    help="checkpoint budget of the recorded rollout in GB (1e9 bytes): checkpoints, segment "
                         "stash, grid ring and grid stores; 0: no bound")
    ap.add_argument("--no-unbounded", action="store_true", help="skip the leg without a checkpoint budget")
    ap.add_argument("--no-walker-codesign", action="store_true",
                    help="skip the walker co-design run through beta = 128 to convergence")
    ap.add_argument("--walker-codesign-only", action="store_true", help="run only the walker co-design leg")
    ap.add_argument("--codesign-converge", type=int, default=0, metavar="MAX",
                    help="also co-design the workload's tasks from a solid design, with the topology held solid "
                         "(the paper's 3D cases), until the convergence rule holds, at most MAX iterations (off by "
                         "default: minutes on the quadruped)")
    ap.add_argument("--codesign-converge-topology", action="store_true",
                    help="with --codesign-converge: optimize the per-particle topology too, from a solid start")
    ap.add_argument("--no-long-horizon", action="store_true",
                    help="skip the walker's rollout and adjoint over 10^5 steps")
    ap.add_argument("--walker-max-iters", type=int, default=1000)
    ap.add_argument("--walker-lr", type=float, default=0.01)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: 3 copies of {args.copy_probe} MiB")
        del src, dst
    kw = {"n_steps": args.n_steps} if args.n_steps else {}
    wl = W.make(args.workload, **kw)
    opts = {}
    for o in args.option:
        k, v = o.split("=")
        opts[k] = int(v)
    log(f"[bench] workload {wl.name}: {wl.description}; {len(wl.instances)} instance(s), "
        f"N={wl.n_particles}, T={wl.n_steps}")
    if args.walker_codesign_only:
        wc = walker_codesign(args.walker_max_iters, lr=args.walker_lr)
        log(f"[bench] walker co-design {wc}")
        print(json.dumps(dict(walker_codesign=wc)), flush=True)
        return
    if args.front_end_only:
        fe = front_end(wl)
        log(f"[bench] front end {fe}")
        print(json.dumps(dict(front_end=fe)), flush=True)
        return
    tuned = None
    if args.autotune:
        from paper_2503_22767_amd import autotune as A
        tuned = A.autotune(wl.instances, wl.precision, log=log)
        log(f"[bench] autotune {tuned['key']}: {tuned['options']} ({'cached' if tuned['cached'] else 'timed'})")
        opts = {**tuned["options"], **opts}
    budget = int(args.budget_gb * 1e9)
    if budget > 0 and "ckpt_budget" not in opts:
        opts["ckpt_budget"] = budget
    sim, tens, dtype = make_sim(wl, opts)
    dloss = torch.ones(len(wl.instances), dtype=dtype, device="cuda")
    base_bytes = sim.device_bytes()
    log(f"[bench] device bytes {base_bytes / 2**30:.2f} GiB (before checkpoints)")
    for w in range(args.warmup):
        run_step(sim, tens, dloss)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    held = sim.device_bytes()
    log(f"[bench] device bytes {held / 2**30:.2f} GiB (with checkpoints and stores; "
        f"{(held - base_bytes) / 1e9:.2f} GB for the reverse sweep, budget {opts.get('ckpt_budget', 0) / 1e9:.1f} GB)")
    t_step = timed(lambda: run_step(sim, tens, dloss), args.steps)
    log(f"[bench] fwd+adj step {t_step * 1e3:.1f} ms")
    scat_bwd = sim.scatter_stats()   # the last call was a backward
    t_fwd = timed(lambda: run_step(sim, tens, dloss, record=False, backward=False), max(1, args.steps))
    log(f"[bench] plain fwd {t_fwd * 1e3:.1f} ms")
    t_rec = timed(lambda: run_step(sim, tens, dloss, record=True, backward=False), 1)
    # scatter fallbacks over the whole recorded rollout, against the block and
    # wave scatters it ran (one P2G per step)
    scat = dict(forward=sim.scatter_stats(), backward=scat_bwd,
                forward_block_scatters=wl.n_steps * sum(-(-int(i.n) // 256) for i in wl.instances),
                forward_wave_scatters=wl.n_steps * sum(-(-int(i.n) // 64) for i in wl.instances))
    log(f"[bench] scatter fallbacks {scat}")
    ps = wl.particle_steps()
    rec = dict(metric=METRIC, value=round(ps / t_step, 1), unit="particle-steps/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(t_step * 1e3, 3),
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32" if wl.precision == 4 else "f64", data="synthetic",
               config=dict(workload=wl.name, description=wl.description, instances=len(wl.instances),
                           particles=wl.n_particles, steps_per_rollout=wl.n_steps,
                           grid=[i.params["n_grid"] for i in wl.instances[:1]][0], parallelism="single-gpu"),
               fwd_value=round(ps / t_fwd, 1), fwd_ms=round(t_fwd * 1e3, 3),
               adj_over_fwd=round((t_step - t_rec) / t_fwd, 3), fwdadj_over_fwd=round(t_step / t_fwd, 3),
               ckpt_budget_bytes=opts.get("ckpt_budget", 0), device_bytes=held,
               reverse_sweep_bytes=held - base_bytes, scatter_fallbacks=scat)
    if tuned is not None:
        rec["tuned_options"] = tuned["options"]
    if args.compare_separate or wl.name == "batch2d":
        t_sep = separate(wl, opts)
        rec["separate_ms_per_step"] = round(t_sep * 1e3, 3)
        rec["batched_speedup"] = round(t_sep / t_step, 3)
        log(f"[bench] {len(wl.instances)} separate handles: {t_sep * 1e3:.1f} ms per fwd+adj pass")
    if not args.no_roofline:
        rl, per_kernel = roofline(sim, tens, dloss, wl.precision, opts.get("streams", 0), wl.name)
        rec["roofline"] = rl
        rec["kernels"] = {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                          for k, v in per_kernel.items()}
        log(f"[bench] roofline {rl}")
    sim.close()
    if budget > 0 and not args.no_unbounded:
        # the same handle options without the bound (grid store as large as the
        # rollout needs, within the free memory)
        u_opts = {k: v for k, v in opts.items() if k != "ckpt_budget"}
        usim, utens, _ = make_sim(wl, u_opts)
        ub = usim.device_bytes()
        run_step(usim, utens, dloss)
        t_u = timed(lambda: run_step(usim, utens, dloss), max(1, min(3, args.steps)))
        t_urec = timed(lambda: run_step(usim, utens, dloss, record=True, backward=False), 1)
        rec["unbounded"] = dict(value=round(ps / t_u, 1), ms_per_step=round(t_u * 1e3, 3),
                                adj_over_fwd=round((t_u - t_urec) / t_fwd, 3), device_bytes=usim.device_bytes(),
                                reverse_sweep_bytes=usim.device_bytes() - ub)
        usim.close()
        log(f"[bench] without the checkpoint budget {rec['unbounded']}")
    if not args.no_front_end:
        rec["front_end"] = front_end(wl)
        log(f"[bench] front end {rec['front_end']}")
    if not args.no_obstacles:
        rec["obstacles"] = obstacles(wl)
        log(f"[bench] obstacles {rec['obstacles']}")
    if args.codesign > 0:
        cd = codesign(wl, args.codesign)
        if cd is not None:
            rec["codesign"] = cd
            log(f"[bench] co-design {cd}")
    if args.codesign_converge > 0:
        rec["codesign_converge"] = codesign_to_convergence(wl, args.codesign_converge,
                                                           topology=args.codesign_converge_topology)
        log(f"[bench] co-design to convergence {rec['codesign_converge']}")
    if not args.no_walker_codesign:
        rec["walker_codesign"] = walker_codesign(args.walker_max_iters, lr=args.walker_lr)
        log(f"[bench] walker co-design {rec['walker_codesign']}")
    if not args.no_long_horizon:
        rec["long_horizon"] = long_horizon()
        log(f"[bench] long horizon {rec['long_horizon']}")
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cb, insts, grads = cpu_baseline(wl.name, wl)
        rec["cpu_baseline"] = cb
        ge = grad_error(wl, insts, grads)
        rec["grad_rel_err_vs_oracle"] = {k: float(f"{v:.3e}") for k, v in ge["own_branches"].items()}
        rec["grad_rel_err_vs_oracle_on_device_branches"] = {k: float(f"{v:.3e}") for k, v in ge["device_branches"].items()}
        rec["branch_decisions_differing"] = ge["branch_decisions_differing"]
        rec["grad_rel_err_sample"] = cb["sample"].split(",")[0] + ", same sample as cpu_baseline"
        log(f"[bench] gradient vs oracle {ge}")
        log(f"[bench] cpu baseline {cb}")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
