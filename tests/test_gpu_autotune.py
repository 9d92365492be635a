"""Every launch option the autotuner may pick gives oracle-parity results, and
the tuner itself returns a valid, cached choice."""
import pytest

from paper_2503_22767_amd import autotune as A
from paper_2503_22767_amd import workloads as W

from gpu_util import compare, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu

OPTION_CASES = [("sort_curve", 1), ("sort_curve", 2), ("box_cap", 64), ("box_cap", 256),
                ("grid_wgs", 16), ("graph", 1), ("fuse_fwd", 0), ("fuse_adj", 0), ("streams", 2),
                ("lane_sort", 0), ("grid_store", 0), ("grid_threads", 256), ("grid_threads", 384), ("grid_threads", 1024),
                ("grid_parts", 1), ("grid_parts", 2), ("grid_parts", 4), ("grid_parts", 8)]


def _case(dim):
    size = (0.4, 0.2, 0.2) if dim == 2 else (0.3, 0.2, 0.25)
    return W.make_tiny(seed=11, dim=dim, n_steps=20, loss_kind=W.LOSS_COM_DISP, floor=True, gravity=1.0,
                       size=size, n_grid=16, n_segments=4)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("key,value", OPTION_CASES, ids=[f"{k}={v}" for k, v in OPTION_CASES])
def test_option_values_keep_oracle_parity(dim, key, value):
    inst = _case(dim)
    ref = oracle_run([inst])
    got = gpu_run([inst], precision=8, options={key: value})
    compare(got, ref, pos_tol=1e-10, grad_tol=1e-9, loss_tol=1e-9, label=f"d{dim} {key}={value} fp64")
    got = gpu_run([inst], precision=4, options={key: value})
    compare(got, ref, pos_tol=1e-4, grad_tol=1e-3, label=f"d{dim} {key}={value} fp32")


def test_autotune_returns_cached_valid_options(tmp_path):
    wl = W.make_walker2d(n_steps=40)
    cache = str(tmp_path / "tune.json")
    rec = A.autotune(wl.instances, 4, steps=10, reps=2, cache_path=cache, log=log)
    log("autotune", rec["key"], rec["options"], f"{rec['seconds'] * 1e3:.2f} ms vs default "
        f"{rec['default_seconds'] * 1e3:.2f} ms")
    assert not rec["cached"]
    for k, v in rec["options"].items():
        assert v in A.SPACE[k]
    assert rec["seconds"] <= rec["default_seconds"]
    again = A.autotune(wl.instances, 4, cache_path=cache)
    assert again["cached"] and again["options"] == rec["options"]
    # the tuned options keep parity on the workload itself
    ref = oracle_run(wl.instances, ckpt_every=8)
    got = gpu_run(wl.instances, precision=4, options=rec["options"])
    compare(got, ref, pos_tol=1e-4, grad_tol=1e-3, label="walker2d[:40] tuned")
