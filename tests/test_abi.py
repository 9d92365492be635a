"""The C-ABI library loads on the host and exports every entry point that the
headers under include/ declare (no device calls)."""
import ctypes
import glob
import os
import re


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def _declared():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(mpm_mag_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("mpm_mag_create", "mpm_mag_rollout", "mpm_mag_backward", "mpm_mag_destroy",
                 "mpm_mag_design_create", "mpm_mag_design_forward", "mpm_mag_design_backward",
                 "mpm_mag_design_destroy"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2503_22767_amd import mpm_mag as M
    L = M.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_status_strings_and_kernel_table():
    from paper_2503_22767_amd import mpm_mag as M
    L = M.lib()
    assert L.mpm_mag_strerror(0) == b"ok"
    assert L.mpm_mag_strerror(7).startswith(b"backward")
    n = L.mpm_mag_num_kernels()
    names = [L.mpm_mag_kernel_name(i).decode() for i in range(n)]
    for k in ("p2g", "grid_update", "g2p", "g2p_adj", "grid_adj", "p2g_adj"):
        assert k in names
    assert L.mpm_mag_kernel_name(n) == b""


def test_create_rejects_bad_arguments_without_touching_the_device():
    from paper_2503_22767_amd import mpm_mag as M
    L = M.lib()
    h = ctypes.c_void_p()
    descs = (M.InstanceDesc * 1)()
    descs[0].dim = 4
    counts = (ctypes.c_int64 * 1)(10)
    assert L.mpm_mag_create(descs, 1, counts, 4, ctypes.byref(h)) == M.EINVAL
    descs[0].dim = 2
    assert L.mpm_mag_create(descs, 1, counts, 5, ctypes.byref(h)) == M.EINVAL
    assert L.mpm_mag_create(descs, 0, counts, 4, ctypes.byref(h)) == M.EINVAL
    descs[0].n_grid = 32
    descs[0].n_segments = 1
    descs[0].dt = 1e-3
    descs[0].particle_volume = 1e-4
    descs[0].mu0 = descs[0].rho = 1.0
    descs[0].nu = 0.3
    zero = (ctypes.c_int64 * 1)(0)
    assert L.mpm_mag_create(descs, 1, zero, 4, ctypes.byref(h)) == M.EINVAL   # no particles
    descs[0].n_steps = -1
    assert L.mpm_mag_create(descs, 1, counts, 4, ctypes.byref(h)) == M.EINVAL  # negative step count
    assert L.mpm_mag_rollout(None, None, None, None, None, None, None, None, None, None, 0) == M.EINVAL
    assert L.mpm_mag_backward(None, None, None, None, None, None, None) == M.EINVAL
    assert L.mpm_mag_set_branch_trace(None, None, 0) == M.EINVAL
    assert L.mpm_mag_trace_nodes(None) == 0
    assert L.mpm_mag_scatter_stats(None, None, 0) == M.EINVAL
    L.mpm_mag_destroy(None)


def test_create_rejects_grids_beyond_32bit_node_offsets():
    """The kernels index the instance grids with 32-bit node offsets: three 3D
    instances at n_grid = 1024 (3 * 2^30 nodes) are refused before any device
    work, two would fit."""
    from paper_2503_22767_amd import mpm_mag as M
    L = M.lib()
    h = ctypes.c_void_p()
    descs = (M.InstanceDesc * 3)()
    for d in descs:
        d.dim = 3
        d.n_grid = 1024
        d.n_steps = 4
        d.n_segments = 1
        d.dt = 1e-4
        d.particle_volume = 1e-9
        d.mu0 = d.rho = d.E = 1.0
        d.nu = 0.3
    counts = (ctypes.c_int64 * 3)(100, 100, 100)
    assert L.mpm_mag_create(descs, 3, counts, 4, ctypes.byref(h)) == M.EINVAL
    assert b"2^31" in L.mpm_mag_last_error(None)
