"""FP64 CPU oracle of the magneto-elastic MLS-MPM step and its adjoint (ctypes).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg load this; the product path (the HIP library) never does, and the
two share no code. The arithmetic lives in mpm_oracle.c; this module only
marshals numpy arrays. Particle arrays cross the boundary with three
components and 3x3 matrices even in 2D (z parts zero, F33 = 1).
"""
from __future__ import annotations

import contextlib
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, EINVAL, ENOMEM, EDOMAIN, EINVERT, ENONFINITE = 0, 1, 2, 4, 5, 6


MAX_OBSTACLES = 4
OBST_HALFSPACE, OBST_SPHERE, OBST_BOX = 1, 2, 3


class Obstacle(C.Structure):
    _fields_ = [("kind", C.c_int), ("attached", C.c_int), ("a", C.c_double * 3), ("b", C.c_double * 3),
                ("mu", C.c_double), ("vel", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n_grid", C.c_int), ("dt", C.c_double), ("n_steps", C.c_int),
        ("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double), ("mu0", C.c_double),
        ("simp_eps", C.c_double), ("simp_q", C.c_double), ("damping", C.c_double),
        ("gravity", C.c_double * 3), ("wall_cells", C.c_int), ("clamp_xmax", C.c_double),
        ("floor_on", C.c_int), ("floor_y", C.c_double), ("floor_mu", C.c_double),
        ("particle_volume", C.c_double),
        ("n_segments", C.c_int), ("seg_steps", C.c_int), ("periodic", C.c_int),
        ("loss_kind", C.c_int), ("loss_dir", C.c_double * 3),
        ("n_obstacles", C.c_int), ("obst", Obstacle * MAX_OBSTACLES),
        ("mass_eps", C.c_double),
    ]


def _vec3(v):
    return (C.c_double * 3)(*([float(x) for x in list(v)] + [0.0] * 3)[:3])


def params(p: dict) -> Params:
    """Parameter struct of one instance; p["obstacles"] (optional) is a list of
    dicts with kind, a, b, mu (default 0), vel (default 0) and attached (default 0)."""
    s = Params()
    obst = list(p.get("obstacles", []))
    if len(obst) > MAX_OBSTACLES:
        raise ValueError("at most 4 obstacles")
    s.n_obstacles = len(obst)
    for j, o in enumerate(obst):
        s.obst[j] = Obstacle(int(o["kind"]), int(o.get("attached", 0)), _vec3(o["a"]), _vec3(o["b"]),
                             float(o.get("mu", 0.0)), _vec3(o.get("vel", [0.0, 0.0, 0.0])))
    for name, _ in Params._fields_:
        if name in ("n_obstacles", "obst"):
            continue
        if name == "mass_eps" and name not in p:
            continue   # default 0: Eq. 33
        val = p[name]
        if name in ("gravity", "loss_dir"):
            arr = (C.c_double * 3)(*[float(v) for v in list(val) + [0.0] * (3 - len(val))][:3])
            setattr(s, name, arr)
        else:
            setattr(s, name, val)
    return s


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        _LIB = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        _LIB.orc_energy_elastic.restype = C.c_double
        _LIB.orc_energy_elastic.argtypes = [dp, C.c_double, C.c_double]
    return _LIB


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a, shape=None):
    if a is None:
        return None
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        out = out.reshape(shape)
    return out


def _u8(a):
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint8))


def _check(code, what):
    if code != 0:
        raise OracleError(code, what)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


# ----------------------------------------------------------------------------
# constitutive pieces
# ----------------------------------------------------------------------------

def moduli(E: float, nu: float):
    G, K = C.c_double(), C.c_double()
    lib().orc_moduli(C.c_double(E), C.c_double(nu), C.byref(G), C.byref(K))
    return G.value, K.value


def stress_elastic(F, G, K):
    F = _f64(F, (9,))
    P = np.zeros(9)
    lib().orc_stress_elastic(_d(F), C.c_double(G), C.c_double(K), _d(P))
    return P.reshape(3, 3)


def stress_elastic_dir(F, G, K, dF):
    F = _f64(F, (9,))
    dF = _f64(dF, (9,))
    dP = np.zeros(9)
    lib().orc_stress_elastic_dir(_d(F), C.c_double(G), C.c_double(K), _d(dF), _d(dP))
    return dP.reshape(3, 3)


def bspline(f: float):
    w = np.zeros(3)
    dw = np.zeros(3)
    lib().orc_bspline(C.c_double(f), _d(w), _d(dw))
    return w, dw


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (n <= 0: the OpenMP default)."""
    lib().orc_set_threads(C.c_int(int(n)))


def get_threads() -> int:
    return int(lib().orc_get_threads())


@contextlib.contextmanager
def branch_trace(p: dict, replay=None, record: bool = False):
    """Replay and/or record the grid operation's per-node decisions (has mass,
    floor branch, wall zeroing, obstacle branches) for the rollouts and
    gradients run inside the block; tables are uint16 [n_steps, n_nodes] in the
    packing mpm_oracle.c documents. Yields the record table (or None)."""
    G = num_nodes(p)
    T = int(p["n_steps"])
    rep = None if replay is None else np.ascontiguousarray(np.asarray(replay, dtype=np.uint16).reshape(T, G))
    rec = np.zeros((T, G), dtype=np.uint16) if record else None
    u16 = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None
    lib().orc_set_branch_trace(u16(rep), u16(rec), C.c_int64(G))
    try:
        yield rec
    finally:
        lib().orc_set_branch_trace(None, None, C.c_int64(0))


def branch_mass_mismatches() -> int:
    """Replayed "has mass" decisions at nodes where the oracle's mass is zero
    (since the last branch_trace began)."""
    lib().orc_branch_mass_mismatches.restype = C.c_longlong
    return int(lib().orc_branch_mass_mismatches())


def segment(p: dict, n: int) -> int:
    return lib().orc_segment(C.byref(params(p)), C.c_int(n))


def num_nodes(p: dict) -> int:
    return lib().orc_num_nodes(C.byref(params(p)))


# ----------------------------------------------------------------------------
# rollout and gradient
# ----------------------------------------------------------------------------

def rollout(p: dict, x0, density, br, b_prog, target=None, mask=None, v0=None, traj=False):
    """Forward rollout of p['n_steps'] steps. Returns a dict with the final state
    (x, v: [N,3]; C, F: [N,3,3]), the loss and optionally all positions."""
    d = p["dim"]
    x0 = _f64(x0)
    n = x0.shape[0]
    phi = _f64(density, (n,))
    br = _f64(br, (n, d))
    prog = _f64(b_prog, (-1, d))
    tgt = _f64(target, (n, d)) if target is not None else None
    msk = _u8(mask)
    v0 = _f64(v0, (n, d)) if v0 is not None else None
    x = np.zeros((n, 3)); v = np.zeros((n, 3)); Cm = np.zeros((n, 9)); F = np.zeros((n, 9))
    loss = C.c_double()
    tr = np.zeros((p["n_steps"] + 1, n, 3)) if traj else None
    code = lib().orc_rollout(C.byref(params(p)), C.c_int(n), _d(x0), _d(v0), _d(phi), _d(br), _d(prog),
                             _d(tgt), msk.ctypes.data_as(C.POINTER(C.c_ubyte)) if msk is not None else None,
                             _d(x), _d(v), _d(Cm), _d(F), C.byref(loss), _d(tr))
    _check(code, "rollout")
    out = dict(x=x, v=v, C=Cm.reshape(n, 3, 3), F=F.reshape(n, 3, 3), loss=loss.value)
    if traj:
        out["traj"] = tr
    return out


def backward(p: dict, x0, density, br, b_prog, target=None, mask=None, dloss: float = 1.0,
             ckpt_every: int = None):
    """Loss and its gradient w.r.t. density [N], remanence [N,d] and the field
    program [S,d] (reverse-mode through every step, checkpointed)."""
    d = p["dim"]
    x0 = _f64(x0)
    n = x0.shape[0]
    phi = _f64(density, (n,))
    br = _f64(br, (n, d))
    prog = _f64(b_prog, (-1, d))
    tgt = _f64(target, (n, d)) if target is not None else None
    msk = _u8(mask)
    if ckpt_every is None:
        ckpt_every = max(1, int(math.isqrt(max(1, p["n_steps"]))))
    gphi = np.zeros(n); gbr = np.zeros((n, d)); gprog = np.zeros_like(prog)
    loss = C.c_double()
    code = lib().orc_backward(C.byref(params(p)), C.c_int(n), _d(x0), _d(phi), _d(br), _d(prog), _d(tgt),
                              msk.ctypes.data_as(C.POINTER(C.c_ubyte)) if msk is not None else None,
                              C.c_double(dloss), C.c_int(ckpt_every), C.byref(loss), _d(gphi), _d(gbr),
                              _d(gprog))
    _check(code, "backward")
    return dict(loss=loss.value, g_density=gphi, g_br=gbr, g_b_prog=gprog)


# ----------------------------------------------------------------------------
# single phases (flat arrays: x,v [N,3]; C,F [N,3,3]; grid m [G], p/v [G,3])
# ----------------------------------------------------------------------------

def p2g(p, x, v, Cm, F, phi, br3, B):
    n = len(phi)
    G = num_nodes(p)
    m = np.zeros(G); mom = np.zeros((G, 3))
    code = lib().orc_p2g_flat(C.byref(params(p)), C.c_int(n), _d(_f64(x, (n, 3))), _d(_f64(v, (n, 3))),
                              _d(_f64(Cm, (n, 9))), _d(_f64(F, (n, 9))), _d(_f64(phi, (n,))),
                              _d(_f64(br3, (n, 3))), _d(_f64(B, (3,))), _d(m), _d(mom))
    _check(code, "p2g")
    return m, mom


def grid(p, m, mom, step=0):
    """Grid update of step `step` (moving obstacles sit at a + v_b step dt)."""
    G = num_nodes(p)
    v = np.zeros((G, 3))
    lib().orc_grid(C.byref(params(p)), int(step), _d(_f64(m, (G,))), _d(_f64(mom, (G, 3))), _d(v))
    return v


def grid_adj(p, m, mom, vbar, step=0):
    G = num_nodes(p)
    pbar = np.zeros((G, 3)); mbar = np.zeros(G)
    lib().orc_grid_adj(C.byref(params(p)), int(step), _d(_f64(m, (G,))), _d(_f64(mom, (G, 3))),
                       _d(_f64(vbar, (G, 3))), _d(pbar), _d(mbar))
    return pbar, mbar


def g2p(p, x, F, vgrid):
    n = np.asarray(x).shape[0]
    x1 = np.zeros((n, 3)); v1 = np.zeros((n, 3)); C1 = np.zeros((n, 9)); F1 = np.zeros((n, 9))
    code = lib().orc_g2p_flat(C.byref(params(p)), C.c_int(n), _d(_f64(x, (n, 3))), _d(_f64(F, (n, 9))),
                              _d(_f64(vgrid, (-1, 3))), _d(x1), _d(v1), _d(C1), _d(F1))
    _check(code, "g2p")
    return x1, v1, C1.reshape(n, 3, 3), F1.reshape(n, 3, 3)


def g2p_adj(p, x, F, vgrid, xb1, vb1, Cb1, Fb1):
    n = np.asarray(x).shape[0]
    G = num_nodes(p)
    vbar = np.zeros((G, 3)); xb0 = np.zeros((n, 3)); Fb0 = np.zeros((n, 9))
    code = lib().orc_g2p_adj_flat(C.byref(params(p)), C.c_int(n), _d(_f64(x, (n, 3))), _d(_f64(F, (n, 9))),
                                  _d(_f64(vgrid, (G, 3))), _d(_f64(xb1, (n, 3))), _d(_f64(vb1, (n, 3))),
                                  _d(_f64(Cb1, (n, 9))), _d(_f64(Fb1, (n, 9))), _d(vbar), _d(xb0), _d(Fb0))
    _check(code, "g2p_adj")
    return vbar, xb0, Fb0.reshape(n, 3, 3)


def p2g_adj(p, x, v, Cm, F, phi, br3, B, pbar, mbar):
    n = len(phi)
    G = num_nodes(p)
    xb = np.zeros((n, 3)); vb = np.zeros((n, 3)); Cb = np.zeros((n, 9)); Fb = np.zeros((n, 9))
    gphi = np.zeros(n); gbr = np.zeros((n, 3)); gB = np.zeros(3)
    code = lib().orc_p2g_adj_flat(C.byref(params(p)), C.c_int(n), _d(_f64(x, (n, 3))), _d(_f64(v, (n, 3))),
                                  _d(_f64(Cm, (n, 9))), _d(_f64(F, (n, 9))), _d(_f64(phi, (n,))),
                                  _d(_f64(br3, (n, 3))), _d(_f64(B, (3,))), _d(_f64(pbar, (G, 3))),
                                  _d(_f64(mbar, (G,))), _d(xb), _d(vb), _d(Cb), _d(Fb), _d(gphi), _d(gbr), _d(gB))
    _check(code, "p2g_adj")
    return dict(x=xb, v=vb, C=Cb.reshape(n, 3, 3), F=Fb.reshape(n, 3, 3), phi=gphi, br=gbr, B=gB)
