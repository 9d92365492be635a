"""FP64 CPU oracle of the design front end: the map from the design variables
(topology variable phi, per-region magnetization magnitude and orientation
vector) to the per-particle density and remanent field that the MPM step takes,
and the transpose of its Jacobian.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg use this; the product path (the HIP library) never does, and the
two share no code. Plain numpy in float64, written for checking by eye, not
for speed: the filter is a brute-force double loop over particle pairs (in
row blocks), with no neighbour search.

What it computes (paper Sec. 3.1, "Design representation"):
  - density filter (Eqs. 23-24): phit_p = sum_q w_pq phi_q / sum_q w_pq over the
    particles q within distance R of p in the initial configuration, with
    w_pq = 1 - |x_q(0) - x_p(0)| / R;
  - Heaviside projection (Eq. 25):
    phibar = (tanh(beta/2) + tanh(beta (phit - 1/2))) / (2 tanh(beta/2));
  - magnetization (Eqs. 26-27): Br~_p = Br_max Br_p zeta_p / sqrt(|zeta_p|^2 + delta);
  - region sharing (Eq. 28): Br_p and zeta_p are those of the particle's region.

Readings (listed in the design notes):
  - Eq. 23's numerator weights phi of the neighbour q (the printed phi_p would
    make the filter the identity).
  - The neighbourhood holds the q with |x_q - x_p| < R, p itself included; the
    weight vanishes at distance R, so the strict or non-strict bound gives the
    same sums.
  - delta enters the orientation only (Eq. 27), so with delta > 0 the
    orientation is slightly shorter than a unit vector.
"""
from __future__ import annotations

import numpy as np

def _rows_per_block(n: int) -> int:
    """Rows of the pair matrix held at once (about 4M pairs)."""
    return max(1, min(512, 4_000_000 // max(1, n)))


def filter_weights_rows(x0: np.ndarray, rows: np.ndarray, radius: float) -> np.ndarray:
    """Weights w_pq (Eq. 24) of the particles p in `rows` against every q; zero
    outside the radius."""
    d = np.sqrt(((x0[rows, None, :] - x0[None, :, :]) ** 2).sum(-1))
    return np.where(d < radius, 1.0 - d / radius, 0.0)


def density_filter(x0: np.ndarray, phi: np.ndarray, radius: float, rows=None) -> np.ndarray:
    """phit = W phi / (W 1) (Eq. 23) at the given rows (default all)."""
    x0 = np.asarray(x0, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    rows = np.arange(len(phi)) if rows is None else np.asarray(rows)
    out = np.empty(len(rows))
    b = _rows_per_block(len(phi))
    for s in range(0, len(rows), b):
        r = rows[s:s + b]
        w = filter_weights_rows(x0, r, radius)
        out[s:s + b] = (w @ phi) / w.sum(1)
    return out


def density_filter_transpose(x0: np.ndarray, g: np.ndarray, radius: float) -> np.ndarray:
    """Transpose of the filter: d phit_p / d phi_q = w_pq / s_p with s_p the row
    sum, so g_phi_q = sum_p w_pq g_p / s_p."""
    x0 = np.asarray(x0, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = len(g)
    out = np.zeros(n)
    b = _rows_per_block(n)
    for s in range(0, n, b):
        r = np.arange(s, min(n, s + b))
        w = filter_weights_rows(x0, r, radius)
        out += (g[r] / w.sum(1)) @ w
    return out


def heaviside(phit: np.ndarray, beta: float) -> np.ndarray:
    """Eq. 25."""
    t = np.tanh(0.5 * beta)
    return (t + np.tanh(beta * (np.asarray(phit, dtype=np.float64) - 0.5))) / (2.0 * t)


def heaviside_derivative(phit: np.ndarray, beta: float) -> np.ndarray:
    """d phibar / d phit of Eq. 25."""
    th = np.tanh(beta * (np.asarray(phit, dtype=np.float64) - 0.5))
    return beta * (1.0 - th * th) / (2.0 * np.tanh(0.5 * beta))


def orientation(zeta: np.ndarray, delta: float) -> np.ndarray:
    """Eq. 27 per row of zeta."""
    zeta = np.asarray(zeta, dtype=np.float64)
    return zeta / np.sqrt((zeta * zeta).sum(-1, keepdims=True) + delta)


def magnetization(region: np.ndarray, br_mag: np.ndarray, zeta: np.ndarray, br_max: float,
                  delta: float) -> np.ndarray:
    """Eqs. 26-28: per-particle remanent field [N][d] from the region variables."""
    region = np.asarray(region)
    b = orientation(zeta, delta)
    return br_max * np.asarray(br_mag, dtype=np.float64)[region, None] * b[region]


def magnetization_transpose(region: np.ndarray, br_mag: np.ndarray, zeta: np.ndarray, br_max: float,
                            delta: float, g_br: np.ndarray):
    """Gradients of the region magnitudes [n_m] and orientation vectors [n_m][d]
    from the per-particle gradient g_br [N][d]: region sums G_m = sum of g_br
    over the region's particles, then g_mag_m = Br_max b_m . G_m and
    g_zeta_m = Br_max Br_m (G_m / r_m - zeta_m (zeta_m . G_m) / r_m^3),
    r_m = sqrt(|zeta_m|^2 + delta)."""
    zeta = np.asarray(zeta, dtype=np.float64)
    br_mag = np.asarray(br_mag, dtype=np.float64)
    n_m, d = zeta.shape
    G = np.zeros((n_m, d))
    np.add.at(G, np.asarray(region), np.asarray(g_br, dtype=np.float64))
    r = np.sqrt((zeta * zeta).sum(-1) + delta)
    b = zeta / r[:, None]
    g_mag = br_max * (b * G).sum(-1)
    zg = (zeta * G).sum(-1)
    g_zeta = br_max * br_mag[:, None] * (G / r[:, None] - zeta * (zg / r ** 3)[:, None])
    return g_mag, g_zeta


def front_end(x0, phi, radius, beta, region, br_mag, zeta, br_max, delta):
    """The whole map: (phit, phibar, Br~) of every particle."""
    phit = density_filter(x0, phi, radius)
    return phit, heaviside(phit, beta), magnetization(region, br_mag, zeta, br_max, delta)


def front_end_backward(x0, phi, radius, beta, region, br_mag, zeta, br_max, delta, g_density, g_br):
    """Gradients of (phi, region magnitudes, region orientations) from the
    gradients of the hot path's inputs (density = phibar, br = Br~)."""
    phit = density_filter(x0, phi, radius)
    g_phit = np.asarray(g_density, dtype=np.float64) * heaviside_derivative(phit, beta)
    g_phi = density_filter_transpose(x0, g_phit, radius)
    g_mag, g_zeta = magnetization_transpose(region, br_mag, zeta, br_max, delta, g_br)
    return g_phi, g_mag, g_zeta


# --------------------------------------------------------------------------
# Harmonic stimulus (Sec. 3.1.2, Eqs. 29-30)
# --------------------------------------------------------------------------
# The rollout's field program holds one row per step when each step is its own
# segment (seg_steps = 1); row n is the field at the start of step n, t_n = n dt.

def harmonic_frequency(f, f_min, f_max):
    """fbar = (f_max - f_min) f + f_min (Eq. 29)."""
    return (f_max - f_min) * np.asarray(f, dtype=np.float64) + f_min


def harmonic_program(b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta):
    """Rows [n_inst * n_steps][d]: instance k, step n gives
    B_max B_a[k] sin(2 pi fbar_k t_n) b(eta_k), b = eta / sqrt(|eta|^2 + delta)."""
    b_a = np.asarray(b_a, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    t = np.arange(n_steps) * dt
    fbar = harmonic_frequency(f, f_min, f_max)
    b = orientation(eta, delta)
    s = np.sin(2.0 * np.pi * fbar[:, None] * t[None, :])            # [n_inst][T]
    return (b_max * b_a[:, None, None] * s[:, :, None] * b[:, None, :]).reshape(-1, eta.shape[1])


def harmonic_program_transpose(b_a, f, eta, n_steps, dt, b_max, f_min, f_max, delta, g_prog):
    """Gradients of (B_a, f, eta) per instance from the program gradient
    g_prog [n_inst * n_steps][d]: with s_n = sin(w t_n), c_n = cos(w t_n),
    w = 2 pi fbar and q_n = b . G_n,
      g_Ba  = B_max sum_n s_n q_n
      g_f   = B_max B_a sum_n c_n 2 pi (f_max - f_min) t_n q_n
      g_eta = B_max B_a (S / r - eta (eta . S) / r^3),  S = sum_n s_n G_n."""
    b_a = np.asarray(b_a, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    n_inst, d = eta.shape
    G = np.asarray(g_prog, dtype=np.float64).reshape(n_inst, n_steps, d)
    t = np.arange(n_steps) * dt
    w = 2.0 * np.pi * harmonic_frequency(f, f_min, f_max)
    s = np.sin(w[:, None] * t[None, :])
    c = np.cos(w[:, None] * t[None, :])
    r = np.sqrt((eta * eta).sum(-1) + delta)
    b = eta / r[:, None]
    q = (G * b[:, None, :]).sum(-1)                                    # [n_inst][T]
    g_ba = b_max * (s * q).sum(1)
    g_f = b_max * b_a * (c * (2.0 * np.pi * (f_max - f_min)) * t[None, :] * q).sum(1)
    S = (s[:, :, None] * G).sum(1)                                     # [n_inst][d]
    g_eta = b_max * b_a[:, None] * (S / r[:, None] - eta * ((eta * S).sum(-1) / r ** 3)[:, None])
    return g_ba, g_f, g_eta


# --------------------------------------------------------------------------
# Optimizer update of the co-design loop (Sec. 3.2)
# --------------------------------------------------------------------------

def adam_step(p, g, m, v, t, lr, beta1, beta2, eps, lo, hi):
    """One Adam update (Kingma and Ba, "Adam: A method for stochastic
    optimization", ICLR 2015, Algorithm 1) at step t >= 1, then the variables
    mapped back into [lo, hi] (the bounds of Eqs. 34c-d and 35c-d). Returns the
    new (p, m, v)."""
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    p = np.asarray(p, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return np.clip(p, lo, hi), m, v
