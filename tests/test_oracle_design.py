"""Pins of the design front end's oracle (density filter, Heaviside projection,
magnetization parametrization with region sharing; Sec. 3.1, Eqs. 23-28)
against what the mathematics fixes: closed forms on small configurations,
limits, invariants, the adjoint identity of the filter and central finite
differences of the whole map."""
import numpy as np
import pytest

from oracle import design as D


def _lattice(nx, ny, nz, h, jitter=0.0, seed=0):
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3) * h
    return g + jitter * h * rng.uniform(-1, 1, g.shape)


def test_filter_of_a_constant_field_is_that_constant():
    x0 = _lattice(6, 5, 4, 0.01, jitter=0.3, seed=1)
    out = D.density_filter(x0, np.full(len(x0), 0.37), radius=0.025)
    assert np.allclose(out, 0.37, rtol=0, atol=1e-15)


def test_filter_radius_below_the_spacing_is_the_identity():
    x0 = _lattice(5, 4, 3, 0.01)
    phi = np.random.default_rng(2).uniform(0, 1, len(x0))
    assert np.array_equal(D.density_filter(x0, phi, radius=0.009), phi)


def test_filter_of_three_collinear_particles_closed_form():
    """Spacing h, R = 1.5 h: neighbours at h weigh 1/3, the pair at 2h lies
    outside; each particle weighs itself 1. The printed numerator index (phi of
    the particle itself) would return phi unchanged."""
    h = 0.1
    x0 = np.array([[0.0, 0, 0], [h, 0, 0], [2 * h, 0, 0]])
    phi = np.array([0.2, 0.9, 0.5])
    out = D.density_filter(x0, phi, radius=1.5 * h)
    w = 1.0 - 1.0 / 1.5
    expect = [(phi[0] + w * phi[1]) / (1 + w),
              (phi[1] + w * (phi[0] + phi[2])) / (1 + 2 * w),
              (phi[2] + w * phi[1]) / (1 + w)]
    assert np.allclose(out, expect, rtol=1e-15, atol=0)


def test_filter_of_two_particles_in_3d_closed_form():
    x0 = np.array([[0.1, 0.2, 0.3], [0.13, 0.16, 0.3]])   # distance 0.05
    phi = np.array([0.8, 0.1])
    R = 0.08
    w = 1 - 0.05 / R
    out = D.density_filter(x0, phi, radius=R)
    assert np.allclose(out, [(0.8 + w * 0.1) / (1 + w), (0.1 + w * 0.8) / (1 + w)], rtol=1e-14, atol=0)


def test_filter_transpose_satisfies_the_adjoint_identity():
    """<F phi, g> = <phi, F^T g>; the row sums differ from particle to particle,
    so dividing by the neighbour's sum instead of the row's fails this."""
    rng = np.random.default_rng(3)
    x0 = rng.uniform(0, 0.1, (700, 3))
    phi, g = rng.uniform(0, 1, 700), rng.standard_normal(700)
    lhs = D.density_filter(x0, phi, 0.02) @ g
    rhs = phi @ D.density_filter_transpose(x0, g, 0.02)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    s = D.filter_weights_rows(x0, np.arange(700), 0.02).sum(1)
    assert s.std() > 0.1 * s.mean()   # the identity is not trivial here


@pytest.mark.parametrize("beta", [1.0, 8.0, 64.0])
def test_heaviside_fixes_zero_half_and_one_and_is_odd_about_the_half(beta):
    assert abs(D.heaviside(0.0, beta)) < 1e-15
    assert abs(D.heaviside(1.0, beta) - 1.0) < 1e-15
    assert abs(D.heaviside(0.5, beta) - 0.5) < 1e-15
    x = np.linspace(0, 1, 41)
    assert np.allclose(D.heaviside(1 - x, beta), 1 - D.heaviside(x, beta), atol=1e-15)
    dh = np.diff(D.heaviside(x, beta))
    assert np.all(dh >= 0)
    if beta <= 8:   # steeper projections saturate to 0 and 1 in double away from the half
        assert np.all(dh > 0)


def test_heaviside_limits():
    x = np.linspace(0, 1, 21)
    # small beta: tanh(b u) ~ b u, the projection tends to the identity
    assert np.allclose(D.heaviside(x, 1e-4), x, atol=1e-8)
    # large beta: a step at one half
    hb = D.heaviside(x, 128.0)
    assert np.all(hb[x < 0.45] < 1e-2) and np.all(hb[x > 0.55] > 1 - 1e-2)


def test_heaviside_derivative_matches_central_differences():
    x = np.linspace(0.02, 0.98, 25)
    for beta in (1.0, 8.0, 32.0):
        e = 1e-6
        fd = (D.heaviside(x + e, beta) - D.heaviside(x - e, beta)) / (2 * e)
        assert np.allclose(D.heaviside_derivative(x, beta), fd, rtol=1e-7, atol=1e-9)


def test_magnetization_magnitude_direction_and_sharing():
    rng = np.random.default_rng(4)
    n_m, n = 5, 40
    zeta = rng.uniform(-1, 1, (n_m, 3))
    mag = rng.uniform(0, 1, n_m)
    region = rng.integers(0, n_m, n)
    br = D.magnetization(region, mag, zeta, br_max=1.3, delta=0.0)
    # delta = 0: a unit orientation, so |Br~| = Br_max Br of the region
    assert np.allclose(np.linalg.norm(br, axis=1), 1.3 * mag[region], rtol=1e-14)
    # parallel to zeta of the region
    assert np.allclose(np.cross(br, zeta[region]), 0, atol=1e-14)
    assert np.all((br * zeta[region]).sum(1) > 0)
    # delta > 0 shortens it by |zeta| / sqrt(|zeta|^2 + delta)
    z2 = (zeta * zeta).sum(1)
    brd = D.magnetization(region, mag, zeta, br_max=1.3, delta=0.05)
    assert np.allclose(np.linalg.norm(brd, axis=1), 1.3 * mag[region] * np.sqrt(z2 / (z2 + 0.05))[region], rtol=1e-14)


def test_region_gradient_is_the_sum_of_its_particles_gradients():
    """n_m regions against n_m = n_p (every particle its own region, Eq. 28's
    special case) carrying the same variables: the region gradient is the sum
    over its particles."""
    rng = np.random.default_rng(5)
    n_m, n = 4, 30
    zeta = rng.uniform(-1, 1, (n_m, 2))
    mag = rng.uniform(0.1, 1, n_m)
    region = rng.integers(0, n_m, n)
    g = rng.standard_normal((n, 2))
    gm, gz = D.magnetization_transpose(region, mag, zeta, 1.0, 1e-3, g)
    pm, pz = D.magnetization_transpose(np.arange(n), mag[region], zeta[region], 1.0, 1e-3, g)
    for m in range(n_m):
        sel = region == m
        assert np.allclose(gm[m], pm[sel].sum(), rtol=1e-13, atol=1e-15)
        assert np.allclose(gz[m], pz[sel].sum(0), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_front_end_gradient_matches_central_differences(dim):
    """d/dv <g_d, phibar(v)> + <g_b, Br~(v)> along a random direction in
    (phi, region magnitudes, region orientations), FP64 central differences."""
    rng = np.random.default_rng(10 + dim)
    n, n_m = 120, 3
    x0 = rng.uniform(0, 0.08, (n, dim))
    phi = rng.uniform(0.1, 0.9, n)
    mag = rng.uniform(0.2, 1, n_m)
    zeta = rng.uniform(-1, 1, (n_m, dim))
    region = rng.integers(0, n_m, n)
    R, beta, bmax, delta = 0.02, 6.0, 1.1, 1e-2
    gd, gb = rng.standard_normal(n), rng.standard_normal((n, dim))
    dphi, dmag, dz = rng.standard_normal(n), rng.standard_normal(n_m), rng.standard_normal((n_m, dim))

    def L(s):
        _, pb, br = D.front_end(x0, phi + s * dphi, R, beta, region, mag + s * dmag, zeta + s * dz, bmax, delta)
        return pb @ gd + (br * gb).sum()

    e = 1e-6
    fd = (L(e) - L(-e)) / (2 * e)
    g_phi, g_mag, g_z = D.front_end_backward(x0, phi, R, beta, region, mag, zeta, bmax, delta, gd, gb)
    adj = g_phi @ dphi + g_mag @ dmag + (g_z * dz).sum()
    assert abs(fd - adj) <= 1e-7 * abs(adj), (fd, adj)


# ---------------------------------------------------------------- harmonic stimulus (Eqs. 29-30)

def test_harmonic_program_shape_zero_start_bound_and_direction():
    rng = np.random.default_rng(20)
    b_a, f, eta = rng.uniform(0.2, 1, 2), rng.uniform(0, 1, 2), rng.uniform(-1, 1, (2, 3))
    P = D.harmonic_program(b_a, f, eta, 400, 1e-3, 2.0, 1.0, 20.0, 0.0).reshape(2, 400, 3)
    assert np.all(P[:, 0] == 0)                                   # sin(0)
    mag = np.linalg.norm(P, axis=-1)
    assert np.all(mag <= 2.0 * b_a[:, None] * (1 + 1e-14))       # |B| <= B_max B_a (delta = 0)
    assert np.allclose(mag.max(1), 2.0 * b_a, rtol=1e-3)         # reached within the 0.4 s window
    assert np.allclose(np.cross(P, eta[:, None, :]), 0, atol=1e-14)


def test_harmonic_frequency_ends_and_period():
    """f = 0 gives f_min and f = 1 gives f_max: the program repeats after
    1 / fbar (here a whole number of steps)."""
    dt = 1e-3
    for f, fbar in ((0.0, 5.0), (1.0, 25.0)):
        P = D.harmonic_program([1.0], [f], [[1.0, 0.0]], 1000, dt, 1.0, 5.0, 25.0, 0.0)
        period = int(round(1.0 / fbar / dt))
        assert np.allclose(P[period:], P[:-period], atol=1e-12)
        # the first crest a quarter period in
        assert abs(P[period // 4, 0] - 1.0) < 1e-12


def test_harmonic_program_is_linear_in_the_magnitude():
    P1 = D.harmonic_program([0.3], [0.4], [[0.2, -0.7, 0.1]], 50, 2e-3, 1.5, 2.0, 9.0, 1e-3)
    P2 = D.harmonic_program([0.6], [0.4], [[0.2, -0.7, 0.1]], 50, 2e-3, 1.5, 2.0, 9.0, 1e-3)
    assert np.allclose(P2, 2 * P1, rtol=1e-15, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_harmonic_transpose_matches_central_differences(dim):
    rng = np.random.default_rng(30 + dim)
    n_inst, T, dt = 3, 300, 1e-3
    b_a, f, eta = rng.uniform(0.2, 1, n_inst), rng.uniform(0, 1, n_inst), rng.uniform(-1, 1, (n_inst, dim))
    g = rng.standard_normal((n_inst * T, dim))
    args = (T, dt, 1.7, 2.0, 30.0, 1e-2)
    dba, dff, de = rng.standard_normal(n_inst), rng.standard_normal(n_inst), rng.standard_normal((n_inst, dim))

    def L(s):
        return (D.harmonic_program(b_a + s * dba, f + s * dff, eta + s * de, *args) * g).sum()

    e = 1e-6
    fd = (L(e) - L(-e)) / (2 * e)
    gba, gf, ge = D.harmonic_program_transpose(b_a, f, eta, *args, g)
    adj = gba @ dba + gf @ dff + (ge * de).sum()
    assert abs(fd - adj) <= 1e-7 * abs(adj), (fd, adj)


# ---------------------------------------------------------------- optimizer update (Sec. 3.2)

def test_adam_first_step_moves_each_variable_by_the_learning_rate():
    """m_hat = g and v_hat = g^2 after one step, so with eps = 0 every variable
    moves by lr against the sign of its gradient."""
    g = np.array([3.0, -0.02, 1e-6, -7.5])
    p, m, v = D.adam_step(np.full(4, 0.5), g, np.zeros(4), np.zeros(4), 1, 0.01, 0.9, 0.999, 0.0, 0.0, 1.0)
    assert np.allclose(p, 0.5 - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_steps_lr_each_iteration():
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    g = np.array([2.0, -1.0, 0.5])
    for t in range(1, 30):
        p, m, v = D.adam_step(p, g, m, v, t, 1e-3, 0.9, 0.999, 0.0, -1.0, 1.0)
        assert np.allclose(p, -1e-3 * t * np.sign(g), rtol=1e-12, atol=1e-15)


def test_adam_maps_back_into_the_bounds_and_stops_without_gradient():
    p, m, v = D.adam_step(np.array([0.995, 0.002]), np.array([-1.0, 1.0]), np.zeros(2), np.zeros(2), 1, 0.01,
                          0.9, 0.999, 1e-8, 0.0, 1.0)
    assert p[0] == 1.0 and p[1] == 0.0
    # a zero gradient from the start leaves the variables where they are
    q, _, _ = D.adam_step(np.array([0.3]), np.array([0.0]), np.zeros(1), np.zeros(1), 1, 0.01, 0.9, 0.999, 1e-8,
                          0.0, 1.0)
    assert q[0] == 0.3


def test_adam_minimizes_a_separable_quadratic():
    c = np.array([0.2, -0.4, 0.9])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 2001):
        p, m, v = D.adam_step(p, 2 * (p - c), m, v, t, 0.01, 0.9, 0.999, 1e-8, -1.0, 1.0)
    assert np.allclose(p, c, atol=1e-3)
