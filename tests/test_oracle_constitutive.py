"""Pins of the oracle's constitutive model and interpolation kernel.

Each test checks the oracle against something other than itself: the energy of
Eq. 4 differentiated numerically, the behaviour a stress must have under rigid
motion, the linear-elastic small-strain limit, closed forms for simple shear and
uniaxial stretch derived by hand, and textbook B-spline values.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _W_e(F, G, K):
    """Eq. 4 written directly (test-side), used only through its numerical gradient."""
    J = np.linalg.det(F)
    I1 = np.sum(F * F)
    return 0.5 * G * (J ** (-2.0 / 3.0) * I1 - 3.0) + 0.5 * K * (J - 1.0) ** 2


def _rand_F(rng, amp, plane=False):
    F = np.eye(3) + amp * rng.standard_normal((3, 3))
    if plane:
        F[2, :] = 0.0
        F[:, 2] = 0.0
        F[2, 2] = 1.0
    if np.linalg.det(F) <= 0.2:
        F = np.eye(3) + 0.1 * (F - np.eye(3))
    return F


def _rot3(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@pytest.mark.parametrize("plane", [False, True])
def test_stress_is_gradient_of_energy(plane):
    """Eq. 7 (elastic part) equals dW_e/dF of Eq. 4 by central differences."""
    G, K = orc.moduli(1.0, 0.3)
    rng = np.random.default_rng(11)
    for trial in range(20):
        F = _rand_F(rng, 0.3, plane)
        P = orc.stress_elastic(F, G, K)
        h = 1e-6
        fd = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                if plane and (i == 2 or j == 2):
                    continue
                E = np.zeros((3, 3)); E[i, j] = h
                fd[i, j] = (_W_e(F + E, G, K) - _W_e(F - E, G, K)) / (2 * h)
        if plane:
            P = P[:2, :2]; fd = fd[:2, :2]
        assert np.max(np.abs(P - fd)) <= 1e-8 * max(1.0, np.max(np.abs(P)))


def test_moduli_from_E_nu():
    """G = E / (2(1+nu)), K = E / (3(1-2nu)): the Lame pair of linear elasticity."""
    G, K = orc.moduli(1.0, 0.3)
    assert G == pytest.approx(1.0 / 2.6, rel=1e-15)
    assert K == pytest.approx(1.0 / 1.2, rel=1e-15)


def test_zero_stress_at_rest_and_under_rotation():
    G, K = orc.moduli(1.0, 0.3)
    assert np.max(np.abs(orc.stress_elastic(np.eye(3), G, K))) < 1e-15
    rng = np.random.default_rng(3)
    for _ in range(10):
        R = _rot3(rng)
        assert np.max(np.abs(orc.stress_elastic(R, G, K))) < 1e-13
    # plane strain: an in-plane rotation embedded with F33 = 1 is stress free
    for th in (0.1, 0.7, 2.5):
        R = np.eye(3)
        R[:2, :2] = [[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]]
        assert np.max(np.abs(orc.stress_elastic(R, G, K))) < 1e-13


def test_objectivity():
    """P(R F) = R P(F) for any rotation R (frame indifference of Eq. 4)."""
    G, K = orc.moduli(1.0, 0.3)
    rng = np.random.default_rng(5)
    for _ in range(10):
        F = _rand_F(rng, 0.25)
        R = _rot3(rng)
        lhs = orc.stress_elastic(R @ F, G, K)
        rhs = R @ orc.stress_elastic(F, G, K)
        assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_small_strain_limit_is_linear_elasticity():
    """P(I + eps S) / eps -> lambda tr(S) I + 2 G sym(S), lambda = K - 2G/3."""
    G, K = orc.moduli(1.0, 0.3)
    lam = K - 2.0 * G / 3.0
    rng = np.random.default_rng(7)
    S = rng.standard_normal((3, 3))
    S = 0.5 * (S + S.T)
    lin = lam * np.trace(S) * np.eye(3) + 2.0 * G * S
    errs = []
    for eps in (1e-3, 1e-4):
        P = orc.stress_elastic(np.eye(3) + eps * S, G, K) / eps
        errs.append(np.max(np.abs(P - lin)))
    assert errs[1] < 2e-3
    assert errs[1] < 0.2 * errs[0]  # error is O(eps)


def test_simple_shear_and_uniaxial_closed_forms():
    """Hand-derived closed forms of Eq. 7 for two deformations.

    Simple shear F = I + g e1 e2^T (J = 1, I1 = 3 + g^2):
      P11 = P22 = P33 = -G g^2 / 3, P12 = G g, P21 = G g (3 + g^2) / 3.
    Uniaxial stretch F = diag(l, 1, 1) (J = l, I1 = l^2 + 2):
      P11 = G l^{-2/3} (2 l^2 - 2) / (3 l) + K (l - 1)."""
    G, K = 0.7, 2.3
    g = 0.4
    F = np.eye(3); F[0, 1] = g
    P = orc.stress_elastic(F, G, K)
    assert P[0, 0] == pytest.approx(-G * g * g / 3, rel=1e-13)
    assert P[1, 1] == pytest.approx(-G * g * g / 3, rel=1e-13)
    assert P[2, 2] == pytest.approx(-G * g * g / 3, rel=1e-13)
    assert P[0, 1] == pytest.approx(G * g, rel=1e-13)
    assert P[1, 0] == pytest.approx(G * g * (3 + g * g) / 3, rel=1e-13)
    l = 1.3
    P = orc.stress_elastic(np.diag([l, 1.0, 1.0]), G, K)
    assert P[0, 0] == pytest.approx(G * l ** (-2 / 3) * (2 * l * l - 2) / (3 * l) + K * (l - 1), rel=1e-13)


def test_stress_tangent_matches_fd_and_is_symmetric():
    """dP_e[dF] (used by the adjoint) against central FD of P_e, and
    <A, dP[B]> = <B, dP[A]> (Hessian of W_e)."""
    G, K = orc.moduli(1.0, 0.3)
    rng = np.random.default_rng(9)
    for _ in range(10):
        F = _rand_F(rng, 0.3)
        A = rng.standard_normal((3, 3)); B = rng.standard_normal((3, 3))
        h = 1e-6
        fd = (orc.stress_elastic(F + h * A, G, K) - orc.stress_elastic(F - h * A, G, K)) / (2 * h)
        dP = orc.stress_elastic_dir(F, G, K, A)
        assert np.max(np.abs(dP - fd)) <= 1e-7 * max(1.0, np.max(np.abs(dP)))
        lhs = np.sum(A * orc.stress_elastic_dir(F, G, K, B))
        rhs = np.sum(B * orc.stress_elastic_dir(F, G, K, A))
        assert lhs == pytest.approx(rhs, rel=1e-11, abs=1e-12)


def test_bspline_golden_values():
    data = json.load(open(os.path.join(GOLDEN, "bspline_quadratic.json")))
    for case in data["cases"]:
        w, _ = orc.bspline(case["f"])
        assert np.allclose(w, case["w"], atol=1e-15, rtol=0)


def test_bspline_moment_identities_and_derivative():
    """sum w = 1, sum w (a - f) = 0, sum w (a - f)^2 = 1/4 for f in [1/2, 3/2), and
    the weight derivative is the derivative of the weights."""
    for f in np.linspace(0.5, 1.5, 41, endpoint=False):
        w, dw = orc.bspline(f)
        a = np.arange(3.0)
        assert abs(w.sum() - 1.0) < 1e-15
        assert abs(np.sum(w * (a - f))) < 1e-15
        assert abs(np.sum(w * (a - f) ** 2) - 0.25) < 1e-15
        h = 1e-7
        fd = (orc.bspline(f + h)[0] - orc.bspline(f - h)[0]) / (2 * h)
        assert np.max(np.abs(fd - dw)) < 1e-8
