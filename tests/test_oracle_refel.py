"""Pins of the oracle's reference element and tableaux against closed forms.

Reference element: paper §2 eqs. soln.points, diff.matrix; App. B eq.
correction.identities (g_R' = l_p(1)/w_p, g_L' = -l_p(0)/w_p, which the oracle
does NOT use: it differentiates the Radau polynomials directly).
Tableaux: Butcher's order conditions (textbook), and the linear time-average
weights b^T A^k 1 = 1/(k+1)! the linear equivalence of §5 rests on.
"""
import math

import numpy as np
import pytest

import oracle

# Gauss-Legendre nodes/weights on [-1, 1] in closed form (textbook values)
GL_CLOSED = {
    0: ([0.0], [2.0]),
    1: ([-1 / math.sqrt(3), 1 / math.sqrt(3)], [1.0, 1.0]),
    2: ([-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)], [5 / 9, 8 / 9, 5 / 9]),
    3: (
        [-math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5)), -math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)),
         math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)), math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))],
        [(18 - math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36, (18 - math.sqrt(30)) / 36],
    ),
    4: (
        [-1 / 3 * math.sqrt(5 + 2 * math.sqrt(10 / 7)), -1 / 3 * math.sqrt(5 - 2 * math.sqrt(10 / 7)), 0.0,
         1 / 3 * math.sqrt(5 - 2 * math.sqrt(10 / 7)), 1 / 3 * math.sqrt(5 + 2 * math.sqrt(10 / 7))],
        [(322 - 13 * math.sqrt(70)) / 900, (322 + 13 * math.sqrt(70)) / 900, 128 / 225,
         (322 + 13 * math.sqrt(70)) / 900, (322 - 13 * math.sqrt(70)) / 900],
    ),
}


@pytest.mark.parametrize("N", [0, 1, 2, 3, 4])
def test_gl_nodes_weights_closed_form(N):
    re = oracle.refel(N)
    x, W = GL_CLOSED[N]
    np.testing.assert_allclose(re["xi"], (np.array(x) + 1) / 2, atol=1e-15)
    np.testing.assert_allclose(re["w"], np.array(W) / 2, atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_quadrature_exactness(N):
    re = oracle.refel(N)
    for k in range(2 * N + 2):
        assert abs(np.sum(re["w"] * re["xi"] ** k) - 1 / (k + 1)) < 1e-15
    k = 2 * N + 2
    assert abs(np.sum(re["w"] * re["xi"] ** k) - 1 / (k + 1)) > 1e-6


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_diff_matrix_exact_on_polynomials(N):
    re = oracle.refel(N)
    x = re["xi"]
    for k in range(N + 1):
        d = k * x ** (k - 1) if k > 0 else 0 * x
        np.testing.assert_allclose(re["D"] @ x**k, d, atol=2e-13)
    # D^{N+1} vanishes on P_N up to round-off relative to |D|^{N+1}
    Dn = np.linalg.matrix_power(re["D"], N + 1)
    assert np.abs(Dn).max() < 1e-12 * np.abs(re["D"]).max() ** (N + 1)


@pytest.mark.parametrize("N", [0, 1, 2, 3, 4])
def test_boundary_interpolation(N):
    re = oracle.refel(N)
    for k in range(N + 1):
        assert abs(re["VL"] @ re["xi"] ** k - (1.0 if k == 0 else 0.0)) < 1e-13
        assert abs(re["VR"] @ re["xi"] ** k - 1.0) < 1e-13


@pytest.mark.parametrize("N", [0, 1, 2, 3, 4])
def test_radau_correction_identities(N):
    """App. B eq. correction.identities: g_R'(xi_p) = l_p(1)/w_p, g_L'(xi_p) = -l_p(0)/w_p."""
    re = oracle.refel(N)
    np.testing.assert_allclose(re["gRp"], re["VR"] / re["w"], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(re["gLp"], -re["VL"] / re["w"], rtol=1e-13, atol=1e-13)
    assert abs(np.sum(re["w"] * re["gRp"]) - 1) < 1e-14
    assert abs(np.sum(re["w"] * re["gLp"]) + 1) < 1e-14


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_orthonormal_legendre(N):
    re = oracle.refel(N)
    L = re["Leg"]
    G = (L * re["w"]) @ L.T
    np.testing.assert_allclose(G, np.eye(N + 1), atol=1e-14)


def _order_conditions(A, b, p):
    """Butcher's order conditions for every rooted tree up to order p (p <= 5)."""
    c = A.sum(axis=1)
    Ac = A @ c
    conds = [(b.sum(), 1.0)]
    if p >= 2:
        conds += [(b @ c, 1 / 2)]
    if p >= 3:
        conds += [(b @ c**2, 1 / 3), (b @ Ac, 1 / 6)]
    if p >= 4:
        conds += [(b @ c**3, 1 / 4), (b @ (c * Ac), 1 / 8), (b @ (A @ c**2), 1 / 12), (b @ (A @ Ac), 1 / 24)]
    if p >= 5:
        conds += [(b @ c**4, 1 / 5), (b @ (c**2 * Ac), 1 / 10), (b @ (c * (A @ c**2)), 1 / 15),
                  (b @ (c * (A @ Ac)), 1 / 30), (b @ Ac**2, 1 / 20), (b @ (A @ c**3), 1 / 20),
                  (b @ (A @ (c * Ac)), 1 / 40), (b @ (A @ (A @ c**2)), 1 / 60), (b @ (A @ (A @ Ac)), 1 / 120)]
    return conds


@pytest.mark.parametrize("N", [0, 1, 2, 3, 4])
def test_tableau_order(N):
    A, b = oracle.tableau(N)
    assert np.allclose(np.triu(A), 0)
    for got, want in _order_conditions(A, b, N + 1):
        assert abs(got - want) < 1e-14
    # the linear time-average weights
    one = np.ones(len(b))
    Ak = np.eye(len(b))
    for k in range(N + 1):
        assert abs(b @ Ak @ one - 1 / math.factorial(k + 1)) < 1e-14
        Ak = Ak @ A


def test_tableau_of_ht112_and_ssp():
    """N=1 and N=2 are the explicit parts of App. C eqs. ht112.butcher and ssp33.butcher."""
    A, b = oracle.tableau(1)
    np.testing.assert_array_equal(A, [[0, 0], [1, 0]])
    np.testing.assert_array_equal(b, [0.5, 0.5])
    A, b = oracle.tableau(2)
    np.testing.assert_allclose(A, [[0, 0, 0], [1, 0, 0], [0.25, 0.25, 0]])
    np.testing.assert_allclose(b, [1 / 6, 1 / 6, 2 / 3])


@pytest.mark.parametrize("N,expect", [(0, 1.0), (1, 1 / 3)])
def test_cfl_closed_forms(N, expect):
    """N=0 is first-order upwind (CFL 1); N=1 is the LW-D2 limit 1/3."""
    assert abs(oracle.cfl_number(N) - expect) < 1e-8
