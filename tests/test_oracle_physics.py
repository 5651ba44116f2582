"""Pins of the oracle's equation systems.

* Wave speeds: the spectral radius of f_d'(u) + B_d(u) (eq. combined.wave.speed)
  is compared with the eigenvalues of a central-difference Jacobian plus the
  B matrix assembled column by column, on random admissible states.
* Primitive forms: the conservative-plus-non-conservative system, evaluated as
  u_t = -(f'(u) + B(u)) u_x with a finite-difference Jacobian, must reproduce the
  textbook primitive equations (shallow water over a bed; for GLM-MHD with the
  Powell and GLM terms the pressure equation p_t + v p_x + gamma p (v1)_x = 0,
  rho(v_t + v1 v_x) = -p_x e1 + (curl B) x B, psi_t + c_h B1_x + v1 psi_x = 0).
  A dropped term or a wrong sign anywhere in f or B breaks one of them.
"""
import numpy as np
import pytest

import oracle

G = 9.81
GAM = 5.0 / 3.0


def fd_jacobian(eq, d, u, ch, h=1e-6):
    n = len(u)
    J = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = h * max(1.0, abs(u[j]))
        fp = oracle.physics(eq, "flux", d, u + e, gamma=GAM, gravity=G, ch=ch)
        fm = oracle.physics(eq, "flux", d, u - e, gamma=GAM, gravity=G, ch=ch)
        J[:, j] = (fp - fm) / (2 * e[j])
    return J


def bmatrix(eq, d, u):
    n = len(u)
    B = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        B[:, j] = oracle.physics(eq, "nc", d, u, e, gamma=GAM, gravity=G)
    return B


def rand_mhd(rng):
    rho = 10 ** rng.uniform(-1, 0.5)
    v = rng.uniform(-2, 2, 3)
    p = 10 ** rng.uniform(-2, 0.5)
    B = rng.uniform(-1.5, 1.5, 3)
    psi = rng.uniform(-0.3, 0.3)
    E = p / (GAM - 1) + 0.5 * rho * v @ v + 0.5 * B @ B + 0.5 * psi**2
    return np.array([rho, *(rho * v), E, *B, psi])


def rand_sw(rng, dim):
    h = 10 ** rng.uniform(-1, 0.5)
    v = rng.uniform(-2, 2, dim)
    b = rng.uniform(-1, 1)
    return np.array([h, *(h * v), b])


@pytest.mark.parametrize("eq,dim", [(oracle.EQ_SW1D, 1), (oracle.EQ_SW2D, 2), (oracle.EQ_MHD2D, 2)])
def test_sigma_is_spectral_radius(eq, dim):
    rng = np.random.default_rng(7)
    for trial in range(300):
        u = rand_mhd(rng) if eq == oracle.EQ_MHD2D else rand_sw(rng, dim)
        for d in range(dim):
            for ch in ([0.0] if eq != oracle.EQ_MHD2D else [0.0, rng.uniform(0, 4)]):
                A = fd_jacobian(eq, d, u, ch) + bmatrix(eq, d, u)
                lam = np.max(np.abs(np.linalg.eigvals(A)))
                sig = oracle.physics(eq, "sigma", d, u, gamma=GAM, gravity=G, ch=ch)[0]
                assert abs(lam - sig) <= 1e-6 * max(1.0, sig), (trial, d, ch, lam, sig)


@pytest.mark.parametrize("eq,dim", [(oracle.EQ_SW1D, 1), (oracle.EQ_SW2D, 2), (oracle.EQ_MHD2D, 2),
                                    (oracle.EQ_LINADV1D, 1), (oracle.EQ_VARADV1D, 1)])
def test_nonzero_columns_of_B(eq, dim):
    """The columns of B_d the stage loop differentiates are exactly the non-zero ones."""
    rng = np.random.default_rng(2)
    n = oracle.NVARS[eq]
    for d in range(dim):
        nz = np.zeros(n, dtype=bool)
        for _ in range(20):
            u = rand_mhd(rng) if eq == oracle.EQ_MHD2D else (
                rand_sw(rng, dim) if eq in (oracle.EQ_SW1D, oracle.EQ_SW2D) else rng.uniform(0.5, 2, n))
            nz |= np.abs(bmatrix(eq, d, u)).max(axis=0) > 0
        assert sorted(np.nonzero(nz)[0].tolist()) == oracle.ncols(eq, d)


def test_varadv_sigma_and_structure():
    u = np.array([0.3, -1.7])
    A = bmatrix(oracle.EQ_VARADV1D, 0, u)
    np.testing.assert_array_equal(A, [[-1.7, 0.0], [0.0, 0.0]])
    assert oracle.physics(oracle.EQ_VARADV1D, "sigma", 0, u)[0] == 1.7


def _dudt(eq, d, u, ux, ch=0.0):
    A = fd_jacobian(eq, d, u, ch) + bmatrix(eq, d, u)
    return -A @ ux


@pytest.mark.parametrize("dim", [1, 2])
def test_shallow_water_primitive_form(dim):
    """h_t + (hv_d)_x = 0 and v_t + v_d v_x + g (h + b)_x e_d = 0 for variation along x_d."""
    eq = oracle.EQ_SW1D if dim == 1 else oracle.EQ_SW2D
    rng = np.random.default_rng(3)
    for _ in range(50):
        h = rng.uniform(0.5, 2)
        v = rng.uniform(-1, 1, dim)
        b = rng.uniform(-1, 1)
        hx, bx = rng.normal(size=2)
        vx = rng.normal(size=dim)
        u = np.array([h, *(h * v), b])
        ux = np.array([hx, *(hx * v + h * vx), bx])
        for d in range(dim):
            if d == 1:  # variation along y: reuse the same derivatives as y-derivatives
                pass
            ut = _dudt(eq, d, u, ux)
            ht = ut[0]
            vt = (ut[1 : 1 + dim] - v * ht) / h
            assert abs(ht + ux[1 + d]) < 1e-7
            want = -v[d] * vx
            want[d] -= G * (hx + bx)
            np.testing.assert_allclose(vt, want, atol=1e-6)
            assert abs(ut[-1]) < 1e-12


def test_mhd_primitive_form():
    """Variation along x only: the conservative GLM-MHD system with the Powell and
    GLM terms must give the primitive ideal-MHD evolution plus the GLM pair."""
    rng = np.random.default_rng(11)
    eq = oracle.EQ_MHD2D
    for _ in range(100):
        rho = rng.uniform(0.5, 2)
        v = rng.uniform(-1, 1, 3)
        p = rng.uniform(0.3, 2)
        B = rng.uniform(-1, 1, 3)
        psi = rng.uniform(-0.2, 0.2)
        ch = rng.uniform(0.1, 3)
        rx, px, psix = rng.normal(size=3)
        vx = rng.normal(size=3)
        Bx = rng.normal(size=3)  # includes a non-zero div B = (B1)_x
        E = p / (GAM - 1) + 0.5 * rho * v @ v + 0.5 * B @ B + 0.5 * psi**2
        Ex = px / (GAM - 1) + 0.5 * rx * v @ v + rho * v @ vx + B @ Bx + psi * psix
        u = np.array([rho, *(rho * v), E, *B, psi])
        ux = np.array([rx, *(rx * v + rho * vx), Ex, *Bx, psix])
        ut = _dudt(eq, 0, u, ux, ch)
        rt = ut[0]
        vt = (ut[1:4] - v * rt) / rho
        Bt = ut[5:8]
        psit = ut[8]
        Et = ut[4]
        pt = (GAM - 1) * (Et - 0.5 * rt * v @ v - rho * v @ vt - B @ Bt - psi * psit)
        tol = 2e-6
        assert abs(rt + v[0] * rx + rho * vx[0]) < tol
        assert abs(pt + v[0] * px + GAM * p * vx[0]) < tol
        J = np.array([0.0, -Bx[2], Bx[1]])  # curl B for x-variation
        lorentz = np.cross(J, B)
        want_vt = -v[0] * vx + lorentz / rho
        want_vt[0] -= px / rho
        np.testing.assert_allclose(vt, want_vt, atol=tol)
        assert abs(psit + ch * Bx[0] + v[0] * psix) < tol
        assert abs(Bt[0] + ch * psix + v[0] * Bx[0]) < tol
        # induction for the transverse components: B_t = curl(v x B) - v div B
        for i in (1, 2):
            want = -(vx[0] * B[i] + v[0] * Bx[i] - Bx[0] * v[i] - B[0] * vx[i]) - v[i] * Bx[0]
            assert abs(Bt[i] - want) < tol


def test_mhd_euler_limit():
    """With B = 0 and psi = 0 the GLM-MHD flux is the Euler flux."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        rho, p = rng.uniform(0.5, 2, 2)
        v = rng.uniform(-1, 1, 3)
        E = p / (GAM - 1) + 0.5 * rho * v @ v
        u = np.array([rho, *(rho * v), E, 0, 0, 0, 0])
        for d in range(2):
            f = oracle.physics(oracle.EQ_MHD2D, "flux", d, u, gamma=GAM, ch=0.7)
            want = np.zeros(9)
            want[0] = rho * v[d]
            want[1:4] = rho * v[d] * v
            want[1 + d] += p
            want[4] = v[d] * (E + p)
            np.testing.assert_allclose(f, want, atol=1e-14)


def test_constraints():
    u = rand_mhd(np.random.default_rng(1))
    c = oracle.physics(oracle.EQ_MHD2D, "constraints", 0, u, gamma=GAM)
    rho, m, E, B, psi = u[0], u[1:4], u[4], u[5:8], u[8]
    p = (GAM - 1) * (E - 0.5 * m @ m / rho - 0.5 * B @ B - 0.5 * psi**2)
    np.testing.assert_allclose(c, [rho, p], rtol=1e-14)
