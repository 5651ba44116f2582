"""Pins of the oracle's time step against what the paper and the mathematics fix.

* free-stream preservation (constant states are steady);
* conservation to round-off of every variable whose non-conservative row is zero
  (§4 below eq. numflux.args: the shared face flux keeps the scheme conservative);
* linear equivalence with the Lax-Wendroff FR scheme (§5 CFL paragraph): for
  f = u the step equals the closed-form Taylor operator, independent of the
  tableau (App. B/§2 construction written as a matrix polynomial);
* Fourier CFL(N): a run at 0.95 CFL stays bounded, one at 1.05 CFL blows up;
* N = 0 reduces to the first order finite volume scheme (App. B eq. fr.fv),
  compared with a plain FV step written here;
* alpha = 1 is the subcell FV scheme (eq. low.order.update), compared with a
  plain subcell FV step written here;
* admissibility: every output state is admissible with Algorithms 1-2 on blocky
  data, also with a 10x time step whenever the lower order update is admissible;
* lake at rest over a continuous, element-wise linear bed is kept to round-off;
* design order on smooth closed-form solutions (Alfven wave, periodic
  variable-coefficient advection);
* forward-mode J v agrees with central finite differences of the step.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2512_08611_amd import workloads as W

G = 9.81
GAM = 5.0 / 3.0


def mass(c, u):
    re = oracle.refel(c.N)
    w = re["w"]
    wn = w if oracle.DIMS[c.eq] == 1 else np.outer(w, w).reshape(-1)
    return (u * wn).sum(axis=(1, 2))


# --------------------------------------------------------- free stream ----
CONST = {
    oracle.EQ_SW1D: np.array([1.3, 0.4, 0.2]),
    oracle.EQ_SW2D: np.array([1.3, 0.4, -0.3, 0.2]),
    oracle.EQ_MHD2D: np.array([1.3, 0.2, -0.1, 0.05, 3.0, 0.4, -0.3, 0.2, 0.01]),
    oracle.EQ_LINADV1D: np.array([0.7]),
    oracle.EQ_VARADV1D: np.array([0.7, 1.2]),
}


@pytest.mark.parametrize("eq", list(CONST))
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_free_stream(eq, N):
    c = oracle.make_cfg(eq, N, 3, 3, blending=2)
    shp = oracle.shape(c)
    u = np.broadcast_to(CONST[eq].reshape(-1, 1, 1), shp).copy()
    r = oracle.step(c, u)
    np.testing.assert_allclose(r["u"], u, atol=1e-14 * np.abs(u).max())
    assert r["flags"].max() == 0


# -------------------------------------------------------- conservation ----
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_conservation_mhd_blocky(N):
    c = oracle.make_cfg(oracle.EQ_MHD2D, N, 6, 6, blending=2)
    re = oracle.refel(N)
    u = W.mhd_blocky(re["xi"], 6, seed=1, nblocks=3)
    r = oracle.step(c, u)
    m0, m1 = mass(c, u), mass(c, r["u"])
    assert abs(m1[0] - m0[0]) < 1e-14 * abs(m0[0])  # rho has a zero non-conservative row


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_conservation_euler_limit(N):
    """B = psi = 0 makes every non-conservative product vanish: all variables conserved."""
    c = oracle.make_cfg(oracle.EQ_MHD2D, N, 5, 5, blending=2)
    re = oracle.refel(N)
    u = W.mhd_blocky(re["xi"], 5, seed=2, nblocks=3)
    u[5:9] = 0.0
    rho, m, p = u[0], u[1:4], None
    u[4] = u[4] - 0.0  # E already excludes magnetic energy after zeroing B? rebuild it:
    r0 = W.mhd_blocky(re["xi"], 5, seed=2, nblocks=3)
    Bsq = (r0[5:8] ** 2).sum(axis=0)
    u[4] = r0[4] - 0.5 * Bsq
    r = oracle.step(c, u)
    m0, m1 = mass(c, u), mass(c, r["u"])
    assert r["flags"].max() & oracle.FLAG_NONFINITE == 0
    np.testing.assert_allclose(m1, m0, atol=2e-14 * np.abs(m0).max())


@pytest.mark.parametrize("N", [1, 3])
def test_conservation_sw(N):
    re = oracle.refel(N)
    c = oracle.make_cfg(oracle.EQ_SW2D, N, 5, 5, blending=2)
    u = W.sw2d_random(re["xi"], 5, seed=3)
    r = oracle.step(c, u)
    m0, m1 = mass(c, u), mass(c, r["u"])
    assert abs(m1[0] - m0[0]) < 1e-14 * m0[0]
    # b = 0: B(u) u = g h b vanishes, so momentum is conserved too.  (A constant
    # non-zero b is not enough: the interface term B(u^{n,±}) U^num of eq.
    # good.numflux.non.cons and the stage average F^nc differ by g b (h^n - H).)
    u[3] = 0.0
    r = oracle.step(c, u)
    m0, m1 = mass(c, u), mass(c, r["u"])
    np.testing.assert_allclose(m1, m0, atol=1e-14 * np.abs(m0).max())


# ------------------------------------------------- linear equivalence ----
def lw_closed_form_step(u, N, nu):
    """u_e <- u_e - nu [D T u_e + g_L'(V_R^T T u_{e-1} - V_L^T T u_e) + g_R'(V_R^T T u_e - V_R^T T u_e)]
    with T = sum_k (-nu D)^k/(k+1)!: the Taylor (Lax-Wendroff) time average for f = u."""
    re = oracle.refel(N)
    D = re["D"]
    T = sum(np.linalg.matrix_power(-nu * D, k) / math.factorial(k + 1) for k in range(N + 1))
    Tu = u @ T.T  # [E, P]
    left = np.roll(Tu, 1, axis=0) @ re["VR"]
    return u - nu * (Tu @ D.T + np.outer(left - Tu @ re["VL"], re["gLp"]))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_linear_equivalence_with_lw(N):
    nx = 7
    c = oracle.make_cfg(oracle.EQ_LINADV1D, N, nx, blending=0)
    rng = np.random.default_rng(N)
    u = rng.normal(size=(1, nx, N + 1))
    dx = 1.0 / nx
    nu = 0.8 * oracle.cfl_number(N)
    r = oracle.step(c, u, dt=nu * dx)
    np.testing.assert_allclose(r["u"][0], lw_closed_form_step(u[0], N, nu), atol=1e-13)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_fourier_cfl_limit(N):
    nx = 16
    c = oracle.make_cfg(oracle.EQ_LINADV1D, N, nx, blending=0)
    rng = np.random.default_rng(0)
    u0 = rng.normal(size=(1, nx, N + 1))
    cfl = oracle.cfl_number(N)
    for fac, stable in ((0.95, True), (1.05, False)):
        u = u0.copy()
        for _ in range(400):
            u = oracle.step(c, u, dt=fac * cfl / nx)["u"]
        growth = np.abs(u).max() / np.abs(u0).max()
        assert (growth < 1.5) == stable, (fac, growth)


# ------------------------------------------------ N = 0 and alpha = 1 ----
def rusanov_pm(eq, d, uL, uR, ch=0.0):
    """f^{num,-}, f^{num,+} of eq. combined.num.flux written out for one pair of states."""
    ph = lambda what, u, w=None: oracle.physics(eq, what, d, u, w, gamma=GAM, gravity=G, ch=ch)
    lam = max(ph("sigma", uL)[0], ph("sigma", uR)[0])
    fc = 0.5 * (ph("flux", uL) + ph("flux", uR)) - 0.5 * lam * (uR - uL)
    avg = 0.5 * (uL + uR)
    return fc + ph("nc", uL, avg), fc + ph("nc", uR, avg)


@pytest.mark.parametrize("eq", [oracle.EQ_SW1D, oracle.EQ_VARADV1D])
def test_n0_is_first_order_fv(eq):
    nx = 9
    rng = np.random.default_rng(2)
    if eq == oracle.EQ_SW1D:
        u = np.stack([1 + 0.3 * rng.random(nx), 0.2 * rng.normal(size=nx), 0.2 * rng.random(nx)])[:, :, None]
    else:
        u = np.stack([rng.normal(size=nx), 1 + 0.3 * rng.random(nx)])[:, :, None]
    c = oracle.make_cfg(eq, 0, nx, blending=0)
    dt = 0.01
    r = oracle.step(c, u, dt=dt)
    dx = 1.0 / nx
    want = np.zeros_like(u)
    for e in range(nx):
        ue, ur, ul = u[:, e, 0], u[:, (e + 1) % nx, 0], u[:, (e - 1) % nx, 0]
        fm, _ = rusanov_pm(eq, 0, ue, ur)
        _, fp = rusanov_pm(eq, 0, ul, ue)
        want[:, e, 0] = ue - dt / dx * (fm - fp)
    np.testing.assert_allclose(r["u"], want, atol=1e-14)


def subcell_fv_1d(eq, u, dt, w, dx):
    """Plain subcell FV step (subcell p of width w_p dx), lower order fluxes at every subface."""
    M, E, P = u.shape
    flat = u.transpose(0, 1, 2).reshape(M, E * P)
    wid = np.tile(w, E) * dx
    out = np.zeros_like(flat)
    n = E * P
    for i in range(n):
        fm, _ = rusanov_pm(eq, 0, flat[:, i], flat[:, (i + 1) % n])
        _, fp = rusanov_pm(eq, 0, flat[:, (i - 1) % n], flat[:, i])
        out[:, i] = flat[:, i] - dt / wid[i] * (fm - fp)
    return out.reshape(M, E, P)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_alpha_one_is_subcell_fv_1d(N):
    nx = 6
    re = oracle.refel(N)
    u = W.sw1d_wave(re["xi"], nx, seed=4)
    c = oracle.make_cfg(oracle.EQ_SW1D, N, nx, blending=1, alpha_force=1.0)
    dt = 1e-3
    r = oracle.step(c, u, dt=dt)
    np.testing.assert_allclose(r["u"], subcell_fv_1d(oracle.EQ_SW1D, u, dt, re["w"], 1.0 / nx), atol=1e-14)


@pytest.mark.parametrize("N", [1, 3])
def test_alpha_one_is_subcell_fv_2d(N):
    n = 3
    re = oracle.refel(N)
    u = W.sw2d_random(re["xi"], n, seed=5)
    c = oracle.make_cfg(oracle.EQ_SW2D, N, n, n, blending=1, alpha_force=1.0)
    dt = 1e-3
    r = oracle.step(c, u, dt=dt)
    n1 = N + 1
    # assemble the global subcell grid [var][Y][X]
    M = u.shape[0]
    g = u.reshape(M, n, n, n1, n1).transpose(0, 1, 3, 2, 4).reshape(M, n * n1, n * n1)
    wid = np.tile(re["w"], n) / n
    want = g.copy()
    X = n * n1
    for j in range(X):
        for i in range(X):
            s = g[:, j, i]
            fmx, _ = rusanov_pm(oracle.EQ_SW2D, 0, s, g[:, j, (i + 1) % X])
            _, fpx = rusanov_pm(oracle.EQ_SW2D, 0, g[:, j, (i - 1) % X], s)
            fmy, _ = rusanov_pm(oracle.EQ_SW2D, 1, s, g[:, (j + 1) % X, i])
            _, fpy = rusanov_pm(oracle.EQ_SW2D, 1, g[:, (j - 1) % X, i], s)
            want[:, j, i] = s - dt * ((fmx - fpx) / wid[i] + (fmy - fpy) / wid[j])
    got = r["u"].reshape(M, n, n, n1, n1).transpose(0, 1, 3, 2, 4).reshape(M, X, X)
    np.testing.assert_allclose(got, want, atol=1e-14)


# ------------------------------------------------------ admissibility ----
@pytest.mark.parametrize("N", [2, 3, 4])
def test_admissible_output_blocky_mhd(N):
    n = 8
    re = oracle.refel(N)
    u = W.mhd_blocky(re["xi"], n, seed=0, nblocks=4)
    c = oracle.make_cfg(oracle.EQ_MHD2D, N, n, n, blending=2)
    for _ in range(3):
        r = oracle.step(c, u)
        u = r["u"]
        assert (r["flags"] & oracle.FLAG_LOW_INADM).max() == 0
        for e in range(u.shape[1]):
            for p in range(u.shape[2]):
                rho, pr = oracle.physics(oracle.EQ_MHD2D, "constraints", 0, u[:, e, p], gamma=GAM)
                assert rho > 0 and pr > 0
    assert (r["flags"] & oracle.FLAG_ALG1).any() or (r["flags"] & oracle.FLAG_ALG2).any()


def test_admissibility_with_large_time_step():
    """With dt x10 Algorithm 2 still returns admissible states wherever u^L is admissible."""
    n, N = 8, 3
    re = oracle.refel(N)
    u = W.mhd_blocky(re["xi"], n, seed=3, nblocks=4)
    c = oracle.make_cfg(oracle.EQ_MHD2D, N, n, n, blending=2)
    dt0, ch = oracle.dt_ch(c, u)
    r = oracle.step(c, u, dt=3 * dt0)
    ok = (r["flags"] & oracle.FLAG_LOW_INADM) == 0
    assert ok.any()
    for e in np.nonzero(ok)[0]:
        for p in range(u.shape[2]):
            rho, pr = oracle.physics(oracle.EQ_MHD2D, "constraints", 0, r["u"][:, e, p], gamma=GAM)
            assert rho > 0 and pr > 0


def test_sw_positivity_near_dry():
    """Dam break into a thin layer: wherever the lower order update is admissible the
    output is admissible (Algorithm 2); the flag marks the rest, whose output is
    the inadmissible u^L itself, and the run stops there (its next input would be
    outside the admissible set the scheme is defined on)."""
    nx, N = 20, 3
    re = oracle.refel(N)
    x = W.coords_1d(re["xi"], nx)
    h = np.where((x > 0.3) & (x < 0.7), 1.0, 0.05)
    u = np.stack([h, 0.5 * h * np.sign(x - 0.5), 0 * h])
    c = oracle.make_cfg(oracle.EQ_SW1D, N, nx, blending=2, cs=0.9)
    limited = 0
    for n in range(40):
        r = oracle.step(c, u)
        ok = (r["flags"] & oracle.FLAG_LOW_INADM) == 0
        assert (r["u"][0][ok] > 0).all()
        limited += int(((r["flags"] & (oracle.FLAG_ALG1 | oracle.FLAG_ALG2)) != 0).sum())
        if not ok.all():
            break
        u = r["u"]
    assert n >= 10 and limited > 0


# ------------------------------------------------------ lake at rest -----
@pytest.mark.parametrize("N,blend", [(2, 0), (3, 2), (4, 2)])
def test_lake_at_rest_1d(N, blend):
    re = oracle.refel(N)
    u = W.sw1d_lake(re["xi"], 12, seed=1)
    c = oracle.make_cfg(oracle.EQ_SW1D, N, 12, blending=blend)
    r = oracle.step(c, u)
    np.testing.assert_allclose(r["u"], u, atol=1e-14)


@pytest.mark.parametrize("N,blend", [(2, 0), (3, 2)])
def test_lake_at_rest_2d(N, blend):
    n = 4
    re = oracle.refel(N)
    x, y = W.coords_2d(re["xi"], n, n)
    rng = np.random.default_rng(0)
    bv = 0.2 * rng.uniform(-1, 1, (n + 1, n + 1))
    bv[n, :] = bv[0, :]
    bv[:, n] = bv[:, 0]
    ix = np.minimum((x * n).astype(int), n - 1)
    iy = np.minimum((y * n).astype(int), n - 1)
    tx, ty = x * n - ix, y * n - iy
    b = (bv[iy, ix] * (1 - tx) * (1 - ty) + bv[iy, ix + 1] * tx * (1 - ty) + bv[iy + 1, ix] * (1 - tx) * ty
         + bv[iy + 1, ix + 1] * tx * ty)
    u = np.stack([1.0 - b, 0 * b, 0 * b, b])
    c = oracle.make_cfg(oracle.EQ_SW2D, N, n, n, blending=blend)
    r = oracle.step(c, u)
    np.testing.assert_allclose(r["u"], u, atol=2e-14)


# ------------------------------------------------------ design order -----
def _alfven_error(N, n, tend):
    re = oracle.refel(N)
    L = math.sqrt(2.0)
    c = oracle.make_cfg(oracle.EQ_MHD2D, N, n, n, lo=(0, 0), hi=(L, L), blending=0)
    u = W.alfven(re["xi"], n)
    t = 0.0
    dt, ch = oracle.dt_ch(c, u)
    nsteps = int(math.ceil(tend / dt))
    dt = tend / nsteps
    for _ in range(nsteps):
        u = oracle.step(c, u, dt=dt)["u"]
    ex = W.alfven(re["xi"], n, t=tend)
    wn = np.outer(re["w"], re["w"]).reshape(-1)
    return math.sqrt(((u[1] - ex[1]) ** 2 * wn).sum() * (L / n) ** 2)


@pytest.mark.parametrize("N,ns", [(1, (4, 8, 16)), (2, (4, 8, 12)), (3, (3, 6))])
def test_design_order_alfven(N, ns):
    errs = [_alfven_error(N, n, 0.2) for n in ns]
    rate = math.log(errs[-2] / errs[-1]) / math.log(ns[-1] / ns[-2])
    assert rate > N + 1 - 0.35, (errs, rate)


def _varadv_error(N, nx, tend):
    """Periodic variable-coefficient advection v_t + a(x) v_x = 0, a = 1 + sin(2pi x)/2:
    characteristics tau(x) = int_0^x ds/a(s); v(x,t) = v0(tau^{-1}(tau(x) - t))."""
    re = oracle.refel(N)
    c = oracle.make_cfg(oracle.EQ_VARADV1D, N, nx, blending=0)
    u = W.varadv_periodic(re["xi"], nx)
    x = W.coords_1d(re["xi"], nx)
    dt = 0.5 * oracle.cfl_number(N) / nx / 1.5
    nsteps = int(math.ceil(tend / dt))
    dt = tend / nsteps
    for _ in range(nsteps):
        u = oracle.step(c, u, dt=dt)["u"]
    # exact: tau(x) = int_0^x ds/(1 + sin(2 pi s)/2), period T0 = tau(1)
    gx, gw = np.polynomial.legendre.leggauss(40)

    def tau(xx):
        s = 0.5 * xx[..., None] * (gx + 1)
        return (0.5 * xx[..., None] * gw / (1 + 0.5 * np.sin(2 * math.pi * s))).sum(-1)

    T0 = tau(np.array(1.0))
    target = (tau(x) - tend) % T0
    xs = x.copy()
    for _ in range(60):  # Newton on tau(xs) = target
        xs = xs - (tau(xs) - target) * (1 + 0.5 * np.sin(2 * math.pi * xs))
    ex = np.sin(2 * math.pi * xs)
    return math.sqrt(((u[0] - ex) ** 2 * re["w"]).sum() / nx)


@pytest.mark.parametrize("N,ns", [(1, (16, 32)), (2, (16, 32)), (3, (8, 16))])
def test_design_order_varadv(N, ns):
    errs = [_varadv_error(N, n, 0.3) for n in ns]
    rate = math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0])
    assert rate > N + 1 - 0.35, (errs, rate)


# ---------------------------------------------------------- indicator ----
def test_indicator_special_cases():
    N, n = 3, 4
    re = oracle.refel(N)
    c = oracle.make_cfg(oracle.EQ_SW2D, N, n, n, blending=2, alpha_max=0.5)
    u = np.zeros((4, n * n, (N + 1) ** 2))
    u[0] = 1.0
    araw, al, _ = oracle.alpha(c, u)
    assert araw.max() == 0.0 and al.max() == 0.0
    # q = pure highest mode L_N(x) L_N(y) on element 5 (plus a constant elsewhere)
    LN = re["Leg"][N]
    u[0, 5] = 1.0 + 0.5 * np.outer(LN, LN).reshape(-1)
    araw, al, _ = oracle.alpha(c, u)
    assert araw[5] == 0.5
    assert al[5] == 0.5 and al[4] == 0.25 and al[6] == 0.25 and al[1] == 0.25 and al[9] == 0.25



@pytest.mark.parametrize("N", [2, 3, 4])
def test_indicator_energy_fractions_closed_form(N):
    """The raw indicator on nodal data built from chosen modal coefficients in the
    orthonormal Legendre basis (§4, Hennemann et al.'s indicator): with q =
    m00 + a B_hi + b B_lo, a mode of degree N and one of degree N-1, the energy
    fractions are a^2/(m00^2+a^2+b^2) and b^2/(m00^2+b^2) exactly, and E is the
    larger.  Targets around the threshold T(N) keep the logistic unclipped;
    the degree of mode (j, k) is max(j, k), so every placement of the two
    modes gives the same E."""
    n1 = N + 1
    re = oracle.refel(N)
    L = re["Leg"]
    T = 0.5 * 10.0 ** (-1.8 * (N + 1.0) ** 0.25)
    s = np.log(9999.0)
    m00 = 1.0 / L[0, 0]  # the constant mode that makes q's mean 1
    # (E_hi, E_lo, mode of degree N, mode of degree N-1); E_* = 0 leaves the mode out
    cases = [(T, 0.0, (N, 0), None), (0.8 * T, 0.0, (0, N), None), (1.3 * T, 0.0, (N, N), None),
             (0.0, T, None, (N - 1, 0)), (0.0, 1.2 * T, None, (N - 1, N - 1)), (0.0, 0.7 * T, None, (0, N - 1)),
             (0.9 * T, 1.1 * T, (N, 1), (1, N - 1)), (1.1 * T, 0.9 * T, (1, N), (N - 1, 0)),
             (0.5, 0.0, (N, N - 1), None), (0.0, 0.0, None, None)]
    n = 4
    c = oracle.make_cfg(oracle.EQ_SW2D, N, n, n, blending=2, alpha_max=1.0, alpha_min=1e-3)
    u = np.zeros((4, n * n, n1 * n1))
    u[0] = 1.0
    want = np.zeros(n * n)
    for e, (Ehi, Elo, hi, lo) in enumerate(cases):
        # b^2 = Elo m00^2/(1-Elo); then a^2 = Ehi (m00^2+b^2)/(1-Ehi)
        b2 = Elo * m00 ** 2 / (1.0 - Elo)
        a2 = Ehi * (m00 ** 2 + b2) / (1.0 - Ehi)
        m = np.zeros((n1, n1))  # m[l, k]: L_k(x) L_l(y)
        m[0, 0] = m00
        if hi is not None:
            m[hi[1], hi[0]] = np.sqrt(a2)
        if lo is not None:
            m[lo[1], lo[0]] = -np.sqrt(b2)
        q = np.einsum("lk,li,kj->ij", m, L, L)  # q[i][j] at node (x_j, y_i)
        u[0, e] = q.reshape(-1)
        E = max(Ehi, Elo)
        a = 1.0 / (1.0 + np.exp(-(s / T) * (E - T)))
        want[e] = 0.0 if a < 1e-3 else (1.0 if a > 1.0 - 1e-3 else a)
    araw, _, _ = oracle.alpha(c, u)
    # the unclipped cases span the logistic's active band
    assert 0.05 < want[1] < 0.5 < want[2] < 0.95 and want[0] == pytest.approx(0.5)
    assert want[8] == 1.0 and want[9] == 0.0
    np.testing.assert_allclose(araw[:len(cases)], want[:len(cases)], rtol=1e-9, atol=1e-12)
    # elements with constant data: E = 0, below alpha_min after the logistic
    assert np.all(araw[len(cases):] == 0.0)

# ----------------------------------------------------------- jvp / FD ----
@pytest.mark.parametrize("eq,N,blend", [(oracle.EQ_MHD2D, 3, 0), (oracle.EQ_MHD2D, 2, 2), (oracle.EQ_SW1D, 4, 2)])
def test_jvp_matches_central_difference(eq, N, blend):
    re = oracle.refel(N)
    if eq == oracle.EQ_MHD2D:
        n = 3
        c = oracle.make_cfg(eq, N, n, n, blending=blend)
        u = W.mhd_smooth(re["xi"], n, seed=1, amp=0.05)
    else:
        c = oracle.make_cfg(eq, N, 8, blending=blend)
        u = W.sw1d_wave(re["xi"], 8, seed=1)
    dt, ch = oracle.dt_ch(c, u)
    rng = np.random.default_rng(0)
    v = rng.normal(size=u.shape) * np.abs(u).mean(axis=(1, 2), keepdims=True)
    _, Jv = oracle.jvp(c, u, v, dt, ch)
    # central difference of the same frozen map: alpha held at its value at u; eps
    # small enough that no theta and no argmax switches
    al = oracle.step(c, u)["alpha"]
    eps = 1e-6
    up = oracle.step(c, u + eps * v, dt=dt, ch=ch, alpha_in=al)["u"]
    um = oracle.step(c, u - eps * v, dt=dt, ch=ch, alpha_in=al)["u"]
    fd = (up - um) / (2 * eps)
    assert np.abs(fd - Jv).max() < 1e-6 * np.abs(Jv).max()
