"""Pins of the oracle's reverse-mode derivative of the step (oracle/reverse.hpp).

The reverse mode tapes the oracle's own arithmetic one element or face line at
a time; these tests tie it to independent derivatives of the same frozen-switch
map (dt, c_h, alpha, every theta and every max/abs branch held at the values at
u):
  * the dot-product identity <lambda, J v> = <J^T lambda, v> against the Dual
    forward mode (a different scalar type and a different order of evaluation),
    for every system, degree and blending mode, smooth and blocky data;
  * whole Jacobians on two-element and 2 x 2 meshes, assembled column by column
    from the forward mode, against rows from the reverse mode, entry by entry;
  * the gradient of a three-step rollout against central differences of the
    same frozen map (smooth data: no theta below 1, so freezing is exact);
  * the same bits for any number of threads.
"""
import numpy as np
import pytest

import oracle
from paper_2512_08611_amd import workloads as W


def _data(eq, N, nx, ny, seed, kind):
    xi = oracle.refel(N)["xi"]
    rng = np.random.default_rng(seed)
    if eq == oracle.EQ_SW1D:
        u = W.sw1d_wave(xi, nx, seed)
        if kind == "rough":
            u[0] *= 1 + 0.2 * rng.uniform(-1, 1, u[0].shape)
        return u
    if eq == oracle.EQ_SW2D:
        u = W.sw2d_random(xi, nx, seed)
        u[1] = 0.2 * u[0] * rng.uniform(-1, 1, u[0].shape[0])[:, None]
        if kind == "rough":
            u[0] *= 1 + 0.3 * rng.uniform(-1, 1, u[0].shape)
        return u
    if eq == oracle.EQ_MHD2D:
        if kind == "smooth":
            return W.mhd_smooth(xi, nx, ny, seed, amp=0.05)
        u = W.mhd_blocky(xi, nx, ny, seed, nblocks=3)
        # moving blocks with a small per-node jitter: no exact tie between the two
        # face states of a max (where both one-sided derivatives are valid)
        gam = 5.0 / 3.0
        p = (gam - 1) * (u[4] - 0.5 * (u[5] ** 2 + u[6] ** 2 + u[7] ** 2))
        u[1:4] = 0.3 * rng.uniform(-1, 1, (3, u.shape[1], 1)) * u[0:1]
        u[8] = 0.05 * rng.uniform(-1, 1, (u.shape[1], 1))
        for v in (0, 1, 2, 3, 5, 6, 7, 8):
            u[v] = u[v] * (1 + 1e-3 * rng.uniform(-1, 1, u[v].shape)) + 1e-4 * rng.uniform(-1, 1, u[v].shape)
        u[4] = p / (gam - 1) + 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / u[0] \
            + 0.5 * (u[5] ** 2 + u[6] ** 2 + u[7] ** 2) + 0.5 * u[8] ** 2
        return u
    if eq == oracle.EQ_LINADV1D:
        return rng.normal(size=(1, nx, N + 1))
    if eq == oracle.EQ_VARADV1D:
        u = W.varadv_periodic(xi, nx, seed)
        if kind == "rough":
            u[1] = np.sign(u[1]) * (0.5 + np.abs(u[1]))
        return u
    raise ValueError(eq)


CASES = [(oracle.EQ_SW1D, "smooth"), (oracle.EQ_SW1D, "rough"), (oracle.EQ_SW2D, "rough"),
         (oracle.EQ_MHD2D, "smooth"), (oracle.EQ_MHD2D, "blocky"), (oracle.EQ_LINADV1D, "smooth"),
         (oracle.EQ_VARADV1D, "rough")]


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("blending", [0, 1, 2])
@pytest.mark.parametrize("eq,kind", CASES)
def test_dot_product_identity(eq, kind, N, blending):
    nx, ny = (9, 1) if oracle.DIMS[eq] == 1 else (4, 3)
    if eq == oracle.EQ_SW2D:
        ny = nx = 3
    c = oracle.make_cfg(eq, N, nx, ny, blending=blending, cfl=0.1)
    u = _data(eq, N, nx, ny, 2, kind)
    dt, ch = oracle.dt_ch(c, u)
    rng = np.random.default_rng(5)
    scale = np.abs(u).mean(axis=(1, 2), keepdims=True) + 1e-3
    for _ in range(2):
        v = rng.normal(size=u.shape) * scale
        lam = rng.normal(size=u.shape)
        _, Jv = oracle.jvp(c, u, v, dt, ch)
        mu = oracle.vjp(c, u, lam, dt, ch)
        a, b = float(np.sum(lam * Jv)), float(np.sum(mu * v))
        assert abs(a - b) <= 1e-13 * float(np.sum(np.abs(lam * Jv))), (a, b)


@pytest.mark.parametrize("eq,N,nx,ny,kind", [
    (oracle.EQ_SW1D, 1, 2, 1, "rough"), (oracle.EQ_SW1D, 4, 2, 1, "rough"),
    (oracle.EQ_VARADV1D, 3, 2, 1, "rough"),
    (oracle.EQ_SW2D, 2, 2, 2, "rough"),
    (oracle.EQ_MHD2D, 1, 2, 1, "blocky"), (oracle.EQ_MHD2D, 2, 2, 2, "blocky"),
    (oracle.EQ_MHD2D, 3, 2, 1, "smooth"), (oracle.EQ_MHD2D, 4, 1, 2, "smooth"),
])
def test_full_jacobian_transpose(eq, N, nx, ny, kind):
    c = oracle.make_cfg(eq, N, nx, ny, blending=2, cfl=0.1)
    u = _data(eq, N, nx, ny, 3, kind)
    dt, ch = oracle.dt_ch(c, u)
    n = u.size
    J = np.zeros((n, n))
    JT = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        J[:, k] = oracle.jvp(c, u, e.reshape(u.shape), dt, ch)[1].reshape(-1)
        JT[k, :] = oracle.vjp(c, u, e.reshape(u.shape), dt, ch).reshape(-1)
    assert np.abs(J - JT).max() <= 1e-13 * np.abs(J).max()


def test_rollout_gradient_against_central_differences():
    """Three steps of GLM-MHD (smooth, blending with Algorithms 1-2; no limiter acts):
    grad of 1/2 sum w rho^2 by the reverse mode against central differences of the
    rollout with each step's dt, c_h and alpha held at their forward values."""
    N, n, K = 2, 4, 3
    c = oracle.make_cfg(oracle.EQ_MHD2D, N, n, n, blending=2)
    re_ = oracle.refel(N)
    u0 = W.mhd_smooth(re_["xi"], n, n, seed=3, amp=0.05)
    wn = np.outer(re_["w"], re_["w"]).reshape(-1)
    states, frozen = [u0], []
    for _ in range(K):
        r = oracle.step(c, states[-1])
        assert (r["flags"] & (oracle.FLAG_ALG1 | oracle.FLAG_ALG2)).max() == 0
        frozen.append((r["dt"], r["ch"], r["alpha"]))
        states.append(r["u"])
    lam = np.zeros_like(u0)
    lam[0] = wn * states[-1][0]
    for k in reversed(range(K)):
        lam = oracle.vjp(c, states[k], lam, frozen[k][0], frozen[k][1])

    def loss(u):
        for dt, ch, al in frozen:
            u = oracle.step(c, u, dt=dt, ch=ch, alpha_in=al)["u"]
        return 0.5 * float(np.sum(wn * u[0] ** 2))

    rng = np.random.default_rng(0)
    for _ in range(3):
        v = rng.normal(size=u0.shape) * (np.abs(u0).mean(axis=(1, 2), keepdims=True) + 1e-3)
        eps = 1e-6
        fd = (loss(u0 + eps * v) - loss(u0 - eps * v)) / (2 * eps)
        ad = float(np.sum(lam * v))
        assert abs(ad - fd) <= 1e-7 * abs(fd), (ad, fd)


def test_thread_count_does_not_change_bits():
    N, n = 3, 6
    c = oracle.make_cfg(oracle.EQ_MHD2D, N, n, n, blending=2)
    u = _data(oracle.EQ_MHD2D, N, n, n, 1, "blocky")
    dt, ch = oracle.dt_ch(c, u)
    lam = np.random.default_rng(2).normal(size=u.shape)
    ref = oracle.vjp(c, u, lam, dt, ch, threads=1)
    for t in (2, 3, 8):
        assert np.array_equal(oracle.vjp(c, u, lam, dt, ch, threads=t), ref)


def test_unsupported_configurations():
    c = oracle.make_cfg(oracle.EQ_SW2D, 2, 3, 3, bc=(1, 1, 0, 0))
    u = _data(oracle.EQ_SW2D, 2, 3, 3, 0, "rough")
    with pytest.raises(AssertionError):
        oracle.vjp(c, u, u, 1e-3, 0.0)
