"""GPU adjoint of the time step against the oracle's forward-mode derivative.

The GPU computes mu = J^T lambda (reverse mode, hand-written) with dt, c_h,
alpha, the Algorithm 1/2 thetas and every max/abs branch frozen at their
forward values; the oracle computes J v with dual numbers through the same
frozen map.  Checks:
  * dot-product identity <lambda, J v> = <J^T lambda, v> (relative 1e-11);
  * full Jacobians on two-element periodic meshes: J^T lambda entry by entry
    against the oracle's J assembled column by column (relative 1e-10 of the
    largest entry).
Test states avoid exact ties of a switch (a max whose two arguments agree to
rounding), where each implementation may take a different, equally valid
one-sided derivative.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_08611_amd import lwfr
from paper_2512_08611_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def make(eq, N, nx, ny=1, blending=2, cfl=0.1):
    cfg = lwfr.make_config(eq, N, (nx, ny), cfl_number=cfl, blending=blending, flags=lwfr.LWFR_CFG_ADJOINT)
    st = lwfr.Stepper(cfg, DEV)
    oc = oracle.make_cfg(eq, N, nx, ny, cfl=cfl, blending=blending)
    return st, oc


def data(eq, N, nx, ny, seed, kind):
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
        u[2] = 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape[0])[:, None]
        if kind == "rough":
            u[0] *= 1 + 0.3 * rng.uniform(-1, 1, u[0].shape)
        return u
    if eq == oracle.EQ_MHD2D:
        u = W.mhd_smooth(xi, nx, ny, seed, amp=0.05) if kind == "smooth" else W.mhd_blocky(xi, nx, ny, seed, nblocks=3)
        if kind == "blocky":
            # piecewise-constant blocks with moving fluid, psi != 0, and a 1e-3 relative
            # jitter per node at fixed pressure: exactly constant data makes the two face
            # values of a block equal up to rounding, so which side wins the max in the
            # wave speed would be decided by the last bit (a tie, where both one-sided
            # derivatives are valid); the jitter keeps every such choice well separated
            gam = 5.0 / 3.0
            p = (gam - 1) * (u[4] - 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / u[0]
                             - 0.5 * (u[5] ** 2 + u[6] ** 2 + u[7] ** 2) - 0.5 * u[8] ** 2)
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
    raise ValueError


def gpu_adjoint(st, u, dt, lam):
    ud = torch.tensor(u, dtype=torch.float64, device=DEV)
    ld = torch.tensor(lam, dtype=torch.float64, device=DEV)
    out = torch.empty_like(ud)
    st.adjoint_step(ud, dt, ld, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def dot_check(eq, N, nx, ny, blending, kind, seed=0):
    st, oc = make(eq, N, nx, ny, blending)
    u = data(eq, N, nx, ny, seed, kind)
    dt, ch = oracle.dt_ch(oc, u)
    rng = np.random.default_rng(seed + 7)
    scale = np.abs(u).mean(axis=(1, 2), keepdims=True) + 1e-3
    worst = 0.0
    for _ in range(3):
        v = rng.normal(size=u.shape) * scale
        lam = rng.normal(size=u.shape)
        _, Jv = oracle.jvp(oc, u, v, dt, ch)
        mu = gpu_adjoint(st, u, dt, lam)
        a, b = float(np.sum(lam * Jv)), float(np.sum(mu * v))
        ref = float(np.sum(np.abs(lam * Jv)))
        worst = max(worst, abs(a - b) / ref)
    return worst


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("blending", [0, 1, 2])
@pytest.mark.parametrize("eq,kind", [(oracle.EQ_SW1D, "smooth"), (oracle.EQ_SW1D, "rough"),
                                     (oracle.EQ_LINADV1D, "smooth"), (oracle.EQ_VARADV1D, "rough")])
def test_dot_product_1d(eq, kind, N, blending):
    assert dot_check(eq, N, 13, 1, blending, kind) < 1e-11


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("blending", [0, 2])
@pytest.mark.parametrize("kind", ["smooth", "rough"])
def test_dot_product_sw2d(N, blending, kind):
    assert dot_check(oracle.EQ_SW2D, N, 5, 5, blending, kind) < 1e-11


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("blending", [0, 1, 2])
@pytest.mark.parametrize("kind", ["smooth", "blocky"])
def test_dot_product_mhd(N, blending, kind):
    assert dot_check(oracle.EQ_MHD2D, N, 5, 4, blending, kind) < 1e-11


@pytest.mark.parametrize("eq,N,nx,ny,kind", [
    (oracle.EQ_SW1D, 3, 2, 1, "rough"),
    (oracle.EQ_VARADV1D, 2, 2, 1, "rough"),
    (oracle.EQ_MHD2D, 1, 2, 1, "blocky"),
    (oracle.EQ_MHD2D, 2, 2, 2, "blocky"),
    (oracle.EQ_MHD2D, 3, 2, 2, "smooth"),
    (oracle.EQ_MHD2D, 4, 2, 1, "smooth"),
])
def test_full_jacobian_two_elements(eq, N, nx, ny, kind):
    st, oc = make(eq, N, nx, ny, 2)
    u = data(eq, N, nx, ny, 3, kind)
    dt, ch = oracle.dt_ch(oc, u)
    n = u.size
    J = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        _, Jv = oracle.jvp(oc, u, e.reshape(u.shape), dt, ch)
        J[:, k] = Jv.reshape(-1)
    rng = np.random.default_rng(1)
    for _ in range(3):
        lam = rng.normal(size=u.shape)
        mu = gpu_adjoint(st, u, dt, lam).reshape(-1)
        ref = J.T @ lam.reshape(-1)
        assert np.abs(mu - ref).max() <= 1e-10 * np.abs(ref).max(), np.abs(mu - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("eq,N,nx,ny,kind", [(oracle.EQ_MHD2D, 3, 5, 4, "blocky"), (oracle.EQ_SW1D, 4, 13, 1, "rough")])
def test_taped_adjoint_equals_recomputing_adjoint(eq, N, nx, ny, kind):
    st, oc = make(eq, N, nx, ny, 2)
    u = torch.tensor(data(eq, N, nx, ny, 4, kind), dtype=torch.float64, device=DEV)
    dt = oracle.dt_ch(oc, u.cpu().numpy())[0]
    lam = torch.randn(u.shape, dtype=torch.float64, device=DEV, generator=torch.Generator(DEV).manual_seed(3))
    tape = st.new_tape()
    out = torch.empty_like(u)
    st.step_taped(u, out, dt, tape)
    ref = torch.empty_like(u)
    st.step(u, ref, dt)
    assert torch.equal(out, ref)
    a, b = torch.empty_like(u), torch.empty_like(u)
    st.adjoint_step(u, dt, lam, a)
    st.adjoint_step(u, dt, lam, b, tape)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_adjoint_requires_flag():
    cfg = lwfr.make_config(lwfr.LWFR_EQ_SW1D, 3, 8)
    st = lwfr.Stepper(cfg, DEV)
    u = torch.ones((3, 8, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(lwfr.LwfrError) as ei:
        st.adjoint_step(u, 1e-3, u, torch.empty_like(u))
    assert ei.value.status == lwfr.LWFR_E_STATE


@pytest.mark.parametrize("eq,N,nx,ny", [(oracle.EQ_SW1D, 3, 13, 1), (oracle.EQ_MHD2D, 3, 5, 4), (oracle.EQ_MHD2D, 4, 4, 4)])
def test_dot_product_gll(eq, N, nx, ny):
    """The adjoint with GLL points and the g_2 correction against the oracle's forward mode.

    Nodal interpolation at GLL points gives both sides of a face the same point,
    so the two face states would be equal and the max of their wave speeds an
    exact tie (both one-sided derivatives valid); a 1e-2 relative jitter per
    point separates them."""
    cfg = lwfr.make_config(eq, N, (nx, ny), cfl_number=0.1, blending=2,
                           flags=lwfr.LWFR_CFG_ADJOINT | lwfr.LWFR_CFG_GLL)
    st = lwfr.Stepper(cfg, DEV)
    oc = oracle.make_cfg(eq, N, nx, ny, cfl=0.1, blending=2, gll=True)
    xi = oracle.refel(N, gll=True)["xi"]
    u = W.sw1d_wave(xi, nx, 2) if eq == oracle.EQ_SW1D else W.mhd_smooth(xi, nx, ny, 2, amp=0.05)
    rng = np.random.default_rng(11)
    u = u * (1 + 1e-2 * rng.uniform(-1, 1, u.shape)) + 1e-3 * rng.uniform(-1, 1, u.shape)
    dt, ch = oracle.dt_ch(oc, u)
    scale = np.abs(u).mean(axis=(1, 2), keepdims=True) + 1e-3
    for _ in range(3):
        v = rng.normal(size=u.shape) * scale
        lam = rng.normal(size=u.shape)
        _, Jv = oracle.jvp(oc, u, v, dt, ch)
        mu = gpu_adjoint(st, u, dt, lam)
        a, b = float(np.sum(lam * Jv)), float(np.sum(mu * v))
        assert abs(a - b) <= 1e-11 * float(np.sum(np.abs(lam * Jv)))
