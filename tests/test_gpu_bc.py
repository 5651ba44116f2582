"""Non-periodic sides on the GPU (outflow, wall, Dirichlet), through the C ABI.

  * one step against the oracle, to the parity bar of the periodic tests
    (1e-12 per value relative to max(|value|, 1e-2 max|u^n|), dt to 1e-13,
    alpha_e to 1e-12, flags bit-exact), for every system and side kind the
    library accepts, degrees 1..4, with and without blending and limiting, on
    meshes with several blocks of elements and ragged tails;
  * Dirichlet inflow + outflow for v_t + x^-2 v_x = 0 on [0.1, 1] (the §5.1
    case with v0 = sin(2 pi x^3)): every step of a run against the oracle, and
    the GPU run's convergence order;
  * walls keep the mass of the shallow water systems over many steps;
  * a batch with wall and outflow sides equals lwfr_step on each problem;
  * the documented errors (Dirichlet data missing, dt <= 0, graph capture).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2512_08611_amd import lwfr
from paper_2512_08611_amd import workloads as W
from test_gpu_parity import DEV, Pair

pytestmark = pytest.mark.gpu
OUT, WALL, DIRI = lwfr.LWFR_BC_OUTFLOW, lwfr.LWFR_BC_WALL, lwfr.LWFR_BC_DIRICHLET


def sw1d_moving(xi, nx, seed):
    """a depth jump and momentum everywhere, also at the walls"""
    rng = np.random.default_rng(seed)
    x = W.coords_1d(xi, nx)
    h = np.where(x < 0.37, 2.0, 1.0) + 0.05 * np.sin(6 * x)
    hv = 0.3 * np.cos(5 * x + rng.uniform(0, 6))
    b = 0.1 * np.sin(3 * x) ** 2
    return np.stack([h, hv, b])


def sw2d_moving(xi, n, seed):
    u = W.sw2d_random(xi, n, seed)
    x, y = W.coords_2d(xi, n, n)
    rng = np.random.default_rng(seed + 7)
    u[0] += np.where((x - 0.4) ** 2 + (y - 0.55) ** 2 < 0.06, 0.8, 0.0)
    u[1] = 0.2 * u[0] * np.sin(3 * y + rng.uniform(0, 6))
    u[2] = -0.15 * u[0] * np.cos(2 * x + rng.uniform(0, 6))
    return u


def ghost_from_state(c, u, rng, rel=1e-2):
    """Dirichlet data near the state's own boundary values: u^n from the node next to each
    boundary face point (perturbed by rel), U a further 1e-3 perturbation of it, F_d the
    oracle's flux of U.  Only the layout matters for parity; the values stay admissible."""
    eq, N = c.eq, c.N
    n1, M, dim = N + 1, oracle.NVARS[eq], oracle.DIMS[eq]
    nfp = oracle.nfp(c)
    nx, ny = c.nx, c.ny
    g = np.zeros(oracle.ghost_size(c))
    off = 0
    for d in range(dim):
        lines = ny if d == 0 else nx
        nb = lines * nfp
        for side in range(2):
            for line in range(lines):
                for q in range(nfp):
                    if d == 0:
                        e = (nx - 1 if side else 0) + nx * line
                        p = (N if side else 0) + n1 * q if dim == 2 else (N if side else 0)
                    else:
                        e = line + nx * (ny - 1 if side else 0)
                        p = q + n1 * (N if side else 0)
                    a = u[:, e, p] * (1 + rel * rng.uniform(-1, 1, M))
                    U = a * (1 + 1e-3 * rng.uniform(-1, 1, M))
                    F = oracle.physics(eq, "flux", d, U, gamma=5.0 / 3.0, gravity=9.81)
                    j = line * nfp + q
                    for v in range(M):
                        g[off + v * nb + j] = a[v]
                        g[off + (M + v) * nb + j] = U[v]
                        g[off + (2 * M + v) * nb + j] = F[v]
            off += 3 * M * nb
    return g


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("blending", [0, 2])
@pytest.mark.parametrize("bc", [(WALL, WALL), (OUT, OUT), (WALL, OUT)])
def test_parity_sw1d(N, blending, bc):
    nx = 137
    pr = Pair(oracle.EQ_SW1D, N, nx, blending=blending, bc=bc + (0, 0))
    for seed in (0, 1):
        pr.check(sw1d_moving(oracle.refel(N)["xi"], nx, seed))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("blending", [0, 1, 2])
@pytest.mark.parametrize("bc", [(WALL,) * 4, (WALL, WALL, 0, 0), (0, 0, OUT, WALL), (OUT, OUT, OUT, OUT)])
def test_parity_sw2d(N, blending, bc):
    n = 11
    pr = Pair(oracle.EQ_SW2D, N, n, n, blending=blending, bc=bc)
    for seed in (0, 1):
        g, o = pr.check(sw2d_moving(oracle.refel(N)["xi"], n, seed))
    if blending == 2:
        assert o["alpha"].max() > 0.05


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("blending", [0, 2])
@pytest.mark.parametrize("kind", ["smooth", "blocky"])
@pytest.mark.parametrize("bc", [(OUT, OUT, 0, 0), (OUT,) * 4, (0, 0, DIRI, OUT), (DIRI,) * 4])
def test_parity_mhd(N, blending, kind, bc):
    nx, ny = 9, 7
    xi = oracle.refel(N)["xi"]
    pr = Pair(oracle.EQ_MHD2D, N, nx, ny, blending=blending, bc=bc)
    rng = np.random.default_rng(N)
    for seed in (0, 1):
        u = W.mhd_smooth(xi, nx, ny, seed) if kind == "smooth" else W.mhd_blocky(xi, nx, ny, seed, nblocks=4)
        ghost = ghost_from_state(pr.oc, u, rng) if DIRI in bc else None
        dt = oracle.dt_ch(pr.oc, u)[0] if DIRI in bc else 0.0
        g, o = pr.check(u, dt=dt, ghost=ghost)
    if kind == "blocky" and blending == 2 and N >= 2:
        assert (o["flags"] & (oracle.FLAG_ALG1 | oracle.FLAG_ALG2)).any()


def test_parity_mhd_limiter_at_boundary_faces():
    """Blocky data with a near-vacuum block on the boundary: Algorithm 1 acts on the
    boundary half faces (flags, which read the left half faces' thetas, bit-exact)."""
    nx, ny, N = 12, 10, 3
    xi = oracle.refel(N)["xi"]
    u = W.mhd_blocky(xi, nx, ny, 3, nblocks=6)
    x, y = W.coords_2d(xi, nx, ny)
    thin = (x < 1.0 / nx) | (y > 1 - 1.0 / ny)
    u[:, thin] *= 1e-3  # density, momenta, energy and field scaled together: pressure ~1e-3 relative
    u[4, thin] = np.maximum(u[4, thin], 0.5 * (u[1, thin] ** 2 + u[2, thin] ** 2 + u[3, thin] ** 2) / u[0, thin]
                            + 0.5 * (u[5, thin] ** 2 + u[6, thin] ** 2 + u[7, thin] ** 2) + 1e-6)
    for bc in [(OUT,) * 4, (OUT, OUT, 0, 0)]:
        pr = Pair(oracle.EQ_MHD2D, N, nx, ny, blending=2, bc=bc)
        g, o = pr.check(u)
        print("BC LIMITER flags", np.bincount(o["flags"].astype(np.int64), minlength=32)[:32].tolist(), flush=True)


def varadv_ghost(c, t, dt, x0):
    g = np.zeros(oracle.ghost_size(c))
    gx, gw = np.polynomial.legendre.leggauss(8)
    ts = t + 0.5 * dt * (gx + 1)
    g[0] = math.sin(2 * math.pi * (x0 ** 3 - 3 * t))
    g[1] = x0 ** -2
    g[2] = 0.5 * (gw * np.sin(2 * math.pi * (x0 ** 3 - 3 * ts))).sum()
    g[3] = x0 ** -2
    return g


def varadv_run(N, nx, tend=0.05, compare_every=0):
    lo, hi = 0.1, 1.0
    cfl = oracle.cfl_number(N)
    pr = Pair(oracle.EQ_VARADV1D, N, nx, blending=0, lo=(lo, 0.0), hi=(hi, 1.0), cfl=cfl,
              bc=(DIRI, OUT, 0, 0))
    x = W.coords_1d(np.array(pr.st.xi), nx, lo, hi)
    u = np.stack([np.sin(2 * math.pi * x ** 3), x ** -2.0])
    dt = 0.9 * cfl * (hi - lo) / nx / lo ** -2  # sigma = max a (the element-mean step is unstable here)
    nsteps = int(math.ceil(tend / dt))
    dt = tend / nsteps
    ghost = torch.zeros(oracle.ghost_size(pr.oc), dtype=torch.float64, device=DEV)
    pr.st.set_boundary_data(ghost)
    ua = torch.tensor(u, dtype=torch.float64, device=DEV)
    ub = torch.empty_like(ua)
    t, worst = 0.0, 0.0
    uo = u.copy()  # the oracle's own run, compared step by step when asked
    for k in range(nsteps):
        gh = varadv_ghost(pr.oc, t, dt, lo)
        ghost.copy_(torch.tensor(gh, dtype=torch.float64))
        pr.st.step(ua, ub, dt)
        if compare_every and k % compare_every == 0:
            o = oracle.step(pr.oc, uo, dt=dt, ghost=gh)["u"]
            g = pr.gpu_step(uo, dt)["u"]
            worst = max(worst, float((np.abs(g - o) / np.maximum(np.abs(o), 1e-2)).max()))
            uo = o
        ua, ub = ub, ua
        t += dt
    torch.cuda.synchronize()
    ex = np.sin(2 * math.pi * (x ** 3 - 3 * tend))
    err = np.sqrt(((ua.cpu().numpy()[0] - ex) ** 2).mean())
    return err, worst


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_varadv_inflow_outflow_every_step(N):
    err, worst = varadv_run(N, 16, tend=0.02, compare_every=1)
    print(f"VARADV N={N} rel={worst:.3e} err={err:.3e}", flush=True)
    assert worst <= 1e-12
    assert err < 0.05


@pytest.mark.parametrize("N,ns", [(1, (32, 64)), (2, (16, 32)), (3, (8, 16)), (4, (8, 16))])
def test_varadv_gpu_order(N, ns):
    errs = [varadv_run(N, n)[0] for n in ns]
    rate = math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0])
    print(f"VARADV ORDER N={N} errs={errs} rate={rate:.2f}", flush=True)
    assert errs[0] < 0.05 and rate > N + 1 - 0.4


@pytest.mark.parametrize("eq", [oracle.EQ_SW1D, oracle.EQ_SW2D])
def test_walls_keep_mass_on_gpu(eq):
    N = 3
    xi = oracle.refel(N)["xi"]
    if eq == oracle.EQ_SW1D:
        n = 300
        u = sw1d_moving(xi, n, 0)
        cfg = lwfr.make_config(eq, N, n, bc=(WALL, WALL, 0, 0))
        wn = torch.tensor(np.array(oracle.refel(N)["w"]), device=DEV, dtype=torch.float64)
    else:
        n = 64
        u = sw2d_moving(xi, n, 0)
        cfg = lwfr.make_config(eq, N, (n, n), bc=(WALL,) * 4)
        w = np.array(oracle.refel(N)["w"])
        wn = torch.tensor(np.outer(w, w).reshape(-1), device=DEV, dtype=torch.float64)
    st = lwfr.Stepper(cfg, DEV)
    ua = torch.tensor(u, dtype=torch.float64, device=DEV)
    ub = torch.empty_like(ua)
    m0 = float((ua[0] * wn).sum())
    for _ in range(200):
        st.step(ua, ub)
        ua, ub = ub, ua
    status, flags = st.query()
    assert status == lwfr.LWFR_OK, flags
    m = float((ua[0] * wn).sum())
    print(f"WALL MASS eq={eq} drift={abs(m - m0) / m0:.2e}", flush=True)
    assert abs(m - m0) <= 1e-12 * m0


def test_batch_with_walls_equals_single_steps():
    specs = [(5, 2, (WALL,) * 4), (7, 3, (OUT, OUT, WALL, WALL)), (4, 4, (0, 0, 0, 0)), (6, 1, (WALL, WALL, 0, 0)),
             (9, 4, (OUT,) * 4)]
    stream = torch.cuda.Stream(DEV)
    cfgs = [lwfr.make_config(lwfr.LWFR_EQ_SW2D, N, (n, n), cfl_number=oracle.cfl_number(N), bc=bc)
            for n, N, bc in specs]
    b = lwfr.Batch(cfgs, DEV, stream=stream)
    u = b.empty()
    states = []
    for i, (n, N, _) in enumerate(specs):
        s = sw2d_moving(oracle.refel(N)["xi"], n, i)
        states.append(s)
        b.view(u, i).copy_(torch.tensor(s, dtype=torch.float64))
    out = b.empty()
    dt = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    b.step(u, out, dt)
    torch.cuda.synchronize()
    for i, cfg in enumerate(cfgs):
        st = lwfr.Stepper(cfg, DEV, stream=stream)
        ud = torch.tensor(states[i], dtype=torch.float64, device=DEV)
        ref = torch.empty_like(ud)
        dtch = torch.zeros(2, dtype=torch.float64, device=DEV)
        torch.cuda.synchronize()
        st.step(ud, ref, 0.0, dtch)
        torch.cuda.synchronize()
        assert float(dt[i]) == float(dtch[0])
        assert torch.equal(b.view(out, i).cpu(), ref.cpu()), i
        st.close()
        n, N, bc = specs[i]
        oc = oracle.make_cfg(oracle.EQ_SW2D, N, n, n, cfl=oracle.cfl_number(N), bc=bc)
        o = oracle.step(oc, states[i])
        scale = np.maximum(np.abs(o["u"]), 1e-2 * np.abs(states[i]).max())
        assert (np.abs(ref.cpu().numpy() - o["u"]) / scale).max() <= 1e-12


def test_boundary_errors():
    cfg = lwfr.make_config(lwfr.LWFR_EQ_VARADV1D, 2, 8, lo=(0.1, 0.0), bc=(DIRI, OUT, 0, 0))
    stream = torch.cuda.Stream(DEV)
    st = lwfr.Stepper(cfg, DEV, stream=stream)
    xi = np.array(st.xi)
    u = torch.tensor(W.varadv_periodic(xi, 8, 0), dtype=torch.float64, device=DEV)
    v = torch.empty_like(u)
    with pytest.raises(lwfr.LwfrError) as ei:
        st.step(u, v, 1e-4)  # no Dirichlet data yet
    assert ei.value.status == lwfr.LWFR_E_STATE
    st.set_boundary_data(torch.zeros(st.boundary_data_size(), dtype=torch.float64, device=DEV))
    with pytest.raises(lwfr.LwfrError) as ei:
        st.step(u, v, 0.0)  # dt from the device: not with Dirichlet sides
    assert ei.value.status == lwfr.LWFR_E_INVALID_ARG
    with pytest.raises(lwfr.LwfrError) as ei:
        st.graph_capture(u, v, 2)
    assert ei.value.status == lwfr.LWFR_E_UNSUPPORTED
    st.step(u, v, 1e-4)
    torch.cuda.synchronize()
    assert st.query()[0] == lwfr.LWFR_OK
