"""Seeded synthetic inputs for the time step (initial states at the solution points).

This module holds none of the method's arithmetic: every function evaluates a
closed-form initial condition at given physical coordinates.  The reference
nodes xi (on [0,1]) are an argument, so the same generator serves the HIP
library and the CPU oracle, each with its own nodes.

State layout (shared by every caller): u[var][elem][node], elements x-fastest,
nodes x-fastest inside an element.

Workloads (sizes are those the time step is measured and checked on):
  * sw1d_wave      1-D shallow water over a smooth bed on [0,1], 200 elements, N=3
  * mhd_smooth     2-D GLM-MHD, Orszag-Tang vortex (paper §5.5 eq. orszag.tang.ic)
                   plus seeded Fourier perturbations of amplitude 1e-2
  * mhd_blocky     2-D GLM-MHD, 16x16 seeded piecewise-constant blocks with jumps
                   inside elements (density ratio <= 10, pressure ratio <= 100)
  * sw2d_random    2-D shallow water, seeded smooth bed and depth 1 + 0.2 noise
  * alfven         2-D GLM-MHD Alfven wave (paper §5.5, exact solution)
  * jinxin_sine    1-D Jin-Xin relaxation for Burgers (paper §5.1 eq. jin.xin.ic) on
                   [-1, 1], in equilibrium v = u^2/2
"""
import math

import numpy as np

GAMMA_MHD = 5.0 / 3.0
GRAVITY = 9.81


def coords_1d(xi, nx, lo=0.0, hi=1.0):
    """x[e, p] of the nodes of a uniform 1-D mesh."""
    dx = (hi - lo) / nx
    e = np.arange(nx).reshape(nx, 1)
    return lo + (e + np.asarray(xi).reshape(1, -1)) * dx


def coords_2d(xi, nx, ny, lo=(0.0, 0.0), hi=(1.0, 1.0)):
    """x[e, p], y[e, p] of a uniform 2-D mesh (elements and nodes x-fastest)."""
    xi = np.asarray(xi)
    n1 = xi.size
    dx = (hi[0] - lo[0]) / nx
    dy = (hi[1] - lo[1]) / ny
    ex = np.tile(np.arange(nx), ny).reshape(-1, 1)
    ey = np.repeat(np.arange(ny), nx).reshape(-1, 1)
    px = np.tile(xi, n1).reshape(1, -1)
    py = np.repeat(xi, n1).reshape(1, -1)
    return lo[0] + (ex + px) * dx, lo[1] + (ey + py) * dy


# ------------------------------------------------------------------ 1-D ----
def sw1d_wave(xi, nx=200, seed=0):
    """h = 2 + 0.1 sin(2 pi x + phi), hv = 0.1 cos(2 pi x), b = 0.5 sin^2(pi x), phi ~ U(0, 2pi)."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    x = coords_1d(xi, nx)
    h = 2.0 + 0.1 * np.sin(2 * math.pi * x + phi)
    hv = 0.1 * np.cos(2 * math.pi * x)
    b = 0.5 * np.sin(math.pi * x) ** 2
    return np.stack([h, hv, b])


def sw1d_lake(xi, nx, seed=0, level=1.0):
    """Lake at rest h + b = level, v = 0, over a continuous bed that is linear inside each
    element with seeded kinks at the element faces."""
    rng = np.random.default_rng(seed)
    bf = 0.3 * rng.uniform(-1, 1, nx)  # bed height at the left face of each element
    bf_right = np.roll(bf, -1)
    x = coords_1d(xi, nx)
    t = (x - np.arange(nx).reshape(-1, 1) / nx) * nx  # local coordinate in [0,1]
    b = bf.reshape(-1, 1) * (1 - t) + bf_right.reshape(-1, 1) * t
    h = level - b
    return np.stack([h, np.zeros_like(h), b])


def linadv_sine(xi, nx, k=1):
    x = coords_1d(xi, nx)
    return np.sin(2 * math.pi * k * x)[None]


def varadv_periodic(xi, nx, seed=0):
    """u = (v, a) with v = sin(2 pi x), a = 1 + sin(2 pi x)/2 (periodic variable coefficient)."""
    x = coords_1d(xi, nx)
    return np.stack([np.sin(2 * math.pi * x), 1.0 + 0.5 * np.sin(2 * math.pi * x)])


def jinxin_sine(xi, nx, lo=-1.0, hi=1.0):
    """u = 2 + sin(pi (x - 0.7)) (eq. jin.xin.ic), v = u^2/2: the equilibrium of the Burgers
    relaxation (the paper gives no initial v)."""
    x = coords_1d(xi, nx, lo, hi)
    u = 2.0 + np.sin(math.pi * (x - 0.7))
    return np.stack([u, 0.5 * u * u])


def jinxin_random(xi, nx, seed=0, lo=-1.0, hi=1.0):
    """smooth u in [1, 3] and v off equilibrium by a seeded smooth perturbation"""
    rng = np.random.default_rng(seed)
    x = coords_1d(xi, nx, lo, hi)
    u = 2.0 + 0.5 * np.sin(math.pi * x + rng.uniform(0, 6)) + 0.3 * np.sin(3 * math.pi * x + rng.uniform(0, 6))
    v = 0.5 * u * u + 0.2 * np.cos(2 * math.pi * x + rng.uniform(0, 6))
    return np.stack([u, v])


# ------------------------------------------------------------------ MHD ----
def _mhd_cons(rho, v1, v2, v3, p, B1, B2, B3, psi, gamma=GAMMA_MHD):
    E = p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2 + v3 * v3) + 0.5 * (B1 * B1 + B2 * B2 + B3 * B3) + 0.5 * psi * psi
    return np.stack([rho, rho * v1, rho * v2, rho * v3, E, B1, B2, B3, psi])


def _fourier(rng, x, y, nmodes=8, kmax=4):
    """sum_k a_k sin(2 pi (m_k x + n_k y) + phi_k), (m,n) in {-kmax..kmax}^2 \\ 0, a_k ~ U(-1,1)/sqrt(nmodes).
    Returns the field and its x- and y-derivatives."""
    f = np.zeros_like(x)
    fx = np.zeros_like(x)
    fy = np.zeros_like(x)
    for _ in range(nmodes):
        while True:
            m, n = rng.integers(-kmax, kmax + 1, size=2)
            if m != 0 or n != 0:
                break
        a = rng.uniform(-1, 1) / math.sqrt(nmodes)
        ph = rng.uniform(0, 2 * math.pi)
        arg = 2 * math.pi * (m * x + n * y) + ph
        f += a * np.sin(arg)
        fx += a * 2 * math.pi * m * np.cos(arg)
        fy += a * 2 * math.pi * n * np.cos(arg)
    return f, fx, fy


def mhd_smooth(xi, nx, ny=None, seed=0, amp=1e-2, gamma=GAMMA_MHD):
    """Orszag-Tang vortex (rho = 1, v = (-sin 2pi y, sin 2pi x, 0), p = 1/gamma,
    B = (-sin(2pi y)/gamma, sin(4pi x)/gamma, 0), psi = 0) on [0,1]^2 plus seeded
    perturbations: rho (1+d_rho), p (1+d_p), v_i + d_vi, B += (dA/dy, -dA/dx)."""
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed)
    x, y = coords_2d(xi, nx, ny)
    s = 2 * math.pi
    d = [amp * _fourier(rng, x, y)[0] for _ in range(5)]
    A, Ax, Ay = _fourier(rng, x, y)
    rho = 1.0 * (1 + d[0])
    v1 = -np.sin(s * y) + d[1]
    v2 = np.sin(s * x) + d[2]
    v3 = np.zeros_like(x) + d[3]
    p = (1.0 / gamma) * (1 + d[4])
    B1 = -np.sin(s * y) / gamma + amp * Ay
    B2 = np.sin(2 * s * x) / gamma - amp * Ax
    B3 = np.zeros_like(x)
    return _mhd_cons(rho, v1, v2, v3, p, B1, B2, B3, np.zeros_like(x), gamma)


def mhd_blocky(xi, nx, ny=None, seed=0, nblocks=16, gamma=GAMMA_MHD):
    """16x16 piecewise-constant blocks with edges at k/16 + 0.4 dx (inside elements);
    per block rho = 10^U(-1,0), p = 10^U(-2,0), B_i ~ 0.5 U(-1,1), v = 0, psi = 0."""
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed)
    x, y = coords_2d(xi, nx, ny)
    shift_x = 0.4 / nx
    shift_y = 0.4 / ny
    bx = np.floor((x - shift_x) * nblocks).astype(int) % nblocks
    by = np.floor((y - shift_y) * nblocks).astype(int) % nblocks
    nb = nblocks * nblocks
    rho_b = 10.0 ** rng.uniform(-1, 0, nb)
    p_b = 10.0 ** rng.uniform(-2, 0, nb)
    B_b = 0.5 * rng.uniform(-1, 1, (3, nb))
    k = bx + nblocks * by
    z = np.zeros_like(x)
    return _mhd_cons(rho_b[k], z, z, z, p_b[k], B_b[0][k], B_b[1][k], B_b[2][k], z, gamma)


def mhd_rotor(xi, n, gamma=1.4):
    """MHD rotor (paper §5.5, eq. rotor.ic) on [0,1]^2: a dense disc (rho = 10,
    r <= 0.1) spinning at angular speed 20 inside a medium at rest, linear taper
    over 0.1 < r <= 0.115, p = 1, B = (5/sqrt(4 pi), 0, 0), psi = 0.  The paper
    does not state gamma for this test; 1.4 is the value of the cited setup
    (Balsara & Spicer)."""
    x, y = coords_2d(xi, n, n)
    r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2)
    r0, r1 = 0.1, 0.115
    f = np.clip((r1 - r) / (r1 - r0), 0.0, 1.0)
    inside = r <= r0
    fr = np.where(inside, 1.0, f)
    rho = 1.0 + 9.0 * fr
    v1 = -20.0 * fr * (y - 0.5)
    v2 = 20.0 * fr * (x - 0.5)
    z = np.zeros_like(x)
    return _mhd_cons(rho, v1, v2, z, z + 1.0, z + 5.0 / math.sqrt(4 * math.pi), z, z, z, gamma)


def alfven(xi, nx, t=0.0, gamma=GAMMA_MHD):
    """Circularly polarised Alfven wave on [0, sqrt 2]^2 (paper §5.5, exact solution at time t):
    rho = 1, p = 0.1, v_perp = 0.1 sin(2 pi (x_perp + t)), v = (-v_perp sin a, v_perp cos a,
    0.1 cos(2 pi (x_perp + t))), B = (cos a + v1, sin a + v2, v3), a = pi/4."""
    L = math.sqrt(2.0)
    x, y = coords_2d(xi, nx, nx, (0.0, 0.0), (L, L))
    a = math.pi / 4
    xp = x * math.cos(a) + y * math.sin(a)
    vp = 0.1 * np.sin(2 * math.pi * (xp + t))
    v1 = -vp * math.sin(a)
    v2 = vp * math.cos(a)
    v3 = 0.1 * np.cos(2 * math.pi * (xp + t))
    one = np.ones_like(x)
    return _mhd_cons(one, v1, v2, v3, 0.1 * one, math.cos(a) + v1, math.sin(a) + v2, v3, 0 * one, gamma)


# ------------------------------------------------------------- 2-D SW ----
def sw2d_random(xi, n, seed=0):
    """Bed b = 0.1 sum_{k<6} c_k cos(2pi(m_k x + n_k y) + phi_k), |m|,|n| <= 3, c_k ~ U(-1,1)/sqrt 6;
    depth h = 1 + 0.2 eta/max|eta| with eta from the same recipe; v = 0."""
    rng = np.random.default_rng(seed)
    x, y = coords_2d(xi, n, n)

    def field():
        f = np.zeros_like(x)
        for _ in range(6):
            while True:
                m, k = rng.integers(-3, 4, size=2)
                if m != 0 or k != 0:
                    break
            c = rng.uniform(-1, 1) / math.sqrt(6)
            ph = rng.uniform(0, 2 * math.pi)
            f += c * np.cos(2 * math.pi * (m * x + k * y) + ph)
        return f

    b = 0.1 * field()
    eta = field()
    h = 1.0 + 0.2 * eta / np.max(np.abs(eta))
    z = np.zeros_like(x)
    return np.stack([h, z, z, b])


def sw2d_batch_specs(count=64, seed=0):
    """Sizes n_i ~ U{32..256} and degrees N_i ~ U{2,3,4} of the batched shallow-water instances."""
    rng = np.random.default_rng(seed)
    n = rng.integers(32, 257, size=count)
    N = rng.integers(2, 5, size=count)
    return [(int(a), int(b)) for a, b in zip(n, N)]


def steep_near_vacuum(xi, eq_dim, nvar, nx, seed=0, kmin=6.0, kmax=10.0, mhd=False, gamma=GAMMA_MHD):
    """Per element a steep exponential depth (shallow water) or density (GLM-MHD,
    then with uniform pressure 1) in x or in y, decaying over the element to near
    zero, toward a seeded side: every node is admissible, but the value a degree
    N >= 1 polynomial through the nodes extrapolates to the element's faces is
    negative on the low side at some degrees.  Small seeded velocities and
    fields, constant per element; zero bed."""
    rng = np.random.default_rng(seed)
    n1 = len(xi)
    E = nx if eq_dim == 1 else nx * nx
    P = n1 if eq_dim == 1 else n1 * n1
    u = np.zeros((nvar, E, P))
    for e in range(E):
        k = rng.uniform(kmin, kmax)
        x = xi if rng.uniform() < 0.5 else 1.0 - np.asarray(xi)
        prof = np.exp(-k * np.asarray(x))
        if eq_dim == 1:
            q = prof
        else:
            q = np.tile(prof, n1) if rng.uniform() < 0.5 else np.repeat(prof, n1)
        if not mhd:
            h = 0.5 * q + 1e-4
            u[0, e] = h
            u[1, e] = 0.05 * h * rng.uniform(-1, 1)
            if eq_dim == 2:
                u[2, e] = 0.05 * h * rng.uniform(-1, 1)
        else:
            rho = q + 1e-3
            v = 0.1 * rng.uniform(-1, 1, 3)
            B = 0.1 * rng.uniform(-1, 1, 3)
            c = [np.full_like(rho, x) for x in (v[0], v[1], v[2], 1.0, B[0], B[1], B[2], 0.0)]
            u[:, e] = _mhd_cons(rho, *c, gamma=gamma)
    return u
