"""Fourier (von Neumann) stability limit CFL(N) of the time-averaged scheme.

TEST INFRASTRUCTURE ONLY.

The paper takes CFL(N) from the Fourier analysis of the linearly equivalent
Lax-Wendroff FR scheme (§5, paragraph after eq. time.step.2d); the table it
cites is not part of the paper, so the number is recomputed here from the
scheme itself.  For u_t + u_x = 0 (f = u, wave speed 1) with nu = dt/dx:

* the stages give the time average U = F = T u_e with
  T = sum_{k=0}^{N} (-nu D)^k/(k+1)!   (D^{N+1} = 0 on P_N, and an order N+1
  tableau reproduces the Taylor weights 1/(k+1)!),
* the Rusanov flux with lambda = 1 is the upwind value F^num_{e+1/2} = V_R^T T u_e,
* the update (eq. crkfr with the Radau correction) is
  u_e^{n+1} = u_e - nu [ D T u_e + g_L' (V_R^T T u_{e-1} - V_L^T T u_e) ].
With u_{e-1} = exp(-i theta) u_e this is u_e^{n+1} = G(theta) u_e; CFL(N) is
the largest nu with spectral radius rho(G(theta)) <= 1 for all theta.

With an IMEX pair (systems with a source) the flux terms use its explicit
part (A~, b~), whose order can be below N+1; then T = sum_i b~_i R_i with the
stage operators R_1 = I, R_i = I + sum_{k<i} a~_ik (-nu D) R_k (the source is
zero in this linear analysis).
"""
import functools
import math

import numpy as np


def time_average_operator(N, nu, D, tableau=None):
    """T with U = T u: the Taylor weights, or the explicit tableau (A~, b~) if given."""
    n1 = N + 1
    if tableau is None:
        T = np.zeros((n1, n1))
        Pk = np.eye(n1)
        for k in range(N + 1):
            T = T + Pk / math.factorial(k + 1)
            Pk = Pk @ (-nu * D)
        return T
    A, b = tableau
    R = []
    for i in range(len(b)):
        Ri = np.eye(n1)
        for k in range(i):
            if A[i, k] != 0.0:
                Ri = Ri + A[i, k] * (-nu * D) @ R[k]
        R.append(Ri)
    return sum(b[i] * R[i] for i in range(len(b)))


def amplification(N, nu, theta, re, tableau=None):
    D = re["D"]
    n1 = N + 1
    T = time_average_operator(N, nu, D, tableau)
    gL = re["gLp"].reshape(n1, 1)
    VR = re["VR"].reshape(1, n1)
    VL = re["VL"].reshape(1, n1)
    return np.eye(n1) - nu * (D @ T + gL @ (np.exp(-1j * theta) * VR - VL) @ T)


def max_growth(N, nu, re, ntheta=721, tableau=None):
    thetas = np.linspace(0.0, np.pi, ntheta)[1:]
    return max(np.max(np.abs(np.linalg.eigvals(amplification(N, nu, t, re, tableau)))) for t in thetas)


@functools.lru_cache(maxsize=None)
def cfl_number(N, gll=False, imex=0):
    """Largest nu with rho(G) <= 1 + tol for degree N (bisection to 1e-10 in nu);
    gll: Gauss-Lobatto-Legendre points with the g_2 correction.

    tol = 1e-12 for N <= 3.  For N = 4 the order-5 Taylor weights leave nearly
    undamped modes a weak growth of order (nu theta)^6 (about 5e-6 per step
    just below the limit); the limit is the sharp loss of stability of the
    high-frequency modes, so there a growth below tol = 1e-5 per step counts as
    stable.  imex: the explicit part of that IMEX pair in place of the degree's
    tableau (same tolerances).
    """
    tol = 1e-12 if N <= 3 else 1e-5
    from . import refel, tableau_imex

    re = refel(N, gll)
    tab = None
    if imex:
        A, b, _, _ = tableau_imex(imex)
        tab = (A, b)
    lo, hi = 0.0, 1.5
    while hi - lo > 1e-10:
        mid = 0.5 * (lo + hi)
        if max_growth(N, mid, re, tableau=tab) <= 1.0 + tol:
            lo = mid
        else:
            hi = mid
    return lo
