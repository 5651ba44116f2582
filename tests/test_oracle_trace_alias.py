"""GLM-MHD flux components that the time-averaged solution fixes.

Three components of the GLM-MHD flux are linear in the state: the mass flux
f_d[0] = u[1+d] and the GLM terms f_d[5+d] = c_h psi and f_d[8] = c_h B_d (§5.5).
Any weighted sum over states therefore keeps them tied to the same sum of u:
for the cRK averages F_d = sum_s b_s f_d(u^(s)) and U = sum_s b_s u^(s) (§3), and
for the approximate Lax-Wendroff averages over Taylor states in time, at every
solution point and so at every face trace:

    F_d[0] = U[1+d],   F_d[5+d] = c_h U[8],   F_d[8] = c_h U[5+d].

The GPU step stores only the other six components of the F_d face traces and
forms these three from the U traces.  Here the oracle's averages are checked
for the identity on smooth and blocky data, N = 1..4, with both time-averaging
procedures.  A c_h term dropped from the oracle's flux, a swapped B component or
a stage weight applied to F and not to U fails.
"""
import numpy as np
import pytest

import oracle
from paper_2512_08611_amd import workloads as W


@pytest.mark.parametrize("alw", [False, True])
@pytest.mark.parametrize("kind", ["smooth", "blocky"])
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_linear_flux_components_follow_from_U(N, kind, alw):
    nx = ny = 4
    c = oracle.make_cfg(oracle.EQ_MHD2D, N, nx, ny, blending=2, alw=alw)
    xi = oracle.refel(N)["xi"]
    u = W.mhd_smooth(xi, nx, ny, seed=3) if kind == "smooth" else W.mhd_blocky(xi, nx, ny, seed=3, nblocks=2)
    dt, ch = oracle.dt_ch(c, u)
    assert ch > 0.0
    F, U, _ = oracle.time_averages(c, u, dt, ch)
    for d in range(2):
        for v, w, scale in ((0, 1 + d, 1.0), (5 + d, 8, ch), (8, 5 + d, ch)):
            want = scale * U[w]
            tol = 1e-13 * max(np.abs(want).max(), np.abs(F[d][v]).max(), 1e-300)
            err = np.abs(F[d][v] - want).max()
            assert err <= tol, (d, v, err, tol)
    # the other components are not fixed by U (a check that the test can fail)
    assert np.abs(F[0][1] - U[1]).max() > 1e-3 * np.abs(U[1]).max()
