"""Approximate Lax-Wendroff time averages on the GPU (LWFR_CFG_ALW), through the C ABI.

  * one step against the oracle to the parity bar of the cRK tests (1e-12 per
    value relative to max(|value|, 1e-2 max|u^n|), dt to 1e-13, alpha_e to
    1e-12, flags bit-exact) for every system, N = 1..4, blending off / indicator /
    limiting, smooth and blocky MHD data, and at the full 256^2 N=4 GLM-MHD size;
  * with non-periodic sides (outflow and walls);
  * the Alfven wave's design order on the GPU (N = 2, 3).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2512_08611_amd import lwfr
from paper_2512_08611_amd import workloads as W
from test_gpu_parity import DEV, Pair, _data

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("blending", [0, 1, 2])
@pytest.mark.parametrize("eq", [oracle.EQ_SW1D, oracle.EQ_LINADV1D, oracle.EQ_VARADV1D])
def test_parity_1d(eq, N, blending):
    nx = 137
    pr = Pair(eq, N, nx, blending=blending, alw=True)
    for seed in (0, 1):
        pr.check(_data(eq, N, nx, 1, seed))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("blending", [0, 2])
def test_parity_sw2d(N, blending):
    pr = Pair(oracle.EQ_SW2D, N, 9, 9, blending=blending, alw=True)
    for seed in (0, 1):
        pr.check(_data(oracle.EQ_SW2D, N, 9, 9, seed))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("blending", [0, 1, 2])
@pytest.mark.parametrize("kind", ["smooth", "blocky"])
def test_parity_mhd(N, blending, kind):
    pr = Pair(oracle.EQ_MHD2D, N, 9, 7, blending=blending, alw=True)
    for seed in (0, 1):
        g, o = pr.check(_data(oracle.EQ_MHD2D, N, 9, 7, seed, kind))
    if kind == "blocky" and blending == 2 and N >= 2:
        assert (o["flags"] & (oracle.FLAG_ALG1 | oracle.FLAG_ALG2)).any()


@pytest.mark.parametrize("bc", [(lwfr.LWFR_BC_OUTFLOW,) * 4, (lwfr.LWFR_BC_WALL,) * 4])
def test_parity_nonperiodic(bc):
    eq = oracle.EQ_SW2D if bc[0] == lwfr.LWFR_BC_WALL else oracle.EQ_MHD2D
    for N in (2, 4):
        pr = Pair(eq, N, 8, 8, blending=2, alw=True, bc=bc)
        pr.check(_data(eq, N, 8, 8, 3, "blocky") if eq == oracle.EQ_MHD2D else _data(eq, N, 8, 8, 3))


def test_parity_mhd_256_n4_full_size():
    """GLM-MHD 256x256 elements, N=4: one step with the approximate LW averages."""
    pr = Pair(oracle.EQ_MHD2D, 4, 256, 256, blending=2, alw=True)
    pr.check(_data(oracle.EQ_MHD2D, 4, 256, 256, 0))


@pytest.mark.parametrize("N,ns", [(2, (8, 12)), (3, (4, 8))])
def test_alfven_order_on_gpu(N, ns):
    L = math.sqrt(2.0)
    errs = []
    for n in ns:
        cfg = lwfr.make_config(lwfr.LWFR_EQ_GLMMHD2D, N, (n, n), lo=(0.0, 0.0), hi=(L, L), blending=0,
                               flags=lwfr.LWFR_CFG_ALW)
        st = lwfr.Stepper(cfg, DEV)
        xi = np.array(st.xi)
        u = torch.tensor(W.alfven(xi, n), dtype=torch.float64, device=DEV)
        v = torch.empty_like(u)
        dtch = torch.zeros(2, dtype=torch.float64, device=DEV)
        st.step(u, v, 0.0, dtch)
        nsteps = int(math.ceil(0.2 / float(dtch[0])))
        for _ in range(nsteps):
            st.step(u, v, 0.2 / nsteps)
            u, v = v, u
        ex = W.alfven(xi, n, t=0.2)
        w = np.array(st.w)
        wn = np.outer(w, w).reshape(-1)
        errs.append(math.sqrt(((u.cpu().numpy()[1] - ex[1]) ** 2 * wn).sum() * (L / n) ** 2))
        st.close()
    rate = math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0])
    print(f"ALW ALFVEN N={N} errs={errs} rate={rate:.2f}", flush=True)
    assert rate > N + 1 - 0.35
