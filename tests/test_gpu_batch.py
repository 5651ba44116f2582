"""Batched stepping of many independent problems (one launch per phase per step).

Checks, all through the C ABI:
  * a mixed batch (sizes 1x1 .. 9x9 elements, degrees 1..4, one problem with a
    fixed ragged shape) equals lwfr_step on each problem alone, bit for bit, and
    each problem's dt is the one lwfr_step computes;
  * every problem of that batch against the oracle, to the parity bar of the
    single-problem tests (1e-12 per value, relative to max(|value|, 1e-2 max|u^n|));
  * every launch shape (tiles of 256 or 128 threads, grid, XCD ranges) gives the
    same result bit for bit;
  * a captured graph of 10 steps, replayed three times with other work and
    synchronisations between the replays, equals 10 eager steps each time;
  * the 64-problem workload (sizes 32^2..256^2, degrees 2..4, seed 0): one
    autotuned batched step equals the single-problem steps bit for bit, every
    problem matches the oracle (dt to 1e-13, values to the parity bar), and 50
    graph-captured steps equal 50 eager batched steps.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2512_08611_amd import lwfr
from paper_2512_08611_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-12


def sw2d_state(xi, n, seed):
    u = W.sw2d_random(xi, n, seed)
    rng = np.random.default_rng(seed + 100)
    u[1] = 0.1 * u[0] * rng.uniform(-1, 1, u[0].shape[0])[:, None]
    u[2] = 0.05 * u[0] * rng.uniform(-1, 1, u[0].shape[0])[:, None]
    return u


def make_batch(specs, stream, **kw):
    # the oracle's CFL numbers, so that the oracle and the GPU take the same dt rule
    cfgs = [lwfr.make_config(lwfr.LWFR_EQ_SW2D, N, (n, n), cfl_number=oracle.cfl_number(N), **kw) for n, N in specs]
    return lwfr.Batch(cfgs, DEV, stream=stream), cfgs


def fill(b, specs, seed0):
    u = b.empty()
    states = []
    for i, (n, N) in enumerate(specs):
        xi = oracle.refel(N)["xi"]
        s = sw2d_state(xi, n, seed0 + i)
        states.append(s)
        b.view(u, i).copy_(torch.tensor(s, dtype=torch.float64))
    return u, states


def single_step(cfg, state, stream):
    st = lwfr.Stepper(cfg, DEV, stream=stream)
    ud = torch.tensor(state, dtype=torch.float64, device=DEV)
    out = torch.empty_like(ud)
    dtch = torch.zeros(2, dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    st.step(ud, out, 0.0, dtch)
    torch.cuda.synchronize()
    res = out.cpu(), float(dtch[0])
    st.close()
    return res


MIXED = [(3, 1), (5, 2), (7, 3), (4, 4), (1, 2), (9, 4), (2, 3), (6, 1), (8, 2), (5, 4), (3, 3)]


@pytest.fixture(scope="module")
def stream():
    return torch.cuda.Stream(DEV)


def test_batch_equals_single_problem_steps(stream):
    b, cfgs = make_batch(MIXED, stream)
    u, states = fill(b, MIXED, 10)
    out = b.empty()
    dt = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    b.step(u, out, dt)
    torch.cuda.synchronize()
    assert b.query() == (lwfr.LWFR_OK, 0)
    for i, cfg in enumerate(cfgs):
        ref, dti = single_step(cfg, states[i], stream)
        got = b.view(out, i).cpu()
        assert float(dt[i]) == dti, (i, float(dt[i]), dti)
        assert torch.equal(got, ref), (i, MIXED[i], float((got - ref).abs().max()))


def test_batch_against_oracle(stream):
    b, cfgs = make_batch(MIXED, stream)
    u, states = fill(b, MIXED, 20)
    out = b.empty()
    dt = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    b.step(u, out, dt)
    torch.cuda.synchronize()
    for i, (n, N) in enumerate(MIXED):
        oc = oracle.make_cfg(oracle.EQ_SW2D, N, n, n, cs=0.9, cfl=oracle.cfl_number(N), blending=2)
        o = oracle.step(oc, states[i])
        g = b.view(out, i).cpu().numpy()
        assert abs(float(dt[i]) - o["dt"]) <= 1e-13 * o["dt"]
        scale = np.maximum(np.abs(o["u"]), 1e-2 * np.abs(states[i]).max())
        err = (np.abs(g - o["u"]) / scale).max()
        print(f"BATCH PARITY problem {i} n={n} N={N} rel={err:.3e}", flush=True)
        assert err <= TOL


def test_launch_shapes_give_identical_results(stream):
    specs = MIXED[:6]
    b, _ = make_batch(specs, stream)
    u, _ = fill(b, specs, 30)
    ref = b.empty()
    torch.cuda.synchronize()
    b.step(u, ref)
    torch.cuda.synchronize()
    out = b.empty()
    for phase in range(4):
        for tt in ((256,) if phase == lwfr.LWFR_PHASE_FACES else (256, 128)):
            for grid in (0, 1, 8, 24):
                for xcd in (0, 1, 2, 4):
                    b.set_launch(phase, tt, grid, xcd)
                    out.fill_(0.0)
                    torch.cuda.synchronize()
                    b.step(u, out)
                    torch.cuda.synchronize()
                    assert torch.equal(out, ref), (phase, tt, grid, xcd)
        b.set_launch(phase, 256, 0, 1)


def test_graph_replays_match_eager_steps(stream):
    specs = MIXED[:7]
    nsteps = 10
    b, _ = make_batch(specs, stream)
    u0, _ = fill(b, specs, 40)
    # eager reference
    ua, ub = u0.clone(), b.empty()
    dts = torch.zeros((nsteps, len(b)), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    for k in range(nsteps):
        b.step(ua, ub, dts[k])
        ua, ub = ub, ua
    torch.cuda.synchronize()
    ref = ua.clone()
    # graph
    ga, gb = b.empty(), b.empty()
    hist = torch.zeros((nsteps, len(b)), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    b.graph_capture(ga, gb, nsteps, hist)
    scratch = b.empty()
    for rep in range(3):
        ga.copy_(u0)
        hist.fill_(0.0)
        torch.cuda.synchronize()
        b.graph_launch()
        torch.cuda.synchronize()
        assert torch.equal(ga, ref), rep
        assert torch.equal(hist, dts), rep
        # other work on the same stream between replays
        b.step(u0, scratch)
        torch.cuda.synchronize()


def test_single_problem_graph_matches_eager(stream):
    cfg = lwfr.make_config(lwfr.LWFR_EQ_GLMMHD2D, 3, (6, 5), blending=2)
    st = lwfr.Stepper(cfg, DEV, stream=stream)
    xi = np.array(st.xi)
    u0 = torch.tensor(W.mhd_blocky(xi, 6, 5, 3, nblocks=3), dtype=torch.float64, device=DEV)
    nsteps = 6
    ua, ub = u0.clone(), torch.empty_like(u0)
    dtch = torch.zeros((nsteps, 2), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    for k in range(nsteps):
        st.step(ua, ub, 0.0, dtch[k])
        ua, ub = ub, ua
    torch.cuda.synchronize()
    ga, gb = u0.clone(), torch.empty_like(u0)
    hist = torch.zeros((nsteps, 2), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    st.graph_capture(ga, gb, nsteps, hist)
    for rep in range(2):
        ga.copy_(u0)
        torch.cuda.synchronize()
        st.graph_launch()
        torch.cuda.synchronize()
        assert torch.equal(ga, ua), rep
        assert torch.equal(hist, dtch), rep


@pytest.mark.parametrize("case", ["mhd4", "mhd3_outflow", "sw1d", "jinxin", "sw2d_walls"])
def test_single_problem_graph_matches_eager_more(stream, case):
    """Captured sequences form each step's element data in the previous step's update
    (no k_pre after the first step): bit-identical to eager steps, which run k_pre."""
    if case == "mhd4":
        cfg = lwfr.make_config(lwfr.LWFR_EQ_GLMMHD2D, 4, (9, 7), blending=2)
        gen = lambda xi: W.mhd_blocky(xi, 9, 7, 5, nblocks=4)
    elif case == "mhd3_outflow":
        # outflow sides: every face's F^+ is stored (a boundary slot holds two faces)
        cfg = lwfr.make_config(lwfr.LWFR_EQ_GLMMHD2D, 3, (7, 6), blending=2, bc=(1, 1, 1, 1))
        gen = lambda xi: W.mhd_blocky(xi, 7, 6, 6, nblocks=3)
    elif case == "sw1d":
        cfg = lwfr.make_config(lwfr.LWFR_EQ_SW1D, 3, 37, blending=2)
        gen = lambda xi: W.sw1d_wave(xi, 37, 2)
    elif case == "jinxin":
        cfg = lwfr.make_config(lwfr.LWFR_EQ_JINXIN1D, 2, 41, lo=(-1.0, 0.0), blending=2,
                               flags=lwfr.LWFR_CFG_IMEX_SSP3, source=(3.0, 1e-3, 0.0, 1.0))
        gen = lambda xi: W.jinxin_sine(xi, 41)
    else:
        cfg = lwfr.make_config(lwfr.LWFR_EQ_SW2D, 3, (8, 8), blending=2, bc=(2, 2, 2, 2))
        gen = lambda xi: sw2d_state(xi, 8, 4)
    st = lwfr.Stepper(cfg, DEV, stream=stream)
    u0 = torch.tensor(gen(np.array(st.xi)), dtype=torch.float64, device=DEV)
    nsteps = 5
    ua, ub = u0.clone(), torch.empty_like(u0)
    dtch = torch.zeros((nsteps, 2), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    for k in range(nsteps):
        st.step(ua, ub, 0.0, dtch[k])
        ua, ub = ub, ua
    torch.cuda.synchronize()
    ga, gb = u0.clone(), torch.empty_like(u0)
    hist = torch.zeros((nsteps, 2), dtype=torch.float64, device=DEV)
    st.graph_capture(ga, gb, nsteps, hist)
    for rep in range(2):
        ga.copy_(u0)
        torch.cuda.synchronize()
        st.graph_launch()
        torch.cuda.synchronize()
        got = ga if nsteps % 2 == 0 else gb
        assert torch.equal(got, ua), rep
        assert torch.equal(hist, dtch), rep
    # eager work after the replays still sees consistent element data
    st.step(u0, ub, 0.0, dtch[0])
    torch.cuda.synchronize()
    assert st.query()[0] == lwfr.LWFR_OK


def test_graph_needs_a_stream():
    cfg = lwfr.make_config(lwfr.LWFR_EQ_SW2D, 2, (3, 3))
    b = lwfr.Batch([cfg], DEV, stream=torch.cuda.default_stream(DEV))
    u, v = b.empty(), b.empty()
    with pytest.raises(lwfr.LwfrError) as ei:
        b.graph_capture(u, v, 2)
    assert ei.value.status == lwfr.LWFR_E_STATE


def test_full_size_batch_64_problems(stream):
    specs = W.sw2d_batch_specs(64, seed=0)
    b, cfgs = make_batch(specs, stream)
    ndof = sum(n * n * (N + 1) ** 2 for n, N in specs)
    print(f"BATCH 64 problems, {ndof} DOF", flush=True)
    u, states = fill(b, specs, 1000)
    out = b.empty()
    torch.cuda.synchronize()
    b.autotune(u, out, reps=2)
    print("BATCH autotuned launch shapes", [b.get_launch(p) for p in range(4)], flush=True)
    dt = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    b.step(u, out, dt)
    torch.cuda.synchronize()
    assert b.query() == (lwfr.LWFR_OK, 0)
    for i, cfg in enumerate(cfgs):
        ref, dti = single_step(cfg, states[i], stream)
        assert float(dt[i]) == dti, i
        assert torch.equal(b.view(out, i).cpu(), ref), (i, specs[i])
    # every problem against the oracle (its element and face loops on the host's cores)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    worst = 0.0
    for i in range(len(specs)):
        n, N = specs[i]
        oc = oracle.make_cfg(oracle.EQ_SW2D, N, n, n, cs=0.9, cfl=oracle.cfl_number(N), blending=2, threads=threads)
        o = oracle.step(oc, states[i])
        assert float(dt[i]) == pytest.approx(o["dt"], rel=1e-13), i
        g = b.view(out, i).cpu().numpy()
        scale = np.maximum(np.abs(o["u"]), 1e-2 * np.abs(states[i]).max())
        err = (np.abs(g - o["u"]) / scale).max()
        worst = max(worst, err)
        assert err <= TOL, (i, n, N, err)
    print(f"BATCH PARITY all 64 problems against the oracle: worst rel={worst:.3e}", flush=True)
    # 50 graph-captured steps against 50 eager batched steps
    nsteps = 50
    ua, ub = u.clone(), b.empty()
    torch.cuda.synchronize()
    for k in range(nsteps):
        b.step(ua, ub)
        ua, ub = ub, ua
    ga, gb = u.clone(), b.empty()
    torch.cuda.synchronize()
    b.graph_capture(ga, gb, nsteps)
    b.graph_launch()
    torch.cuda.synchronize()
    assert torch.equal(ga, ua)
    assert b.query() == (lwfr.LWFR_OK, 0)
