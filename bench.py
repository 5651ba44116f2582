"""Throughput of the time step on one MI355X, with roofline and CPU-oracle baseline.

Workload of the headline line (the largest single-problem configuration):
2-D ideal GLM-MHD on 512 x 512 periodic elements, N = 3 (16 Gauss-Legendre
points per element, 4,194,304 solution points), blocky data (16 x 16 constant
blocks with density and pressure ratios up to 10 and 100 and random fields,
at rest, jumps inside elements; seed 0), FP64, C_s = 0.9 with CFL(N) from the
library's Fourier analysis, subcell blending with Algorithms 1 and 2 active,
dt computed on the device every step.  The secondary line is the smooth
Orszag-Tang workload (256 x 256, N = 4).

One "step" is one full time step (means/indicator, dt and c_h, element stages,
faces, update).  The state is resident in HBM before the timed region.  The
timed region is K consecutive steps captured as one HIP graph (the library's
lwfr_graph_capture; dt is computed on the device every step) and replayed
once, bracketed by device synchronisation, after one untimed replay.  The same
K steps launched one by one with HIP events around every kernel give the
per-kernel durations and ms_per_step_eager.

Output: one JSON line (see the keys below).  value = DOF-updates/s =
elements * points per element * K / wall time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FP64 DOF-updates/s per LWFR step (1 GPU, % roofline); adjoint/forward time"
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X FP64 vector, published
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published

# Algorithmic floating point operations per solution point of the element-local
# stage loop (inner stages, local operator, time averages F, U, B^loc), counted
# by the oracle's counting scalar (+, -, *, / each one operation) over the
# tableau's non-zero entries and the non-zero columns of B_d.
STAGE_LOOP_FLOPS_PER_DOF = {
    ("GLMMHD2D", 4): 3561,
    ("GLMMHD2D", 3): 2153,
}
# The work of the dominant kernel, k_stages: the stage loop and the face traces
# of F_d, U and u^n (the oracle's next phase, 231.2 and 235 flops per point at
# N = 4 and 3).  The kernel also forms the folded correction offsets, which the
# oracle counts with its faces and update; they are not counted here, so the
# achieved rate is a lower bound.  tests/test_bench_contract.py re-counts both.
STAGE_KERNEL_FLOPS_PER_DOF = {
    ("GLMMHD2D", 4): 3792.2,
    ("GLMMHD2D", 3): 2388.0,
}
# Algorithmic floating point operations per solution point of a whole step
# (means, dt and c_h, indicator; stage loop; face traces; faces with Algorithm
# 1; update with the subcell scheme and Algorithm 2), counted by the oracle's
# counting scalar on a 16x16-element sample of the workload's recipe (the
# count does not depend on the data to 0.1 flop per point).  The indicator is
# counted in the oracle's plain form (each Legendre mode as a full double sum),
# a few percent above the factored projection the kernel uses.
# tests/test_bench_contract.py re-counts.
STEP_FLOPS_PER_DOF = {
    (3, "blocky"): 5015.8,
    (4, "smooth"): 6392.4,
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mhd512_n3_blocky", choices=sorted(WORKLOADS),
                    help="the timed workload (the other one is measured as the secondary line)")
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary workload's line")
    ap.add_argument("--graph-trace", action="store_true",
                    help="profiling runs: only the warm-up and the graph-replayed steps run (no event-timed pass)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps of the CPU baseline sample")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward time measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-problem measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the rotor run and the variants (GLL, approximate LW, Jin-Xin IMEX): profiling runs")
    ap.add_argument("--no-references", action="store_true",
                    help="skip the measured device references (a 1 GiB copy and an FP64 matrix product; "
                         "also skipped with --no-extras or --copy-calibration)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of 256 MiB (reference kernel for the HBM byte counters)")
    return ap.parse_args()


def device_references(torch, reps=5):
    """What this GPU reaches on plain reference work, beside the published peaks the
    roofline uses: a 1 GiB device-to-device copy (read + write bytes per second) and
    an 8192^3 FP64 matrix product through the ROCm BLAS library (dense FP64 flops per
    second).  Each is timed with events on the current stream, best of `reps`."""
    dev = torch.device("cuda:0")
    res = {}
    a = torch.ones(128 * 1024 * 1024, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    res["copy_GBs"] = 2 * a.numel() * 8 / min(ts) / 1e9
    del a, b
    n = 8192
    A = torch.rand((n, n), dtype=torch.float64, device=dev)
    B = torch.rand((n, n), dtype=torch.float64, device=dev)
    C = torch.matmul(A, B)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.matmul(A, B, out=C)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    res["fp64_gemm_TFLOPs"] = 2.0 * n ** 3 / min(ts) / 1e12
    res["note"] = ("measured on this GPU for context; the roofline fractions use the published peaks "
                   "(8 TB/s HBM, 78.6 TFLOP/s FP64 vector)")
    return res


def cpu_baseline(u0, n, N, steps):
    """The oracle, as it stands, on the host: `steps` steps of the same workload."""
    import numpy as np

    import oracle

    c = oracle.make_cfg(oracle.EQ_MHD2D, N, n, n, blending=2, cs=0.9)
    u = np.ascontiguousarray(u0)
    t0 = time.perf_counter()
    for _ in range(steps):
        u = oracle.step(c, u)["u"]
    dt = time.perf_counter() - t0
    dofs = u.shape[1] * u.shape[2]
    return {
        "value": dofs * steps / dt,
        "unit": "DOF-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} steps of the full {n}x{n} N={N} GLM-MHD workload, single-threaded C++ oracle "
                  f"({dt:.1f} s)",
        "host": host_info(),
    }


def adjoint_over_forward(torch, lwfr, workloads, np, n=128, N=3, steps=20, every=5, reps=3):
    """Backward (checkpoint recomputation + adjoint steps) time over forward time of a
    differentiable rollout: GLM-MHD n x n, degree N, `steps` steps, checkpoint every `every`."""
    from paper_2512_08611_amd import rollout

    dev = torch.device("cuda:0")
    cfg = lwfr.make_config(lwfr.LWFR_EQ_GLMMHD2D, N, (n, n), blending=2, flags=lwfr.LWFR_CFG_ADJOINT)
    st = lwfr.Stepper(cfg, dev)
    u0 = torch.tensor(workloads.mhd_smooth(np.array(st.xi), n, n, seed=0), dtype=torch.float64, device=dev)
    tf, tb = [], []
    for r in range(reps + 1):
        x = u0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = rollout.rollout(x, st, steps, every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = 0.5 * torch.sum(y[0] ** 2)
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r > 0:  # the first repetition warms up
            tf.append(t1 - t0)
            tb.append(t2 - t1)
    f, b = min(tf), min(tb)
    return {"ratio": b / f, "forward_ms": f * 1e3, "backward_ms": b * 1e3,
            "workload": f"GLM-MHD {n}x{n} N={N}, {steps} steps, checkpoint every {every}"}


def batched(torch, lwfr, workloads, np, steps=50, count=64):
    """64 independent 2-D shallow-water problems (sizes n ~ U{32..256}, degrees
    N ~ U{2,3,4}, seed 0; bed and depth from seeded cosine modes), advanced with
    one launch per phase per step, launch shapes from the library's autotuner,
    `steps` steps captured in one HIP graph and replayed (the first replay warms up)."""
    dev = torch.device("cuda:0")
    specs = workloads.sw2d_batch_specs(count, seed=0)
    cfgs = [lwfr.make_config(lwfr.LWFR_EQ_SW2D, N, (n, n), cfl_safety=0.9, blending=2) for n, N in specs]
    stream = torch.cuda.Stream(dev)
    b = lwfr.Batch(cfgs, dev, stream=stream)
    u0 = b.empty()
    for i, (n, N) in enumerate(specs):
        xi, _ = lwfr.lwfr_reference_nodes(b.problem(i), N + 1)
        b.view(u0, i).copy_(torch.tensor(workloads.sw2d_random(np.array(xi), n, seed=1000 + i)))
    dofs = sum(n * n * (N + 1) ** 2 for n, N in specs)
    scratch = b.empty()
    torch.cuda.synchronize()
    b.autotune(u0, scratch, reps=3)
    shapes = {name: b.get_launch(ph) for ph, name in enumerate(("pre", "stages", "faces", "update"))}
    # eager steps with per-kernel timing
    b.timing_begin(64)
    b.step(u0, scratch)
    kern = b.timing_end()
    ua, ub = b.empty(), b.empty()
    ua.copy_(u0)
    torch.cuda.synchronize()
    b.graph_capture(ua, ub, steps)
    b.graph_launch()  # warm-up replay
    torch.cuda.synchronize()
    ua.copy_(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.graph_launch()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t0 = time.perf_counter()
    for k in range(steps):
        b.step(ua if k % 2 == 0 else ub, ub if k % 2 == 0 else ua)
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0
    status, flags = b.query()
    return {
        "workload": f"{count} 2-D shallow-water problems with bathymetry, n~U{{32..256}}^2 elements, "
                    f"N~U{{2,3,4}} (seed 0), {dofs} DOF, {steps} graph-captured steps",
        "value": dofs * steps / wall,
        "unit": "DOF-updates/s",
        "ms_per_step": wall / steps * 1e3,
        "ms_per_step_eager": wall_eager / steps * 1e3,
        "dof": dofs,
        "launch_shapes": {k: {"tile_threads": v[0], "grid": v[1], "xcd": v[2]} for k, v in shapes.items()},
        "kernels_ms_per_step": {k: ms for k, (ms, cnt) in kern.items() if cnt},
        "step_status": int(status),
        "flags_or": int(flags),
    }


def variant_timing(torch, lwfr, workloads, np, n, N, flags, steps, name):
    """ms per step of the default workload with other lwfr_config.flags (e.g. GLL points)."""
    dev = torch.device("cuda:0")
    cfg = lwfr.make_config(lwfr.LWFR_EQ_GLMMHD2D, N, (n, n), cfl_safety=0.9, blending=2, flags=flags)
    st = lwfr.Stepper(cfg, dev)
    ua = torch.tensor(workloads.mhd_smooth(np.array(st.xi), n, n, seed=0), dtype=torch.float64, device=dev)
    ub = torch.empty_like(ua)
    for _ in range(3):
        st.step(ua, ub)
        ua, ub = ub, ua
    lwfr.lwfr_timing_begin(st.ctx, 8 * steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step(ua, ub)
        ua, ub = ub, ua
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = lwfr.lwfr_timing_end(st.ctx)
    status, flags_or = st.query()
    dofs = n * n * (N + 1) ** 2
    return {
        "variant": name,
        "workload": f"GLM-MHD {n}x{n}, N={N}, same data and settings as the main line",
        "value": dofs * steps / wall,
        "unit": "DOF-updates/s",
        "ms_per_step": wall / steps * 1e3,
        "cfl_number": lwfr.lwfr_cfl_number(N, flags),
        "kernels_ms_per_launch": {k: ms / c for k, (ms, c) in kern.items() if c},
        "step_status": int(status),
        "flags_or": int(flags_or),
    }


def jinxin_timing(torch, lwfr, workloads, np, steps, nx=1 << 20, N=3, eps=1e-12):
    """The Jin-Xin relaxation system (eq. jin.xin.ic on [-1, 1], a = 3, Burgers flux) with
    SSP3-IMEX(4,3,3) at the paper's stiffest eps, N = 3, nx elements: DOF-updates/s."""
    dev = torch.device("cuda:0")
    cfg = lwfr.make_config(lwfr.LWFR_EQ_JINXIN1D, N, nx, lo=(-1.0, 0.0), hi=(1.0, 1.0), blending=2,
                           flags=lwfr.LWFR_CFG_IMEX_SSP3, source=(3.0, eps, 0.0, 1.0))
    st = lwfr.Stepper(cfg, dev)
    ua = torch.tensor(workloads.jinxin_sine(np.array(st.xi), nx), dtype=torch.float64, device=dev)
    ub = torch.empty_like(ua)
    for _ in range(3):
        st.step(ua, ub)
        ua, ub = ub, ua
    lwfr.lwfr_timing_begin(st.ctx, 8 * steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step(ua, ub)
        ua, ub = ub, ua
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = lwfr.lwfr_timing_end(st.ctx)
    status, flags_or = st.query()
    dofs = nx * (N + 1) * 2
    return {
        "workload": f"Jin-Xin relaxation (Burgers, a=3, eps={eps:g}), {nx} elements, N={N}, SSP3-IMEX(4,3,3)",
        "value": nx * (N + 1) * steps / wall, "unit": "DOF-updates/s (solution points x steps)",
        "ms_per_step": wall / steps * 1e3, "variables": 2, "doubles_per_state": dofs,
        "kernels_ms_per_launch": {k: ms / c for k, (ms, c) in kern.items() if c},
        "step_status": int(status), "flags_or": int(flags_or),
    }


def rotor_run(torch, lwfr, workloads, np, n=256, N=4, tend=0.15, gamma=1.4):
    """The MHD rotor (eq. rotor.ic) to t = 0.15 with N = 4 on n x n elements, dt from the
    CFL rule on the device each step, blending with Algorithms 1 and 2."""
    dev = torch.device("cuda:0")
    cfg = lwfr.make_config(lwfr.LWFR_EQ_GLMMHD2D, N, (n, n), gamma=gamma, blending=2)
    st = lwfr.Stepper(cfg, dev)
    ua = torch.tensor(workloads.mhd_rotor(np.array(st.xi), n, gamma), dtype=torch.float64, device=dev)
    ub = torch.empty_like(ua)
    hist = torch.zeros((20000, 2), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t, k = 0.0, 0
    while t < tend and k < hist.shape[0]:
        # dt read back every 64 steps only: the device computes each step's dt
        st.step(ua, ub, 0.0, hist[k])
        ua, ub = ub, ua
        k += 1
        if k % 64 == 0:
            t = float(hist[:k, 0].sum())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t = float(hist[:k, 0].sum())
    status, flags = st.query()
    dofs = n * n * (N + 1) ** 2
    return {"workload": f"MHD rotor (eq. rotor.ic, gamma {gamma}) {n}x{n}, N={N}, to t >= {tend}",
            "steps": k, "t_end": t, "ms_per_step": wall / k * 1e3, "value": dofs * k / wall,
            "unit": "DOF-updates/s", "step_status": int(status), "flags_or": int(flags)}


def host_info():
    """The host CPU model and the cores this process may use (the oracle's baseline runs on them)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


WORKLOADS = {
    # name: (elements per direction, degree, data)
    "mhd512_n3_blocky": (512, 3, "blocky"),
    "mhd256_n4_smooth": (256, 4, "smooth"),
}


def workload_state(workloads, np, xi, n, data):
    if data == "blocky":
        return workloads.mhd_blocky(np.array(xi), n, n, seed=0)
    return workloads.mhd_smooth(np.array(xi), n, n, seed=0)


def workload_text(n, N, data):
    dofs = n * n * (N + 1) ** 2
    if data == "blocky":
        return (f"2-D GLM-MHD, 16x16 piecewise-constant blocks (rho 10^U(-1,0), p 10^U(-2,0), B 0.5 U(-1,1), "
                f"at rest; jumps inside elements; seed 0), {n}x{n} periodic elements, N={N} Gauss-Legendre "
                f"({dofs} DOF, 9 variables), blending + Algorithms 1-2, C_s=0.9")
    return (f"2-D GLM-MHD Orszag-Tang + 1e-2 seeded Fourier perturbations, {n}x{n} periodic elements, "
            f"N={N} Gauss-Legendre ({dofs} DOF, 9 variables), blending + Algorithms 1-2, C_s=0.9")


def kernel_rooflines(table, per_kernel, K):
    """Every kernel of a step against both rooflines, and the HBM bytes of one
    graph-replayed step: counter figures (table: counters.read_table of the
    committed summary) with the live eager durations (per_kernel)."""
    by_kernel = None
    step_bytes = None
    if table:
        by_kernel, step_bytes = {}, 0.0
        for name, row in table.items():
            base = name.split("<")[0]
            key = next((k for k in per_kernel if base == k or base.startswith(k + "2")), None)
            if key is None or not per_kernel[key]["ms_per_launch"]:
                continue
            # a captured K-step sequence runs k_pre once, the update that also
            # forms the next step's element data K-1 times and the plain update
            # once; every other kernel once a step
            chained = name.endswith(", true>")
            per_graph_step = {"k_pre": 1.0 / K}.get(key, 1.0)
            if key == "k_update":
                per_graph_step = (K - 1) / K if chained else 1.0 / K
            if "bytes" in row:
                step_bytes += row["bytes"] * per_graph_step
            if chained:
                continue  # the live durations are those of the eager steps' plain update
            sec = per_kernel[key]["ms_per_launch"] * 1e-3
            ent = {"counted_kernel": name, "ms_per_launch": per_kernel[key]["ms_per_launch"]}
            if "bytes" in row:
                gbs = row["bytes"] / sec / 1e9
                ent.update(hbm_bytes=row["bytes"], hbm_GBs=gbs, hbm_frac=gbs / HBM_PEAK_GBS)
            if "fp64_ops" in row:
                tf = row["fp64_ops"] / sec / 1e12
                ent.update(fp64_hw_ops=row["fp64_ops"], fp64_TFLOPs=tf, fp64_frac=tf / FP64_VECTOR_PEAK_TFLOPS)
            by_kernel[key] = ent
    return by_kernel, step_bytes


def measure(torch, np, lwfr, workloads, counters, n, N, data, K, Wm, graph_trace=False):
    """One workload: Wm warm-up steps, K steps launched one by one with HIP events
    around every kernel (per-kernel durations, ms_per_step_eager), then the timed
    region: the same K steps as one HIP graph replayed once after an untimed replay."""
    dev = torch.device("cuda:0")
    cfg = lwfr.make_config(lwfr.LWFR_EQ_GLMMHD2D, N, (n, n), cfl_safety=0.9, blending=2)
    stream = torch.cuda.Stream(dev)  # graph capture needs a non-default stream
    st = lwfr.Stepper(cfg, dev, stream=stream)
    u0 = workload_state(workloads, np, st.xi, n, data)
    ua = torch.tensor(u0, dtype=torch.float64, device=dev)
    ub = torch.empty_like(ua)
    dtch = torch.zeros(2, dtype=torch.float64, device=dev)
    E, P = n * n, (N + 1) ** 2
    dofs = E * P
    for _ in range(Wm):
        st.step(ua, ub, 0.0, dtch)
        ua, ub = ub, ua
    torch.cuda.synchronize()
    per_kernel, wall_eager = {}, None
    if not graph_trace:
        lwfr.lwfr_timing_begin(st.ctx, 8 * K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            st.step(ua, ub, 0.0, dtch)
            ua, ub = ub, ua
        torch.cuda.synchronize()
        wall_eager = time.perf_counter() - t0
        kern = lwfr.lwfr_timing_end(st.ctx)
        per_kernel = {k: {"ms_per_launch": (ms / cnt if cnt else None), "launches": cnt, "ms_total": ms}
                      for k, (ms, cnt) in kern.items() if cnt}
    ga, gb = ua.clone(), torch.empty_like(ua)
    torch.cuda.synchronize()
    st.graph_capture(ga, gb, K)
    st.graph_launch()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st.graph_launch()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t2
    status, flags = st.query()
    res = {
        "value": dofs * K / wall,
        "ms_per_step": wall / K * 1e3,
        "ms_per_step_eager": wall_eager / K * 1e3 if wall_eager else None,
        "workload": workload_text(n, N, data),
        "elements": E, "degree": N, "dof": dofs,
        "per_kernel": per_kernel,
        "step_status": int(status), "flags_or": int(flags),
        "u0": u0,
    }
    if graph_trace:
        return res
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_total"])
    avg_ms = per_kernel["k_stages"]["ms_per_launch"]
    flops = STAGE_KERNEL_FLOPS_PER_DOF.get(("GLMMHD2D", N))
    achieved = flops * dofs / (avg_ms * 1e-3) / 1e12 if flops else None
    summary = os.path.join(ROOT, "profiles", f"counters_mhd{n}_n{N}.md")
    traffic, traffic_us = counters.read_traffic(summary, f"k_stages<MHD2D, {N},")
    res["roofline"] = {
        "kernel": "k_stages",
        "bound": "alu",
        "achieved": achieved,
        "peak": FP64_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / FP64_VECTOR_PEAK_TFLOPS if achieved else None,
        "traffic": traffic,
        "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE scaled by a device copy)",
        "traffic_profile_mean_us": traffic_us,
        "algorithmic_flops_per_launch": flops * dofs if flops else None,
        "dominant_kernel_by_time": dom,
    }
    # every kernel of the step against both rooflines (counter figures from the
    # committed summary while it matches the sources, durations measured live)
    by_kernel, step_bytes = kernel_rooflines(counters.read_table(summary), per_kernel, K)
    res["rooflines_by_kernel"] = by_kernel
    # the whole step (graph-replayed) against both rooflines: algorithmic FP64
    # operations of every phase (oracle counts per solution point) and the HBM
    # bytes of every kernel of a step (counter summary)
    sec = wall / K
    step_flops = STEP_FLOPS_PER_DOF.get((N, data))
    res["step_roofline"] = {
        "seconds_per_step": sec,
        "fp64": None if step_flops is None else {
            "flops_per_dof": step_flops, "flops_per_step": step_flops * dofs,
            "achieved_TFLOPs": step_flops * dofs / sec / 1e12,
            "frac": step_flops * dofs / sec / 1e12 / FP64_VECTOR_PEAK_TFLOPS},
        "hbm": None if not step_bytes else {
            "bytes_per_step": step_bytes, "achieved_GBs": step_bytes / sec / 1e9,
            "frac": step_bytes / sec / 1e9 / HBM_PEAK_GBS,
            "state_min_bytes_per_step": 2 * 9 * 8 * dofs,
            "bytes_over_state_min": step_bytes / (2 * 9 * 8 * dofs)},
    }
    res["kernels_ms_per_launch"] = {k: v["ms_per_launch"] for k, v in per_kernel.items()}
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU "
              f"path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2512_08611_amd import counters, lwfr, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lwfr.lib()  # raises if the HIP library is not built
    n, N, data = WORKLOADS[args.workload]
    K, Wm = args.steps, args.warmup
    dev = torch.device("cuda:0")
    main_line = measure(torch, np, lwfr, workloads, counters, n, N, data, K, Wm, args.graph_trace)
    u0 = main_line.pop("u0")
    out = {
        "metric": METRIC,
        "value": main_line["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": main_line["ms_per_step"],
        "ms_per_step_eager": main_line["ms_per_step_eager"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": main_line["workload"], "name": args.workload, "elements": main_line["elements"],
                   "degree": N, "dof": main_line["dof"]},
        "roofline": main_line.get("roofline"),
        "step_roofline": main_line.get("step_roofline"),
        "rooflines_by_kernel": main_line.get("rooflines_by_kernel"),
        "kernels_ms_per_launch": main_line.get("kernels_ms_per_launch"),
        "step_status": main_line["step_status"],
        "flags_or": main_line["flags_or"],
        "secondary": None,
        "adjoint_over_forward": None,
        "batched": None,
    }
    if args.graph_trace:
        print(json.dumps(out), flush=True)
        return
    if not args.no_secondary:
        for name in WORKLOADS:
            if name == args.workload:
                continue
            sn, sN, sdata = WORKLOADS[name]
            sec = measure(torch, np, lwfr, workloads, counters, sn, sN, sdata, K, Wm)
            sec.pop("u0")
            sec.pop("per_kernel")
            sec["name"] = name
            out["secondary"] = sec
    if not args.no_adjoint:
        out["adjoint_over_forward"] = adjoint_over_forward(torch, lwfr, workloads, np)
    if not args.no_batch:
        out["batched"] = batched(torch, lwfr, workloads, np)
    if not args.no_extras:
        out["rotor"] = rotor_run(torch, lwfr, workloads, np)
        out["gll_g2"] = variant_timing(torch, lwfr, workloads, np, 256, 4, lwfr.LWFR_CFG_GLL, K,
                                       "Gauss-Lobatto-Legendre points with the g_2 correction")
        out["alw"] = variant_timing(torch, lwfr, workloads, np, 256, 4, lwfr.LWFR_CFG_ALW, K,
                                    "approximate Lax-Wendroff time averages in place of the cRK stages")
        out["imex_jinxin"] = jinxin_timing(torch, lwfr, workloads, np, K)
    if not (args.no_references or args.no_extras or args.copy_calibration):
        # not in profiling runs: the counter calibration takes the largest copy
        out["device_references"] = device_references(torch)
    if args.copy_calibration:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": a.numel() * 8, "write": b.numel() * 8}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(u0, n, N, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
