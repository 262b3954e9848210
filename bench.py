"""Benchmark of the DGSEM RK-stage hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload euler3d]

A step is one SSP-RK3 step (three fused dg_rk_stage launches: volume integral,
Rusanov faces, surface lift, Jacobian scaling and the stage update) over the
3-D Euler workload: periodic [0, 2pi]^3, 32^3 hexahedra, N = 3 (64 nodes per
element), smooth random state, dt from CFL 0.5.  Inputs are resident in HBM
before the timed region.  The headline is FP64; the FP32 form and the discrete
adjoint stage are timed in the same run and reported beside it.

Prints one JSON line: DOF-updates/s per RK stage (DOF = nodes x 5 variables),
the roofline of the dominant kernel (algorithmic bytes per launch over its mean
HIP-event duration, against 8 TB/s HBM), and the CPU oracle's throughput on a
bounded sample of the same workload.
"""

import argparse
import json
import os
import platform
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import dginputs as di  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFS = 78.6


def split_flops_per_element(dim, N):
    """Algorithmic FP64 operations of the split-form volume sum of one
    element (an FMA counts 2): one two-point flux per unordered node pair of
    every line (the flux is symmetric), each pair adding D_im F# to node i and
    D_mi F# to node m.  The flux as evaluated: two log means (24 and 19
    operations: sum, difference, a reciprocal of 5, the series through u^4,
    a second reciprocal or the products), arithmetic means and v_i . v_m
    (4 dim - 1), and the rows (13 + dim), i.e. 55 + 5 dim; plus 2 x (dim + 2)
    FMAs of accumulation."""
    n = N + 1
    flux = 55 + 5 * dim
    acc = 2 * 2 * (dim + 2)
    lines = dim * n ** (dim - 1)
    return lines * (n * (n - 1) // 2) * (flux + acc)
# Algorithmic state traffic of one SSP-RK3 step: stage 1 reads U^n and writes
# U1, stages 2 and 3 read U^n and U_k and write U_(k+1): 8 arrays over 3
# stages, i.e. 8/3 words per DOF per stage on average.
WORDS_PER_DOF_STAGE = 8.0 / 3.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def warm_up(solver, U, dt, steps, t1, t2, block=100):
    """Untimed SSP-RK3 steps on a scratch copy of U, reset to U every `block`
    steps (the copy never drifts from the workload's state; U itself is left
    untouched).  Under sustained load the device settles at its board power
    limit within a few tens of milliseconds, after an initial overshoot of
    the clock governor; the default warm-up covers that settling so that the
    timed steps see the steady state a long run sees."""
    W = U.clone()
    for k in range(steps):
        if k % block == 0:
            W.copy_(U)
        solver.ssprk3_step(W, dt, t1, t2)
    torch.cuda.synchronize()
    del W


def time_stages(solver, U, dt, steps, warmup, steady=False):
    """Run warmup + timed SSP-RK3 steps; returns (wall seconds of the timed
    steps, mean duration of one dg_rk_stage launch in seconds).  The timed
    steps run back to back (no host work or markers between the launches);
    one pair of HIP events on the launch stream brackets them, so the mean
    launch duration is the GPU time of the timed region over its 3K launches
    (consecutive dependent launches start as the previous one retires).
    With steady=True, after that measurement a further >= 0.2 s of untimed
    steps bring the device to the clock it sustains under this load, and
    the same number of steps is timed again: the third value returned (None
    otherwise) is that steady-state mean launch duration, reported beside
    the headline, never as it."""
    t1 = solver.empty()
    t2 = solver.empty()
    stream = torch.cuda.current_stream()
    U0 = U.clone()
    warm_up(solver, U, dt, warmup, t1, t2)

    def timed():
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record(stream)
        for _ in range(steps):
            solver.ssprk3_step(U, dt, t1, t2)
        b.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, a.elapsed_time(b) * 1e-3 / (3 * steps)

    wall, kern = timed()
    kern_steady = None
    if steady:
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < 0.2:
            if k % 100 == 0:
                U.copy_(U0)
            solver.ssprk3_step(U, dt, t1, t2)
            k += 1
            if k % 50 == 0:
                torch.cuda.synchronize()
        U.copy_(U0)
        _, kern_steady = timed()
    return wall, kern, kern_steady


def time_adjoint(solver, U, dt, steps, warmup, recompute=False):
    """Adjoint of SSP-RK3 steps with stored stage states: per step three
    dg_rk_stage_adjoint launches; with recompute=True (step checkpoints) the
    two forward stages of the step are recomputed from U^n first, as the
    rollout's "steps" checkpointing does.  Returns (wall s per step, mean
    launch s)."""
    Us = [U.clone(), solver.empty(), solver.empty()]
    solver.rk_stage(None, Us[0], Us[1], 0.0, 1.0, dt)
    solver.rk_stage(Us[0], Us[1], Us[2], 0.75, 0.25, 0.25 * dt)
    lam = torch.randn_like(U)
    mu2, mu1, acc, out = solver.empty(), solver.empty(), solver.empty(), solver.empty()

    def step():
        if recompute:
            solver.rk_stage(None, Us[0], Us[1], 0.0, 1.0, dt)
            solver.rk_stage(Us[0], Us[1], Us[2], 0.75, 0.25, 0.25 * dt)
        solver.ssprk3_step_adjoint(Us, dt, lam, out, acc, mu2, mu1)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(steps):
        step()
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall / steps, a.elapsed_time(b) * 1e-3 / steps


def cpu_baseline(p, budget_s=15.0):
    """The CPU oracle (torch-CPU float64) timed on the host's cores on a
    bounded sample: full RK stages on the full-size mesh until ~budget_s, then
    one stage on a single thread."""
    from oracle.dgsem import Operator
    from oracle.mesh import cartesian_mesh
    from oracle.physics import Euler
    from oracle.timestep import rk_stage, dt_cfl

    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    mesh = cartesian_mesh(3, p["N"], p["nel"], p["lo"], p["hi"])
    op = Operator(mesh, Euler(3))
    U = torch.tensor(di.random_euler(mesh.coords(), p["lo"], p["hi"]))[None]
    dt = dt_cfl(op, U, p["cfl"])
    nstage = 0
    t0 = time.perf_counter()
    Uk = U
    coefs = ((0.0, 1.0, 1.0), (0.75, 0.25, 0.25), (1 / 3, 2 / 3, 2 / 3))
    while True:
        a, b, c = coefs[nstage % 3]
        Uk = rk_stage(op, U, Uk, a, b, c * dt)
        nstage += 1
        if time.perf_counter() - t0 > budget_s or nstage >= 60:
            break
    el = time.perf_counter() - t0
    dof = mesh.E * mesh.Np * 5
    threads = torch.get_num_threads()
    torch.set_num_threads(1)
    t1 = time.perf_counter()
    rk_stage(op, U, U, 0.0, 1.0, dt)
    single = dof / (time.perf_counter() - t1)
    torch.set_num_threads(threads)
    return dict(value=dof * nstage / el, unit="DOF-updates/s per RK stage", cores=threads,
                kind="oracle", single_thread_value=single, cpu_model=cpu_model(),
                sample=f"{nstage} full RK stages of the 32^3 N=3 mesh ({dof} DOF) in {el:.1f} s, "
                f"torch-CPU float64 on {threads} threads of {cpu_model()}; plus one stage on 1 thread")


def copy_ceiling(nbytes, reps=20):
    """Bandwidth of a plain device copy (torch's elementwise copy kernel) of
    nbytes into a second buffer: bytes read plus bytes written over the GPU
    time of one copy (HIP events around `reps` back-to-back copies, after
    warm-up copies) -- the practical ceiling of a streaming kernel at that
    footprint."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / t / 1e9


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), else the machine type."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.machine()


def kernel_source_hash():
    """sha256 over the sources the headline stage kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("k_stage.hip", "dg_device.hpp", "dg_internal.hpp", "dg_split.hpp"):
        with open(os.path.join(ROOT, "paper_2605_26388_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(bytes_per_launch):
    """HBM bytes per launch of the headline kernel from the committed counter
    summary (FETCH_SIZE / WRITE_SIZE KiB per dispatch, scaled by the factors a
    plain device copy of known size gives); None when the kernel sources have
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_stage_n3_euler3d_f64_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        c = json.load(fh)
    if c.get("source_sha256") != kernel_source_hash():
        return None
    t = (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0
    return {"bytes_per_launch": t, "over_algorithmic": t / bytes_per_launch}


def time_calls(fn, reps, warmup=2, settle_s=0.05, reset=None):
    """Mean wall time of fn() (seconds) with the stream synchronised around,
    after at least `warmup` untimed calls and at least settle_s seconds of
    untimed calls (the device's clock settling under load).  When fn advances
    a state in place, reset() restores it every 16 untimed calls and once
    before the timed calls, so the timed calls start from the workload's
    initial state."""
    t0 = time.perf_counter()
    k = 0
    while k < warmup or time.perf_counter() - t0 < settle_s:
        if reset is not None and k % 16 == 0:
            reset()
        fn()
        k += 1
        if k % 16 == 0:
            torch.cuda.synchronize()
    if reset is not None:
        reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def steady_summary(res, note):
    f64, f32 = res["f64"], res["f32"]
    if f64["kern_steady"] is None or f32["kern_steady"] is None:
        return None
    return {"f64_kernel_us": f64["kern_steady"] * 1e6, "f32_kernel_us": f32["kern_steady"] * 1e6,
            "f64_roofline_frac": f64["bytes"] / f64["kern_steady"] / 1e9 / HBM_PEAK_GBS,
            "fp32_speedup_vs_fp64": f64["kern_steady"] / f32["kern_steady"], "note": note}


def bench_large(steps, warmup):
    """The same stage at 64^3 (671 MB per FP64 state array, past the 256 MB
    last-level cache), FP64 and FP32, same protocol as the headline (the
    seeded state is evaluated on the device)."""
    from paper_2605_26388_amd import Solver
    p = di.PRESETS["euler3d_L"]
    res = {}
    for prec in ("f64", "f32"):
        s = Solver(3, p["N"], p["nel"], p["lo"], p["hi"], precision=prec)
        X = s.node_coords()
        U = di.random_euler(X, p["lo"], p["hi"])[None].to(s.dtype).contiguous()
        del X
        dt = s.dt_cfl(U, p["cfl"])
        dof = s.E * s.Np * s.nv
        wall, kern, kern_steady = time_stages(s, U, dt, steps, warmup, steady=True)
        st = s.status()
        assert st["nonphysical"] == 0, st
        byt = WORDS_PER_DOF_STAGE * (8 if prec == "f64" else 4) * dof
        res[prec] = {"kernel_us": kern * 1e6, "value": dof * 3 * steps / wall, "bytes_per_launch": byt,
                     "roofline_frac": byt / kern / 1e9 / HBM_PEAK_GBS,
                     "steady_kernel_us": kern_steady * 1e6,
                     "steady_roofline_frac": byt / kern_steady / 1e9 / HBM_PEAK_GBS}
        log(f"64^3 {prec}: kernel {kern * 1e6:.1f} us/launch ({res[prec]['roofline_frac']:.3f} of HBM), "
            f"steady {kern_steady * 1e6:.1f} us")
        del U
        s.close()
        torch.cuda.empty_cache()
    res["fp32_speedup_vs_fp64"] = res["f64"]["kernel_us"] / res["f32"]["kernel_us"]
    res["workload"] = ("euler3d_L: 3-D Euler 64^3 hex elements, N=3 (83.9M DOF), smooth random state, "
                       "SSP-RK3 at CFL 0.5")
    return res


def bench_navier_stokes(reps, nel=None, volume="standard", warp=0.0):
    from paper_2605_26388_amd import Solver
    p = di.PRESETS["tgv3d"]
    nel = tuple(nel) if nel else tuple(p["nel"])
    out = {}
    for prec in ("f64", "f32"):
        s = Solver(3, p["N"], nel, p["lo"], p["hi"], physics="navier_stokes", precision=prec,
                   mu=p["mu"], prandtl=p["prandtl"], volume=volume, warp=warp)
        X = s.node_coords().cpu().numpy()
        U = torch.tensor(di.taylor_green(X, mach=p["mach"]))[None].to(s.device, s.dtype).contiguous()
        dt = s.dt_cfl(U, p["cfl"])
        t1, t2 = s.empty(), s.empty()
        U0 = U.clone()
        step = time_calls(lambda: s.ssprk3_step(U, dt, t1, t2), reps, reset=lambda: U.copy_(U0))
        dof = s.E * s.Np * s.nv
        out[prec] = {"ms_per_stage": step / 3 * 1e3, "dof_updates_per_s": 3 * dof / step}
        s.close()
    out["workload"] = (f"tgv3d: Navier-Stokes TGV {nel[0]}^3, N=4, Re 1600, Mach 0.1, BR1 (two passes per stage)"
                       + (", split-form (Ranocha) inviscid volume integral" if volume == "split" else "")
                       + (f", box warped by {warp} (per-node metrics)" if warp else ""))
    return out


def bench_reacting(reps):
    from paper_2605_26388_amd import Solver
    p = di.PRESETS["air5_2d"]
    mech = di.preset_mechanism(p)
    s = Solver(2, 3, p["nel"], p["lo"], p["hi"], physics="reacting", patch_lo=p["patch_lo"],
               patch_hi=p["patch_hi"], mech=mech)
    X = s.node_coords().cpu().numpy()
    U0 = torch.tensor(di.reacting_state(X, p["lo"], p["hi"], mech, rho0=p["rho0"]))[None].to(s.device).contiguous()
    dt = s.dt_cfl(U0, p["cfl"])
    nodes = s.E * s.Np
    U, t1, t2 = U0.clone(), s.empty(), s.empty()
    restore = lambda: U.copy_(U0)  # noqa: E731
    stage = time_calls(lambda: s.ssprk3_step(U, dt, t1, t2), reps, reset=restore) / 3
    out0 = torch.zeros_like(U0)
    src0 = time_calls(lambda: s.source_chem(U0, out0, 0.0, 0), reps)
    out1 = s.empty()
    s.status(reset=True)
    src1 = time_calls(lambda: s.source_chem(U0, out1, 0.5 * dt, 1), reps)
    st = s.status()
    strang = time_calls(lambda: s.strang_step(U, dt, t1, t2), max(2, reps // 4), reset=restore)
    t3 = s.empty()
    strang54 = time_calls(lambda: s.strang_step(U, 1.508 * dt, t1, t2, t3, transport="ssprk54"), max(2, reps // 4),
                          reset=restore)
    st2 = s.status()
    s.close()
    return {"workload": "air5_2d: reacting Euler 64^2 + 2:1 16^2 patch, N=3, 5-species air, rho about 0.1 kg/m^3, "
                        "backward rates over the forward range, FP64",
            "stage_ms": stage * 1e3, "source_mode0_node_evals_per_s": nodes / src0,
            "source_mode1_nodes_per_s": nodes / src1, "source_mode1_ms": src1 * 1e3,
            "newton_iters_max": st["newton_iters_max"], "newton_unconverged": st["newton_unconverged"],
            "strang_step_ms": strang * 1e3,
            "strang_ssprk54_step_ms": strang54 * 1e3, "strang_ssprk54_dt_over_ssprk3": 1.508,
            "strang_nonphysical": st2["nonphysical"],
            "strang_newton_unconverged": st2["newton_unconverged"]}


def bench_split(steps, warmup):
    """Split-form stage (entropy-conservative volume integral, Ranocha flux)
    on the headline workload, FP64 and FP32 storage: the kernel's mean launch
    time, its throughput, and its ALU roofline (algorithmic FP64 operations
    per launch over the launch time, against the FP64 vector peak)."""
    from paper_2605_26388_amd import Solver
    p = di.PRESETS["euler3d"]
    out = {}
    for prec in ("f64", "f32"):
        s = Solver(3, p["N"], p["nel"], p["lo"], p["hi"], precision=prec, volume="split")
        X = s.node_coords().cpu().numpy()
        U = torch.tensor(di.random_euler(X, p["lo"], p["hi"]))[None].to(s.device, s.dtype).contiguous()
        dt = s.dt_cfl(U, p["cfl"])
        wall, kern, _ = time_stages(s, U, dt, steps, warmup)
        st = s.status()
        assert st["nonphysical"] == 0, st
        dof = s.E * s.Np * s.nv
        flops = split_flops_per_element(3, p["N"]) * s.E
        achieved = flops / kern / 1e12
        out[prec] = {"kernel_us": kern * 1e6, "value": dof * 3 * steps / wall,
                     "ms_per_step": wall / steps * 1e3,
                     "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFS,
                                  "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFS,
                                  "flops_per_launch": flops},
                     "hbm_frac": WORDS_PER_DOF_STAGE * (8 if prec == "f64" else 4) * dof / kern / 1e9
                     / HBM_PEAK_GBS}
        log(f"split {prec}: kernel {kern * 1e6:.1f} us/launch, {achieved:.2f} TFLOP/s algorithmic")
        s.close()
    out["workload"] = ("euler3d split form: 3-D Euler 32^3, N=3, entropy-conservative volume integral "
                       "(Ranocha flux), Rusanov interfaces, SSP-RK3 at CFL 0.5")
    return out


def bench_ssprk54(steps, warmup):
    """SSPRK54 steps (five fused stage launches, the fourth writing two
    combinations) on the headline mesh, standard form and the paper's
    production setting (split form, positivity floor rho >= 1e-6,
    p >= 5e-7), FP64.  Reports the step time, the mean stage launch and the
    cost per unit simulated time relative to SSP-RK3 at the same fraction of
    each method's SSP step bound (SSP coefficients 1.508 and 1)."""
    from paper_2605_26388_amd import Solver
    p = di.PRESETS["euler3d"]
    out = {}
    for name, kw in (("standard", {}), ("split_floor", dict(volume="split", rho_floor=1e-6, p_floor=5e-7))):
        s = Solver(3, p["N"], p["nel"], p["lo"], p["hi"], **kw)
        X = s.node_coords().cpu().numpy()
        U = torch.tensor(di.random_euler(X, p["lo"], p["hi"]))[None].to(s.device).contiguous()
        dt = s.dt_cfl(U, p["cfl"])
        t1, t2, t3, W = s.empty(), s.empty(), s.empty(), U.clone()
        for k in range(warmup):
            if k % 100 == 0:
                W.copy_(U)
            s.ssprk54_step(W, 1.508 * dt, t1, t2, t3)
        stream = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a.record(stream)
        for _ in range(steps):
            s.ssprk54_step(U, 1.508 * dt, t1, t2, t3)
        b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu = a.elapsed_time(b) * 1e-3
        st = s.status()
        assert st["nonphysical"] == 0, st
        dof = s.E * s.Np * s.nv
        out[name] = {"ms_per_step": wall / steps * 1e3, "stage_us": gpu / (5 * steps) * 1e6,
                     "dof_updates_per_s": 5 * dof * steps / wall, "floored": st["floored"]}
        s.close()
    out["cost_per_simulated_time_vs_ssprk3"] = (5 / 1.508) / 3
    out["workload"] = ("euler3d: 3-D Euler 32^3, N=3, SSPRK54 at 1.508 x the SSP-RK3 step (CFL 0.5), FP64; "
                       "split_floor: split form with the positivity floor")
    return out


def bench_reacting_2t(reps):
    """Two-temperature version of the reacting workload: stage, source mode 0,
    implicit substep (mode 1) at h = dt/2 and a Strang step, FP64."""
    from paper_2605_26388_amd import Solver
    p = di.PRESETS["air5_2t_2d"]
    mech = di.preset_mechanism(p)
    vib = di.air5_vibration(mech)
    s = Solver(2, 3, p["nel"], p["lo"], p["hi"], physics="reacting_2t", patch_lo=p["patch_lo"],
               patch_hi=p["patch_hi"], mech=mech, vib=vib)
    X = s.node_coords().cpu().numpy()
    U0 = torch.tensor(di.reacting2t_state(X, p["lo"], p["hi"], mech, vib, u0=250.0))[None].to(s.device).contiguous()
    dt = s.dt_cfl(U0, p["cfl"])
    nodes = s.E * s.Np
    U, t1, t2 = U0.clone(), s.empty(), s.empty()
    restore = lambda: U.copy_(U0)  # noqa: E731
    stage = time_calls(lambda: s.ssprk3_step(U, dt, t1, t2), reps, reset=restore) / 3
    out0 = torch.zeros_like(U0)
    src0 = time_calls(lambda: s.source_chem(U0, out0, 0.0, 0), reps)
    out1 = s.empty()
    s.status(reset=True)
    src1 = time_calls(lambda: s.source_chem(U0, out1, 0.5 * dt, 1), reps)
    st = s.status()
    strang = time_calls(lambda: s.strang_step(U, dt, t1, t2), max(2, reps // 4), reset=restore)
    s.close()
    return {"workload": "air5_2t_2d: two-temperature reacting Euler 64^2 + 2:1 16^2 patch, N=3, 5-species air, FP64",
            "stage_ms": stage * 1e3, "source_mode0_node_evals_per_s": nodes / src0,
            "source_mode1_nodes_per_s": nodes / src1, "source_mode1_ms": src1 * 1e3,
            "newton_iters_max": st["newton_iters_max"], "newton_unconverged": st["newton_unconverged"],
            "strang_step_ms": strang * 1e3}


def bench_curvilinear(steps, warmup):
    """Curvilinear stage on the headline mesh warped (warp 0.03, periodic),
    FP64: mean launch time and the HBM roofline with the metric planes
    (1/J and Ja^l: 10 doubles per node, read once per launch) added to the
    state traffic."""
    from paper_2605_26388_amd import Solver
    p = di.PRESETS["euler3d"]
    out = {}
    for volume, prec in (("standard", "f64"), ("split", "f64"), ("standard", "f32")):
        s = Solver(3, p["N"], p["nel"], p["lo"], p["hi"], warp=0.03, volume=volume, precision=prec)
        X = s.node_coords().cpu().numpy()
        U = torch.tensor(di.random_euler(X, p["lo"], p["hi"]))[None].to(s.device, s.dtype).contiguous()
        dt = s.dt_cfl(U, p["cfl"])
        wall, kern, _ = time_stages(s, U, dt, steps, warmup)
        st = s.status()
        assert st["nonphysical"] == 0, st
        nodes = s.E * s.Np
        dof = nodes * s.nv
        byt = WORDS_PER_DOF_STAGE * 8 * dof + 10 * 8 * nodes
        s.close()
        if prec == "f32":
            out["f32"] = {"kernel_us": kern * 1e6, "value": dof * 3 * steps / wall}
        elif volume == "standard":
            out.update({"kernel_us": kern * 1e6, "value": dof * 3 * steps / wall, "bytes_per_launch": byt,
                        "roofline": {"bound": "hbm", "achieved": byt / kern / 1e9, "peak": HBM_PEAK_GBS,
                                     "unit": "GB/s", "frac": byt / kern / 1e9 / HBM_PEAK_GBS}})
        else:
            out["split"] = {"kernel_us": kern * 1e6, "value": dof * 3 * steps / wall}
    out["workload"] = ("euler3d warped: 3-D Euler 32^3, N=3, warp 0.03 (per-node metrics), periodic, FP64; "
                       "split: the same with the split-form volume integral; f32: FP32 state, standard form")
    return out


def bench_adjoint(steps):
    """Adjoint workload (16^3, N=3, batch 8) in FP32: forward SSP-RK3 step vs
    its reverse sweep with stored stage states."""
    from paper_2605_26388_amd import Solver
    p = di.PRESETS["adjoint3d"]
    out = {}
    for prec in ("f32", "f64"):
        s = Solver(3, 3, p["nel"], p["lo"], p["hi"], batch=p["batch"], precision=prec)
        X = s.node_coords().cpu().numpy()
        base = di.random_euler(X, p["lo"], p["hi"])
        U = torch.tensor(np.stack([di.perturb_density(base, b) for b in range(p["batch"])]))
        U = U.to(s.device, s.dtype).contiguous()
        dt = s.dt_cfl(U, p["cfl"])
        t1, t2 = s.empty(), s.empty()
        U0 = U.clone()
        fwd = time_calls(lambda: s.ssprk3_step(U, dt, t1, t2), steps, reset=lambda: U.copy_(U0))
        bwd_step, _ = time_adjoint(s, U, dt, steps, 2)
        bwd_rec, _ = time_adjoint(s, U, dt, steps, 2, recompute=True)
        out[prec] = {"forward_ms_per_step": fwd * 1e3, "backward_ms_per_step": bwd_step * 1e3,
                     "backward_over_forward": bwd_step / fwd,
                     "backward_recompute_ms_per_step": bwd_rec * 1e3,
                     "backward_recompute_over_forward": bwd_rec / fwd}
        s.close()
    out["workload"] = "adjoint3d: 3-D Euler 16^3, N=3, batch 8 (10,485,760 DOF), stored stage states"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=600,
                    help="untimed steps before the timed region (about 0.1 s at the default workload)")
    ap.add_argument("--workload", default="euler3d", choices=["euler3d", "euler3d_L"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
    ap.add_argument("--only", choices=["f64", "f32"], default=None,
                    help="time one form only (profiling runs)")
    ap.add_argument("--side", choices=["adjoint", "navier_stokes", "navier_stokes_L", "navier_stokes_split",
                                       "navier_stokes_curvilinear", "reacting",
                                       "reacting_2t", "split",
                                       "ssprk54", "curvilinear"],
                    default=None,
                    help="instead: run one side workload alone and print its JSON (profiling runs)")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="instead: run a plain device copy of this many MiB 10 times (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: measures one GPU; runs on several GPUs are not supported "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        n = args.calib_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.calib_copy} MiB x 10")
        return

    if args.side:
        reps = max(5, args.steps // 10)
        fn = {"adjoint": lambda: bench_adjoint(reps),
              "navier_stokes": lambda: bench_navier_stokes(reps),
              "navier_stokes_L": lambda: bench_navier_stokes(reps, nel=(32, 32, 32)),
              "navier_stokes_split": lambda: bench_navier_stokes(reps, volume="split"),
              "navier_stokes_curvilinear": lambda: bench_navier_stokes(reps, warp=0.03),
              "reacting": lambda: bench_reacting(reps),
              "reacting_2t": lambda: bench_reacting_2t(reps),
              "split": lambda: bench_split(args.steps, args.warmup),
              "ssprk54": lambda: bench_ssprk54(args.steps, args.warmup // 2),
              "curvilinear": lambda: bench_curvilinear(args.steps, args.warmup)}[args.side]
        print(json.dumps({args.side: fn()}), flush=True)
        return

    from paper_2605_26388_amd import Solver

    p = di.PRESETS[args.workload]
    res = {}
    forms = [args.only] if args.only else ["f64", "f32"]
    for form in forms:
        prec = form
        s = Solver(3, p["N"], p["nel"], p["lo"], p["hi"], precision=prec)
        U = di.random_euler(s.node_coords(), p["lo"], p["hi"])[None].to(s.dtype).contiguous()
        dt = s.dt_cfl(U, p["cfl"])
        dof = s.E * s.Np * s.nv
        wall, kern, kern_steady = time_stages(s, U, dt, args.steps, args.warmup, steady=not args.only)
        st = s.status()
        assert st["nonphysical"] == 0, st
        bytes_per_launch = WORDS_PER_DOF_STAGE * (8 if prec == "f64" else 4) * dof
        res[form] = dict(wall=wall, kern=kern, dof=dof, bytes=bytes_per_launch, kern_steady=kern_steady,
                         value=dof * 3 * args.steps / wall, ms_per_step=wall / args.steps * 1e3)
        log(f"{form}: {wall / args.steps * 1e3:.3f} ms/step, kernel {kern * 1e6:.1f} us/launch, "
            f"{bytes_per_launch / kern / 1e9:.0f} GB/s algorithmic")
        s.close()
    if args.only:
        return

    f64 = res["f64"]
    achieved = f64["bytes"] / f64["kern"] / 1e9
    traffic = measured_traffic(f64["bytes"])
    out = {
        "metric": "DOF-updates/s per RK stage (FP64 vs FP32 vs adjoint), % HBM roofline",
        "value": f64["value"],
        "unit": "DOF-updates/s per RK stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: 3-D compressible Euler, periodic [0,2pi]^3, "
                               f"{p['nel'][0]}^3 hex elements, N=3 (64 nodes/elem), smooth random state, "
                               f"SSP-RK3 at CFL 0.5, FP64",
                   "elements": int(np.prod(p["nel"])), "degree": 3, "dof": f64["dof"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic["bytes_per_launch"],
                     "traffic_over_algorithmic": None if traffic is None else traffic["over_algorithmic"],
                     "kernel": "k_stage_n3 (3-D Euler, N=3, FP64)",
                     "kernel_us": f64["kern"] * 1e6, "bytes_per_launch": f64["bytes"]},
        "fp32": {"value": res["f32"]["value"], "kernel_us": res["f32"]["kern"] * 1e6,
                 "speedup_vs_fp64": f64["kern"] / res["f32"]["kern"],
                 "roofline_frac": res["f32"]["bytes"] / res["f32"]["kern"] / 1e9 / HBM_PEAK_GBS},
        "steady_state": steady_summary(res, "after >= 0.2 s more of back-to-back steps (the clock the device "
                                            "sustains under this load); the headline is the measurement above"),
    }
    # the practical ceiling: a plain copy moving the stage's algorithmic bytes
    # (read half, write half; cache-resident like the stage) and one of 1 GiB
    # per buffer (past the Infinity Cache), after the headline measurement
    c_stage = copy_ceiling(int(f64["bytes"]) // 2 // 8 * 8)
    c_large = copy_ceiling(1 << 30)
    out["roofline"]["copy_ceiling"] = {
        "gbs_at_stage_bytes": c_stage, "gbs_1gib": c_large,
        "frac_of_copy_at_stage_bytes": achieved / c_stage,
        "note": "torch's device copy; bytes read + written per copy over its GPU time"}
    if not args.no_extras:
        log("64^3 workload ...")
        out["euler3d_L"] = bench_large(args.steps, args.warmup)
        log("adjoint workload ...")
        out["adjoint"] = bench_adjoint(max(5, args.steps // 10))
        log("Navier-Stokes workload ...")
        out["navier_stokes"] = bench_navier_stokes(max(5, args.steps // 10))
        out["navier_stokes_L"] = bench_navier_stokes(max(5, args.steps // 10), nel=(32, 32, 32))
        out["navier_stokes_split"] = bench_navier_stokes(max(5, args.steps // 10), volume="split")
        out["navier_stokes_curvilinear"] = bench_navier_stokes(max(5, args.steps // 10), warp=0.03)
        log("reacting workload ...")
        out["reacting"] = bench_reacting(max(5, args.steps // 10))
        log("two-temperature reacting workload ...")
        out["reacting_2t"] = bench_reacting_2t(max(5, args.steps // 10))
        log("split-form workload ...")
        out["split"] = bench_split(args.steps, args.warmup)
        log("SSPRK54 workload ...")
        out["ssprk54"] = bench_ssprk54(args.steps, args.warmup // 2)
        log("curvilinear workload ...")
        out["curvilinear"] = bench_curvilinear(args.steps, args.warmup)
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(dict(p, N=3))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
