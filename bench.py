"""Throughput of the curved-space D3Q19 step on one MI355X.

Workload: the 256x128x128 channel (4,128,768 fluid nodes) with a Gaussian
bump of amplitude 0.08*128 on the top wall, tau 0.6, body force 1e-6, initial
velocity noise +-1e-4 (seed 2).  The headline value is the FP32 deviation-form
step in MLUPS (fluid-node updates per second); the FP64 step is measured on
the same workload and reported beside it.  Inputs are synthetic and resident
in HBM before the timed region.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic HBM bytes per fluid-node update of one step with a static
# metric: populations read + written (19 each), forcing history read +
# written (10 each), geometry read (28).
BYTES_PER_LUP = {"fp32": 4 * (19 + 19 + 10 + 10 + 28), "fp64": 8 * (19 + 19 + 10 + 10 + 28)}
HBM_PEAK_GBPS = 8000.0
# The committed rocprofv3 summary of the step kernel's HBM counters, and the
# sources it was taken from: traffic is reported only while they are unchanged.
COUNTER_PROFILE = os.path.join(ROOT, "profiles", "step_fused_c2_256x128x128.md")
STEP_SOURCES = ["paper_1803_07822_amd/csrc/lbm_step_fused.hip", "paper_1803_07822_amd/csrc/lbm_device.h",
                "paper_1803_07822_amd/csrc/lbm_internal.h", "paper_1803_07822_amd/build.py"]


def step_kernel_name(variant, stage):
    """The FP32 step kernel a launch shape runs (lbm_get_tuning's variant and stage)."""
    if variant == 1:
        return "k_moments<float> + k_collide<float> (two-pass step; time of both)"
    return f"k_step_fused<float, 64, 4, {stage}, false, false, false> (whole step, one launch)"
METRIC = "MLUPS + HBM GB/s (% peak) FP32 vs FP64 step; adjoint/forward time ratio"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--workload", default="c2_bump_256x128x128")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward timing")
    p.add_argument("--fp64-steps", type=int, default=None)
    p.add_argument("--no-extra", action="store_true",
                   help="skip the oscillating-wall loop, the 512x256x256 runs and the flag channel")
    p.add_argument("--part", choices=["all", "adjoint", "c3", "c5", "c5adj", "flag", "open", "cpu_c5"],
                   default="all",
                   help="run one measurement alone (for profiling): the 128x64x64 adjoint, the oscillating-wall "
                        "loop, the 512x256x256 runs, the 512x256x256 adjoint alone (from rest), the flag channel, "
                        "the open channel at scale, or the oracle on the 512x256x256 workload; prints that part's "
                        "JSON only")
    p.add_argument("--variant", type=int, default=0,
                   help="launch variant of the step (lbm_set_tuning): 0 fused (default), 1 two-pass")
    p.add_argument("--stage", type=int, default=-1,
                   help="staging of the FP32 fused step (lbm_set_tuning): -1 the default, 0 none, 1 registers")
    p.add_argument("--counters", action="store_true",
                   help="no timing: a 256 MiB calibration copy, then --steps FP32 steps, for rocprofv3 --pmc runs")
    return p.parse_args()


def setup(w, precision, variant=0, stage=-1):
    import numpy as np

    from paper_1803_07822_amd import lbm, synth

    S = lbm.Solver(w.nx, w.ny, w.nz, w.tau, precision)
    if variant or stage != -1:
        lbm.lbm_set_tuning(S.ctx, 0, variant, stage)
    S.set_body_force(w.force)
    S.set_wall_displacement(lbm.LBM_WALL_YMAX, w.disp())
    uc = synth.uniform_noise_velocity(w.nx, w.ny, w.nz, 1e-4, seed=2)
    S.init_equilibrium(None, uc)
    S.sync()
    return S, uc


# The bump channel at tau 0.6 is unstable under the scheme (the explicit
# velocity-gradient forcing C^ij outweighs the low BGK viscosity where the
# 8 % bump bends the metric): the instability guard trips after about 55
# steps from rest, so steps are timed in windows that each start from the
# equilibrium initial state.
WINDOW = 30
LEAD_IN = 5


def time_steps(S, uc, steps, warmup):
    """Time exactly `steps` steps: windows of at most WINDOW steps, each after a
    fresh equilibrium start and LEAD_IN untimed steps, bracketed by HIP events
    on the library's stream.  A step is one launch of the fused step kernel,
    so the mean step time is also that kernel's mean launch duration (launch
    gaps included).  Returns it with the host wall time of the windows."""
    import torch

    S.step(warmup)
    S.sync()
    done, tot_ms, wall = 0, 0.0, 0.0
    while done < steps:
        n = min(WINDOW, steps - done)
        S.init_equilibrium(None, uc)
        S.step(LEAD_IN)
        S.sync()
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record(S.stream)
        S.step(n)
        stop.record(S.stream)
        S.sync()
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        tot_ms += start.elapsed_time(stop)
        done += n
    return tot_ms / steps, wall


def adjoint_ratio(repeats=3):
    """The 128x64x64 adjoint workload (FP64, K = 200, checkpoint every 20):
    time of lbm_forward_record and of lbm_backward, from stream events."""
    import numpy as np
    import torch

    from paper_1803_07822_amd import lbm, synth

    w = synth.workload("c4_adjoint_128x64x64")
    K, N = w.steps, w.extra["ckpt_every"]
    S = lbm.Solver(w.nx, w.ny, w.nz, w.tau, "fp64", adjoint_K=K, ckpt_every=N)
    S.set_body_force(w.force)
    S.set_wall_displacement(lbm.LBM_WALL_YMAX, w.disp().astype(np.float32).astype(np.float64))
    S.init_equilibrium()
    f0 = S.populations()
    W = torch.zeros((K, 3), dtype=torch.float64, device=S.device)
    W[:, 0] = 1.0
    fwd, bwd = [], []
    for r in range(repeats + 1):
        S.set_populations(f0)
        S.sync()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(S.stream)
        lbm.lbm_forward_record(S.ctx, K, N, lbm.LBM_WALL_YMAX, torch.empty((K, 3), dtype=torch.float64, device=S.device))
        e1.record(S.stream)
        gd = torch.empty((w.nz, w.nx), dtype=torch.float64, device=S.device)
        gf = torch.empty((19, w.nz, w.ny - 2, w.nx), dtype=torch.float64, device=S.device)
        lbm.lbm_backward(S.ctx, W, gd, None, gf)
        e2.record(S.stream)
        S.sync()
        if r > 0:
            fwd.append(e0.elapsed_time(e1))
            bwd.append(e1.elapsed_time(e2))
    f, b = sum(fwd) / len(fwd), sum(bwd) / len(bwd)
    return {"workload": w.name, "K": K, "ckpt_every": N, "forward_ms": round(f, 3), "backward_ms": round(b, 3),
            "ratio": round(b / f, 3), "forward_mlups": round(w.fluid_nodes * K / (f * 1e-3) / 1e6, 1)}


def moving_wall_loop(w, wall_at, every, steps, keep_state=False, general_updates=0):
    """FP32 run of workload `w` under a moving top wall: `steps` steps, the
    wall shape and velocity (wall_at(t) -> d [nz, nx], dd/dt [nz, nx]) updated
    with re-projection every `every` steps, the top-wall force recorded every
    step into device memory (lbm_step_force: the force of each state a step
    starts from, states 0 .. steps-1, formed by the fused step itself).  GPU time per phase from events on the library's
    stream, and the host wall time of the whole loop.  keep_state: also
    return the final populations (FP64, on the host).

    Charts built from a wall displacement move the nodes along y only and the
    library updates them on a path of its own; general_updates > 0 then also
    times that many updates with the loop's last two wall charts given whole
    (lbm_set_metric, the general path) on the final state, for comparison."""
    import numpy as np
    import torch

    from paper_1803_07822_amd import lbm, synth

    S = lbm.Solver(w.nx, w.ny, w.nz, w.tau, "fp32")
    S.set_body_force(w.force)

    def wall(t):
        d, v = wall_at(float(t))
        vc = np.zeros((w.nz, w.nx, 3))
        vc[..., 1] = v
        return torch.as_tensor(d, device=S.device), torch.as_tensor(vc, device=S.device)

    d, vc = wall(0)
    lbm.lbm_set_wall_displacement(S.ctx, lbm.LBM_WALL_YMAX, d, 0)
    lbm.lbm_set_wall_velocity(S.ctx, lbm.LBM_WALL_YMAX, vc)
    S.init_equilibrium()
    walls = [wall(t) for t in range(every, steps + 1, every)]  # uploaded before timing
    forces = torch.empty((steps, 3), dtype=torch.float64, device=S.device)
    nup = steps // every
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(nup)]
    S.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for u in range(nup):
        e = ev[u]
        e[0].record(S.stream)
        lbm.lbm_step_force(S.ctx, every, lbm.LBM_WALL_YMAX, forces[u * every:(u + 1) * every])
        e[1].record(S.stream)
        d, vc = walls[u]
        lbm.lbm_set_wall_displacement(S.ctx, lbm.LBM_WALL_YMAX, d, 1)
        e[2].record(S.stream)
        lbm.lbm_set_wall_velocity(S.ctx, lbm.LBM_WALL_YMAX, vc)
        e[3].record(S.stream)
    S.sync()
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    step_ms = sum(e[0].elapsed_time(e[1]) for e in ev)
    rp_ms = sum(e[1].elapsed_time(e[2]) for e in ev)
    vel_ms = sum(e[2].elapsed_time(e[3]) for e in ev)
    total_ms = ev[0][0].elapsed_time(ev[-1][3])
    f = forces.cpu().numpy()
    gen_ms = None
    if general_updates > 0:
        charts = [torch.as_tensor(synth.chart_from_displacement(w.nx, w.ny, w.nz, np.asarray(walls[u][0].cpu())),
                                  device=S.device) for u in (nup - 2, nup - 1)]
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        lbm.lbm_set_metric(S.ctx, charts[0], 1)
        g0.record(S.stream)
        for r in range(general_updates):
            lbm.lbm_set_metric(S.ctx, charts[(r + 1) % 2], 1)
        g1.record(S.stream)
        S.sync()
        torch.cuda.synchronize()
        gen_ms = round(g0.elapsed_time(g1) / general_updates, 4)
    res = {"workload": w.name, "precision": "fp32", "steps": steps, "updates": nup,
           "gpu_ms": round(total_ms, 2), "wall_s": round(wall_s, 3),
           "mlups_with_updates": round(w.fluid_nodes * steps / (total_ms * 1e-3) / 1e6, 1),
           "step_and_force_ms_per_step": round(step_ms / steps, 5),
           "metric_update_and_reprojection_ms": round(rp_ms / nup, 4),
           "wall_velocity_ms": round(vel_ms / nup, 4),
           "general_chart_update_ms": gen_ms,
           "force_finite": bool(np.isfinite(f).all()), "final_force": [float(x) for x in f[-1]]}
    state = S.populations().cpu() if keep_state else None
    del S, walls, forces
    torch.cuda.empty_cache()
    return (res, state) if keep_state else res


def c3_loop():
    """The oscillating-wall workload in FP32: 4000 steps, the metric and wall
    velocity updated with re-projection every 10 steps (moving_wall_loop)."""
    from paper_1803_07822_amd import synth

    w = synth.workload("c3_oscillating_256x128x128")
    return moving_wall_loop(w, lambda t: synth.oscillating_wall(w.nx, w.nz, t=t), w.extra["update_every"], w.steps,
                            general_updates=10)


def open_channel(steps=50, repeats=2):
    """Open ends at scale: a 256x130x128 channel (4.19M fluid nodes) with a
    parabolic inlet (peak 0.05) and an open outlet, FP32 and FP64, timed
    with the fused step (periodic fused kernel plus the two end-column
    passes) and with the two-pass step, from the developed inlet profile."""
    import numpy as np
    import torch

    from paper_1803_07822_amd import lbm, synth

    nx, ny, nz, tau = 256, 130, 128, 0.6
    H = ny - 2
    out = {"workload": "open_channel_256x130x128", "fluid_nodes": nx * H * nz}
    for prec in ("fp32", "fp64"):
        S = lbm.Solver(nx, ny, nz, tau, prec)
        uin = synth.parabolic_inlet(nz, H, 0.05)
        S.set_open_x(uin)
        S.set_wall_displacement(lbm.LBM_WALL_YMAX, np.zeros((nz, nx)))
        uc = np.zeros((3, nz, H, nx))
        uc[0] = uin[..., 0][:, :, None]
        res = {}
        for name, variant in (("fused_ms", 0), ("two_pass_ms", 1)):
            lbm.lbm_set_tuning(S.ctx, 0, variant, -1)
            tot = 0.0
            for _ in range(repeats):
                S.init_equilibrium(None, uc)
                S.step(5)
                S.sync()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(S.stream)
                S.step(steps)
                e1.record(S.stream)
                S.sync()
                tot += e0.elapsed_time(e1)
            res[name] = round(tot / (steps * repeats), 4)
        res["fused_mlups"] = round(nx * H * nz / (res["fused_ms"] * 1e-3) / 1e6, 1)
        out[prec] = res
        del S
        torch.cuda.empty_cache()
    return out


def c5_travelling(keep_state=False):
    """The 512x256x256 patch wave travelling, in FP32 at the run amplitude:
    3000 steps, the wall shape and velocity updated with re-projection every
    10 steps (moving_wall_loop); keep_state: also the final populations."""
    from paper_1803_07822_amd import synth

    w = synth.workload("c5_patch_wave_512x256x256")
    A = w.extra["A_run"]
    return moving_wall_loop(w, lambda t: synth.patch_wave(A=A, t=t), w.extra["update_every"], w.steps, keep_state)


def c5_adjoint(f_start, d_end=None, start="state after the 3000-step FP32 travelling run (FP64), "
                                             "wall frozen at its t = 3000 shape, at rest"):
    """The FP64 adjoint of the 512x256x256 workload over K = 100 steps with a
    checkpoint every 10 (about 245 GiB of workspace), from f_start (the state
    the 3000-step FP32 travelling run ended in, on the host, FP64): the wall
    frozen at its shape at t = 3000, at rest; loss = sum of the top-wall
    x-force over states 1..K.  Forward-record and backward times."""
    import torch

    from paper_1803_07822_amd import lbm, synth

    w = synth.workload("c5_patch_wave_512x256x256")
    K, N = w.extra["K"], w.extra["ckpt_every"]
    if d_end is None:
        d_end, _ = synth.patch_wave(A=w.extra["A_run"], t=float(w.steps))
    try:
        S = lbm.Solver(w.nx, w.ny, w.nz, w.tau, "fp64", adjoint_K=K, ckpt_every=N)
        S.set_body_force(w.force)
        S.set_wall_displacement(lbm.LBM_WALL_YMAX, d_end)
        S.set_populations(f_start)
        Wt = torch.zeros((K, 3), dtype=torch.float64, device=S.device)
        Wt[:, 0] = 1.0
        gd = torch.empty((w.nz, w.nx), dtype=torch.float64, device=S.device)
        forces = torch.empty((K, 3), dtype=torch.float64, device=S.device)
        S.sync()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(S.stream)
        lbm.lbm_forward_record(S.ctx, K, N, lbm.LBM_WALL_YMAX, forces)
        ev[1].record(S.stream)
        lbm.lbm_backward(S.ctx, Wt, gd, None, None)
        ev[2].record(S.stream)
        S.sync()
        f, b = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
        out = {"K": K, "ckpt_every": N, "start": start, "forward_ms": round(f, 2), "backward_ms": round(b, 2),
               "ratio": round(b / f, 3), "grad_finite": bool(torch.isfinite(gd).all().item())}
        del S
    except (RuntimeError, lbm.LBMError) as e:  # e.g. not enough device memory for the workspace
        out = {"error": str(e)[:200]}
    torch.cuda.empty_cache()
    return out


def flag_channel(steps=None):
    """The flag channel (Sec. VI.A without the structure), FP32: parabolic
    inlet, open outlet, a plate flapping with a prescribed motion, its chart
    rebuilt and the state re-projected every step.  GPU time per step
    (step + chart + geometry + re-projection + plate velocity) from events on
    the library's stream over the whole run, with the plate shapes uploaded
    beforehand; the guard is checked at the end."""
    import numpy as np
    import torch

    from paper_1803_07822_amd import lbm, synth

    w = synth.workload("flag_channel_257x65")
    steps = steps or w.steps
    H = w.ny - 2
    jp, i0, i1 = w.extra["plate"]
    A, om = w.extra["A"], w.extra["omega"]
    S = lbm.Solver(w.nx, w.ny, w.nz, w.tau, "fp32")
    S.set_open_x(synth.parabolic_inlet(w.nz, H, w.extra["U"]))
    S.set_plate(jp, i0, i1)
    S.set_wall_displacement(lbm.LBM_WALL_YMAX, np.zeros((w.nz, w.nx)))
    uc = np.zeros((3, w.nz, H, w.nx))
    uc[0] = synth.parabolic_inlet(w.nz, H, w.extra["U"])[..., 0][:, :, None]
    S.init_equilibrium(None, uc)
    shapes = [synth.flapping_plate(w.nx, w.nz, i0, i1, A=A, omega=om, t=float(t)) for t in range(1, steps + 1)]
    dev = [(torch.as_tensor(d, device=S.device), torch.as_tensor(v, device=S.device)) for d, v in shapes]
    force = torch.empty((steps, 3), dtype=torch.float64, device=S.device)
    S.sync()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(S.stream)
    for t in range(steps):
        lbm.lbm_step(S.ctx, 1)
        d, v = dev[t]
        lbm.lbm_set_plate_displacement(S.ctx, d, 1)
        lbm.lbm_set_plate_velocity(S.ctx, v)
        lbm.lbm_plate_force(S.ctx, force[t])
    e1.record(S.stream)
    stable = True
    try:
        S.sync()
    except lbm.LBMError:
        stable = False
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    f = force.cpu().numpy()
    rho, u = S.moments(cartesian=True) if stable else (None, None)
    del S
    torch.cuda.empty_cache()
    graph_ms = flag_channel_graph(w, steps) if stable else None
    res = {"workload": w.name, "precision": "fp32", "steps": steps, "tau": round(w.tau, 5),
           "Re_channel": 325, "stable": stable, "gpu_ms": round(ms, 2),
           "ms_per_step_with_reprojection": round(ms / steps, 5),
           "mlups_with_reprojection": round(w.fluid_nodes * steps / (ms * 1e-3) / 1e6, 1),
           "max_u": float(u.abs().max()) if stable else None,
           "plate_force_last": [float(x) for x in f[-1]],
           "plate_force_lift_range": [float(f[:, 1].min()), float(f[:, 1].max())],
           "ms_per_step_graph": round(graph_ms / steps, 5) if graph_ms else None}
    return res


def flag_channel_graph(w, steps):
    """The same loop captured as one HIP graph of a flapping period (the
    shapes repeat with it) on the context's own stream and replayed
    steps/period times; GPU time of the replays from events."""
    import numpy as np
    import torch

    from paper_1803_07822_amd import lbm, synth

    H = w.ny - 2
    jp, i0, i1 = w.extra["plate"]
    A, om = w.extra["A"], w.extra["omega"]
    period = int(round(2 * np.pi / om))
    assert steps % period == 0 and period % 2 == 0
    side = torch.cuda.Stream()
    S = lbm.Solver(w.nx, w.ny, w.nz, w.tau, "fp32", stream=side)
    S.set_open_x(synth.parabolic_inlet(w.nz, H, w.extra["U"]))
    S.set_plate(jp, i0, i1)
    S.set_wall_displacement(lbm.LBM_WALL_YMAX, np.zeros((w.nz, w.nx)))
    uc = np.zeros((3, w.nz, H, w.nx))
    uc[0] = synth.parabolic_inlet(w.nz, H, w.extra["U"])[..., 0][:, :, None]
    S.init_equilibrium(None, uc)
    shapes = [synth.flapping_plate(w.nx, w.nz, i0, i1, A=A, omega=om, t=float(t)) for t in range(1, period + 1)]
    dev = [(torch.as_tensor(d, device=S.device), torch.as_tensor(v, device=S.device)) for d, v in shapes]
    force = torch.empty((period, 3), dtype=torch.float64, device=S.device)

    def calls():
        for t in range(period):
            lbm.lbm_step(S.ctx, 1)
            lbm.lbm_set_plate_displacement(S.ctx, dev[t][0], 1)
            lbm.lbm_set_plate_velocity(S.ctx, dev[t][1])
            lbm.lbm_plate_force(S.ctx, force[t])

    calls()  # eager first period (launch shapes chosen outside the capture)
    S.sync()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        calls()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(side):
        e0.record(side)
        for _ in range(steps // period):
            g.replay()
        e1.record(side)
    S.sync()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del g, S
    torch.cuda.empty_cache()
    return ms


def c5_runs(steps=200):
    """The 512x256x256 patch-wave workload (33.3M fluid nodes, run amplitude
    0.04*256): FP32 step throughput over `steps` steps from the equilibrium
    start with the wave frozen, the travelling wave over its 3000 steps with
    re-projection every 10 (c5_travelling), then the FP64 adjoint over K = 100
    with a checkpoint every 10 (about 245 GiB of workspace) from the state the
    travelling run ended in (c5_adjoint): forward-record and backward times."""
    import torch

    from paper_1803_07822_amd import lbm, synth

    w = synth.workload("c5_patch_wave_512x256x256")
    out = {"workload": w.name, "amplitude": w.extra["A_run"]}
    S = lbm.Solver(w.nx, w.ny, w.nz, w.tau, "fp32")
    S.set_body_force(w.force)
    S.set_wall_displacement(lbm.LBM_WALL_YMAX, w.disp())
    S.init_equilibrium()
    S.step(5)
    S.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(S.stream)
    S.step(steps)
    e1.record(S.stream)
    S.sync()
    ms = e0.elapsed_time(e1) / steps
    out["fp32"] = {"steps": steps, "ms_per_step": round(ms, 5), "mlups": round(w.fluid_nodes / (ms * 1e-3) / 1e6, 1),
                   "effective_GBps": round(w.fluid_nodes * BYTES_PER_LUP["fp32"] / (ms * 1e-3) / 1e9, 1),
                   "launch": dict(zip(("zchunk", "variant", "stage"), lbm.lbm_get_tuning(S.ctx)))}
    del S
    torch.cuda.empty_cache()
    out["travelling"], f_end = c5_travelling(keep_state=True)
    out["adjoint"] = c5_adjoint(f_end)
    return out


def c5_adjoint_rest():
    """The 512x256x256 FP64 adjoint alone (K = 100, checkpoint every 10), from
    the equilibrium state at rest under the frozen wave: the program the
    adjoint's counter runs profile (the kernels' work does not depend on the
    start state)."""
    import torch

    from paper_1803_07822_amd import lbm, synth

    w = synth.workload("c5_patch_wave_512x256x256")
    S = lbm.Solver(w.nx, w.ny, w.nz, w.tau, "fp64")
    S.set_body_force(w.force)
    S.set_wall_displacement(lbm.LBM_WALL_YMAX, w.disp())
    S.init_equilibrium()
    f0 = S.populations().cpu()
    del S
    torch.cuda.empty_cache()
    return c5_adjoint(f0, d_end=w.disp(), start="equilibrium at rest under the frozen wave (t = 0)")


def cpu_model():
    """The host CPU as /proc/cpuinfo names it (model name, family, model,
    stepping) and the cores this process may run on."""
    info = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                k, _, v = ln.partition(":")
                k = k.strip()
                if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                    info[k] = v.strip()
    except OSError:
        pass
    return {"model_name": info.get("model name", "unknown"), "family": info.get("cpu family"),
            "model": info.get("model"), "stepping": info.get("stepping"),
            "cores_available": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def oracle_rate(w, warm, timed, seed_noise=True):
    """The FP64 oracle stepping workload w on all the cores it uses: `warm`
    untimed steps, then `timed` timed steps; fluid-node updates per second."""
    import oracle
    from paper_1803_07822_amd import synth

    O = oracle.Oracle(w.nx, w.ny, w.nz, w.tau)
    O.set_body_force(w.force)
    O.set_wall_displacement(1, w.disp())
    O.init_equilibrium(None, synth.uniform_noise_velocity(w.nx, w.ny, w.nz, 1e-4, seed=2) if seed_noise else None)
    O.step(warm)
    t0 = time.perf_counter()
    O.step(timed)
    t = time.perf_counter() - t0
    return w.fluid_nodes * timed / t, t, O


def cpu_baseline(w, warm=2, timed=20):
    """The FP64 oracle on this host's cores, on the same workload: `warm`
    warm-up steps, then `timed` timed steps with all cores, then one step on a
    single thread."""
    import oracle

    cores = oracle.threads()
    rate, t, O = oracle_rate(w, warm, timed)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    O.step(1)
    t1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    return {"value": round(rate / 1e6, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{timed} FP64 steps of the full {w.nx}x{w.ny}x{w.nz} workload after {warm} warm-up steps "
                      f"({t:.1f} s)",
            "single_thread": {"value": round(w.fluid_nodes / t1 / 1e6, 3), "unit": "MLUPS",
                              "sample": f"1 FP64 step of the same workload on one thread ({t1:.1f} s)"},
            "cpu": cpu_model()}


def cpu_c5():
    """The oracle on the 512x256x256 workload (33.3M fluid nodes), all cores:
    2 warm-up steps, 5 timed (about a minute of CPU time, so not part of the
    default run)."""
    import oracle
    from paper_1803_07822_amd import synth

    w = synth.workload("c5_patch_wave_512x256x256")
    print("cpu_c5: oracle set-up and 7 steps of the 512x256x256 workload", file=sys.stderr, flush=True)
    rate, t, _ = oracle_rate(w, 2, 5, seed_noise=False)
    return {"workload": w.name, "value": round(rate / 1e6, 3), "unit": "MLUPS", "cores": oracle.threads(),
            "sample": f"5 FP64 steps after 2 warm-up steps ({t:.1f} s)", "cpu": cpu_model()}


def step_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload):
    """HBM bytes per launch of the FP32 step kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated), or None if the summary is
    for another workload or the kernel sources changed since it was taken."""
    try:
        with open(COUNTER_PROFILE) as fh:
            lines = [ln for ln in fh if ln.startswith("counters:")]
    except OSError:
        return None
    if not lines:
        return None
    kv = dict(item.split("=", 1) for item in lines[-1][len("counters:"):].split())
    if kv.get("workload") != workload or kv.get("source_sha256") != step_source_hash():
        return None
    return int(kv["fetch_bytes"]) + int(kv["write_bytes"])


def copy_rate():
    """Device-to-device copy of 1 GiB (the runtime's copy kernel), as a
    practical bandwidth reference beside the 8 TB/s peak: GB/s counting the
    bytes read plus the bytes written."""
    import torch

    a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / 10
    r = 2 * a.numel() * 4 / t / 1e9
    del a, b
    torch.cuda.empty_cache()
    return round(r, 1)


def stream_floor(n, precision, reps=10):
    """Time of lbm_stream_probe over n nodes: the step's 57 read and 29
    written planes as pure streams, no arithmetic (ms per launch)."""
    import torch

    from paper_1803_07822_amd import lbm

    dt = torch.float64 if precision == "fp64" else torch.float32
    a = torch.zeros(57 * n, dtype=dt, device="cuda")
    b = torch.empty(29 * n, dtype=dt, device="cuda")
    st = torch.cuda.current_stream()
    code = lbm.LBM_FP64 if precision == "fp64" else lbm.LBM_FP32_DEV
    for _ in range(3):
        lbm.lbm_stream_probe(code, n, a, b, st.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        lbm.lbm_stream_probe(code, n, a, b, st.cuda_stream)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return ms


def counter_run(w, steps, stage=-1):
    """What the HBM counters are read over: a device-to-device copy of
    256 MiB into a fresh buffer (calibrates FETCH_SIZE and WRITE_SIZE against
    known bytes), then `steps` FP32 steps of the workload with the default
    launch shape (or the staging asked for)."""
    import torch

    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()
    S, uc = setup(w, "fp32", 0, stage)
    S.step(steps)
    S.sync()
    from paper_1803_07822_amd import lbm

    z, v, st = lbm.lbm_get_tuning(S.ctx)
    print(json.dumps({"counter_run": w.name, "steps": steps, "zchunk": z, "variant": v, "stage": st}), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1803_07822_amd import lbm, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = synth.workload(a.workload)
    if a.counters:
        counter_run(w, a.steps, a.stage)
        return
    if a.part != "all":
        part = {"adjoint": adjoint_ratio, "c3": c3_loop, "c5": c5_runs, "flag": flag_channel,
                "open": open_channel, "cpu_c5": cpu_c5, "c5adj": c5_adjoint_rest}[a.part]()
        print(json.dumps({"part": a.part, **part}), flush=True)
        return
    N = w.fluid_nodes
    res = {}
    for prec, steps in (("fp32", a.steps), ("fp64", a.fp64_steps or max(10, a.steps // 2))):
        S, uc = setup(w, prec, a.variant, a.stage)
        ms, wall = time_steps(S, uc, steps, a.warmup)
        res[prec] = dict(ms=ms, steps=steps, wall=wall, tuning=lbm.lbm_get_tuning(S.ctx),
                         mlups=N / (ms * 1e-3) / 1e6,
                         eff_gbps=N * BYTES_PER_LUP[prec] / (ms * 1e-3) / 1e9)
        del S
        torch.cuda.empty_cache()
    f32 = res["fp32"]
    achieved = N * BYTES_PER_LUP["fp32"] / (f32["ms"] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(f32["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(f32["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "fluid_nodes": N, "tau": w.tau,
                   "form": "fp32 deviation storage, fp64 metric precompute"},
        "roofline": {
            "bound": "hbm",
            "kernel": step_kernel_name(f32["tuning"][1], f32["tuning"][2]),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": recorded_traffic(w.name) if a.variant == 0 and a.stage == -1 else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "bytes_per_lup": BYTES_PER_LUP["fp32"],
            "kernel_ms": round(f32["ms"], 5),
            "launch": dict(zip(("zchunk", "variant", "stage"), f32["tuning"])),
        },
        "fp64": {
            "mlups": round(res["fp64"]["mlups"], 2),
            "ms_per_step": round(res["fp64"]["ms"], 5),
            "effective_GBps": round(res["fp64"]["eff_gbps"], 1),
            "frac": round(res["fp64"]["eff_gbps"] / HBM_PEAK_GBPS, 4),
            "bytes_per_lup": BYTES_PER_LUP["fp64"],
            "launch": dict(zip(("zchunk", "variant", "stage"), res["fp64"]["tuning"])),
            "steps": res["fp64"]["steps"],
        },
        "fp32_effective_GBps": round(f32["eff_gbps"], 1),
        "device_copy_GBps": copy_rate(),
        "stream_floor": {},
        "adjoint_forward_ratio": None,
    }
    for prec in ("fp32", "fp64"):
        fm = stream_floor(N, prec)
        out["stream_floor"][prec] = {
            "ms": round(fm, 5), "GBps": round(N * BYTES_PER_LUP[prec] / (fm * 1e-3) / 1e9, 1),
            "step_over_floor": round(res[prec]["ms"] / fm, 3)}
    if not a.no_adjoint:
        out["adjoint"] = adjoint_ratio()
        out["adjoint_forward_ratio"] = out["adjoint"]["ratio"]
    if not a.no_extra:
        out["c3_time_varying_metric"] = c3_loop()
        out["c5_at_scale"] = c5_runs()
        out["flag_channel"] = flag_channel()
        out["open_channel"] = open_channel()
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
