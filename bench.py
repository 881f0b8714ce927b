#!/usr/bin/env python3
"""Throughput of the fused fire-mesh time step on one MI355X.

Default workload: the FP32 8192 x 8192 patchy fire (dx = 6 m, 13 Voronoi fuel
categories, 8 Gaussian hills, 16-mode Fourier wind re-drawn every 10 steps
from 4 fields resident in HBM, 4 line ignitions, dt = 0.25 s, refinement 10
-> 820 x 820 atmosphere cells).  One step is one call of fire_step(): the
whole method (ignition, both Heun stages, ignition times, fuel fraction,
fluxes, atmosphere averaging) in one fused kernel launch.

Prints one JSON line: cell-steps/s, the roofline of the step kernel measured
with HIP events on the launch stream (algorithmic bytes 37 B per cell-step in
FP32, 73 B in FP64, against 8 TB/s) and the FP64 CPU oracle timed on a bounded
sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
B_ALG = {"f32": 37.0, "f64": 73.0}   # bytes per cell-step the method must move
KERNEL = "k_step"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import numpy as np
    from paper_1102_1343_amd import synth
    if name == "patchy8192":
        p = synth.patchy_fire(n=8192, steps=1000, nwind=4, wind_period=10,
                              field_dtype=np.float32)
        return p, "f32"
    if name == "patchy8192_burning":
        p = synth.patchy_fire(n=8192, steps=1000, nwind=4, wind_period=10,
                              field_dtype=np.float32)
        return p, "f32"
    if name == "patchy2048":
        p = synth.patchy_fire(n=2048, steps=2000, field_dtype=np.float32)
        return p, "f32"
    if name == "uniform128":
        return synth.uniform_fire(128), "f64"
    if name == "adjoint1024":
        return synth.adjoint_case(n=1024, steps=500, field_dtype=np.float32), "f32"
    if name == "wind8192":
        return synth.atmosphere(820, 820, nz=40, dx=60.0, dy=60.0, dtype=np.float32), "f32"
    if name == "ensemble256":
        return synth.ensemble(ndom=256, side_min=256, side_max=1024, steps=500,
                              field_dtype=np.float32), "f32"
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash(files=("fire_kernels.hip", "fire_internal.h")):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1102_1343_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(name, dtype, tile, kernel=KERNEL,
                files=("fire_kernels.hip", "fire_internal.h")):
    """HBM bytes per launch of the kernel from the committed rocprofv3
    counter summary for this workload, if it was taken on the current kernel
    source with the same tile shape (None: no tile); else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{name}_{dtype}_pmc.txt")
    if tile is not None:   # one summary per tile shape where several were taken
        per_tile = os.path.join(ROOT, "profiles",
                                f"{kernel}_{name}_{dtype}_{tile[0]}x{tile[1]}_pmc.txt")
        if os.path.exists(per_tile):
            path = per_tile
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    t = re.search(r"tile:\s*(\d+)x(\d+)", txt)
    if not m or not b or m.group(1) != kernel_source_hash(files):
        return None
    if tile is not None and (not t or (int(t.group(1)), int(t.group(2))) != tuple(tile)):
        return None
    return float(b.group(1))


def host_cpu():
    """The host's processor model and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        ncpu = os.cpu_count()
    return {"model": model, "cpus_available": ncpu}


def cpu_baseline(prob, dtype, seconds):
    """The FP64 oracle on a window of the same workload (1024 x 1024 cells
    around the first ignition, the full mesh's initial level set), run for
    whole steps until ``seconds`` of wall time have passed on all the
    oracle's threads, then again from t = 0 on one thread for a third of
    that time."""
    import numpy as np
    import oracle
    from paper_1102_1343_amd import synth

    w = min(1024, prob.nx)
    h = min(1024, prob.ny)
    g0 = prob.ignitions[0] if prob.ignitions else dict(ax=prob.nx * prob.dx / 2,
                                                       ay=prob.ny * prob.dy / 2)
    sr = prob.sr_x
    i0 = int(min(max(0, g0["ax"] / prob.dx - w / 2), prob.nx - w)) // sr * sr
    j0 = int(min(max(0, g0["ay"] / prob.dy - h / 2), prob.ny - h)) // prob.sr_y * prob.sr_y
    win = synth.window(prob, i0, j0, w, h)
    if dtype == "f32":
        win = win.cast(np.float32)
    psi0 = math.hypot(prob.nx * prob.dx, prob.ny * prob.dy)

    def run(budget):
        """Cumulative wall time after each step."""
        o = oracle.OracleFire(win, psi_init=psi0)
        t0 = time.perf_counter()
        el = []
        while not el or el[-1] < budget or len(el) < 2:
            o.step(*win.wind_at(len(el)), win.dt)
            el.append(time.perf_counter() - t0)
        return el

    cores = oracle.threads()
    el = run(seconds)
    oracle.set_threads(1)
    try:
        el1 = run(seconds / 3)
    finally:
        oracle.set_threads(cores)
    steps, steps1 = len(el), len(el1)
    # the threads' speed-up over the steps both runs took
    k = min(steps, steps1) - 1
    return {"value": w * h * steps / el[-1], "unit": "cell-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"FP64 oracle, {w}x{h} window of the {prob.nx}x{prob.ny} workload at "
                      f"({i0},{j0}), first {steps} steps from t=0, {el[-1]:.1f} s wall",
            "single_thread": {"value": w * h * steps1 / el1[-1], "cores": 1,
                              "sample": f"the same window, first {steps1} steps, "
                                        f"{el1[-1]:.1f} s wall",
                              "threads_speedup_same_steps": el1[k] / el[k]},
            "host": host_cpu()}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's own step count, at most 1000)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="patchy8192",
                    choices=("patchy8192", "patchy8192_burning", "patchy2048", "uniform128",
                             "ensemble256",
                             "adjoint1024", "wind8192"))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", type=str, default="", help="tile_x,tile_y override")
    ap.add_argument("--every", type=int, default=50,
                    help="adjoint workload: checkpoint interval (steps)")
    ap.add_argument("--loop-steps", type=int, default=0,
                    help="ensemble workload: steps of the loop of plain contexts to time "
                         "(0: the same window as the ensemble)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run 5 device copies of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.copy_probe_mib:
        import torch
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                          "copies": 5}))
        return 0

    if args.gpus != 1:
        print(f"bench.py: the fire step runs on one GPU; --gpus {args.gpus} is not "
              "supported (several GPUs would each own a 2-D block of the fire mesh with a "
              "halo exchange every step, which is not implemented)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1102_1343_amd import fire as F

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)

    log(f"generating workload {args.workload}")
    t = time.perf_counter()
    prob, dtype = workload(args.workload)
    log(f"generated in {time.perf_counter() - t:.1f} s")
    if args.workload == "adjoint1024":
        return run_adjoint(args, *prob, dtype)
    if args.workload == "wind8192":
        return run_wind(args, prob, dtype)
    if args.steps is None:
        args.steps = min(1000, (prob[0] if isinstance(prob, list) else prob).steps)
    if args.workload == "ensemble256":
        return run_ensemble(args, prob, dtype)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    stream = torch.cuda.current_stream()
    fire = F.Fire.from_problem(prob, dtype=tdt)
    if args.workload == "patchy8192_burning":
        from paper_1102_1343_amd import synth
        psi, tign, frac, t0 = synth.burning_state(prob)
        fire.set_state(psi, tign, frac, t0)
        log(f"state set at t = {t0} s with {float((psi < 0).mean()):.3f} of the mesh burning")
    if args.tile:
        fire.set_tile(*[int(x) for x in args.tile.split(",")])
    winds = [(torch.from_numpy(np.ascontiguousarray(u)).to("cuda", tdt),
              torch.from_numpy(np.ascontiguousarray(v)).to("cuda", tdt)) for u, v in prob.wind]
    fs, fl = fire.new_flux()
    torch.cuda.synchronize()
    log(f"inputs resident; tile {fire.get_tile()}; warmup {args.warmup} steps")

    def wind(k):
        if prob.wind_period <= 0:
            return winds[0]
        return winds[(k // prob.wind_period) % len(winds)]

    step = 0
    for _ in range(args.warmup):
        u, v = wind(step)
        fire.step(u, v, prob.dt, fs, fl)
        step += 1
    torch.cuda.synchronize()

    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t_start.record(stream)
    for k in range(K):
        u, v = wind(step)
        ev[k][0].record(stream)
        fire.step(u, v, prob.dt, fs, fl)
        ev[k][1].record(stream)
        step += 1
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    total_ms = t_start.elapsed_time(t_end)
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    avg_kernel_s = sum(kern_ms) / len(kern_ms) / 1e3
    elapsed = max(total_ms / 1e3, 1e-12)
    cells = prob.nx * prob.ny
    value = cells * K / elapsed
    status = fire.status()
    burning = float((fire.psi < 0).float().mean())
    q = max(1, K // 10)
    log(f"{K} steps in {elapsed * 1e3:.2f} ms (wall {wall * 1e3:.1f} ms), kernel avg "
        f"{avg_kernel_s * 1e6:.1f} us (first tenth {sum(kern_ms[:q]) / q * 1e3:.1f}, last "
        f"{sum(kern_ms[-q:]) / q * 1e3:.1f}), status {status}, burning {burning:.4f}")

    bytes_per_launch = B_ALG[dtype] * cells
    achieved = bytes_per_launch / avg_kernel_s / 1e9
    traffic = pmc_traffic(args.workload, dtype, fire.get_tile())
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": KERNEL, "avg_kernel_us": round(avg_kernel_s * 1e6, 2),
            "alg_bytes_per_cell_step": B_ALG[dtype]}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host (cpu_baseline)")
        cpu = cpu_baseline(prob, dtype, args.cpu_seconds)
        log(f"oracle {cpu['value']:.3e} cell-steps/s on {cpu['cores']} threads, "
            f"{cpu['single_thread']['value']:.3e} on one ({cpu['host']['model']})")

    out = {
        "metric": "fire cell-steps/s",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": total_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {prob.nx}x{prob.ny} fire mesh, dx={prob.dx} m, "
                               f"{len(prob.fuels)} fuels, {len(prob.ignitions)} ignitions, "
                               f"dt={prob.dt} s, refinement {prob.sr_x} "
                               f"-> {fire.nax}x{fire.nay} atmosphere cells",
                   "nx": prob.nx, "ny": prob.ny, "dt": prob.dt, "sr": prob.sr_x,
                   "wind_fields": len(prob.wind), "wind_period": prob.wind_period,
                   "tile": list(fire.get_tile()), "status": status,
                   "burning_frac_end": round(burning, 5)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def cpu_baseline_members(probs, dtype, seconds):
    """The FP64 oracle on the ensemble's members in order, each for the
    workload's steps from t = 0, until ``seconds`` of wall time have passed
    (the last member stops at a whole step)."""
    import numpy as np
    import oracle

    cells_steps = 0
    done = []
    t0 = time.perf_counter()
    el = 0.0
    for p in probs:
        q = p.cast(np.float32) if dtype == "f32" else p
        o = oracle.OracleFire(q)
        k = 0
        while k < p.steps:
            o.step(*q.wind_at(k), q.dt)
            k += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                break
        cells_steps += p.nx * p.ny * k
        done.append((p.nx, k))
        if el >= seconds:
            break
    full = sum(1 for _, k in done if k == probs[0].steps)
    return {"value": cells_steps / el, "unit": "cell-steps/s", "cores": oracle.threads(),
            "kind": "oracle", "host": host_cpu(),
            "sample": f"FP64 oracle on the first {len(done)} members in order (sides "
                      f"{', '.join(str(n) for n, _ in done)}), {full} of them for all "
                      f"{probs[0].steps} steps from t=0, the last for {done[-1][1]}; "
                      f"{el:.1f} s wall"}


BWD_REPS = 3


def run_adjoint(args, prob, pert, dtype):
    """Cost of the hand-written adjoint: a run of `steps` fire steps under
    one wind, then the backward pass of L = 1/2 sum (F_end - F_target)^2 to
    the per-cell wind, the category multipliers and the ignition shifts,
    against the same run as plain fire_step calls."""
    import numpy as np
    import torch
    from paper_1102_1343_amd import fire as F

    tdt = torch.float32 if dtype == "f32" else torch.float64
    K = args.steps or prob.steps
    stream = torch.cuda.current_stream()
    u = torch.from_numpy(np.ascontiguousarray(prob.wind[0][0])).to("cuda", tdt)
    v = torch.from_numpy(np.ascontiguousarray(prob.wind[0][1])).to("cuda", tdt)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # target: the perturbed run
    fuels = [dict(f, ros_mult=float(m)) for f, m in zip(prob.fuels, pert["mult"])]
    tgt = F.Fire(prob.nx, prob.ny, prob.dx, prob.dy, prob.sr_x, prob.sr_y, fuels, prob.cat,
                 prob.dzdx, prob.dzdy, F.shifted_ignitions(prob.ignitions, pert["shift"]),
                 dtype=tdt, **{k: prob.params[k] for k in ("viscosity", "ros_cap",
                                                            "boundary_policy")})
    fs, fl = tgt.new_flux()
    us, vs = u * pert["wind_scale"], v * pert["wind_scale"]
    for _ in range(K):
        tgt.step(us, vs, prob.dt, fs, fl)
    target = tgt.frac.clone()
    tgt.close()

    # plain forward
    plain = F.Fire.from_problem(prob, dtype=tdt)
    fs, fl = plain.new_flux()
    plain.step(u, v, prob.dt, fs, fl)      # warm-up launch
    plain.close()
    plain = F.Fire.from_problem(prob, dtype=tdt)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(stream)
    for _ in range(K):
        plain.step(u, v, prob.dt, fs, fl)
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1)
    F_plain = plain.frac.clone()
    plain.close()

    # warm-up: a 2-step adjoint loads every kernel of the recording forward
    # and the backward before anything is timed
    warm = F.Fire.from_problem(prob, dtype=tdt)
    wadj = F.FireAdjoint(warm, 2, 1)
    wF = wadj.forward(u, v, prob.dt)
    wadj.backward((wF - 1).contiguous())
    wadj.close()
    warm.close()

    # recording forward, then the backward: one untimed call, then the mean
    # of BWD_REPS timed calls (each replays the same checkpoints; the
    # gradients must come out bit for bit the same every time)
    fire = F.Fire.from_problem(prob, dtype=tdt)
    adj = F.FireAdjoint(fire, K, args.every)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(stream)
    Fend = adj.forward(u, v, prob.dt)
    e1.record(stream)
    torch.cuda.synchronize()
    rec_ms = e0.elapsed_time(e1)
    dF = (Fend - target).contiguous()
    gu, gv, gm, gs = adj.backward(dF)
    torch.cuda.synchronize()
    e1.record(stream)
    reps = [adj.backward(dF) for _ in range(BWD_REPS)]
    e2 = ev()
    e2.record(stream)
    torch.cuda.synchronize()
    bwd_ms = e1.elapsed_time(e2) / BWD_REPS
    repeat_equal = all(torch.equal(ru, gu) and torch.equal(rv, gv) and np.array_equal(rm, gm)
                       and np.array_equal(rs, gs) for ru, rv, rm, rs in reps)
    del reps
    same = bool(torch.equal(Fend, F_plain))
    loss = 0.5 * float(((Fend - target).double() ** 2).sum())
    log(f"{K} steps: plain forward {fwd_ms:.1f} ms, recording forward {rec_ms:.1f} ms, "
        f"backward {bwd_ms:.1f} ms; loss {loss:.4e}; F_end equal to the plain run: {same}")
    out = {
        "metric": "gradient cost: (recording forward + backward) / plain forward",
        "value": (rec_ms + bwd_ms) / fwd_ms,
        "unit": "x",
        "n_gpus": 1,
        "steps": K,
        "warmup": 1,
        "ms_per_step": (rec_ms + bwd_ms) / K,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"adjoint1024: {prob.nx}x{prob.ny} fire mesh, dx={prob.dx} m, "
                               f"{len(prob.fuels)} fuels, 2 instant circular ignitions, "
                               f"dt={prob.dt} s, {K} steps, checkpoint every {args.every}; "
                               "loss 1/2 sum (F_end - F_target)^2",
                   "nx": prob.nx, "ny": prob.ny, "every": args.every},
        "adjoint": {"forward_ms": fwd_ms, "recording_forward_ms": rec_ms, "backward_ms": bwd_ms,
                    "backward_reps": BWD_REPS, "backward_repeats_bit_equal": repeat_equal,
                    "backward_over_forward": bwd_ms / fwd_ms,
                    "loss": loss, "F_end_equals_plain_run": same,
                    "grad_norms": {"u": float(gu.double().norm()), "v": float(gv.double().norm()),
                                   "mult": float(np.linalg.norm(gm)),
                                   "shift": float(np.linalg.norm(gs))}},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def run_wind(args, atm, dtype):
    """Coupling input: the staggered atmosphere wind (820 x 820 columns of
    60 m, 40 levels) to the 8192 x 8192 fire mesh at 6.1 m, K calls."""
    import numpy as np
    import torch
    import oracle.wind as W
    from paper_1102_1343_amd import fire as F

    nx = ny = 8192
    sr = 10
    tdt = torch.float32 if dtype == "f32" else torch.float64
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).to("cuda", tdt) for k, v in atm.items()}
    nz, nay, nax1 = dev["u3"].shape
    nax = nax1 - 1
    nb = F.wind_scratch_bytes(nax, nay, nz, nx, ny, sr, sr, tdt)
    scratch = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    u = torch.empty((ny, nx), dtype=tdt, device="cuda")
    v = torch.empty_like(u)
    stream = torch.cuda.current_stream()
    inputs = [dev[k] for k in ("u3", "v3", "phi", "hgt", "z0")]

    def call():
        F.wind_interp(*inputs, nx, ny, sr, sr, out=(u, v), scratch=scratch)

    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    K = args.steps or 200
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for k in range(K):
        ev[k][0].record(stream)
        call()
        ev[k][1].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    avg_s = sum(a.elapsed_time(b) for a, b in ev) / K / 1e3
    value = nx * ny * K / (total_ms / 1e3)
    es = 4 if dtype == "f32" else 8
    alg = 2 * es * nx * ny            # the two outputs; the staggered inputs are ~1 % of it
    log(f"{K} calls in {total_ms:.2f} ms, avg {avg_s * 1e6:.1f} us per call")
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host (cpu_baseline)")
        sub = {k: np.asarray(atm[k], dtype=np.float64) for k in atm}
        w = 40                          # 40 x 40 columns -> 400 x 400 fire cells
        win = dict(u3=sub["u3"][:, :w, :w + 1], v3=sub["v3"][:, :w + 1, :w],
                   phi=sub["phi"][:, :w, :w], hgt=sub["hgt"][:w, :w], z0=sub["z0"][:w, :w])
        n = 0
        t = time.perf_counter()
        while time.perf_counter() - t < args.cpu_seconds or n == 0:
            W.fire_wind(win["u3"], win["v3"], win["phi"], win["hgt"], win["z0"], w * sr, w * sr,
                        sr, sr)
            n += 1
        el = time.perf_counter() - t
        cpu = {"value": (w * sr) ** 2 * n / el, "unit": "fire cells/s", "cores": 1,
               "kind": "oracle", "host": host_cpu(),
               "sample": f"FP64 oracle (numpy, one thread), the {w}x{w}-column corner of the "
                         f"atmosphere to its {w * sr}x{w * sr} fire cells, {n} times, {el:.1f} s"}
        log(f"oracle {cpu['value']:.3e} fire cells/s")
    out = {
        "metric": "surface wind fire cells/s",
        "value": value,
        "unit": "fire cells/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": total_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"wind8192: {nax}x{nay} atmosphere columns of 60 m, {nz} levels, "
                               f"staggered u/v -> {nx}x{ny} fire mesh (6 m) at 6.1 m",
                   "nax": nax, "nay": nay, "nz": nz, "nx": nx, "ny": ny},
        "roofline": {"bound": "hbm", "achieved": round(alg / avg_s / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": pmc_traffic("wind8192", dtype, None, kernel="k_wind",
                                            files=("fire_wind.hip", "fire_internal.h")),
                     "kernel": "k_wind_vertical + k_wind_bilinear",
                     "avg_kernel_us": round(avg_s * 1e6, 2),
                     "alg_bytes_per_fire_cell": 2 * es},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


ENS_TILES = [(120, 20), (120, 10), (60, 20), (120, 30), (120, 40), (60, 10), (60, 40)]


def run_ensemble(args, probs, dtype):
    """All members in one launch per step (HIP graph replay of fire_ens_step),
    under both schedules of the step kernel (one work-group per tile; resident
    work-groups), each from t = 0 over the same step window, against a loop of
    one plain fire_step per member and step over that window too."""
    import numpy as np
    import torch
    from paper_1102_1343_amd import fire as F

    tdt = torch.float32 if dtype == "f32" else torch.float64
    stream = torch.cuda.current_stream()
    dt = probs[0].dt
    K, W = args.steps, args.warmup
    tile = tuple(int(x) for x in args.tile.split(",")) if args.tile else None

    def timed(resident):
        ens = F.FireEnsemble.from_problems(probs, dtype=tdt)
        u = ens.concat([p.wind[0][0] for p in probs])
        v = ens.concat([p.wind[0][1] for p in probs])
        fs, fl = ens.new_flux()
        ens.set_schedule(resident)
        torch.cuda.synchronize()
        if tile is None:
            log(f"ensemble of {ens.ndom}, {ens.ncells} cells resident; autotuning tiles "
                f"({'resident' if resident else 'grid'} schedule)")
            best = ens.autotune(u, v, dt, ENS_TILES, reps=3)
        else:
            best = tile
            ens.set_tile(*best)
        for _ in range(W):
            ens.step(u, v, dt, fs, fl)
        torch.cuda.synchronize()
        # capture one step; each replay is one step of every member
        side = torch.cuda.Stream()
        ens.set_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                ens.step(u, v, dt, fs, fl)
        ens.set_stream(stream)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(K)]
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for k in range(K):
            ev[k][0].record(stream)
            graph.replay()
            ev[k][1].record(stream)
        t1.record(stream)
        torch.cuda.synchronize()
        total_ms = t0.elapsed_time(t1)
        step_us = [x.elapsed_time(y) * 1e3 for x, y in ev]
        status = ens.status()
        burning = float((ens.psi < 0).float().mean())
        q = max(1, K // 10)
        r = {"value": ens.ncells * K / (total_ms / 1e3), "ms_per_step": total_ms / K,
             "avg_step_us": sum(step_us) / K, "first_tenth_us": sum(step_us[:q]) / q,
             "last_tenth_us": sum(step_us[-q:]) / q, "flagged": int((status != 0).sum()),
             "burning": burning, "cells": ens.ncells, "tile": list(best)}
        log(f"resident {resident}, tile {best}: {K} graph steps in {total_ms:.2f} ms, avg "
            f"{r['avg_step_us']:.1f} us/step (first tenth {r['first_tenth_us']:.1f}, last "
            f"{r['last_tenth_us']:.1f}), {r['flagged']} members flagged, burning {burning:.4f}")
        del graph
        ens.close()
        return r

    sched = {"grid": timed(False), "resident": timed(True)}
    main_name = "grid"    # the library's default schedule
    main = sched[main_name]
    cells = main["cells"]
    tile = tuple(main["tile"])

    # the same members as plain contexts, one fire_step each per step, over
    # the same window (W untimed steps, then K timed); --loop-steps L > 0
    # times L steps after one untimed step instead (a short check)
    plain = [F.Fire.from_problem(p, dtype=tdt) for p in probs]
    pw = [(torch.from_numpy(np.ascontiguousarray(p.wind[0][0])).to("cuda", tdt),
           torch.from_numpy(np.ascontiguousarray(p.wind[0][1])).to("cuda", tdt)) for p in probs]
    pf = [g.new_flux() for g in plain]
    KL, WL = (K, W) if args.loop_steps <= 0 else (max(1, min(args.loop_steps, K)), 1)
    for _ in range(WL):
        for g, (uu, vv), (a, b) in zip(plain, pw, pf):
            g.step(uu, vv, dt, a, b)
    torch.cuda.synchronize()
    l0, l1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    l0.record(stream)
    for _ in range(KL):
        for g, (uu, vv), (a, b) in zip(plain, pw, pf):
            g.step(uu, vv, dt, a, b)
    l1.record(stream)
    torch.cuda.synchronize()
    loop_ms = l0.elapsed_time(l1)
    loop_value = cells * KL / (loop_ms / 1e3)
    log(f"loop of {len(plain)} plain steps over steps {WL}..{WL + KL - 1}: "
        f"{loop_ms / KL:.3f} ms/step")
    for g in plain:
        g.close()

    avg_step_s = main["avg_step_us"] / 1e6
    bytes_per_launch = B_ALG[dtype] * cells
    achieved = bytes_per_launch / avg_step_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": pmc_traffic(args.workload, dtype, tile, kernel="k_ens_step"),
            "kernel": "k_ens_step", "avg_kernel_us": round(main["avg_step_us"], 2),
            "alg_bytes_per_cell_step": B_ALG[dtype],
            "note": "duration per graph replay (geometry, step and one-thread clock kernels)"}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host (cpu_baseline)")
        cpu = cpu_baseline_members(probs, dtype, args.cpu_seconds)
        log(f"oracle {cpu['value']:.3e} cell-steps/s on {cpu['cores']} threads")
    sides = [p.nx for p in probs]
    out = {
        "metric": "fire cell-steps/s",
        "value": main["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": main["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"ensemble256: {len(probs)} square fire domains, sides "
                               f"{min(sides)}-{max(sides)} (sum {cells} cells), dx=6 m, "
                               f"dt={dt} s, refinement 10, one HIP-graph replay per step",
                   "members": len(probs), "cells": cells, "tile": list(tile),
                   "schedule": main_name,
                   "members_flagged": main["flagged"],
                   "burning_frac_end": round(main["burning"], 5)},
        "ensemble": {"schedules": sched, "loop_value": loop_value, "loop_steps": KL,
                     "loop_window": [WL, WL + KL],
                     "loop_ms_per_step": loop_ms / KL,
                     "speedup_vs_loop": main["value"] / loop_value,
                     "resident_over_grid": sched["resident"]["value"] / sched["grid"]["value"]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
