"""Benchmark: adjoint-state FWI gradient throughput on one MI355X.

One step = one complete gradient of the least-squares misfit for every shot
of the workload (forward sweep keeping checkpoints, misfit, per segment a
recompute storing the pressure and the adjoint sweep with imaging,
finalization), chain-ruled into the K-rho, Vp-rho, Ip-rho and Vp-Ip
parameterizations.  The default workload is smooth-1001: 1001^2 at 5 m + 40
PML, 64 shots, 4000 steps, checkpoints every 64 steps (its live state is far
beyond the 256 MB Infinity Cache, so the sweeps stream from HBM).  The
library keeps the whole pressure history instead when it fits in half the
HBM (gauss-401: 97 GB), and then the checkpointed form is timed beside it.
value = padded cells x time steps x shots / seconds per step
(Gcell-updates/s; each cell-step counted once although the forward,
recompute and adjoint sweeps all touch it).

Beside the timed steps: the forward-only modelling rate (traces of every
shot, nothing kept), the plain path (one shot per launch) on the same
workload, a served stream of gradient requests of mixed sizes (p50 / p99
latency and aggregate rate), and the FP64 oracle on a sample of the
workload on the host cores.

Prints one JSON line.  Inputs are synthetic (workloads.py), generated and
resident in HBM before the timed region.  The timed steps run without
per-launch instrumentation; one further step with per-launch timing
(dispatch-stamped events for the sweep kernels) gives the per-kernel
figures and the roofline entry.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "Gcell-updates/s (fwd+adjoint grad, FP32) vs plain; p50/p99 gradient latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="smooth1001",
                    choices=["gauss401", "smooth1001", "layered2001"])
    ap.add_argument("--shots", type=int, default=0,
                    help="evenly spaced subset of the shots (default: all; layered2001: 32, one GPU's "
                         "share of 256 shots over 8)")
    ap.add_argument("--band-rows", type=int, default=0)
    ap.add_argument("--shots-per-group", type=int, default=0)
    ap.add_argument("--lane-cols", type=int, default=0)
    ap.add_argument("--ckpt-every", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true",
                    help="use the library's default decomposition instead of the autotuned "
                         "one (the tuner also runs unless a decomposition is given)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forward", action="store_true",
                    help="no forward-only modelling leg")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="time steps of the CPU sample (default: all of the workload's)")
    ap.add_argument("--cpu-shots", type=int, default=1, help="shots of the CPU sample")
    ap.add_argument("--cpu-single-steps", type=int, default=64,
                    help="time steps of the single-thread CPU sample (0: none)")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests of the served Poisson stream (0: no serving leg)")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="offered load of the served stream, as a fraction of the gradient "
                         "rate measured in the timed steps")
    ap.add_argument("--time-steps", type=int, default=0,
                    help="run the workload for this many time steps instead of its own "
                         "(short runs under hardware-counter profiling; per-launch work is "
                         "unchanged)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="no per-launch event timing (for hardware-counter runs); the "
                         "roofline entry is then omitted")
    ap.add_argument("--born", action="store_true",
                    help="schemes I/II instead: one Born gradient per step (frequency-domain "
                         "form of the 401² Gaussian benchmark), one JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB elementwise kernel (reads 1 GiB, writes 1 GiB) and "
                         "exit: the reference for the HBM traffic counters")
    return ap.parse_args()


def workload(name, shots=0):
    from paper_1804_01184_amd import workloads as W
    w = {"gauss401": W.gauss401, "smooth1001": W.smooth1001, "layered2001": W.layered2001}[name]()
    if name == "layered2001" and not shots:
        shots = 32
    if shots and shots < w.nshots:
        idx = np.linspace(0, w.nshots - 1, shots).round().astype(int)
        w = w.subset(shots=idx, name=f"{w.name}-{shots}of{w.nshots}")
    return w


def algorithmic_bytes(plan_info, S, k):
    """Algorithmic HBM bytes per cell-step of each sweep (FP32 streaming,
    the model and the gradient read once per pass over the S shots):
      forward    24 + 8 fp + 8/S + 12/k   read and write vx, vz, p; the
                                          absorbing-layer split (fp = layer
                                          fraction); K and the buoyancies;
                                          checkpoint writes every k steps
      recompute  forward + 4              the pressure stored for the adjoint
      adjoint    24 + 8 fp + 8/S + 4 + 16/S   adjoint state read and write,
                                          its split, the model, the stored
                                          pressure read once (carried over
                                          from the previous reverse step),
                                          gK and the buoyancy gradient pair
                                          read and written once
    and, per kernel class, the cell-steps one launch advances (a two-step
    forward launch advances two).  The forward kernels in a gradient store
    the pressure, so both are charged the recompute figure.  The kernels'
    own minimum for one launch (a one-step adjoint must read both pressure
    levels and their splits, and in this design reads the model and
    read-modify-writes the gradient once per shot group) is larger; the
    counter traffic shows what they move."""
    N = plan_info["Nz"] * plan_info["Nx"]
    fp = plan_info["pml_cells"] / N
    fwd = 24 + 8 * fp + 8 / S + 12 / k
    rec = fwd + 4
    adj = 24 + 8 * fp + 8 / S + 4 + 16 / S
    per_cell = {"fwd_step": rec, "fwd_pair": rec, "adj_step": adj, "adj_pair": adj}
    cells = {"fwd_step": N * S, "fwd_pair": 2 * N * S, "adj_step": N * S, "adj_pair": 2 * N * S}
    return {"pml_fraction": fp, "per_cell": per_cell, "cell_steps": cells,
            "gradient_per_cell": rec + rec + adj - 4 - 12 / k}


KERNEL_SOURCE = os.path.join(ROOT, "paper_1804_01184_amd", "csrc", "k_fused.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
BORN_SOURCE = os.path.join(ROOT, "paper_1804_01184_amd", "csrc", "k_born.hip")
BORN_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_born.json")


def measured_traffic(kernel, decomposition, traffic_file=TRAFFIC_FILE, source=KERNEL_SOURCE):
    """HBM bytes per launch of `kernel` from the committed counter profile
    (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or None if
    the profile was taken with another kernel source or decomposition."""
    try:
        with open(traffic_file) as fh:
            prof = json.load(fh)
        with open(source, "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, ValueError):
        return None
    # entries are keyed "<kernel class>@<workload>" (or by the class alone)
    kern = prof.get("kernels", {})
    k = kern.get(f"{kernel}@{decomposition.get('workload')}", kern.get(kernel))
    if prof.get("source_sha256") != sha or k is None or k.get("decomposition") != decomposition:
        return None
    return int(k["bytes_per_launch"])


def copy_calibration():
    import torch
    torch.cuda.set_device(0)
    n = 256 * 1024 * 1024
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a).fill_(0.0)
    torch.cuda.synchronize()
    torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n}}))


def host_cpu():
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(w, shots, steps, single_steps):
    """The FP64 oracle on a bounded sample of the same workload: the full
    grid, `shots` evenly spaced shots, `steps` time steps (checkpoints every
    ceil(sqrt(steps)), as the GPU plan), the gradient in Vp-rho; all host
    threads (over grid rows when there are fewer shots than threads), then
    one thread on a shorter run.  Observed data zero (same cost as any)."""
    import math
    import oracle as O

    def run(nt):
        idx = np.linspace(0, w.nshots - 1, shots).round().astype(int)
        sub = w.subset(shots=idx, nt=nt)
        g = O.Grid(sub.nz, sub.nx, sub.dz, sub.dx, sub.npml, sub.nt, sub.dt, sub.vmax,
                   sub.pml_r)
        f = sub.wavelet()
        obs = np.zeros((shots, sub.nrec, sub.nt))
        k = int(math.ceil(math.sqrt(nt)))
        t = time.perf_counter()
        O.gradient(g, O.VP_RHO, sub.vp_start, sub.rho_start, sub.src_xz, sub.rec_xz, f, obs, k)
        dt = time.perf_counter() - t
        Nz, Nx = sub.padded
        return Nz * Nx * nt * shots / dt / 1e9, dt

    nth = O.num_threads()
    print(f"bench: CPU oracle, {shots} shot(s) x {steps} steps on {nth} threads",
          file=sys.stderr, flush=True)
    rate, dt = run(steps)
    out = {"value": round(rate, 5), "unit": "Gcell-updates/s", "cores": nth, "kind": "oracle",
           "seconds": round(dt, 2), "host": host_cpu(),
           "sample": f"{shots} shot(s) x {steps} of {w.nt} time steps of the full "
                     f"{w.padded[0]}x{w.padded[1]} padded grid: a complete gradient of those "
                     f"shots in Vp-rho (FP64, checkpoints every "
                     f"{int(np.ceil(np.sqrt(steps)))} steps, OpenMP over "
                     f"{'rows' if shots < nth else 'shots'})"}
    if single_steps:
        O.set_num_threads(1)
        try:
            r1, d1 = run(single_steps)
        finally:
            O.set_num_threads(nth)
        out["single_thread"] = {"value": round(r1, 5), "seconds": round(d1, 2),
                                "sample": f"{shots} shot(s) x {single_steps} time steps, "
                                          f"one thread"}
    return out


def serve_leg(dev, rate_gcells, n, load):
    """A seeded Poisson stream of `n` gradient requests of mixed sizes (the
    serving workload: sides 201..1201 + 40 PML, 8-64 shots, 1000-4000 steps,
    Gaussian-anomaly models) served by continuous batching on 4 streams.
    Arrivals are scaled so the offered load is `load` of the batched
    gradient rate measured in the timed steps.  Returns p50 / p99 latency
    (arrival to completion) and the aggregate rate over the makespan."""
    import torch
    from paper_1804_01184_amd import serve, workloads as W
    specs = W.serving_requests(n, rate_hz=1.0)
    t = time.perf_counter()
    reqs = serve.make_requests(specs, device=dev)
    torch.cuda.synchronize()
    prep = time.perf_counter() - t
    cells = np.array([q.cell_steps for q in reqs], dtype=np.float64)
    mean_service = float(cells.mean()) / (rate_gcells * 1e9)
    gap = float(np.mean(np.diff([0.0] + [s["arrival"] for s in specs])))
    scale = mean_service / load / gap
    for q, sp in zip(reqs, specs):
        q.arrival = sp["arrival"] * scale
    print(f"bench: serving {n} requests (Poisson, mean gap {mean_service / load:.2f} s)",
          file=sys.stderr, flush=True)
    srv = serve.GradientServer(max_slots=4, device=dev)
    res = srv.run(reqs)
    summ = serve.summary(res, srv.makespan)
    return {"requests": n, "slots": 4, "offered_load": load,
            "p50_ms": round(summ["p50_ms"], 1), "p99_ms": round(summ["p99_ms"], 1),
            "mean_ms": round(summ["mean_ms"], 1),
            "aggregate_gcells": round(summ["aggregate_gcells"], 3),
            "makespan_s": round(srv.makespan, 2), "prepare_s": round(prep, 1),
            "cell_steps": int(cells.sum())}


def born_cpu_baseline(w, xk, xr, flops):
    """The FP64 oracle's Born data on a bounded sample: one frequency, one
    source, half the receivers, every cell."""
    from oracle import born as OB
    f = len(w.freqs) // 2
    rec = w.rec_xz[::2]
    t = time.perf_counter()
    OB.scattered(w.omega[f:f + 1], w.src_xz[:1], rec, w.cells, w.dA, w.K0, w.rho0, xk, xr)
    dt = time.perf_counter() - t
    frac = 1.0 / (len(w.freqs) * len(w.src_xz)) * len(rec) / len(w.rec_xz)
    return {"value": round(flops * frac / dt / 1e12, 6), "unit": "TFLOP/s", "kind": "oracle",
            "cores": 1, "seconds": round(dt, 2),
            "sample": f"Born data of one frequency, one source, {len(rec)} receivers and all "
                      f"{len(xk)} cells (FP64 numpy/scipy); rate counted as 24 flops per "
                      f"(frequency, source, receiver, cell)"}


def born_main(args):
    """One step = one scheme-II gradient: contrast map, Born data, misfit,
    adjoint (gradient in the inverse contrasts), chain rule; the Green
    tables are built once per geometry, before the timed region."""
    import torch
    from paper_1804_01184_amd import born, workloads as W
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    w = W.born_gauss401()
    sz = w.sizes()
    m = born.measure(w, reps=max(args.steps, 1), device=dev)
    prob = born.BornProblem.of(w, dev)
    xa = torch.tensor(w.xa.ravel(), dtype=torch.float32, device=dev)
    xb = torch.tensor(w.xb.ravel(), dtype=torch.float32, device=dev)
    q = prob.data(*born.contrasts(2, w.param, xa, xb))
    za, zb = torch.zeros_like(xa), torch.zeros_like(xb)
    d = torch.empty_like(q)

    def step():
        xk, xr = born.contrasts(2, w.param, za, zb)
        prob.data(xk, xr, out=d)
        _, r = prob.misfit(d, q)
        gK, gR = prob.gradient(r)
        return born.chain(2, w.param, za, zb, gK, gR)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / args.steps
    flops = m["flops_per_launch"]
    dom = "data" if m["data"]["ms"] >= m["gradient"]["ms"] else "gradient"
    kname = "k_born_data_mfma" if dom == "data" else "k_born_grad_mfma"
    roof = {"bound": "mfma", "achieved": round(m[dom]["tflops"], 3),
            "peak": born.PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(m[dom]["tflops"] / born.PEAK_FP32_TFLOPS, 4),
            "traffic": measured_traffic(kname, {"workload": w.name, **sz}, BORN_TRAFFIC_FILE,
                                        BORN_SOURCE),
            "traffic_unit": "bytes per launch", "kernel": kname,
            "flops_per_launch": flops, "avg_ms": round(m[dom]["ms"], 4)}
    xk, xr = (t_.cpu().numpy().astype(np.float64) for t_ in m["contrasts"])
    cpu = None if args.no_cpu else born_cpu_baseline(w, xk, xr, flops)
    rec = {"metric": "Born gradient (schemes I/II): TFLOP/s of the data and adjoint sums",
           "value": round(2 * flops / (ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"{w.name}: {w.nz}x{w.nx} cells at {w.dx:g} m, "
                                  f"{sz['S']} sources x {sz['R']} receivers, {sz['F']} "
                                  f"frequencies, scheme II in {w.param}",
                      **sz},
           "kernels_ms": {"green_tables": round(m["green"]["ms"], 3),
                          "data": round(m["data"]["ms"], 3),
                          "gradient": round(m["gradient"]["ms"], 3)},
           "roofline": roof, "cpu_baseline": cpu}
    print(json.dumps(rec), flush=True)


def main():
    args = parse()
    if args.born:
        born_main(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (shots would "
              "shard across GPUs with one all-reduce of the gradient; not built here)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1804_01184_amd import api

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    w = workload(args.workload, args.shots)
    if args.time_steps:
        w = w.subset(nt=args.time_steps)
    grid = api.Grid.of(w)
    f = torch.tensor(w.wavelet(), dtype=torch.float32, device=dev)
    vp0 = torch.tensor(w.vp_start, dtype=torch.float32, device=dev)
    rho0 = torch.tensor(w.rho_start, dtype=torch.float32, device=dev)
    decomp = {"band_rows": args.band_rows, "shots_per_group": args.shots_per_group,
              "lane_cols": args.lane_cols}
    tuned = None
    if not args.no_tune and not any(decomp.values()):
        # the autotuner times the candidate decompositions on a short run of
        # this shape (cached per shape and GPU), outside the timed region
        from paper_1804_01184_amd import autotune
        t = time.perf_counter()
        decomp = autotune.tune(grid, w.src_xz, w.rec_xz)
        tuned = {"seconds": round(time.perf_counter() - t, 2)}
        print(f"bench: decomposition {decomp} ({tuned['seconds']} s)", file=sys.stderr,
              flush=True)
    plan = api.Plan(grid, w.src_xz, w.rec_xz, ckpt_every=args.ckpt_every, **decomp)
    info = plan.info
    obs = plan.forward("vp-rho", w.vp_true, w.rho_true, f)
    torch.cuda.synchronize()
    print(f"bench: {w.name}, observed data modelled; {info['segments']} segment(s)",
          file=sys.stderr, flush=True)
    K0, r0 = api.model_convert("vp-rho", "k-rho", vp0, rho0)
    Jb = torch.empty(1, dtype=torch.float32, device=dev)
    gK, gr = torch.empty_like(K0), torch.empty_like(K0)
    others = {p: api.model_convert("k-rho", p, K0, r0) for p in ("vp-rho", "ip-rho", "vp-ip")}
    out = {}

    def step():
        plan.gradient("k-rho", K0, r0, f, obs, out=(Jb, gK, gr))
        for p, (m1, m2) in others.items():
            out[p] = api.chain_rule(p, m1, m2, gK, gr)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # timed steps: no per-launch instrumentation
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        step()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # one more step with per-launch timing for the kernel figures
    per_class = {}
    if not args.no_kernel_timing:
        plan.timing(True)
        step()
        torch.cuda.synchronize()
        per_class = plan.timing_read(reset=True)
        plan.timing(False)
    lat = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    ms = wall / args.steps * 1e3
    cells = w.cell_steps()
    value = cells / (ms * 1e-3) / 1e9

    S, G = w.nshots, info["shot_groups"]
    ab = algorithmic_bytes(info, S, info["ckpt_every"])
    roof, roof_all = None, {}
    if not args.no_kernel_timing:
        # every sweep kernel that ran: achieved = its per-cell-step algorithmic
        # bytes x the cell-steps of one launch / its average launch time; the
        # entry of the kernel with the largest total time is `roofline`
        prefix = {"fwd_pair": "two_step_", "adj_pair": "adj_two_step_"}
        for kc in ab["per_cell"]:
            n_launch, kc_ms = per_class.get(kc, (0, 0.0))
            if not n_launch:
                continue
            avg_s = kc_ms / n_launch * 1e-3
            per_launch = ab["per_cell"][kc] * ab["cell_steps"][kc]
            achieved = per_launch / avg_s / 1e9
            pre = prefix.get(kc, "")
            kdec = {"band_rows": info[pre + "band_rows"],
                    "shots_per_group": info["two_step_shots_per_group" if kc == "fwd_pair"
                                            else "shots_per_group"],
                    "lane_cols": info[pre + "lane_cols"], "workload": w.name}
            roof_all[kc] = {
                "bound": "hbm", "kernel": kc, "achieved": round(achieved, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": measured_traffic(kc, kdec),
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)",
                "avg_launch_us": round(avg_s * 1e6, 2), "launches": n_launch,
                "total_ms": round(kc_ms, 2), "decomposition": kdec,
                "cell_steps_per_launch": ab["cell_steps"][kc],
                "bytes_per_cell_step": round(ab["per_cell"][kc], 3),
                "bytes_per_launch": int(per_launch),
                "gradient_bytes_per_cell_step": round(ab["gradient_per_cell"], 2),
                "gradient_roof_gcells": round(PEAK_HBM_GBS / ab["gradient_per_cell"], 1),
                "pml_fraction": round(ab["pml_fraction"], 4)}
            tr = roof_all[kc]["traffic"]
            if tr:
                # what the kernel moves (counters) at this launch time
                roof_all[kc]["traffic_achieved"] = round(tr / avg_s / 1e9, 1)
                roof_all[kc]["traffic_frac"] = round(tr / avg_s / 1e9 / PEAK_HBM_GBS, 4)
            if kc.endswith("_pair"):
                roof_all[kc]["note"] = (
                    "two time steps per launch: the state between them stays on chip, so "
                    "the per-cell-step algorithmic bytes include bytes this kernel never "
                    "moves (traffic is what it moves)")
        if roof_all:
            roof = roof_all[max(roof_all, key=lambda k: roof_all[k]["total_ms"])]
    classes = {k: {"launches": v[0], "ms": round(v[1], 3)} for k, v in per_class.items()
               if v[0]}

    # the same gradient with sqrt(nt) checkpoints and segment recompute (the
    # memory-bounded form the autograd path uses on large grids)
    ckpt = None
    if not args.no_plain and info["segments"] == 1:
        import math
        kc = int(math.ceil(math.sqrt(w.nt)))
        pc = api.Plan(grid, w.src_xz, w.rec_xz, ckpt_every=kc, **decomp)
        pc.gradient("k-rho", K0, r0, f, obs)          # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        pc.gradient("k-rho", K0, r0, f, obs)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t
        ckpt = {"ckpt_every": kc, "value": round(cells / tc / 1e9, 3),
                "ms_per_step": round(tc * 1e3, 2)}
        del pc

    # forward-only modelling (traces of every shot, no pressure kept), the
    # same batched kernels; forward-only algorithmic bytes 24 + 8 fp + 8/S
    fwd_only = None
    if not args.no_forward:
        tr = torch.empty(plan._traces_shape(), dtype=torch.float32, device=dev)
        plan.forward("k-rho", K0, r0, f, traces=tr)          # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(2):
            plan.forward("k-rho", K0, r0, f, traces=tr)
        torch.cuda.synchronize()
        tf = (time.perf_counter() - t) / 2
        b_fwd = 24 + 8 * ab["pml_fraction"] + 8 / S
        fwd_only = {"value": round(cells / tf / 1e9, 3), "ms_per_forward": round(tf * 1e3, 2),
                    "bytes_per_cell_step": round(b_fwd, 3),
                    "roof_gcells": round(PEAK_HBM_GBS / b_fwd, 1),
                    "frac_of_roof": round(cells / tf / 1e9 / (PEAK_HBM_GBS / b_fwd), 4)}
        del tr

    plain = None
    if not args.no_plain:
        print("bench: plain path (one shot per launch)", file=sys.stderr, flush=True)
        pp = api.Plan(grid, w.src_xz, w.rec_xz, mode="plain")
        pp.workspace(2)             # allocated outside the timed call
        torch.cuda.synchronize()
        t = time.perf_counter()
        Jp, gKp, grp = pp.gradient("k-rho", K0, r0, f, obs)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        rel = float((gKp - gK).abs().max() / gK.abs().max())
        plain = {"value": round(cells / tp / 1e9, 3), "ms_per_step": round(tp * 1e3, 2),
                 "speedup_batched_vs_plain": round(tp * 1e3 / ms, 3),
                 "grad_K_maxrel_vs_batched": rel}
        del pp

    served = None
    if args.serve_requests > 0:
        del plan
        torch.cuda.empty_cache()
        served = serve_leg(dev, value, args.serve_requests, args.serve_load)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, min(args.cpu_shots, w.nshots), args.cpu_steps or w.nt,
                           args.cpu_single_steps)

    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.nz}x{w.nx} at {w.dx:g} m + {w.npml} PML "
                               f"({info['Nz']}x{info['Nx']} padded), {w.nt} steps, "
                               f"{w.nshots} shots x {w.nrec} receivers, gradient in K-rho "
                               f"chain-ruled to Vp-rho, Ip-rho, Vp-Ip",
                   "cell_steps": cells, "band_rows": info["band_rows"],
                   "shots_per_group": info["shots_per_group"], "lane_cols": info["lane_cols"],
                   "shot_groups": G, "two_step": info["two_step"],
                   "two_step_band_rows": info["two_step_band_rows"],
                   "two_step_shots_per_group": info["two_step_shots_per_group"],
                   "two_step_lane_cols": info["two_step_lane_cols"],
                   "adj_two_step": info["adj_two_step"],
                   "adj_two_step_band_rows": info["adj_two_step_band_rows"],
                   "adj_two_step_lane_cols": info["adj_two_step_lane_cols"],
                   "decomposition": "autotuned" if tuned else "given" if any(
                       v for k, v in decomp.items() if k != "two_step") else "default",
                   "ckpt_every": info["ckpt_every"], "segments": info["segments"]},
        "step_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                            "p99": round(float(np.percentile(lat, 99)), 3),
                            "over": f"{args.steps} back-to-back gradient calls"},
        "roofline": roof,
        "roofline_by_kernel": roof_all,
        "kernels": classes,
        "checkpointed": ckpt,
        "forward_only": fwd_only,
        "plain": plain,
        "serve": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
