#!/usr/bin/env python3
"""Benchmark of the KKT hot path on one MI355X.

A step is one pass of the whole path over one seeded state: assemble K
from the state, factor it (blocks, then the border), solve one right-hand
side.  Default workload: 500-bus grid x 256 branch-outage contingencies
with PV/PQ complementarity rows (N = 1,104,380), rho = 1e5, FP64, states
from a 50-step seeded trajectory, all resident in HBM before timing.
``--config 4`` runs the batched workload (64 uneven networks in one
handle) and reports it against the same networks factored one handle at
a time, and against a hipGraph replay of the batched step.

Prints one JSON line.  `value` is steps per second (assembly included, so
it is a lower bound of factor+solve/s).  The line carries the roofline of
the dominant kernel (its launches bracketed by HIP events on the launch
stream during the timed region; algorithmic bytes from the library's
per-kernel model), the per-phase times, the backward error of checked
solves and the CPU oracle timed on the host on a bounded sample.

``python bench.py --summarize-pmc FETCH_DIR WRITE_DIR --kernel NAME`` turns
two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script into the
per-dispatch HBM traffic summary under profiles/ that later runs report.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KKT factor+solve/s and HBM GB/s, 500-bus×256-cont, FP64 bwd err ≤1e-12"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    1: "single ACOPF KKT, 30-bus synthetic grid (N=214), rho=1e3, FP64",
    2: "500-bus synthetic grid x 16 branch-outage contingencies (N=59420), rho=1e4, FP64",
    3: "500-bus synthetic grid x 256 branch-outage contingencies with PV/PQ complementarity rows "
       "(N=1104380), rho=1e5, FP64",
    4: "64 uneven synthetic grids (118..2000 buses log-uniform, 4..32 branch-outage contingencies each) "
       "in one batched handle, rho=1e4, FP64",
    5: "2000-bus synthetic grid x 64 branch-outage contingencies (N=907760), rho=1e4, FP64",
    6: "contingency screening of the 500-bus grid's 256 branch-outage contingencies with PV/PQ rows, "
       "first-stage variables fixed: 256 independent blocks, no border (N=1100800), rho=1e5, FP64",
    7: "500-bus synthetic grid x 256 branch-outage contingencies with PV/PQ and AGC droop complementarity "
       "rows (N=1335036), rho=1e5, FP64",
    8: "contingency screening of the 500-bus grid's 256 branch-outage contingencies with PV/PQ and AGC droop "
       "rows, first-stage variables fixed: 256 independent blocks, no border (N=1331456), rho=1e5, FP64",
    9: "2000-bus synthetic grid x 64 branch-outage contingencies with AGC droop complementarity rows "
       "(N=1138224), rho=1e5, FP64",
}
COPY_DOUBLES = 64 * 2 ** 20          # the plain copy whose counters calibrate FETCH_SIZE / WRITE_SIZE
PROFILE_STRIDE = 7                   # one launch in 7 of the dominant kernel is event-timed in the timed region
KERNELS_SRC = os.path.join(ROOT, "paper_2510_13333_amd", "csrc", "kernels.hip")


def kernels_sha():
    with open(KERNELS_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_file(kernel, cfg):
    return os.path.join(ROOT, "profiles", f"{kernel}_c{cfg}_traffic.json")


def load_traffic(kernel, cfg):
    """HBM bytes per dispatch from the committed counter summary, or None
    when there is none or the kernels changed since it was taken."""
    p = traffic_file(kernel, cfg)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("kernels_sha") != kernels_sha():
        return None
    return t["traffic_bytes_per_dispatch"]


def dominant_kernel(k, step):
    """Profile each kernel kind over one step; the kind with the most time wins."""
    from paper_2510_13333_amd.ncl import KERNELS
    import torch
    per = {}
    for kind, name in enumerate(KERNELS):
        if name in ("values", "status_init"):
            continue
        k.profile(kind)
        step()
        torch.cuda.synchronize()
        n, ms = k.profile_read()
        if n:
            per[kind] = ms
    k.profile(-1)
    return max(per, key=per.get), per


PHASE_OF = {"interleave": "assemble", "assemble": "assemble", "sol_load": "solve", "sol_fwd_gather": "solve",
            "sol_fwd_diag": "solve",
            "sol_bpart": "solve", "sol_border": "solve", "sol_bwd_border": "solve", "sol_bwd": "solve",
            "sol_store": "solve",
            "berr_rows": "gate", "berr_border": "gate", "berr_final": "gate"}


def phase_of(kind):
    from paper_2510_13333_amd.ncl import KERNELS
    return PHASE_OF.get(KERNELS[kind], "factor")


def phase_bytes(k, nrhs):
    """Algorithmic HBM bytes per step of each phase, as the method must move
    them (every value read or written once; index arrays not counted):
    assembly writes K's lower triangle and reads the state z and Sigma;
    the factorisation reads K and writes L and D; a solve reads L twice
    (forward and backward), D once, and reads b and writes x per
    right-hand side."""
    return {"assemble": 8 * k.nnzK + 16 * k.N,
            "factor": 8 * (k.nnzK + k.nnzL + k.N),
            "solve": 16 * k.nnzL + 8 * k.N + 16 * k.N * nrhs}


def roofline(k, kind, n_launch, ms_total, pbytes):
    """Roofline of one kernel kind: its phase's algorithmic bytes per step
    spread over the kind's launches per step, over the mean event-timed
    launch; the library's own per-launch byte model beside it."""
    launches, model_bytes = k.kernel_model(kind)
    phase = phase_of(kind)
    per_launch_bytes = pbytes[phase] / launches
    t_launch = ms_total / n_launch * 1e-3
    achieved = per_launch_bytes / t_launch / 1e9
    name = k.kernel_name(kind)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(name, k.cfg), "kernel": name,
            "phase": phase, "algorithmic_bytes_per_launch": per_launch_bytes,
            "implementation_bytes_per_launch": model_bytes / launches, "launches_per_step": launches,
            "avg_launch_us": t_launch * 1e6, "launches_timed": n_launch, "timed_every": PROFILE_STRIDE}


def copy_peak(reps=10):
    """Bandwidth of the library's plain streaming copy over COPY_DOUBLES
    doubles (read + write), median of reps event-timed copies; its counters
    also calibrate FETCH_SIZE and WRITE_SIZE in the profiled runs."""
    import torch
    from paper_2510_13333_amd.ncl import stream_copy
    src = torch.ones(COPY_DOUBLES, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream_copy(src, dst)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        stream_copy(src, dst)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return 16.0 * COPY_DOUBLES / float(np.median(ts)) / 1e9


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = min(avail, int(omp)) if omp and omp.isdigit() and int(omp) > 0 else avail
    return model, os.cpu_count(), threads


def cpu_baseline(nets, cfg, steps, batched=False):
    """The oracle timed on the host: C left-looking LDL^T and solve of one
    right-hand side per network and step, single-threaded and with OpenMP
    over the blocks on every available core.  Its K values (numpy
    assembly) and symbolic analysis are prepared untimed, as the GPU's
    factor+solve rate excludes assembly too."""
    import gridgen as G
    import oracle as O
    model, ncpu, threads = cpu_info()
    work = []
    for it in range(steps):
        for i, net in enumerate(nets):
            z, s = G.draw_point(net, cfg, instance=i if batched else 0, iteration=it)
            cp, ri, v, pos = O.kkt(net, z, s)
            work.append((i, cp, ri, v, G.draw_rhs(pos.N, 1, cfg, iteration=it)[0], np.array(pos.block_off)))
    facs = {}
    for i, cp, ri, v, b, boff in work:
        if i not in facs:
            facs[i] = O.Factor(len(b), cp, ri, boff)
    rates = {}
    for nt in (1, threads):
        if nt in rates:
            continue
        t0 = time.perf_counter()
        for i, cp, ri, v, b, _ in work:
            facs[i].factor(cp, ri, v, nthreads=nt)
            facs[i].solve(b)
        rates[nt] = len(work) / (time.perf_counter() - t0)
    return rates, threads, model, ncpu


def run_single(args):
    import torch
    import gridgen as G
    from paper_2510_13333_amd import KKT

    cfg = args.config
    net = G.config_network(cfg)
    t0 = time.perf_counter()
    k = KKT(net)
    k.cfg = cfg
    t_analyze = time.perf_counter() - t0
    nrhs = args.nrhs
    k.bind(nrhs_max=nrhs)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    nst = max(1, min(args.states, args.steps + args.warmup))
    z0, s0 = G.draw_point(net, cfg)
    states = []
    for it in range(nst):
        z, s = G.draw_trajectory_point(net, cfg, it, z0, s0)
        b = G.draw_rhs(k.N, nrhs, cfg, iteration=it)
        b = b[0] if nrhs == 1 else b
        states.append((dev(z), dev(s), dev(b)))
    x = torch.empty((k.N,) if nrhs == 1 else (nrhs, k.N), dtype=torch.float64, device="cuda")
    print(f"[bench] config {cfg}: N={k.N} nnzK={k.nnzK} nnzL={k.nnzL} supernodes={k.nsuper} "
          f"analyze={t_analyze:.3f}s states={nst}", file=sys.stderr, flush=True)

    # gate[i] = (eta, omega) of each right-hand side of step i, computed on
    # the device after the solve (no host synchronisation in the loop)
    gate = torch.full((args.steps, nrhs, 2), float("nan"), dtype=torch.float64, device="cuda")

    def step(i=0, ev=None, g=None):
        z, s, b = states[i % nst]
        if ev is not None:
            ev[0].record()
        k.assemble(z, s, net.rho)
        if ev is not None:
            ev[1].record()
        k.factor_solve(b, out=x)
        if ev is not None:
            ev[2].record()
        if g is not None:
            k.backward_error(b, x, out=g)
            if ev is not None:
                ev[3].record()

    def step_split(i, ev):
        """The same step with the factorisation and the solve as two calls
        (no overlap), for the per-phase times."""
        z, s, b = states[i % nst]
        k.assemble(z, s, net.rho)
        ev[0].record()
        k.factor_blocks()
        k.factor_border()
        ev[1].record()
        k.solve(b, out=x)
        ev[2].record()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    dom, per_kind = dominant_kernel(k, step)
    # timed region: wall clock over exactly `steps` steps, each bracketed
    # per phase by events and checked by the device's backward-error gate;
    # meanwhile every PROFILE_STRIDE-th launch of the dominant kernel is
    # bracketed by events on its stream (a stride coprime with the launches
    # per step samples every level evenly)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    k.profile(dom)
    k.profile_stride(PROFILE_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i, evs[i], gate[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_dom, ms_dom = k.profile_read()
    k.profile(-1)
    info = k.info()
    ph = np.array([[e[j].elapsed_time(e[j + 1]) * 1e-3 for j in range(3)] for e in evs])
    t_asm, t_fs, t_gate = (np.median(ph[:, j]) for j in range(3))
    # the factorisation and the solve as separate calls, for the phase table
    nsplit = min(args.steps, 20)
    evs2 = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(nsplit)]
    for i in range(nsplit):
        step_split(args.warmup + i, evs2[i])
    torch.cuda.synchronize()
    ph2 = np.array([[e[j].elapsed_time(e[j + 1]) * 1e-3 for j in range(2)] for e in evs2])
    t_fac, t_sol = np.median(ph2[:, 0]), np.median(ph2[:, 1])
    g = gate.cpu().numpy()
    eta_max, omega_max = float(np.max(g[..., 0])), float(np.max(g[..., 1]))
    passed = int(np.sum(np.all(g[..., 0] <= 1e-12, axis=1)))
    pb = phase_bytes(k, nrhs)
    roof = roofline(k, dom, n_dom, ms_dom, pb)
    print(f"[bench] timed {args.steps} steps: {wall / args.steps * 1e3:.3f} ms/step wall; factor+solve median "
          f"{t_fs * 1e3:.3f} ms (as two calls: {(t_fac + t_sol) * 1e3:.3f} ms); gate eta<=1e-12 on {passed}/"
          f"{args.steps} (max eta {eta_max:.2e}, omega {omega_max:.2e}); dominant {roof['kernel']} "
          f"{roof['avg_launch_us']:.1f} us/launch x {roof['launches_per_step']}", file=sys.stderr, flush=True)

    # one refinement step on the last state: its cost and the componentwise error after it
    z, s, b = states[(args.warmup + args.steps - 1) % nst]
    step(args.warmup + args.steps - 1)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record()
    k.refine(b, x)
    e[1].record()
    gr = k.backward_error(b, x).cpu().numpy()
    t_ref = e[0].elapsed_time(e[1]) * 1e-3

    peak_copy = copy_peak()
    phases = {}
    for name, t in (("assemble", t_asm), ("factor", t_fac), ("solve", t_sol)):
        gbs = pb[name] / t / 1e9
        phases[name] = {"ms": t * 1e3, "algorithmic_MB": pb[name] / 1e6, "GBs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS,
                        "frac_copy": gbs / peak_copy}

    eta_or = None
    if not args.no_check:
        import oracle as O
        etas = []
        picks = sorted({args.warmup % nst, (args.warmup + args.steps // 2) % nst, (args.warmup + args.steps - 1) % nst})
        for it in picks:
            z, s, b = states[it]
            step(it)
            xs = x.cpu().numpy()
            cp, ri, v, _ = O.kkt(net, z.cpu().numpy(), s.cpu().numpy())
            etas.append(O.backward_error(cp, ri, v, xs, b.cpu().numpy()))
        eta_or = float(max(etas))
        print(f"[bench] oracle-assembled backward error on states {picks}: {eta_or:.2e}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu and args.cpu_steps > 0:
        rates, threads, model, ncpu = cpu_baseline([net], cfg, args.cpu_steps)
        cpu = {"value": rates[threads], "unit": "factor+solve/s", "cores": threads, "kind": "oracle",
               "single_thread_value": rates[1], "cpu_model": model, "os_cpu_count": ncpu,
               "sample": f"{args.cpu_steps} states of the same workload, one factor+solve (nrhs=1) each, "
                         f"C left-looking LDL^T with OpenMP over the blocks on {threads} threads, and again on "
                         f"1 thread; K assembled by numpy and the symbolic analysis done beforehand, untimed"}

    ipm = None
    if not args.no_ipm and not getattr(net, "screen", False):
        ipm = ipm_steps(k, net, cfg, args.ipm_steps)
        print(f"[bench] IPM step: {ipm['ms_median']:.3f} ms median over {ipm['steps']} points, "
              f"{ipm['factorizations_mean']:.1f} factorisations each", file=sys.stderr, flush=True)

    ncl = None
    if not args.no_ncl and args.gpus == 1:
        ncl = ncl_solve_run(args.ncl_config, args.ncl_load_scale)
        print(f"[bench] NCL solve: {ncl['s']:.3f} s, status {ncl['status']}, {ncl['outer']} outer / {ncl['inner']} "
              f"inner iterations, {ncl['factorizations']} factorisations", file=sys.stderr, flush=True)
        if not args.no_cpu:
            ncl["cpu_oracle"] = ncl_oracle_beside(args.ncl_load_scale)
            co = ncl["cpu_oracle"]
            print(f"[bench] NCL solve, 500-bus x 4: oracle {co['oracle_s']:.1f} s ({co['oracle_inner']} inner), "
                  f"library {co['gpu_s']:.3f} s ({co['gpu_inner']} inner)", file=sys.stderr, flush=True)
        sc = ncl.get("screening")
        if sc:
            print(f"[bench] screening at that first stage: {sc['s']:.3f} s ({sc['ms_per_contingency']:.3f} ms per "
                  f"contingency), status {sc['status']}, {sc['outer']} outer / {sc['inner']} inner iterations",
                  file=sys.stderr, flush=True)

    disp = None
    if cfg == 5 and not args.no_dispatch:
        disp = dispatch_backward(net, args.steps)
        print(f"[bench] dispatch map: forward {disp['forward_s']:.2f} s ({disp['newton_steps']} Newton steps), "
              f"backward {disp['backward_ms']:.3f} ms", file=sys.stderr, flush=True)

    from paper_2510_13333_amd.ncl import KERNELS
    nbd = sum(i["nbd"] for i in k.instances)
    step_bytes = sum(k.kernel_model(kind)[1] for kind in range(len(KERNELS)))
    out = {
        "metric": METRIC,
        "value": 1.0 / t_fs,
        "unit": "factor+solve/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[cfg], "value": "1 / median over the timed steps of the event time of "
                   "ncl_kkt_factor_solve (factor and solve in one call, the border's factorisation overlapped with "
                   "the blocks' forward substitution); ms_per_step is the wall clock of the whole step (assembly "
                   "and the gate included); phases.factor / phases.solve time the two as separate calls",
                   "step": f"assemble+factor_solve+gate, nrhs={nrhs}", "N": k.N, "nnzK_lower": k.nnzK,
                   "nnzL": k.nnzL, "blocks": net.nblk, "border": nbd},
        "roofline": roof,
        "phases": phases,
        "factor_solve_ms": t_fs * 1e3,
        "factor_plus_solve_separate_ms": (t_fac + t_sol) * 1e3,
        "copy_peak_GBs": peak_copy,
        "gate_ms": t_gate * 1e3,
        "steps_per_s_wall": args.steps / wall,
        "kernel_ms_per_step": {k.kernel_name(kd): ms for kd, ms in sorted(per_kind.items(), key=lambda x: -x[1])},
        "implementation_GB_per_step": step_bytes / 1e9,
        "gate": {"eta_max": eta_max, "omega_max": omega_max, "steps_eta_le_1e-12": passed,
                 "refine_ms": t_ref * 1e3, "eta_after_refine": float(gr[..., 0].max()),
                 "omega_after_refine": float(gr[..., 1].max())},
        "bwd_err_oracle_assembled": eta_or,
        "inertia": [info["npos"], info["nneg"], info["nzero"]],
        "status": info["status"],
        "cpu_baseline": cpu,
    }
    if disp is not None:
        out["dispatch_map"] = disp
    if ipm is not None:
        out["ipm_step"] = ipm
    if ncl is not None:
        out["ncl_solve"] = ncl
    print(json.dumps(out), flush=True)


def ipm_steps(k, net, cfg, steps):
    """The IPM step of the NCL subproblem on this network (ncl_kkt_ipm_step:
    sigma, the inertia-corrected factorisation, the right-hand side, one
    solve and the recovery) at `steps` seeded interior points, each shift
    warm-started from the previous point's as an IPM run does; wall clock
    per step (the inertia loop reads each factorisation's report)."""
    import torch
    import gridgen as G
    from paper_2510_13333_amd.ncl import InertiaOpts
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda")
    N = k.N
    pts = []
    for it in range(steps + 1):
        d, pd = G.draw_ipm_point(net, cfg, iteration=it)
        prob = dict(pd=dev(pd), lo=dev(d["lo"]), hi=dev(d["hi"]), y_n=dev(d["y_n"]), qd_ratio=0.3, qmax=3.0, pmax=8.0,
                    smax2=100.0, eps=1.0, mu=0.1, rho=net.rho)
        pts.append((prob, {n: dev(d[n]) for n in ("z", "rt", "s", "zl", "zu")}))
    dirs = {n: torch.empty(N, dtype=torch.float64, device="cuda") for n in ("dz", "drt", "ds", "dzl", "dzu")}
    work = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    opts = InertiaOpts(0.0, 0, 0)
    k.ipm_step(*pts[0], dirs, opts, work)          # warm-up
    torch.cuda.synchronize()
    ts, nf, dws = [], [], []
    for prob, st in pts[1:]:
        t0 = time.perf_counter()
        k.ipm_step(prob, st, dirs, opts, work)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        nf.append(opts.nfactor)
        dws.append(opts.dw_last)
    ms = np.array(ts) * 1e3
    return {"what": "one Newton direction of the NCL subproblem's IPM at seeded interior points: sigma, "
                    "inertia-corrected assemble+factor (shift sequence warm-started from the previous point), "
                    "right-hand side from the KKT residuals, one solve, recovery of the eliminated directions",
            "steps": steps, "ms_median": float(np.median(ms)), "ms_min": float(ms.min()),
            "factorizations_mean": float(np.mean(nf)), "factorizations": nf,
            "ms_per_factorization": float(np.median(ms / np.array(nf))), "shifts": dws}


NCL_LOAD_SCALE = 0.1     # the NCL workload's loads: this fraction of the seeded pd


def ncl_solve_run(cfg, load_scale=NCL_LOAD_SCALE):
    """The NCL method end to end (ncl_kkt_ncl_solve) on config cfg's network
    (by default the 500-bus x 256 grid with PV/PQ and AGC droop rows): from
    the fixed interior start, loads load_scale x the seeded pd, the
    network's rho as the first penalty, tolerance 1e-6 and smallest barrier
    parameter 1e-7 (Section V); wall clock of the whole solve, the analysis
    before it untimed.  One warm-up solve of the same problem first."""
    import torch
    import gridgen as G
    from paper_2510_13333_amd import KKT
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda")
    net = G.config_network(cfg)
    t0 = time.perf_counter()
    k = KKT(net).bind(nrhs_max=1)
    t_an = time.perf_counter() - t0
    st0 = G.ncl_start(net)
    pd = load_scale * G.draw_loads(net, cfg)
    prob = dict(pd=dev(pd), lo=dev(st0["lo"]), hi=dev(st0["hi"]), qd_ratio=0.3, qmax=3.0, pmax=8.0, smax2=100.0,
                eps=1.0, rho=net.rho)
    work = torch.empty(17 * k.N + 64, dtype=torch.float64, device="cuda")

    def run():
        state = {n: dev(st0[n]) for n in ("z", "rt", "s", "zl", "zu")}
        state["y_n"] = torch.zeros(k.N, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t = time.perf_counter()
        rep = k.ncl_solve(prob, state, work=work)
        torch.cuda.synchronize()
        return rep, time.perf_counter() - t, state

    run()
    rep, t, state = run()
    screen = ncl_screen_run(net, cfg, pd, state) if cfg == 7 else None
    return {"what": "the NCL method end to end (outer multiplier / penalty updates around the subproblem's "
                    "primal-dual IPM, every step on the GPU) on " + WORKLOADS[cfg] + f", loads {load_scale} x "
                    "the seeded pd, from the fixed interior start; tol 1e-6, smallest mu 1e-7",
            "N": k.N, "s": t, "status": rep["status"], "outer": rep["outer"], "inner": rep["inner"],
            "factorizations": rep["factorizations"], "ms_per_inner": 1e3 * t / max(1, rep["inner"]),
            "rho": rep["rho"], "r_inf": rep["r_inf"], "kkt_err": rep["kkt_err"], "analyze_s": t_an,
            "screening": screen}


def ncl_sweep(ks, load_scale=NCL_LOAD_SCALE):
    """The NCL solve as the number of contingencies K grows (the shape of
    Table II): the 500-bus grid with PV/PQ and AGC rows and K outages (the
    grid and loads of config 3's seed; each K draws its own outage set),
    from the fixed start, one warm-up and one timed solve each."""
    import torch
    import gridgen as G
    from paper_2510_13333_amd import KKT
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda")
    rows = []
    for K in ks:
        net = G.make_network(3, 500, 700, 90, K, pvpq=True, rho=1e5, agc=True)
        k = KKT(net).bind(nrhs_max=1)
        st0 = G.ncl_start(net)
        pd = load_scale * G.draw_loads(net, 3)
        prob = dict(pd=dev(pd), lo=dev(st0["lo"]), hi=dev(st0["hi"]), qd_ratio=0.3, qmax=3.0, pmax=8.0,
                    smax2=100.0, eps=1.0, rho=net.rho)
        work = torch.empty(17 * k.N + 64, dtype=torch.float64, device="cuda")
        for timed in (False, True):
            st = {n: dev(st0[n]) for n in ("z", "rt", "s", "zl", "zu")}
            st["y_n"] = torch.zeros(k.N, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t = time.perf_counter()
            rep = k.ncl_solve(prob, st, work=work)
            torch.cuda.synchronize()
            t = time.perf_counter() - t
        row = {"K": K, "N": k.N, "s": t, "status": rep["status"], "outer": rep["outer"], "inner": rep["inner"],
               "factorizations": rep["factorizations"], "ms_per_inner": 1e3 * t / max(1, rep["inner"])}
        rows.append(row)
        print(f"[bench] NCL sweep K={K}: N={k.N} {t:.3f} s, status {rep['status']}, {rep['outer']} outer / "
              f"{rep['inner']} inner, {rep['factorizations']} factorisations", file=sys.stderr, flush=True)
        del k, work
    return rows


def ncl_oracle_beside(load_scale=NCL_LOAD_SCALE):
    """The oracle's NCL solve (oracle/ncl.py, numpy with the C LDL^T on one
    thread) timed beside the library's on one bounded instance: the 500-bus
    grid with PV/PQ and AGC rows and 4 contingencies (N = 24384), the same
    start, loads and options.  Both solves and their iteration counts."""
    import torch
    import gridgen as G
    from oracle import ipm as OI
    from oracle import ncl as ON
    from paper_2510_13333_amd import KKT
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda")
    net = G.make_network(3, 500, 700, 90, 4, pvpq=True, rho=1e5, agc=True)
    st0 = G.ncl_start(net)
    pd = load_scale * G.draw_loads(net, 3)
    N = st0["z"].shape[0]
    prob = OI.Problem(pd=pd, lo=st0["lo"], hi=st0["hi"], y_n=np.zeros(N), mu=0.1, rho=net.rho)
    t = time.perf_counter()
    _, _, rep_o = ON.solve(net, prob, OI.State(st0["z"], st0["rt"], st0["s"], st0["zl"], st0["zu"]))
    t_o = time.perf_counter() - t
    k = KKT(net).bind(nrhs_max=1)
    gprob = dict(pd=dev(pd), lo=dev(st0["lo"]), hi=dev(st0["hi"]), qd_ratio=0.3, qmax=3.0, pmax=8.0, smax2=100.0,
                 eps=1.0, rho=net.rho)
    work = torch.empty(17 * k.N + 64, dtype=torch.float64, device="cuda")
    for _ in range(2):
        st = {n: dev(st0[n]) for n in ("z", "rt", "s", "zl", "zu")}
        st["y_n"] = torch.zeros(k.N, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t = time.perf_counter()
        rep = k.ncl_solve(gprob, st, work=work)
        torch.cuda.synchronize()
        t_g = time.perf_counter() - t
    return {"what": "the oracle's NCL solve (numpy, C LDL^T on 1 thread) beside the library's on the 500-bus grid "
                    "with PV/PQ and AGC rows and 4 contingencies, the same start, loads and options",
            "N": N, "oracle_s": t_o, "oracle_outer": rep_o.outer, "oracle_inner": rep_o.inner, "gpu_s": t_g,
            "gpu_outer": rep["outer"], "gpu_inner": rep["inner"], "cores": 1}


def ncl_screen_run(net, cfg, pd, state):
    """Contingency screening (eq. (screening)) at the first stage of the NCL
    solution just computed: the same grid's 256 contingencies with the
    first-stage pg and vm0 fixed at that solution, their feasibility
    problems solved together by one NCL solve (no border); wall clock, and
    per contingency."""
    import torch
    import gridgen as G
    from paper_2510_13333_amd import KKT
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda")
    kind, _, block, _ = G.layout(net)
    z = state["z"].cpu().numpy()
    pg0 = z[(kind == G.PG) & (block < 0)]
    vm0 = z[kind == G.VM0]
    scr = G.config_network(8)
    k = KKT(scr).bind(nrhs_max=1)
    st0 = G.ncl_start(scr)
    prob = dict(pd=dev(pd), lo=dev(st0["lo"]), hi=dev(st0["hi"]), qd_ratio=0.3, qmax=3.0, pmax=8.0, smax2=100.0,
                eps=1.0, rho=scr.rho, pg0=dev(pg0), vm0=dev(vm0))
    work = torch.empty(17 * k.N + 64, dtype=torch.float64, device="cuda")

    def run():
        st = {n: dev(st0[n]) for n in ("z", "rt", "s", "zl", "zu")}
        st["y_n"] = torch.zeros(k.N, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t = time.perf_counter()
        rep = k.ncl_solve(prob, st, work=work)
        torch.cuda.synchronize()
        return rep, time.perf_counter() - t

    run()
    rep, t = run()
    return {"what": "screening of the same grid's " + str(scr.ncont) + " contingencies at the solution's first "
                    "stage: one NCL solve over the contingencies' feasibility problems (" + WORKLOADS[8] + ")",
            "N": k.N, "s": t, "ms_per_contingency": 1e3 * t / scr.ncont, "status": rep["status"],
            "outer": rep["outer"], "inner": rep["inner"], "factorizations": rep["factorizations"],
            "r_inf": rep["r_inf"], "kkt_err": rep["kkt_err"]}


def dispatch_backward(net, steps):
    """The differentiable dispatch map on this network: one forward pass
    (the library's Newton solve, untimed beyond its wall clock) and the
    backward pass (adjoint right-hand side, one adjoint solve on the stored
    factors, reduction to the loads) timed by events, median of `steps`."""
    import torch
    import gridgen as G
    from paper_2510_13333_amd.dispatch import DispatchSolver
    pd = torch.from_numpy(G.draw_loads(net, 5)).to("cuda")
    s = DispatchSolver(net)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z = s.newton(pd)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    s._pd_of = (pd,)
    gphi = torch.ones((), dtype=torch.float64, device="cuda")
    s.vjp(z, gphi, None)
    ts = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.vjp(z, gphi, None)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return {"what": "d phi*/d pd for the 2000 bus loads: adjoint right-hand side, one adjoint KKT solve on the "
                    "factors of the converged forward pass, reduction over the blocks' balance rows",
            "newton_steps": s.iterations, "forward_s": t_fwd, "backward_ms": float(np.median(ts))}


def run_batched(args):
    """64 uneven networks: one batched handle (eager, and its step replayed
    from a hipGraph) against one handle per network run back to back."""
    import torch
    import gridgen as G
    from paper_2510_13333_amd import KKT
    from paper_2510_13333_amd import autotune

    cfg = 4
    nets = G.batched_networks(64)
    table = autotune.load_table()
    relax = [autotune.relax_for(table, n) for n in nets] if table else None
    t0 = time.perf_counter()
    kb = KKT(nets=nets, relax=relax)
    t_analyze = time.perf_counter() - t0
    kb.bind(nrhs_max=1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    zs, ss = [], []
    for i, n in enumerate(nets):
        z, s = G.draw_point(n, cfg, instance=i)
        zs.append(z)
        ss.append(s)
    z = dev(np.concatenate(zs))
    s = dev(np.concatenate(ss))
    b = dev(G.draw_rhs(kb.N, 1, cfg)[0])
    x = torch.empty_like(b)
    rho = nets[0].rho
    print(f"[bench] batched: {len(nets)} networks N={kb.N} nnzL={kb.nnzL} analyze={t_analyze:.2f}s "
          f"amalgamation={sorted(set(relax)) if relax else 'default'}", file=sys.stderr, flush=True)

    def step():
        kb.assemble(z, s, rho)
        kb.factor()
        kb.solve(b, out=x)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    info = kb.info()
    dom, per_kind = dominant_kernel(kb, step)
    kb.profile(dom)
    kb.profile_stride(PROFILE_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_dom, ms_dom = kb.profile_read()
    kb.profile(-1)
    kb.cfg = cfg
    roof = roofline(kb, dom, n_dom, ms_dom, phase_bytes(kb, 1))
    x_eager = x.clone()

    # the same step captured once in a hipGraph and replayed
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    g.replay()
    torch.cuda.synchronize()
    graph_ok = bool(torch.equal(x, x_eager))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t0
    graph_ok = graph_ok and bool(torch.equal(x, x_eager))

    # unbatched: one handle per network, run back to back on the same stream
    singles = []
    for i, n in enumerate(nets):
        k1 = KKT(n, relax=relax[i] if relax else None).bind(nrhs_max=1)
        I = kb.instances[i]
        singles.append((k1, z[I["col0"]:I["col0"] + I["N"]].contiguous(), s[I["col0"]:I["col0"] + I["N"]].contiguous(),
                        b[I["col0"]:I["col0"] + I["N"]].contiguous(), torch.empty(I["N"], dtype=torch.float64,
                                                                                   device="cuda")))

    def step_single():
        for k1, z1, s1, b1, x1 in singles:
            k1.assemble(z1, s1, rho)
            k1.factor()
            k1.solve(b1, out=x1)

    step_single()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_single()
    torch.cuda.synchronize()
    wall_single = time.perf_counter() - t0
    same = all(torch.equal(x1, x_eager[kb.instances[i]["col0"]:kb.instances[i]["col0"] + kb.instances[i]["N"]])
               for i, (_, _, _, _, x1) in enumerate(singles))
    peak_copy = copy_peak()

    eta = None
    if not args.no_check:
        import oracle as O
        xs = x_eager.cpu().numpy()
        bs = b.cpu().numpy()
        etas = []
        for i, n in enumerate(nets[:8]):
            I = kb.instances[i]
            sl = slice(I["col0"], I["col0"] + I["N"])
            cp, ri, v, _ = O.kkt(n, zs[i], ss[i])
            etas.append(O.backward_error(cp, ri, v, xs[sl], bs[sl]))
        eta = float(max(etas))

    cpu = None
    if not args.no_cpu and args.cpu_steps > 0:
        rates, threads, model, ncpu = cpu_baseline(nets[:8], cfg, 1, batched=True)
        cpu = {"value": rates[threads], "unit": "factor+solve/s", "cores": threads, "kind": "oracle",
               "single_thread_value": rates[1], "cpu_model": model, "os_cpu_count": ncpu,
               "sample": "the first 8 of the 64 networks, one factor+solve each (C left-looking LDL^T with OpenMP "
                         "over blocks, and on 1 thread; K assembled by numpy beforehand, untimed); one "
                         "factor+solve = one network"}

    n = len(nets)
    out = {
        "metric": METRIC,
        "value": n * args.steps / wall,
        "unit": "factor+solve/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[cfg], "step": "assemble+factor+solve of all 64 networks, nrhs=1",
                   "N": kb.N, "nnzL": kb.nnzL, "networks": n,
                   "amalgamation": ("per size class from the tuner's table: " + ", ".join(
                       "/".join(map(str, r)) for r in sorted(set(relax)))) if relax else "default 16/1/4"},
        "roofline": roof,
        "copy_peak_GBs": peak_copy,
        "batched_graph_per_s": n * args.steps / wall_graph,
        "unbatched_per_s": n * args.steps / wall_single,
        "batched_over_unbatched": wall_single / wall,
        "graph_replay_bitwise_equal": graph_ok,
        "batched_equals_unbatched_bitwise": bool(same),
        "kernel_ms_per_step": {kb.kernel_name(kd): ms for kd, ms in sorted(per_kind.items(), key=lambda x: -x[1])},
        "bwd_err_max": eta,
        "inertia": [info["npos"], info["nneg"], info["nzero"]],
        "status": info["status"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def summarize_pmc(fetch_dir, write_dir, kernel, cfg):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE of `kernel`, scaled by the same
    counters of the plain copy (COPY_DOUBLES doubles read and written)."""
    def per_kernel(d, counter):
        vals = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    if row.get("Counter_Name") != counter:
                        continue
                    name = row["Kernel_Name"].split("(")[0].replace("ncl::", "")
                    vals.setdefault(name, []).append(float(row["Counter_Value"]))
        return vals
    fe, wr = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    copy_bytes = 8 * COPY_DOUBLES
    copy_f = max(fe["k_copy"])
    copy_w = max(wr["k_copy"])
    sf, sw = copy_bytes / (copy_f * 1024), copy_bytes / (copy_w * 1024)
    f_kib, w_kib = float(np.mean(fe[kernel])), float(np.mean(wr[kernel]))
    res = {"kernel": kernel, "workload": WORKLOADS[cfg], "kernels_sha": kernels_sha(),
           "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib, "dispatches": len(fe[kernel]),
           "copy_fetch_kib": copy_f, "copy_write_kib": copy_w, "copy_bytes_each_way": copy_bytes,
           "scale_fetch": sf, "scale_write": sw,
           "traffic_bytes_per_dispatch": f_kib * 1024 * sf + w_kib * 1024 * sw}
    with open(traffic_file(kernel, cfg), "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3, choices=sorted(WORKLOADS))
    ap.add_argument("--states", type=int, default=50, help="distinct trajectory states, cycled")
    ap.add_argument("--nrhs", type=int, default=1, help="right-hand sides per solve (single-network workloads)")
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle steps timed on the host")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-dispatch", action="store_true", help="skip the dispatch-map backward timing (config 5)")
    ap.add_argument("--no-ipm", action="store_true", help="skip the IPM-step timing")
    ap.add_argument("--no-ncl", action="store_true", help="skip the NCL-solve timing")
    ap.add_argument("--ncl-config", type=int, default=7, help="network of the NCL-solve timing")
    ap.add_argument("--ncl-sweep", default=None,
                    help="comma-separated contingency counts: time the NCL solve on the 500-bus grid with PV/PQ "
                         "and AGC rows at each, and report only that")
    ap.add_argument("--ncl-load-scale", type=float, default=NCL_LOAD_SCALE,
                    help="the NCL workload's loads as a fraction of the seeded pd")
    ap.add_argument("--ipm-steps", type=int, default=5, help="interior points of the IPM-step timing")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--kernel", default=None)
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.kernel, args.config)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is documented, "
              "not built", file=sys.stderr)
        sys.exit(2)
    if args.ncl_sweep:
        ks = [int(x) for x in args.ncl_sweep.split(",")]
        print(json.dumps({"what": "NCL solve against the number of contingencies (the shape of Table II): the "
                                  "500-bus synthetic grid with PV/PQ and AGC rows, loads "
                                  f"{args.ncl_load_scale} x the seeded pd, tol 1e-6",
                          "rows": ncl_sweep(ks, args.ncl_load_scale)}))
    elif args.config == 4:
        run_batched(args)
    else:
        run_single(args)


if __name__ == "__main__":
    main()
