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


def roofline(k, kind, n_launch, ms_total, cfg):
    launches, model_bytes = k.kernel_model(kind)
    per_launch_bytes = model_bytes / launches
    t_launch = ms_total / n_launch * 1e-3
    achieved = per_launch_bytes / t_launch / 1e9
    name = k.kernel_name(kind)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(name, cfg), "kernel": name,
            "algorithmic_bytes_per_launch": per_launch_bytes, "launches_per_step": launches,
            "avg_launch_us": t_launch * 1e6, "launches_timed": n_launch, "timed_every": PROFILE_STRIDE}


def copy_calibration():
    """A plain copy of known size, for scaling the HBM counters of a profiled run."""
    import torch
    src = torch.empty(COPY_DOUBLES, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def cpu_baseline(nets, cfg, steps, batched=False):
    """The oracle timed on the host: numpy assembly, C LDL^T and solve per
    network and step (its symbolic analysis done once, untimed)."""
    import gridgen as G
    import oracle as O
    threads = min(os.cpu_count() or 1, 16)
    facs = []
    for i, net in enumerate(nets):
        z, s = G.draw_point(net, cfg, instance=i if batched else 0)
        cp, ri, v, pos = O.kkt(net, z, s)
        facs.append(O.Factor(pos.N, cp, ri, np.array(pos.block_off)))
    t0 = time.perf_counter()
    done = 0
    for it in range(steps):
        for i, net in enumerate(nets):
            z, s = G.draw_point(net, cfg, instance=i if batched else 0, iteration=it)
            cp, ri, v, pos = O.kkt(net, z, s)
            facs[i].factor(cp, ri, v, nthreads=threads)
            facs[i].solve(G.draw_rhs(pos.N, 1, cfg, iteration=it)[0])
            done += 1
    tc = time.perf_counter() - t0
    return done / tc, threads


def run_single(args):
    import torch
    import gridgen as G
    from paper_2510_13333_amd import KKT

    cfg = args.config
    net = G.config_network(cfg)
    t0 = time.perf_counter()
    k = KKT(net)
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

    def step(i=0, ev=None):
        z, s, b = states[i % nst]
        if ev is not None:
            ev[0].record()
        k.assemble(z, s, net.rho)
        if ev is not None:
            ev[1].record()
        k.factor_blocks()
        if ev is not None:
            ev[2].record()
        k.factor_border()
        if ev is not None:
            ev[3].record()
        k.solve(b, out=x)
        if ev is not None:
            ev[4].record()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    info = k.info()
    dom, per_kind = dominant_kernel(k, step)
    # timed region: wall clock over exactly `steps` steps; meanwhile every
    # PROFILE_STRIDE-th launch of the dominant kernel is bracketed by events
    # on its stream (a stride coprime with the launches per step samples
    # every level evenly and keeps the event records few)
    k.profile(dom)
    k.profile_stride(PROFILE_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_dom, ms_dom = k.profile_read()
    k.profile(-1)
    roof = roofline(k, dom, n_dom, ms_dom, cfg)
    print(f"[bench] timed {args.steps} steps: {wall / args.steps * 1e3:.3f} ms/step; dominant "
          f"{roof['kernel']} {roof['avg_launch_us']:.1f} us/launch x {roof['launches_per_step']} per step "
          f"({n_dom} launches sampled)", file=sys.stderr,
          flush=True)
    # phase timing with events (separate pass over the same steps)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    for i in range(args.steps):
        step(args.warmup + i, evs[i])
    torch.cuda.synchronize()
    ph = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(4)] for e in evs]).mean(axis=0) * 1e-3
    t_asm, t_fblk, t_fbrd, t_sol = (float(v) for v in ph)
    copy_calibration()

    eta = None
    if not args.no_check:
        import oracle as O
        etas = []
        for it in sorted({args.warmup % nst, (args.warmup + args.steps - 1) % nst}):
            z, s, b = states[it]
            k.assemble(z, s, net.rho)
            k.factor()
            xs = k.solve(b).cpu().numpy()
            cp, ri, v, _ = O.kkt(net, z.cpu().numpy(), s.cpu().numpy())
            etas.append(O.backward_error(cp, ri, v, xs, b.cpu().numpy()))
        eta = float(max(etas))
        print(f"[bench] backward error {eta:.2e}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu and args.cpu_steps > 0:
        rate, threads = cpu_baseline([net], cfg, args.cpu_steps)
        cpu = {"value": rate, "unit": "factor+solve/s", "cores": threads, "kind": "oracle",
               "sample": f"{args.cpu_steps} steps of the same workload (numpy assembly, C left-looking LDL^T "
                         f"with OpenMP over blocks, solve); symbolic analysis untimed"}

    from paper_2510_13333_amd.ncl import KERNELS
    nbd = sum(i["nbd"] for i in k.instances)
    step_bytes = sum(k.kernel_model(kind)[1] for kind in range(len(KERNELS)))
    out = {
        "metric": METRIC,
        "value": args.steps / wall,
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
        "config": {"workload": WORKLOADS[cfg], "step": f"assemble+factor+solve, nrhs={nrhs}", "N": k.N,
                   "nnzK_lower": k.nnzK, "nnzL": k.nnzL, "blocks": net.nblk, "border": nbd},
        "roofline": roof,
        "phases_ms": {"assemble": t_asm * 1e3, "factor_blocks": t_fblk * 1e3, "factor_border": t_fbrd * 1e3,
                      "solve": t_sol * 1e3},
        "factor_solve_per_s": 1.0 / (t_fblk + t_fbrd + t_sol),
        "kernel_ms_per_step": {k.kernel_name(kd): ms for kd, ms in sorted(per_kind.items(), key=lambda x: -x[1])},
        "step_algorithmic_GB": step_bytes / 1e9,
        "bwd_err_max": eta,
        "inertia": [info["npos"], info["nneg"], info["nzero"]],
        "status": info["status"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


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
          f"tiles={'autotuned' if table else 'default'}", file=sys.stderr, flush=True)

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
    roof = roofline(kb, dom, n_dom, ms_dom, cfg)
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
    copy_calibration()

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
        rate, threads = cpu_baseline(nets[:8], cfg, 1, batched=True)
        cpu = {"value": rate, "unit": "factor+solve/s", "cores": threads, "kind": "oracle",
               "sample": "the first 8 of the 64 networks, one factor+solve each (numpy assembly, C left-looking "
                         "LDL^T with OpenMP over blocks, solve); one factor+solve = one network"}

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
                   "N": kb.N, "nnzL": kb.nnzL, "networks": n, "tiles": "autotuned" if table else "default"},
        "roofline": roof,
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
    copy_f = max(max(v) for n, v in fe.items() if not n.startswith("k_"))
    copy_w = max(max(v) for n, v in wr.items() if not n.startswith("k_"))
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
    if args.config == 4:
        run_batched(args)
    else:
        run_single(args)


if __name__ == "__main__":
    main()
