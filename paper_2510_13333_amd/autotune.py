"""Supernode tile autotuner for the batched path.

The tile shape of the supernodal factorisation is set by the relaxed
amalgamation parameters (widest merged supernode, admitted explicit-zero
fraction): wider supernodes mean fewer levels and launches but more padded
work per row.  The best choice depends on the network's size, so the
tuner groups networks into shape classes (rounded log2 of the bus count)
and, per class, times assemble+factor+solve of representative networks
for each candidate on the GPU, keeping the fastest.  The result is a small
JSON table (class -> (maxw, znum, zden)) that the batched handle applies
per instance; the parameters are ordinary analysis options, so the CPU
oracle's symbolic analysis reproduces any of them exactly.

    python -m paper_2510_13333_amd.autotune [--out FILE]   (needs a GPU)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles_mi355x.json")
CANDIDATES = [(4, 1, 4), (8, 1, 4), (16, 1, 4), (32, 1, 4), (16, 1, 2), (32, 1, 2)]
DEFAULT = (16, 1, 4)


def shape_class(net) -> int:
    return int(round(math.log2(max(int(net.nb), 2))))


def load_table(path: str = TABLE):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def relax_for(table, net):
    if not table:
        return DEFAULT
    return tuple(table["classes"].get(str(shape_class(net)), table.get("default", DEFAULT)))


def time_network(net, relax, cfg, instance, reps=5):
    """Median event time (ms) of assemble+factor+solve of one network."""
    import numpy as np
    import torch
    import gridgen as G
    from paper_2510_13333_amd import KKT
    k = KKT(net, relax=relax).bind(nrhs_max=1)
    z, s = G.draw_point(net, cfg, instance=instance)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    z, s, b = dev(z), dev(s), dev(G.draw_rhs(k.N, 1, cfg)[0])
    x = torch.empty_like(b)

    def step():
        k.assemble(z, s, net.rho)
        k.factor()
        k.solve(b, out=x)

    step()
    torch.cuda.synchronize()
    if k.info()["status"] != 0:
        return math.inf
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune(nets, cfg=4, per_class=3, reps=5, log=print):
    classes = {}
    for i, n in enumerate(nets):
        classes.setdefault(shape_class(n), []).append(i)
    table = {"default": list(DEFAULT), "classes": {}, "timings_ms": {}, "candidates": [list(c) for c in CANDIDATES]}
    for c, idx in sorted(classes.items()):
        sample = idx[:per_class]
        best, best_t = DEFAULT, math.inf
        times = {}
        for cand in CANDIDATES:
            t = sum(time_network(nets[i], cand, cfg, i, reps) for i in sample)
            times[str(list(cand))] = t
            if t < best_t:
                best, best_t = cand, t
        table["classes"][str(c)] = list(best)
        table["timings_ms"][str(c)] = times
        log(f"[autotune] class 2^{c} buses ({len(idx)} networks, {len(sample)} timed): best {best} "
            f"{best_t:.3f} ms")
    return table


def main():
    import gridgen as G
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    t0 = time.perf_counter()
    table = tune(G.batched_networks(64), reps=args.reps)
    table["tuned_on"] = "MI355X (gfx950)"
    table["seconds"] = time.perf_counter() - t0
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(table["classes"]))


if __name__ == "__main__":
    main()
