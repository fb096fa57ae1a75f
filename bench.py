#!/usr/bin/env python
"""Faces meshed per second by analytic marching on one MI355X.

One step is one pass of the whole hot path over one shape: dichotomy seeding
of 1,024 rays, marching every reachable analytic cell (chain, clip, vertex
solves, neighbour flips, hash deduplication) and emitting the CSR mesh.  The
network weights and the rays are resident in HBM before the timed region.

Workload (default): a 3->[90]x6->1 ReLU MLP fitted to the signed distance of
a union of 8 random spheres (frozen fixture am_workloads/data/c2.npz), seeded
by 128 Fibonacci directions from each sphere centre; it stands in for the
paper's D6-W60 ShapeNet fits (Table 4).

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (durations from HIP events on the library's stream) and the CPU
oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "faces meshed/sec on 1 MI355X (plain vs learned+BF16 form); exact cell-set match"
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def workload(name: str):
    from am_workloads import nets, seeds
    if name == "c2":
        net = nets.load_fitted("c2")
        prim = np.load(os.path.join(nets.DATA_DIR, "c2_primitives.npz"))
        o, d = seeds.centre_rays(prim["p0"], 128)
        desc = ("C2 plain FP64: 3->[90]x6->1 ReLU SDF fit of 8 random spheres (FP32 weights, FP64 geometry), "
                "1024 dichotomy rays")
        return net, o, d, desc
    if name == "c1":
        net = nets.c1_net()
        o, d = seeds.axis_ray()
        return net, o, d, "C1 plain FP64: 0.1*MLP(3->64->64->1)+max-norm-0.5, one ray along +x"
    raise SystemExit(f"unknown workload {name}")


def chain_flops_per_cell(net, codes: np.ndarray) -> float:
    """Algorithmic FLOPs of the affine chain per cell, from the cells' codes.

    Block (l <- j), j >= 1: 2 * 4 * n_l * (active units of layer j) (the four
    homogeneous columns; inactive units contribute exact zeros).  Blocks from
    the input (Z_0 = [I | 0]) are copies and count 0.
    """
    offs = np.cumsum([0] + net.widths[1:-1])
    N = net.n_hidden
    bits = np.unpackbits(codes.view(np.uint8), axis=1, bitorder="little")[:, :N].astype(np.float64)
    active = {}
    for j in range(1, len(net.widths) - 1):
        active[j] = bits[:, offs[j - 1]:offs[j - 1] + net.widths[j]].sum(axis=1).mean()
    total = 0.0
    for d, s, W in net.blocks:
        if s >= 1:
            total += 8.0 * net.widths[d] * active[s]
    return total


def cpu_baseline(net, o, d, budget_s: float):
    """The oracle (single thread, as it stands) on a BFS prefix of the workload."""
    from oracle import oracle as O
    on = O.OracleNet(net)
    t0 = time.perf_counter()
    codes, ams, pts, sts = on.seed_rays(o, d)
    t_seed = time.perf_counter() - t0
    # size the prefix from a short calibration run
    t1 = time.perf_counter()
    probe = on.march(codes, ams, max_cells=2000)
    dt = time.perf_counter() - t1
    per_cell = dt / max(1, probe.stats["cells"])
    cells = int(max(2000, min(2_000_000, budget_s / max(per_cell, 1e-7))))
    t2 = time.perf_counter()
    mesh = on.march(codes, ams, max_cells=cells)
    t_march = time.perf_counter() - t2
    faces = mesh.n_faces
    rate = faces / (t_seed + t_march)
    return {"value": rate, "unit": "faces/s", "cores": 1, "kind": "oracle",
            "sample": f"dichotomy seeding of {len(o)} rays ({t_seed:.2f} s) + FIFO march of the first "
                      f"{min(cells, mesh.stats['cells'])} cells ({faces} faces, {t_march:.2f} s), "
                      f"single-threaded C oracle, FP64"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--max-cells", type=int, default=1 << 21)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="plain,bf16", help="forms to time besides the plain one")
    a = ap.parse_args(argv)

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the marching path runs on a single MI355X "
              "(multi-GPU sharding is described in DESIGN.md, not built).", file=sys.stderr)
        return 2

    import torch
    from paper_2106_10031_amd import binding as B

    net, o, d, desc = workload(a.workload)
    ctx = B.Context(0).load_net(net)
    dev = torch.device("cuda", 0)
    o_d = torch.as_tensor(o, dtype=torch.float64, device=dev)
    d_d = torch.as_tensor(d, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def step(time_kernels=False, precision=0):
        ctx.seed_rays(o_d, d_d)
        st = ctx.march(max_cells=a.max_cells, time_kernels=time_kernels, precision=precision)
        out = ctx.fetch()
        return st, out

    def timed(precision):
        for _ in range(a.warmup):
            step(precision=precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for _ in range(a.steps):
            st, out = step(precision=precision)
            stats.append(st)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        f = stats[-1]["faces"]
        assert all(s["faces"] == f for s in stats), "face count changed between steps"
        return f, (t1 - t0) * 1e3 / a.steps, f * a.steps / (t1 - t0), stats

    faces, ms_per_step, value, stats = timed(0)
    forms = {"plain": {"faces_per_s": round(value, 1), "ms_per_step": round(ms_per_step, 3),
                       "precision": "FP64 chain (MFMA), FP64 clip and vertex solves"}}
    if "bf16" in a.forms.split(","):
        f16, ms16, v16, st16 = timed(1)
        assert f16 == faces, "split-BF16 form changed the face count"
        forms["bf16"] = {"faces_per_s": round(v16, 1), "ms_per_step": round(ms16, 3),
                         "escalated_cells": st16[-1]["escalated"],
                         "precision": "split-BF16 chain (3 terms, 6 MFMA products, FP32 accumulate); "
                                      "FP64 sign tests within margin 4e-6 + the vertex's error estimate and vertex solves; "
                                      "uncertified cells redone in FP64"}

    # per-kernel durations (HIP events on the library's stream), separate pass
    kst, kout = step(time_kernels=True)
    torch.cuda.synchronize()
    codes = kout["codes"].cpu().numpy().view(np.uint64)
    flops_cell = chain_flops_per_cell(net, codes)
    cells = kst["cells"]
    chain_avg_ms = kst["chain_ms"] / max(1, kst["chain_launches"])
    clip_avg_ms = kst["clip_ms"] / max(1, kst["clip_launches"])
    cells_per_launch = cells / max(1, kst["chain_launches"])
    chain_tflops = flops_cell * cells_per_launch / (chain_avg_ms * 1e-3) / 1e12 if chain_avg_ms > 0 else 0.0
    roofline = {"kernel": "k_chain_f64", "bound": "mfma", "achieved": round(chain_tflops, 4),
                "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": round(chain_tflops / PEAK_FP64_MFMA_TFLOPS, 6), "traffic": None,
                "algorithmic_per_cell": flops_cell, "cells_per_launch": round(cells_per_launch, 1),
                "avg_launch_ms": round(chain_avg_ms, 4),
                "time_split_ms": {"chain": round(kst["chain_ms"], 3), "clip": round(kst["clip_ms"], 3),
                                  "hash": round(kst["hash_ms"], 3), "march_total": round(kst["march_ms"], 3)}}
    if kst["clip_ms"] > kst["chain_ms"]:
        roofline["dominant_by_time"] = "k_clip_f64"

    res = {"metric": METRIC, "value": round(value, 1), "unit": "faces/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "forms": forms,
           "config": {"workload": desc, "form": "plain", "faces": faces, "face_verts": stats[-1]["face_verts"],
                      "triangles": stats[-1]["triangles"], "cells": stats[-1]["cells"],
                      "march_steps": stats[-1]["steps"], "seeds": stats[-1]["seed_cells"],
                      "degenerate": stats[-1]["degenerate"]},
           "roofline": roofline}
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(net, o, d, a.cpu_budget)
    print(json.dumps(res), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
